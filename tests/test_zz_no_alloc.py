"""The allocation-free loss/gradient entry point against the workspace one (GPU).

fde_mlp_loss_grad_static keeps its partial gradients in a scratch array the
library holds per GPU; it must give exactly what fde_mlp_loss_grad gives with a
caller workspace, call after call, also when a smaller call follows a larger one
(the array keeps the larger call's contents)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1406_7803_amd import fde

import parity_cases as pc

pytestmark = pytest.mark.gpu


def _pair(be, n, seed):
    S = pc.fdev(be, pc.mlp_samples(n, seed))
    th = pc.fdev(be, pc.mlp_params(seed + 1))
    tr = fde.MlpTrainer(be, S, th)
    loss_ref, grad_ref = tr.loss_grad()
    grad = torch.full((fde.MLP_NPARAM,), float("nan"), dtype=torch.float32, device=be.device)
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device=be.device)
    # through the C ABI directly (the binding only marshals the same pointers)
    st = be.lib.fde_mlp_loss_grad_static(n, ctypes.c_void_p(S.data_ptr()), ctypes.c_void_p(th.data_ptr()),
                                         ctypes.c_void_p(grad.data_ptr()), ctypes.c_void_p(loss.data_ptr()),
                                         be.stream())
    assert st == 0, be.lib.fde_last_error().decode()
    be.sync()
    return loss_ref.cpu().numpy(), grad_ref.cpu().numpy(), loss.cpu().numpy(), grad.cpu().numpy()


def test_static_scratch_matches_workspace_entry_point():
    be = fde.gpu_backend("cuda:0")
    # a large call, then a smaller one (fewer blocks than the first left in the array),
    # then a call that needs more samples per block than either
    for n, seed in ((70000, 301), (3000, 303), (200000, 305)):
        lr, gr, ls, gs = _pair(be, n, seed)
        assert np.isfinite(ls).all() and np.isfinite(gs).all()
        assert np.array_equal(ls, lr), (n, ls, lr)
        assert np.array_equal(gs, gr), (n, float(np.max(np.abs(gs - gr))))


def test_static_scratch_rejects_bad_sizes():
    be = fde.gpu_backend("cuda:0")
    z = ctypes.c_void_p(0)
    assert be.lib.fde_mlp_loss_grad_static(0, z, z, z, z, be.stream()) == -1
    assert be.lib.fde_mlp_loss_grad_static((1 << 28) + 1, z, z, z, z, be.stream()) == -2
