"""The C ABI: both builds load and export every symbol include/fde.h declares;
host-side argument checks return errors (CPU only, no compute on a GPU)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1406_7803_amd import fde

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fde.h")


def declared():
    src = open(HEADER).read()
    names = set(re.findall(r"^\s*(?:fde_status|void|const char\*)\s+(fde_\w+)\s*\(", src, re.M))
    return names


def exported(path):
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True, check=True).stdout
    return {line.split()[-1] for line in out.splitlines() if " T " in line}


@pytest.mark.parametrize("path", [fde.LIB_PATH, fde.EMU_PATH])
def test_library_exports_header(path):
    assert os.path.exists(path), f"{path} missing: run `python -m paper_1406_7803_amd.build`"
    names = declared()
    assert len(names) >= 19
    assert names <= exported(path)
    assert set(fde.SYMBOLS) == names
    lib = ctypes.CDLL(path)
    for n in names:
        getattr(lib, n)


def test_device_library_is_gfx950():
    # the offload bundle of our own build names its target
    assert b"amdgcn-amd-amdhsa--gfx950" in open(fde.LIB_PATH, "rb").read()


def test_plan_errors():
    be = fde.emulation_backend()
    with pytest.raises(fde.FdeError, match="product of 2, 3, 5"):
        fde.Plan((6.0, 6.0, 7.0), (12, 12, 14), 2.2, [(0, 0, 0)], backend=be)
    with pytest.raises(fde.FdeError, match="too small"):
        fde.Plan((10.0, 10.0, 10.0), (20, 24, 24), 7.0, [(0, 0, 0)], backend=be)
    with pytest.raises(fde.FdeError, match="prec"):
        fde.Plan((6.0, 6.0, 7.0), (12, 12, 15), 2.2, [(0, 0, 0)], prec=7, backend=be)
    p = fde.Plan((6.0, 6.0, 7.0), (12, 12, 15), 2.2, [(0, 0, 0)], max_nb=2, max_nproj=1, backend=be)
    psi = p.zeros_bands(2, 0)
    v = p.zeros_grid()
    with pytest.raises(fde.FdeError, match="max_nproj"):
        beta = p.zeros_bands(3, 0)
        p.apply_h(0, psi, v, beta, __import__("torch").zeros(3, dtype=__import__("torch").float64))
    with pytest.raises(fde.FdeError, match="k-point"):
        p.npw(3)
    with pytest.raises(fde.FdeError, match="m <= 2 max_nb"):
        p.subspace_rr(0, p.zeros_bands(5, 0), p.zeros_bands(5, 0), 2)
    with pytest.raises(fde.FdeError):
        p.apply_h(0, psi, v.to(dtype=__import__("torch").float32))


def test_empty_calls_are_noops():
    import torch
    be = fde.emulation_backend()
    p = fde.Plan((6.0, 6.0, 7.0), (12, 12, 15), 2.2, [(0, 0, 0)], max_nb=2, backend=be)
    psi = p.zeros_bands(0, 0)
    out = p.apply_h(0, psi, p.zeros_grid())
    assert out.shape == (0, p.npw(0))
    rho = p.zeros_grid()
    p.density(0, psi, torch.zeros(0, dtype=torch.float64), rho)
    assert float(rho.abs().sum()) == 0.0
