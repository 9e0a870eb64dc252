"""Python binding of the C ABI in include/fde.h (argument marshalling only).

PyTorch provides device memory and streams; every step of the method runs in
the HIP kernels of libfde.so. The binding raises if the library is missing:
there is no CPU path.

Names follow include/fde.h: ``Plan`` wraps fde_plan_* and the compute calls
are methods with the same names as the C functions minus the ``fde_`` prefix.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfde.so")
EMU_PATH = os.path.join(HERE, "libfde_emu.so")

F64, F32 = 0, 1
XC_NONE, XC_LDA, XC_PBE = 0, 1, 2
KIN_NONE, KIN_TF, KIN_LC94, KIN_REVAPBEK = 0, 1, 2, 3
OCC_INTEGER, OCC_FERMI_DIRAC, OCC_METHFESSEL_PAXTON = 0, 1, 2
PULAY_MAX = 8
NE = 8
E_XC, E_XCNAD, E_KIN, E_LOC, E_HEMB, E_HSELF, E_DEBAND, E_CHARGE = range(NE)

SYMBOLS = [
    "fde_last_error", "fde_plan_create", "fde_plan_destroy", "fde_plan_info", "fde_plan_miller",
    "fde_plan_workspace_bytes", "fde_plan_set_workspace", "fde_apply_h", "fde_density",
    "fde_embed_potential", "fde_subspace_rr", "fde_precondition", "fde_occupations", "fde_mix",
    "fde_local_potential", "fde_kb_projectors", "fde_init_bands", "fde_band_energies", "fde_grid_dot",
    "fde_subspace_rr_batched", "fde_precondition_batched", "fde_grid_mean", "fde_precondition_mlp_batched",
    "fde_mlp_forward", "fde_mlp_workspace_bytes", "fde_mlp_loss_grad", "fde_mlp_adam", "fde_plan_set_gemm_mode",
    "fde_plan_set_tuning", "fde_energy_total", "fde_mlp_loss_grad_static", "fde_mix_pulay", "fde_density_l1",
    "fde_frozen_environment", "fde_apply_s", "fde_aug_charges", "fde_aug_density",
]
TUNE_APPLY_BPW = 1
TUNE_STICK_GROUP = 2
TUNE_Z_REGISTER = 3
TUNE_PLANE_KIND = 4
TUNE_PLANE_ROWS = 5
TUNE_RR_SPLIT = 6
PLANE_REG, PLANE_LDS, PLANE_TWO_FACTOR = 1, 2, 3
GEMM_FP64, GEMM_BF16X3, GEMM_BF16X6 = 0, 1, 2
MLP_NPARAM, MLP_NIN, MLP_SAMPLE = 4545, 4, 7


class FdeError(RuntimeError):
    pass


class Functionals(ctypes.Structure):
    _fields_ = [("xc", ctypes.c_int), ("xc_nad", ctypes.c_int), ("kin_nad", ctypes.c_int),
                ("rho_thr", ctypes.c_double)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_S = ctypes.c_size_t


class Block(ctypes.Structure):
    """fde_block: one (subsystem, k-point) band block of the solver."""
    _fields_ = [("ik", _I), ("nb", _I), ("m", _I), ("v", _P), ("hv", _P), ("active", _P), ("t_active", _P),
                ("eval", _P), ("rnorm", _P), ("info", _P), ("sv", _P)]


def _declare(lib):
    lib.fde_last_error.restype = ctypes.c_char_p
    lib.fde_plan_create.argtypes = [_P, _P, _D, _I, _P, _I, ctypes.POINTER(_P)]
    lib.fde_plan_destroy.argtypes = [_P]
    lib.fde_plan_destroy.restype = None
    lib.fde_plan_info.argtypes = [_P, _I, _P, _P]
    lib.fde_plan_miller.argtypes = [_P, _I, _P]
    lib.fde_plan_workspace_bytes.argtypes = [_P, _I, _I, _I, ctypes.POINTER(_S)]
    lib.fde_plan_set_workspace.argtypes = [_P, _P, _S, _I, _I, _I]
    lib.fde_subspace_rr_batched.argtypes = [_P, _I, _P, _D, _P]
    lib.fde_precondition_batched.argtypes = [_P, _I, _P, _P]
    lib.fde_apply_h.argtypes = [_P, _I, _I, _P, _P, _P, _I, _P, _P, _P]
    lib.fde_density.argtypes = [_P, _I, _I, _P, _P, _P, _P]
    lib.fde_embed_potential.argtypes = [_P, _I, _P, _P, ctypes.POINTER(Functionals), _P, _P, _P, _P]
    lib.fde_subspace_rr.argtypes = [_P, _I, _I, _I, _P, _P, _P, _D, _P, _P, _P]
    lib.fde_precondition.argtypes = [_P, _I, _I, _P, _P, _P, _P, _P, _P, _P]
    lib.fde_occupations.argtypes = [_I, _I, _P, _P, _D, _I, _D, _P, _P, _P, _P]
    lib.fde_mix.argtypes = [_S, _D, _P, _P, _I, _P]
    lib.fde_mix_pulay.argtypes = [_P, _I, _I, _P, _P, _P, _P, _P, _D, _D, _P, _P]
    lib.fde_local_potential.argtypes = [_P, _I, _P, _P, _P, _P, _P]
    lib.fde_kb_projectors.argtypes = [_P, _I, _I, _P, _P, _P, _P, _P, _P]
    lib.fde_init_bands.argtypes = [_P, _I, _I, _P, _P, _P]
    lib.fde_band_energies.argtypes = [_P, _I, _I, _P, _P, _P, _I, _P, _P, _P, _P]
    lib.fde_energy_total.argtypes = [_I, _P, _P, _P, _P, _P]
    lib.fde_grid_dot.argtypes = [_P, _P, _P, _P, _P]
    lib.fde_grid_mean.argtypes = [_P, _P, _P, _P]
    lib.fde_density_l1.argtypes = [_P, _I, _P, _P, _P, _P]
    lib.fde_frozen_environment.argtypes = [_P, _I, _P, _P, _S, _P]
    lib.fde_apply_s.argtypes = [_P, _I, _I, _P, _P, _I, _P, _P, _P]
    lib.fde_aug_charges.argtypes = [_P, _I, _I, _P, _P, _I, _P, _P, _P, _P, _P]
    lib.fde_aug_density.argtypes = [_P, _I, _P, _P, _P, _P]
    lib.fde_plan_set_gemm_mode.argtypes = [_P, _I]
    lib.fde_plan_set_tuning.argtypes = [_P, _I, _I]
    lib.fde_precondition_mlp_batched.argtypes = [_P, _I, _P, _P, _P, _P]
    lib.fde_mlp_forward.argtypes = [_I, _P, _P, _P, _P]
    lib.fde_mlp_workspace_bytes.argtypes = [_I, ctypes.POINTER(_S)]
    lib.fde_mlp_loss_grad.argtypes = [_I, _P, _P, _P, _P, _P, _S, _P]
    lib.fde_mlp_loss_grad_static.argtypes = [_I, _P, _P, _P, _P, _P]
    _F = ctypes.c_float
    lib.fde_mlp_adam.argtypes = [_P, _P, _P, _P, _I, _F, _F, _F, _F, _P]
    for name in SYMBOLS:
        if name not in ("fde_last_error", "fde_plan_destroy"):
            getattr(lib, name).restype = _I
    return lib


_LIBS = {}


def load(path: str = LIB_PATH):
    """Load a build of the library (default: the gfx950 product library)."""
    if path in _LIBS:
        return _LIBS[path]
    if not os.path.exists(path):
        raise FdeError(f"{path} not found: build it with `python -m paper_1406_7803_amd.build`")
    lib = _declare(ctypes.CDLL(path))
    _LIBS[path] = lib
    return lib


class Backend:
    """Where buffers live and which library runs the kernels."""

    def __init__(self, lib, device: torch.device, emulated: bool):
        self.lib = lib
        self.device = device
        self.emulated = emulated

    def stream(self):
        if self.emulated:
            return None
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def sync(self):
        if not self.emulated:
            torch.cuda.synchronize(self.device)


def gpu_backend(device="cuda:0") -> Backend:
    if not torch.cuda.is_available():
        raise FdeError("no GPU visible: the library runs on MI355X (gfx950) only")
    return Backend(load(LIB_PATH), torch.device(device), emulated=False)


def emulation_backend() -> Backend:
    """Host emulation of the kernels, for the CPU test suite only."""
    return Backend(load(EMU_PATH), torch.device("cpu"), emulated=True)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Plan:
    """fde_plan_create + an attached workspace tensor owned by this object."""

    def __init__(self, L: Sequence[float], grid: Sequence[int], ecut: float, kfrac, prec: int = F64,
                 max_nb: int = 64, max_nproj: int = 0, max_batch: int = 1, backend: Optional[Backend] = None):
        self.be = backend or gpu_backend()
        self.lib = self.be.lib
        kf = np.ascontiguousarray(np.asarray(kfrac, dtype=np.float64).reshape(-1, 3))
        Lc = (ctypes.c_double * 3)(*[float(x) for x in L])
        gc = (ctypes.c_int * 3)(*[int(n) for n in grid])
        h = ctypes.c_void_p()
        self._check(self.lib.fde_plan_create(Lc, gc, float(ecut), len(kf), kf.ctypes.data_as(_P), int(prec),
                                             ctypes.byref(h)))
        self.h = h
        self.L = tuple(float(x) for x in L)
        self.grid = tuple(int(n) for n in grid)
        self.ecut = float(ecut)
        self.kfrac = kf
        self.prec = prec
        self.rdtype = torch.float64 if prec == F64 else torch.float32
        self.cdtype = torch.complex128 if prec == F64 else torch.complex64
        self.max_nb = max_nb
        self.max_nproj = max_nproj
        self.max_batch = max_batch
        nbytes = ctypes.c_size_t()
        self._check(self.lib.fde_plan_workspace_bytes(self.h, max_nb, max_nproj, max_batch, ctypes.byref(nbytes)))
        self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.be.device)
        base = self.ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._check(self.lib.fde_plan_set_workspace(self.h, ctypes.c_void_p(aligned), nbytes.value, max_nb,
                                                    max_nproj, max_batch))

    # -- helpers ---------------------------------------------------------------
    def _check(self, st: int):
        if st != 0:
            raise FdeError(f"fde error {st}: {self.lib.fde_last_error().decode()}")

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.fde_plan_destroy(self.h)
                self.h = None
        except Exception:
            pass

    @property
    def shape(self):
        N1, N2, N3 = self.grid
        return (N3, N2, N1)

    def npw(self, ik: int) -> int:
        n = ctypes.c_int()
        self._check(self.lib.fde_plan_info(self.h, ik, ctypes.byref(n), None))
        return n.value

    def ncol(self, ik: int) -> int:
        n = ctypes.c_int()
        self._check(self.lib.fde_plan_info(self.h, ik, None, ctypes.byref(n)))
        return n.value

    def miller(self, ik: int) -> np.ndarray:
        out = np.zeros((self.npw(ik), 3), dtype=np.int32)
        self._check(self.lib.fde_plan_miller(self.h, ik, out.ctypes.data_as(_P)))
        return out

    def zeros_bands(self, nb: int, ik: int) -> torch.Tensor:
        return torch.zeros((nb, self.npw(ik)), dtype=self.cdtype, device=self.be.device)

    def zeros_grid(self, *lead) -> torch.Tensor:
        return torch.zeros(tuple(lead) + self.shape, dtype=self.rdtype, device=self.be.device)

    def _bands(self, t: torch.Tensor, ik: int, name: str):
        if t.dtype != self.cdtype or not t.is_contiguous() or t.device != self.be.device:
            raise FdeError(f"{name}: expected a contiguous {self.cdtype} tensor on {self.be.device}")
        if t.shape[-1] != self.npw(ik):
            raise FdeError(f"{name}: last dimension {t.shape[-1]} != npw {self.npw(ik)}")

    def _grid(self, t: torch.Tensor, name: str):
        if t.dtype != self.rdtype or not t.is_contiguous() or t.device != self.be.device:
            raise FdeError(f"{name}: expected a contiguous {self.rdtype} tensor on {self.be.device}")
        if tuple(t.shape[-3:]) != self.shape:
            raise FdeError(f"{name}: grid shape {tuple(t.shape[-3:])} != {self.shape}")

    def _f64(self, t: torch.Tensor, name: str):
        if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.be.device:
            raise FdeError(f"{name}: expected a contiguous float64 tensor on {self.be.device}")

    # -- the C ABI -------------------------------------------------------------
    def apply_h(self, ik: int, psi: torch.Tensor, veff: torch.Tensor, beta=None, dkb=None, out=None):
        self._bands(psi, ik, "psi")
        self._grid(veff, "veff")
        nb = psi.shape[0]
        out = torch.empty_like(psi) if out is None else out
        self._bands(out, ik, "hpsi")
        nproj = 0 if beta is None else beta.shape[0]
        if nproj:
            self._bands(beta, ik, "beta")
            self._f64(dkb, "dkb")
        self._check(self.lib.fde_apply_h(self.h, ik, nb, _ptr(psi), _ptr(out), _ptr(veff), nproj,
                                         _ptr(beta) if nproj else None, _ptr(dkb) if nproj else None,
                                         self.be.stream()))
        return out

    def density(self, ik: int, psi: torch.Tensor, occw: torch.Tensor, rho: torch.Tensor):
        self._bands(psi, ik, "psi")
        self._f64(occw, "occw")
        self._grid(rho, "rho")
        if occw.numel() < psi.shape[0]:
            raise FdeError("occw shorter than the number of bands")
        self._check(self.lib.fde_density(self.h, ik, psi.shape[0], _ptr(psi), _ptr(occw), _ptr(rho),
                                         self.be.stream()))
        return rho

    def embed_potential(self, rho_sub: torch.Tensor, vloc: torch.Tensor, xc=XC_LDA, xc_nad=XC_LDA,
                        kin_nad=KIN_LC94, rho_thr=1e-10, veff=None, energies=None, info=None):
        self._grid(rho_sub, "rho_sub")
        self._grid(vloc, "vloc")
        ns = rho_sub.shape[0]
        veff = torch.empty_like(rho_sub) if veff is None else veff
        self._grid(veff, "veff")
        dev = self.be.device
        energies = torch.zeros((ns + 1, NE), dtype=torch.float64, device=dev) if energies is None else energies
        info = torch.zeros(1, dtype=torch.int32, device=dev) if info is None else info
        f = Functionals(int(xc), int(xc_nad), int(kin_nad), float(rho_thr))
        self._check(self.lib.fde_embed_potential(self.h, ns, _ptr(rho_sub), _ptr(vloc), ctypes.byref(f),
                                                 _ptr(veff), _ptr(energies), _ptr(info), self.be.stream()))
        return veff, energies, info

    def subspace_rr(self, ik: int, v: torch.Tensor, hv: torch.Tensor, nb: int, active=None, drop_tol=1e-10,
                    eval=None, info=None):
        self._bands(v, ik, "v")
        self._bands(hv, ik, "hv")
        m = v.shape[0]
        dev = self.be.device
        eval = torch.empty(nb, dtype=torch.float64, device=dev) if eval is None else eval
        info = torch.zeros(1, dtype=torch.int32, device=dev) if info is None else info
        if active is not None and (active.dtype != torch.uint8 or active.numel() < m):
            raise FdeError("active must be a uint8 tensor of length m")
        self._check(self.lib.fde_subspace_rr(self.h, ik, m, nb, _ptr(v), _ptr(hv), _ptr(active), float(drop_tol),
                                             _ptr(eval), _ptr(info), self.be.stream()))
        return eval, info

    def subspace_rr_batched(self, blocks, drop_tol=1e-10):
        """blocks: list of Block (see make_block)."""
        arr = (Block * len(blocks))(*blocks)
        self._check(self.lib.fde_subspace_rr_batched(self.h, len(blocks), arr, float(drop_tol), self.be.stream()))

    def precondition_batched(self, blocks):
        arr = (Block * len(blocks))(*blocks)
        self._check(self.lib.fde_precondition_batched(self.h, len(blocks), arr, self.be.stream()))

    def make_block(self, ik: int, nb: int, m: int, v, hv, active=None, t_active=None, eval=None, rnorm=None,
                   info=None, sv=None) -> Block:
        """sv: the rows S v of a generalised problem (fde_apply_s), or None (S = 1)."""
        self._bands(v, ik, "v")
        self._bands(hv, ik, "hv")
        if v.shape[0] < m or hv.shape[0] < m:
            raise FdeError("block: v and hv need m rows")
        if sv is not None:
            self._bands(sv, ik, "sv")
            if sv.shape[0] < m:
                raise FdeError("block: sv needs m rows")
        return Block(ik, nb, m, v.data_ptr(), hv.data_ptr(), None if active is None else active.data_ptr(),
                     None if t_active is None else t_active.data_ptr(), None if eval is None else eval.data_ptr(),
                     None if rnorm is None else rnorm.data_ptr(), None if info is None else info.data_ptr(),
                     None if sv is None else sv.data_ptr())

    def precondition(self, ik: int, x: torch.Tensor, hx: torch.Tensor, eval: torch.Tensor, t: torch.Tensor,
                     active: torch.Tensor, rnorm: torch.Tensor):
        for a, nme in ((x, "x"), (hx, "hx"), (t, "t")):
            self._bands(a, ik, nme)
        self._f64(eval, "eval")
        self._f64(rnorm, "rnorm")
        self._check(self.lib.fde_precondition(self.h, ik, x.shape[0], _ptr(x), _ptr(hx), _ptr(eval), _ptr(t),
                                              _ptr(active), _ptr(rnorm), self.be.stream()))

    def local_potential(self, pos, Z, width, vloc=None):
        pos = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 3))
        Z = np.ascontiguousarray(np.asarray(Z, dtype=np.float64))
        width = np.ascontiguousarray(np.asarray(width, dtype=np.float64))
        vloc = self.zeros_grid() if vloc is None else vloc
        self._check(self.lib.fde_local_potential(self.h, len(pos), pos.ctypes.data_as(_P), Z.ctypes.data_as(_P),
                                                 width.ctypes.data_as(_P), _ptr(vloc), self.be.stream()))
        return vloc

    def kb_projectors(self, ik: int, pos, lmax, rbeta):
        pos = np.ascontiguousarray(np.asarray(pos, dtype=np.float64).reshape(-1, 3))
        lmax = np.ascontiguousarray(np.asarray(lmax, dtype=np.int32))
        rbeta = np.ascontiguousarray(np.asarray(rbeta, dtype=np.float64))
        nproj = int(sum(0 if l < 0 else (1 if l == 0 else 4) for l in lmax))
        beta = self.zeros_bands(max(nproj, 1), ik)
        n = ctypes.c_int()
        self._check(self.lib.fde_kb_projectors(self.h, ik, len(pos), pos.ctypes.data_as(_P),
                                               lmax.ctypes.data_as(_P), rbeta.ctypes.data_as(_P), _ptr(beta),
                                               ctypes.byref(n), self.be.stream()))
        return beta[:n.value]

    def init_bands(self, ik: int, raw: torch.Tensor, out=None):
        self._bands(raw, ik, "raw")
        out = torch.empty_like(raw) if out is None else out
        self._check(self.lib.fde_init_bands(self.h, ik, raw.shape[0], _ptr(raw), _ptr(out), self.be.stream()))
        return out

    def band_energies(self, ik: int, psi, occw, beta=None, dkb=None, out=None, eval=None):
        """out[0] += sum_n occw_n T_n (kinetic), out[1] += sum_n occw_n E_NL,n (nonlocal),
        out[2] += sum_n occw_n eval_n (when eval is given)."""
        self._bands(psi, ik, "psi")
        self._f64(occw, "occw")
        if occw.numel() < psi.shape[0]:
            raise FdeError("occw shorter than the number of bands")
        if psi.shape[0] > self.max_nb:
            raise FdeError("band_energies: more bands than the workspace's max_nb")
        nout = 2 if eval is None else 3
        out = torch.zeros(nout, dtype=torch.float64, device=self.be.device) if out is None else out
        self._f64(out, "out")
        if out.numel() < nout:
            raise FdeError(f"out needs {nout} values")
        if eval is not None:
            self._f64(eval, "eval")
            if eval.numel() < psi.shape[0]:
                raise FdeError("eval shorter than the number of bands")
        nproj = 0 if beta is None else beta.shape[0]
        if nproj:
            self._bands(beta, ik, "beta")
            self._f64(dkb, "dkb")
            if dkb.numel() < nproj:
                raise FdeError("dkb shorter than the number of projectors")
        self._check(self.lib.fde_band_energies(self.h, ik, psi.shape[0], _ptr(psi), _ptr(occw), _ptr(eval), nproj,
                                               _ptr(beta) if nproj else None, _ptr(dkb) if nproj else None,
                                               _ptr(out), self.be.stream()))
        return out

    def grid_dot(self, a, b, out=None):
        """out[0] += sum_j a_j b_j dV (b None: b = 1)."""
        self._grid(a, "a")
        if b is not None:
            self._grid(b, "b")
        out = torch.zeros(1, dtype=torch.float64, device=self.be.device) if out is None else out
        self._f64(out, "out")
        self._check(self.lib.fde_grid_dot(self.h, _ptr(a), _ptr(b), _ptr(out), self.be.stream()))
        return out

    def set_tuning(self, key: int, value: int):
        self._check(self.lib.fde_plan_set_tuning(self.h, int(key), int(value)))

    def set_gemm_mode(self, mode: int):
        """Arithmetic of the Rayleigh-Ritz subspace products (GEMM_FP64, GEMM_BF16X3, GEMM_BF16X6)."""
        self._check(self.lib.fde_plan_set_gemm_mode(self.h, int(mode)))

    def density_l1(self, rho_sub, rho_ref, out=None):
        """out[0] += int |sum_I rho_sub[I] - rho_ref| dV (rho_sub [ns][N] or [N])."""
        self._grid(rho_sub, "rho_sub")
        self._grid(rho_ref, "rho_ref")
        if rho_ref.numel() != int(np.prod(self.shape)):
            raise FdeError("rho_ref must be one grid")
        ns = rho_sub.numel() // int(np.prod(self.shape))
        out = torch.zeros(1, dtype=torch.float64, device=self.be.device) if out is None else out
        self._f64(out, "out")
        self._check(self.lib.fde_density_l1(self.h, ns, _ptr(rho_sub), _ptr(rho_ref), _ptr(out), self.be.stream()))
        return out

    def apply_s(self, ik: int, psi: torch.Tensor, beta, q, out=None):
        """out = S psi = psi + beta q beta^H psi (q: float64 [nproj][nproj] device)."""
        self._bands(psi, ik, "psi")
        out = torch.empty_like(psi) if out is None else out
        self._bands(out, ik, "out")
        nproj = 0 if beta is None else beta.shape[0]
        if nproj:
            self._bands(beta, ik, "beta")
            self._f64(q, "q")
            if tuple(q.shape) != (nproj, nproj):
                raise FdeError("q must be [nproj][nproj]")
        self._check(self.lib.fde_apply_s(self.h, ik, psi.shape[0], _ptr(psi), _ptr(out), nproj, _ptr(beta),
                                         _ptr(q), self.be.stream()))
        return out

    def aug_charges(self, ik: int, psi: torch.Tensor, occw, beta, q, atom_of, charges):
        """charges[atom_of[i]] += sum_n occw_n Re(conj(P_in) (q P)_in), P = beta^H psi."""
        self._bands(psi, ik, "psi")
        self._bands(beta, ik, "beta")
        self._f64(occw, "occw")
        self._f64(q, "q")
        self._f64(charges, "charges")
        if atom_of.dtype != torch.int32 or atom_of.numel() != beta.shape[0]:
            raise FdeError("atom_of must be int32 [nproj]")
        if occw.numel() < psi.shape[0]:
            raise FdeError("occw needs one weight per band")
        self._check(self.lib.fde_aug_charges(self.h, ik, psi.shape[0], _ptr(psi), _ptr(occw), beta.shape[0],
                                             _ptr(beta), _ptr(q), _ptr(atom_of), _ptr(charges), self.be.stream()))
        return charges

    def aug_density(self, atoms, charges, rho):
        """rho += sum_a c_a g_a (atoms: float64 [natom][4] = x, y, z, width, on the device)."""
        self._f64(atoms, "atoms")
        self._f64(charges, "charges")
        self._grid(rho, "rho")
        if atoms.dim() != 2 or atoms.shape[1] != 4 or charges.numel() != atoms.shape[0]:
            raise FdeError("atoms must be [natom][4] with one charge each")
        self._check(self.lib.fde_aug_density(self.h, atoms.shape[0], _ptr(atoms), _ptr(charges), _ptr(rho),
                                             self.be.stream()))
        return rho

    def frozen_environment(self, rho_sub, out):
        """out[I] = sum_{J != I} rho_sub[J] (out [ns][N]), or into the second density of
        [ns][2][N] pairs {rho_I, env_I}."""
        self._grid(rho_sub, "rho_sub")
        self._grid(out, "out")
        n = int(np.prod(self.shape))
        ns = rho_sub.numel() // n
        if out.shape[0] != ns or out.numel() not in (ns * n, 2 * ns * n):
            raise FdeError("out must be [ns][N] or [ns][2][N]")
        ld = out.numel() // ns
        dst = out if ld == n else out[:, 1]
        self._check(self.lib.fde_frozen_environment(self.h, ns, _ptr(rho_sub), dst.data_ptr(), ld,
                                                    self.be.stream()))
        return out

    def grid_mean(self, a, out=None):
        self._grid(a, "a")
        out = torch.zeros(1, dtype=torch.float64, device=self.be.device) if out is None else out
        self._check(self.lib.fde_grid_mean(self.h, _ptr(a), _ptr(out), self.be.stream()))
        return out

    def mix_pulay(self, state: torch.Tensor, x_hist: torch.Tensor, r_hist: torch.Tensor, rho_in: torch.Tensor,
                  rho_out: torch.Tensor, beta: float, q0: float, info=None):
        """fde_mix_pulay: state int32 [3] (zero to start), histories [nhmax][ns][N3][N2][N1]."""
        self._grid(rho_in, "rho_in")
        self._grid(rho_out, "rho_out")
        self._grid(x_hist, "x_hist")
        self._grid(r_hist, "r_hist")
        ns = rho_in.shape[0] if rho_in.dim() == 4 else 1
        nhmax = x_hist.shape[0]
        if x_hist.shape != r_hist.shape or x_hist.numel() != nhmax * rho_in.numel() or rho_out.shape != rho_in.shape:
            raise FdeError("x_hist, r_hist must be [nhmax] + rho_in.shape")
        if state.dtype != torch.int32 or state.numel() < 3 or state.device != self.be.device:
            raise FdeError("state must be an int32 device tensor of 3 values")
        info = torch.zeros(1, dtype=torch.int32, device=self.be.device) if info is None else info
        self._check(self.lib.fde_mix_pulay(self.h, ns, nhmax, _ptr(state), _ptr(x_hist), _ptr(r_hist), _ptr(rho_in),
                                           _ptr(rho_out), float(beta), float(q0), _ptr(info), self.be.stream()))
        return rho_in, info

    def precondition_mlp_batched(self, blocks, params: torch.Tensor, vbar: torch.Tensor):
        """fde_precondition_batched with the learned network; vbar: [len(blocks)] float64 device."""
        _check_params(params, self.be)
        self._f64(vbar, "vbar")
        if vbar.numel() < len(blocks):
            raise FdeError("vbar needs one value per block")
        arr = (Block * len(blocks))(*blocks)
        self._check(self.lib.fde_precondition_mlp_batched(self.h, len(blocks), arr, _ptr(params), _ptr(vbar),
                                                          self.be.stream()))


def occupations(be: Backend, eval: torch.Tensor, wk: torch.Tensor, nelec: float, mode: int, sigma: float,
                occw=None, mu=None, info=None):
    nk, nb = eval.shape
    dev = be.device
    occw = torch.empty((nk, nb), dtype=torch.float64, device=dev) if occw is None else occw
    mu = torch.empty(1, dtype=torch.float64, device=dev) if mu is None else mu
    info = torch.zeros(1, dtype=torch.int32, device=dev) if info is None else info
    st = be.lib.fde_occupations(nk, nb, _ptr(eval), _ptr(wk), float(nelec), int(mode), float(sigma), _ptr(occw),
                                _ptr(mu), _ptr(info), be.stream())
    if st != 0:
        raise FdeError(f"fde error {st}: {be.lib.fde_last_error().decode()}")
    return occw, mu, info


def energy_total(be: Backend, embed_energies: torch.Tensor, band_terms: torch.Tensor, dots: torch.Tensor,
                 out=None) -> torch.Tensor:
    """fde_energy_total: [ns+4] = (E_K per subsystem, T^nad, E_xc^nad, E_FDE direct, E_FDE via fragments)."""
    ns = band_terms.shape[0]
    for t, shape, nme in ((embed_energies, (ns + 1, NE), "embed_energies"), (band_terms, (ns, 3), "band_terms"),
                          (dots, (ns, 2), "dots")):
        if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != shape or t.device != be.device:
            raise FdeError(f"{nme}: expected a contiguous float64 tensor {shape} on {be.device}")
    out = torch.zeros(ns + 4, dtype=torch.float64, device=be.device) if out is None else out
    if out.dtype != torch.float64 or out.numel() < ns + 4 or out.device != be.device:
        raise FdeError("out: expected float64 [ns+4]")
    st = be.lib.fde_energy_total(ns, _ptr(embed_energies), _ptr(band_terms), _ptr(dots), _ptr(out), be.stream())
    if st != 0:
        raise FdeError(f"fde error {st}: {be.lib.fde_last_error().decode()}")
    return out


def mix(be: Backend, rho_in: torch.Tensor, rho_out: torch.Tensor, beta: float):
    prec = F64 if rho_in.dtype == torch.float64 else F32
    st = be.lib.fde_mix(rho_in.numel(), float(beta), _ptr(rho_in), _ptr(rho_out), prec, be.stream())
    if st != 0:
        raise FdeError(f"fde error {st}: {be.lib.fde_last_error().decode()}")
    return rho_in


# ---------------------------------------------------------------------------
# Learned preconditioner network (FP32 parameters, layout of FDE_MLP_NPARAM)
# ---------------------------------------------------------------------------
def _check_params(params: torch.Tensor, be: Backend):
    if params.dtype != torch.float32 or params.numel() != MLP_NPARAM or not params.is_contiguous():
        raise FdeError(f"params must be a contiguous float32 vector of {MLP_NPARAM}")
    if params.device != be.device:
        raise FdeError("params on the wrong device")


def _raise(be: Backend, st: int):
    if st != 0:
        raise FdeError(f"fde error {st}: {be.lib.fde_last_error().decode()}")


def mlp_forward(be: Backend, u: torch.Tensor, params: torch.Tensor, y=None) -> torch.Tensor:
    """y[s] = network(u[s]) for u [n][4] float32."""
    _check_params(params, be)
    if u.dtype != torch.float32 or u.dim() != 2 or u.shape[1] != MLP_NIN or not u.is_contiguous():
        raise FdeError("u must be contiguous float32 [n][4]")
    y = torch.empty(u.shape[0], dtype=torch.float32, device=be.device) if y is None else y
    _raise(be, be.lib.fde_mlp_forward(u.shape[0], _ptr(u), _ptr(params), _ptr(y), be.stream()))
    return y


def mlp_loss_grad_static(be: Backend, samples: torch.Tensor, params: torch.Tensor, grad: torch.Tensor,
                         loss: torch.Tensor):
    """fde_mlp_loss_grad_static: loss and gradient with the library's own scratch (no
    workspace, nothing allocated; for callers that cannot allocate)."""
    _check_params(params, be)
    if samples.dtype != torch.float32 or samples.dim() != 2 or samples.shape[1] != MLP_SAMPLE \
            or not samples.is_contiguous() or samples.device != be.device:
        raise FdeError("samples must be contiguous float32 [n][7] on the backend's device")
    if grad.dtype != torch.float32 or grad.numel() != MLP_NPARAM or not grad.is_contiguous():
        raise FdeError(f"grad must be a contiguous float32 vector of {MLP_NPARAM}")
    if loss.dtype != torch.float64 or loss.numel() < 1:
        raise FdeError("loss must be a float64 tensor")
    _raise(be, be.lib.fde_mlp_loss_grad_static(samples.shape[0], _ptr(samples), _ptr(params), _ptr(grad),
                                               _ptr(loss), be.stream()))
    return loss, grad


class MlpTrainer:
    """Loss/gradient passes and Adam steps on one sample set (all on the device)."""

    def __init__(self, be: Backend, samples: torch.Tensor, params: torch.Tensor, lr=1e-3, beta1=0.9, beta2=0.999,
                 eps=1e-8):
        _check_params(params, be)
        if samples.dtype != torch.float32 or samples.dim() != 2 or samples.shape[1] != MLP_SAMPLE \
                or not samples.is_contiguous():
            raise FdeError("samples must be contiguous float32 [n][7]")
        self.be, self.samples, self.params = be, samples, params
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps
        n = samples.shape[0]
        nbytes = ctypes.c_size_t()
        _raise(be, be.lib.fde_mlp_workspace_bytes(n, ctypes.byref(nbytes)))
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=be.device)
        self.grad = torch.zeros(MLP_NPARAM, dtype=torch.float32, device=be.device)
        self.m = torch.zeros_like(self.grad)
        self.v = torch.zeros_like(self.grad)
        self.loss = torch.zeros(1, dtype=torch.float64, device=be.device)
        self.t = 0

    def loss_grad(self):
        n = self.samples.shape[0]
        _raise(self.be, self.be.lib.fde_mlp_loss_grad(n, _ptr(self.samples), _ptr(self.params), _ptr(self.grad),
                                                      _ptr(self.loss), _ptr(self.ws), self.ws.numel(),
                                                      self.be.stream()))
        return self.loss, self.grad

    def step(self):
        """One full-batch loss/gradient pass and one Adam step."""
        self.loss_grad()
        self.t += 1
        _raise(self.be, self.be.lib.fde_mlp_adam(_ptr(self.grad), _ptr(self.params), _ptr(self.m), _ptr(self.v),
                                                 self.t, self.lr, self.beta1, self.beta2, self.eps,
                                                 self.be.stream()))
        return self.loss
