"""Naive separable DFT (test infrastructure, FP64).

Transform pair of the plane-wave basis (Hartree atomic units, grid
r_j = (j1 L1/N1, j2 L2/N2, j3 L3/N3)):

    f(G)   = (1/N) sum_j f(r_j) exp(-i G.r_j)        (to_reciprocal)
    f(r_j) =       sum_G f(G)   exp(+i G.r_j)        (to_real)

Each axis is applied as a dense n x n DFT matrix whose phases are reduced
exactly, (j*k mod n), before the cosine/sine, so the matrices are exact to
rounding. Arrays are C-order [..., N3, N2, N1] (x fastest); the output index
along an axis is the Miller index modulo N.

Parseval, inverse-after-forward and the single-plane-wave delta pin these
routines (tests/test_oracle_basis.py).

A second mode evaluates the same pair with scipy.fft (pocketfft, FP64) for
timing the oracle on the larger cells; it is used only by the benchmark's CPU
baseline and is checked equal to the dense-matrix mode to 1e-13 on grids up to
24^3 (tests/test_oracle_basis.py). Select it with set_mode("fft", workers).
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np


@lru_cache(maxsize=64)
def dft_matrix(n: int, sign: int) -> np.ndarray:
    """M[k, j] = exp(sign * 2 pi i * (j k mod n) / n)."""
    j = np.arange(n)
    jk = np.outer(j, j) % n
    ang = 2.0 * np.pi * jk / n
    return np.cos(ang) + (1j * sign) * np.sin(ang)


def _apply_axis(a: np.ndarray, axis: int, M: np.ndarray) -> np.ndarray:
    a = np.moveaxis(a, axis, -1)
    out = a @ M.T
    return np.moveaxis(out, -1, axis)


_MODE = {"kind": "naive", "workers": 1}


def set_mode(kind: str, workers: int = 1) -> None:
    """'naive' (dense per-axis DFT matrices, the parity mode) or 'fft' (scipy.fft)."""
    if kind not in ("naive", "fft"):
        raise ValueError(kind)
    _MODE["kind"] = kind
    _MODE["workers"] = int(workers)


def to_reciprocal(f: np.ndarray) -> np.ndarray:
    """(1/N) sum_j f(r_j) e^{-iG.r_j} over the last three axes [N3, N2, N1]."""
    if _MODE["kind"] == "fft":
        import scipy.fft as sf
        return sf.fftn(np.asarray(f, dtype=np.complex128), axes=(-3, -2, -1), norm="forward",
                       workers=_MODE["workers"])
    a = np.asarray(f, dtype=np.complex128)
    N3, N2, N1 = a.shape[-3:]
    a = _apply_axis(a, -1, dft_matrix(N1, -1))
    a = _apply_axis(a, -2, dft_matrix(N2, -1))
    a = _apply_axis(a, -3, dft_matrix(N3, -1))
    return a / (N1 * N2 * N3)


def to_real(F: np.ndarray) -> np.ndarray:
    """sum_G F(G) e^{+iG.r_j} over the last three axes [N3, N2, N1]."""
    if _MODE["kind"] == "fft":
        import scipy.fft as sf
        return sf.ifftn(np.asarray(F, dtype=np.complex128), axes=(-3, -2, -1), norm="forward",
                        workers=_MODE["workers"])
    a = np.asarray(F, dtype=np.complex128)
    N3, N2, N1 = a.shape[-3:]
    a = _apply_axis(a, -1, dft_matrix(N1, +1))
    a = _apply_axis(a, -2, dft_matrix(N2, +1))
    a = _apply_axis(a, -3, dft_matrix(N3, +1))
    return a
