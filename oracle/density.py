"""Subsystem density from bands (test infrastructure, FP64).

Sec. 2 defines rho_I(r) = (2/Omega_BZ) int_BZ dk sum_j n_jk |u_jk(r)|^2 with
0 <= n <= 1. On a k mesh with weights w_k (sum w_k = 1) and f = 2n in [0, 2]:

    rho_I(r_j) = sum_k w_k sum_n f_nk |u_nk(r_j)|^2,
    u(r) = Omega^{-1/2} sum_G c(G) e^{iG.r}.

The caller passes occw[n] = w_k f_nk for one k-point; contributions of the
k-points are summed.

Pins: charge conservation sum_j rho dV = sum occw; a single plane wave gives
the uniform density f/Omega (tests/test_oracle_basis.py).
"""
from __future__ import annotations

import numpy as np

from . import basis, dft


def density(cell: basis.Cell, sph: basis.Sphere, psi: np.ndarray, occw: np.ndarray) -> np.ndarray:
    """sum_n occw[n] |u_n(r)|^2 on the grid [N3, N2, N1]."""
    psi = np.asarray(psi, dtype=np.complex128).reshape(-1, sph.npw)
    u = dft.to_real(basis.to_grid(cell, sph, psi))
    return np.einsum("n,nzyx->zyx", np.asarray(occw, dtype=np.float64), np.abs(u) ** 2) / cell.omega
