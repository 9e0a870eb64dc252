"""H_I applied to plane-wave bands (test infrastructure, FP64).

Eq. KS: [-(nabla + ik)^2 / 2 + V_eff^I(r)] u = eps u, with the nonlocal
projectors of the subsystem's own atoms (Appendix, non-local
pseudopotentials). In the coefficients of u, for G in S_k:

    y(G) = |k+G|^2/2 c(G) + [DFT_fwd(V_eff * DFT_inv(c))](G)
           + sum_i beta_i(G) D_i <beta_i | c>

Pins: free electrons (constant V) give eigenvalues |k+G|^2/2 + V0; the
matrix-free product equals the explicit matrix
H_GG' = |k+G|^2/2 delta + V(m - m' mod N) + sum_i beta_i(G) D_i beta_i(G')^*;
Hermiticity; a rank-one projector adds D |<beta|psi>|^2
(tests/test_oracle_hamiltonian.py).
"""
from __future__ import annotations

import numpy as np

from . import basis, dft


def apply_h(cell: basis.Cell, sph: basis.Sphere, psi: np.ndarray, veff: np.ndarray,
            beta: np.ndarray | None = None, dkb: np.ndarray | None = None) -> np.ndarray:
    """H psi for band-major psi [nb, npw]; veff real [N3, N2, N1]."""
    psi = np.asarray(psi, dtype=np.complex128).reshape(-1, sph.npw)
    u = dft.to_real(basis.to_grid(cell, sph, psi))
    w = dft.to_reciprocal(np.asarray(veff, dtype=np.float64)[None] * u)
    y = basis.from_grid(sph, w) + sph.kin[None, :] * psi
    if beta is not None and len(beta):
        P = beta.conj() @ psi.T                       # [nproj, nb] = <beta_i | psi_n>
        y = y + (beta.T @ (np.asarray(dkb)[:, None] * P)).T
    return y


def explicit_h(cell: basis.Cell, sph: basis.Sphere, veff: np.ndarray,
               beta: np.ndarray | None = None, dkb: np.ndarray | None = None) -> np.ndarray:
    """Dense H_GG' [npw, npw] (small grids only)."""
    VG = dft.to_reciprocal(np.asarray(veff, dtype=np.float64))
    N1, N2, N3 = cell.grid
    m = sph.miller
    d1 = np.mod(m[:, None, 0] - m[None, :, 0], N1)
    d2 = np.mod(m[:, None, 1] - m[None, :, 1], N2)
    d3 = np.mod(m[:, None, 2] - m[None, :, 2], N3)
    H = VG[d3, d2, d1] + np.diag(sph.kin)
    if beta is not None and len(beta):
        H = H + (beta.T * np.asarray(dkb)[None, :]) @ beta.conj()
    return H


def kinetic_band(sph: basis.Sphere, psi: np.ndarray) -> np.ndarray:
    """<psi_n| -(nabla+ik)^2/2 |psi_n> per band (the Janak kinetic term, Sec. 2)."""
    return np.einsum("g,ng->n", sph.kin, np.abs(psi) ** 2)


def nonlocal_band(psi: np.ndarray, beta: np.ndarray | None, dkb: np.ndarray | None) -> np.ndarray:
    """sum_i D_i |<beta_i|psi_n>|^2 per band."""
    if beta is None or not len(beta):
        return np.zeros(psi.shape[0])
    P = beta.conj() @ psi.T
    return np.einsum("i,in->n", np.asarray(dkb), np.abs(P) ** 2)
