"""Embedding potential of every subsystem (test infrastructure, FP64).

Appendix, recast of the effective potential: with the Hartree potential of
the total density computed by a Fourier-space Poisson solve (Sec. 2, the
plane-wave Hartree remark), the effective potential of subsystem I is

    V_eff^I = V_eN + V_H[rho] + V_XC[rho_I] + V_kin^nad[rho, rho_I] + V_XC^nad[rho, rho_I]

where V_eN groups all nuclei, V_kin^nad = dT/drho[rho] - dT/drho[rho_I] and
V_XC^nad = dE~xc/drho[rho] - dE~xc/drho[rho_I] (Eq. embedding), and
rho = sum_I rho_I (Eq. int1).

Discretisation: V_H(G) = 4 pi rho(G) / |G|^2 on D without G = 0; gradients
and divergences are spectral, grad X = DFT_inv(i G X(G)) and
div h = DFT_inv(sum_i i G_i h_i(G)), both over G in D only, which makes -div
the exact adjoint of grad on the grid. The kinetic potential follows the
appendix's functional derivative (dG/drho - div dG/dgrad rho) in the regular
form h = C_TF C_s^2 (F'(s)/s) grad X / X.

Energies per row (subsystems 0..ns-1, then the total density in row ns):
    0 E_xc[X]            1 E~xc[X] (nonadditive xc functional)
    2 T~[X] (KEDF)       3 int V_loc X
    4 int V_H[rho] X     5 E_H[X] = 1/2 int V_H[X] X
    6 -int (V_eff^I - V_loc) rho_I  (the band-energy correction of the
      Appendix recast of the total energy; zero in the total row)
    7 int X

Pins: Hartree energy of a Gaussian charge against the direct lattice sum;
uniform-density Thomas-Fermi energy and potential; T^nad[rho_A, 0] = 0;
finite differences of the total potential energy against every V_eff^I
(tests/test_oracle_embed.py).
"""
from __future__ import annotations

import math

import numpy as np

from . import basis, dft, functionals as fn

NE = 8
E_XC, E_XCT, E_KIN, E_LOC, E_HEMB, E_HSELF, E_DEBAND, E_CHARGE = range(NE)


def _g(cell, ecut):
    g1, g2, g3 = basis.grid_g(cell)
    mask = basis.density_mask(cell, ecut)
    return (g1, g2, g3), mask


def hartree(cell: basis.Cell, ecut: float, rho: np.ndarray):
    """(V_H(r), E_H) of a real density on the grid."""
    (g1, g2, g3), mask = _g(cell, ecut)
    G2 = g1 * g1 + g2 * g2 + g3 * g3
    rG = dft.to_reciprocal(rho)
    nz = mask & (G2 > 0)
    VG = np.zeros_like(rG)
    VG[nz] = 4.0 * math.pi * rG[nz] / G2[nz]
    V = dft.to_real(VG).real
    return V, 0.5 * float(np.sum(V * rho)) * cell.dV


def hartree_energy(cell: basis.Cell, ecut: float, rho: np.ndarray) -> float:
    """E_H = (Omega/2) sum_{G in D, G != 0} 4 pi |rho(G)|^2 / |G|^2, in Fourier space."""
    (g1, g2, g3), mask = _g(cell, ecut)
    G2 = g1 * g1 + g2 * g2 + g3 * g3
    rG = dft.to_reciprocal(rho)
    nz = mask & (G2 > 0)
    return 0.5 * cell.omega * float(np.sum(4.0 * math.pi * np.abs(rG[nz]) ** 2 / G2[nz]))


def gradient(cell: basis.Cell, ecut: float, X: np.ndarray):
    (g1, g2, g3), mask = _g(cell, ecut)
    XG = np.where(mask, dft.to_reciprocal(X), 0.0)
    return [dft.to_real(1j * g * XG).real for g in (g1, g2, g3)]


def divergence(cell: basis.Cell, ecut: float, h):
    (g1, g2, g3), mask = _g(cell, ecut)
    acc = np.zeros(cell.shape, dtype=np.complex128)
    for g, hi in zip((g1, g2, g3), h):
        acc += 1j * g * dft.to_reciprocal(hi)
    return dft.to_real(np.where(mask, acc, 0.0)).real


def kedf(cell: basis.Cell, ecut: float, X: np.ndarray, thr: float = 1e-10, kind: str = "lc94"):
    """(T~[X], V~_kin[X]) for kind in {'lc94', 'revapbek', 'tf', 'none'}."""
    X = np.asarray(X, dtype=np.float64)
    if kind == "none":
        return 0.0, np.zeros_like(X)
    ok = X >= thr
    Xs = np.where(ok, X, 1.0)
    if kind == "tf":
        e = np.where(ok, fn.C_TF * Xs ** (5.0 / 3.0), 0.0)
        v = np.where(ok, fn.C_TF * (5.0 / 3.0) * Xs ** (2.0 / 3.0), 0.0)
        return float(np.sum(e)) * cell.dV, v
    if kind not in ("lc94", "revapbek"):
        raise ValueError(kind)
    grad = gradient(cell, ecut, X)
    gabs = np.sqrt(grad[0] ** 2 + grad[1] ** 2 + grad[2] ** 2)
    s = fn.C_S * gabs / Xs ** (4.0 / 3.0)
    if kind == "lc94":
        F = fn.lc94_F(s)
        dF = fn.lc94_dF(s)
        dFs = fn.lc94_dF_over_s(s)
    else:
        F = fn.revapbek_F(s)
        dFs = fn.revapbek_dF_over_s(s)
        dF = dFs * s
    e = np.where(ok, fn.C_TF * Xs ** (5.0 / 3.0) * F, 0.0)
    v = np.where(ok, fn.C_TF * Xs ** (2.0 / 3.0) * (5.0 / 3.0 * F - 4.0 / 3.0 * s * dF), 0.0)
    h = [np.where(ok, fn.C_TF * fn.C_S ** 2 * dFs * gi / Xs, 0.0) for gi in grad]
    V = v - divergence(cell, ecut, h)
    return float(np.sum(e)) * cell.dV, V


def xc(X: np.ndarray, cell: basis.Cell, thr: float = 1e-10, kind: str = "lda", ecut: float = None):
    """(E_xc[X], v_xc[X]) for kind in {'lda', 'pbe', 'none'}. PBE: v = e_rho - div(2 e_sigma
    grad X) with the spectral gradient and divergence on D (ecut needed)."""
    X = np.asarray(X, dtype=np.float64)
    if kind == "none":
        return 0.0, np.zeros_like(X)
    if kind == "lda":
        e, v = fn.lda(X, thr)
        return float(np.sum(e)) * cell.dV, v
    if kind != "pbe":
        raise ValueError(kind)
    ok = X >= thr
    Xs = np.where(ok, X, 1.0)
    grad = gradient(cell, ecut, X)
    sigma = grad[0] ** 2 + grad[1] ** 2 + grad[2] ** 2
    e, er, es = fn.complex_step(fn.pbe_energy, Xs, sigma)
    e = np.where(ok, e, 0.0)
    h = [np.where(ok, 2.0 * es * gi, 0.0) for gi in grad]
    v = np.where(ok, er, 0.0) - divergence(cell, ecut, h)
    return float(np.sum(e)) * cell.dV, v


def embed_potential(cell: basis.Cell, ecut: float, rho_sub: np.ndarray, vloc: np.ndarray,
                    thr: float = 1e-10, xc_kind="lda", xc_nad="lda", kin_nad="lc94"):
    """(V_eff [ns, N3, N2, N1], energies [ns+1, NE])."""
    rho_sub = np.asarray(rho_sub, dtype=np.float64)
    ns = rho_sub.shape[0]
    rho = np.sum(rho_sub, axis=0)
    dV = cell.dV
    VH, EH = hartree(cell, ecut, rho)
    Ext, vxt = xc(rho, cell, thr, xc_nad, ecut)
    Ekt, vkt = kedf(cell, ecut, rho, thr, kin_nad)
    Exc_tot, _ = xc(rho, cell, thr, xc_kind, ecut)
    veff = np.zeros_like(rho_sub)
    en = np.zeros((ns + 1, NE))
    for I in range(ns):
        rI = rho_sub[I]
        ExcI, vxcI = xc(rI, cell, thr, xc_kind, ecut)
        ExtI, vxtI = xc(rI, cell, thr, xc_nad, ecut)
        EkI, vkI = kedf(cell, ecut, rI, thr, kin_nad)
        _, EHI = hartree(cell, ecut, rI)
        veff[I] = vloc + VH + vxcI + (vxt - vxtI) + (vkt - vkI)
        en[I, E_XC] = ExcI
        en[I, E_XCT] = ExtI
        en[I, E_KIN] = EkI
        en[I, E_LOC] = float(np.sum(vloc * rI)) * dV
        en[I, E_HEMB] = float(np.sum(VH * rI)) * dV
        en[I, E_HSELF] = EHI
        en[I, E_DEBAND] = -float(np.sum((veff[I] - vloc) * rI)) * dV
        en[I, E_CHARGE] = float(np.sum(rI)) * dV
    en[ns, E_XC] = Exc_tot
    en[ns, E_XCT] = Ext
    en[ns, E_KIN] = Ekt
    en[ns, E_LOC] = float(np.sum(vloc * rho)) * dV
    en[ns, E_HEMB] = float(np.sum(VH * rho)) * dV
    en[ns, E_HSELF] = EH
    en[ns, E_CHARGE] = float(np.sum(rho)) * dV
    return veff, en


def potential_energy(cell: basis.Cell, ecut: float, rho_sub: np.ndarray, vloc: np.ndarray,
                     thr: float = 1e-10, xc_kind="lda", xc_nad="lda", kin_nad="lc94") -> float:
    """The density-dependent part of E_FDE (Sec. 2), whose derivative in rho_I is V_eff^I:

    sum_I int V_loc rho_I + E_H[rho] + sum_I E_xc[rho_I] + (E~xc[rho] - sum E~xc[rho_I])
    + (T~[rho] - sum T~[rho_I]).  Evaluated from energies only (no potentials).
    """
    rho_sub = np.asarray(rho_sub, dtype=np.float64)
    rho = rho_sub.sum(axis=0)
    dV = cell.dV
    E = float(np.sum(vloc * rho)) * dV
    E += hartree_energy(cell, ecut, rho)
    E += xc(rho, cell, thr, xc_nad, ecut)[0] + kedf(cell, ecut, rho, thr, kin_nad)[0]
    for rI in rho_sub:
        E += xc(rI, cell, thr, xc_kind, ecut)[0] - xc(rI, cell, thr, xc_nad, ecut)[0]
        E -= kedf(cell, ecut, rI, thr, kin_nad)[0]
    return E
