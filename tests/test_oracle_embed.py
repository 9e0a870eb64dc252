"""Pins of the oracle's embedding potential (CPU only)."""
import math

import numpy as np
import pytest

import fde_synth
from oracle import basis, density, embed, subspace


def _smooth_densities(cell, ecut, ns=2, nb=3, seed=20):
    sph = basis.sphere(cell, ecut, (0.0, 0.0, 0.0))
    out = []
    for I in range(ns):
        c = fde_synth.random_complex(seed + I, (nb, sph.npw)) / (1 + 2 * sph.kin)[None] ** 2
        X = subspace.orthonormalise(c)
        out.append(density.density(cell, sph, X, np.full(nb, 2.0)))
    return np.array(out)


def test_gaussian_charge_hartree_lattice_sum():
    cell = basis.Cell((10.0, 10.0, 10.0), (24, 24, 24))
    ecut, q, sig = 7.0, 1.7, 1.2
    x, y, z = cell.positions()
    c = np.array([3.1, 5.0, 6.3])
    n = np.zeros(cell.shape)
    for sx in (-1, 0, 1):           # periodic images (the Gaussian is < 1e-9 beyond one cell)
        for sy in (-1, 0, 1):
            for sz in (-1, 0, 1):
                r2 = (x - c[0] - sx * 10) ** 2 + (y - c[1] - sy * 10) ** 2 + (z - c[2] - sz * 10) ** 2
                n += q * (2 * math.pi * sig ** 2) ** -1.5 * np.exp(-r2 / (2 * sig ** 2))
    _, EH = embed.hartree(cell, ecut, n)
    # E_H = (2 pi q^2 / Omega) sum_{G != 0} e^{-G^2 s^2} / G^2, summed directly
    b = 2 * math.pi / 10.0
    m = np.arange(-20, 21)
    M1, M2, M3 = np.meshgrid(m, m, m, indexing="ij")
    G2 = b * b * (M1 ** 2 + M2 ** 2 + M3 ** 2).astype(float)
    G2 = G2[G2 > 0]
    ref = 2 * math.pi * q * q / 1000.0 * np.sum(np.exp(-G2 * sig ** 2) / G2)
    assert abs(EH - ref) < 1e-12 * abs(ref)
    assert abs(embed.hartree_energy(cell, ecut, n) - ref) < 1e-12 * abs(ref)


def test_uniform_density_kedf_closed_form():
    cell = basis.Cell((7.0, 8.0, 9.0), (12, 12, 15))
    rho0 = 0.037
    X = np.full(cell.shape, rho0)
    T, V = embed.kedf(cell, 2.0, X)
    from oracle.functionals import C_TF
    assert abs(T - C_TF * rho0 ** (5 / 3) * cell.omega) < 1e-14 * T
    assert np.max(np.abs(V - 5 / 3 * C_TF * rho0 ** (2 / 3))) < 1e-14


def test_tnad_of_single_density_vanishes_bitwise():
    cell = basis.Cell((8.0, 8.0, 8.0), (15, 15, 15))
    ecut = 2.5
    rho = _smooth_densities(cell, ecut, ns=1)
    both = np.array([rho[0], np.zeros(cell.shape)])
    veff, en = embed.embed_potential(cell, ecut, both, np.zeros(cell.shape))
    tnad = en[2, embed.E_KIN] - en[0, embed.E_KIN] - en[1, embed.E_KIN]
    assert tnad == 0.0
    # V_kin^nad[rho, rho_A] = 0 and V_xc^nad = 0 bitwise when rho_B = 0: V_eff^A = V_H + V_xc[rho]
    VH, _ = embed.hartree(cell, ecut, rho[0])
    _, vxc = embed.xc(rho[0], cell)
    assert np.array_equal(veff[0], np.zeros(cell.shape) + VH + vxc + (vxc - vxc) + 0.0)


def test_single_subsystem_is_kohn_sham_and_xc_invariant():
    cell = basis.Cell((8.0, 8.0, 8.0), (15, 15, 15))
    ecut = 2.5
    rs = _smooth_densities(cell, ecut, ns=3)
    vloc = fde_synth.random_real(3, cell.shape, -0.2, 0.2)
    veff, _ = embed.embed_potential(cell, ecut, rs, vloc, kin_nad="none")
    VH, _ = embed.hartree(cell, ecut, rs.sum(0))
    _, vxc_tot = embed.xc(rs.sum(0), cell)
    for I in range(3):   # LDA for both xc functionals: xc part equals V_xc[rho]
        assert np.max(np.abs(veff[I] - (vloc + VH + vxc_tot))) < 1e-13
    v1, _ = embed.embed_potential(cell, ecut, rs[:1], vloc)
    VH1, _ = embed.hartree(cell, ecut, rs[0])
    _, vxc1 = embed.xc(rs[0], cell)
    assert np.max(np.abs(v1[0] - (vloc + VH1 + vxc1))) < 1e-13


def test_gradient_divergence_adjoint():
    cell = basis.Cell((6.0, 7.0, 8.0), (10, 12, 15))
    X = fde_synth.random_real(30, cell.shape)
    h = [fde_synth.random_real(31 + i, cell.shape) for i in range(3)]
    g = embed.gradient(cell, 2.0, X)
    lhs = sum(np.sum(gi * hi) for gi, hi in zip(g, h))
    rhs = -np.sum(X * embed.divergence(cell, 2.0, h))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("kind", ["lc94", "tf"])
def test_kedf_potential_finite_difference(kind):
    cell = basis.Cell((6.0, 6.0, 7.0), (12, 12, 14))
    ecut = 2.2
    X = _smooth_densities(cell, ecut, ns=1)[0]
    _, V = embed.kedf(cell, ecut, X, kind=kind)
    for idx in [(0, 0, 0), (3, 5, 7), (7, 2, 9), (13, 11, 1)]:
        h = 1e-5 * X[idx]
        Xp = X.copy(); Xp[idx] += h
        Xm = X.copy(); Xm[idx] -= h
        fd = (embed.kedf(cell, ecut, Xp, kind=kind)[0] - embed.kedf(cell, ecut, Xm, kind=kind)[0]) / (2 * h * cell.dV)
        assert abs(fd - V[idx]) < 1e-7 * max(1.0, abs(V[idx]))


def test_veff_is_derivative_of_potential_energy():
    cell = basis.Cell((6.0, 6.0, 7.0), (12, 12, 14))
    ecut = 2.2
    rs = _smooth_densities(cell, ecut, ns=2)
    vloc = fde_synth.random_real(5, cell.shape, -0.3, 0.3)
    veff, _ = embed.embed_potential(cell, ecut, rs, vloc)
    for I in range(2):
        for idx in [(1, 2, 3), (9, 4, 0), (5, 10, 6)]:
            h = 1e-5 * rs[I][idx]
            rp = rs.copy(); rp[I][idx] += h
            rm = rs.copy(); rm[I][idx] -= h
            fd = (embed.potential_energy(cell, ecut, rp, vloc) - embed.potential_energy(cell, ecut, rm, vloc)) / (2 * h * cell.dV)
            assert abs(fd - veff[I][idx]) < 1e-7 * max(1.0, abs(veff[I][idx]))
