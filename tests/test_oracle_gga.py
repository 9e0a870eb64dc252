"""Pins of the oracle's PBE exchange-correlation and revAPBEK kinetic functional (CPU only)."""
import math

import numpy as np
import pytest

import fde_synth
from oracle import basis, embed, functionals as fn

RHO = np.array([1e-4, 3e-3, 0.02, 0.1, 0.5, 2.0])


def test_pbe_uniform_gas_is_slater_plus_pw92():
    e, er, es = fn.complex_step(fn.pbe_energy, RHO, np.zeros_like(RHO))
    ex, vx = fn.slater(RHO)
    rs = np.cbrt(3 / (4 * math.pi * RHO))
    ec = fn.pw92_eps(rs)
    assert np.allclose(e, RHO * (ex + ec), rtol=1e-14, atol=0)
    # d(rho eps_c)/drho by central differences of the PW92 formula in rho
    h = 1e-6 * RHO
    fd = ((RHO + h) * fn.pw92_eps(np.cbrt(3 / (4 * math.pi * (RHO + h))))
          - (RHO - h) * fn.pw92_eps(np.cbrt(3 / (4 * math.pi * (RHO - h))))) / (2 * h)
    assert np.allclose(er, vx + fd, rtol=1e-8, atol=0)


def test_pw92_matches_pz81_and_the_high_density_limit():
    # two parametrisations of the same correlation energies of the electron gas
    rs = np.array([0.5, 1.0, 2.0, 5.0, 10.0])
    rho = 3 / (4 * math.pi * rs ** 3)
    pz, _ = fn.pz81(rho)
    assert np.max(np.abs(fn.pw92_eps(rs) - pz)) < 1.5e-3
    # eps_c ~ a ln r_s for r_s -> 0 with a = (1 - ln 2)/pi^2 (Gell-Mann-Brueckner)
    r1, r2 = 1e-6, 1e-7
    slope = (fn.pw92_eps(r1) - fn.pw92_eps(r2)) / math.log(r1 / r2)
    assert abs(slope - (1 - math.log(2)) / math.pi ** 2) < 2e-4
    assert abs(fn.PBE["gamma"] - (1 - math.log(2)) / math.pi ** 2) < 1e-15
    assert abs(fn.PW92["a"] - fn.PBE["gamma"]) < 1e-7


def test_pbe_gradient_limits():
    rho = 0.05
    kf = (3 * math.pi ** 2 * rho) ** (1 / 3)
    # exchange: F_x = 1 + mu s^2 + O(s^4), mu = beta pi^2 / 3
    s = 1e-3
    sigma = (s * 2 * kf * rho) ** 2
    ex0 = fn.pbe_x_energy(np.array([rho]), np.array([0.0]))[0]
    ex1 = fn.pbe_x_energy(np.array([rho]), np.array([sigma]))[0]
    assert abs((ex1 / ex0 - 1) / s ** 2 - fn.PBE["mu"]) < 1e-6
    assert abs(fn.PBE["mu"] - 0.2195149727645171) < 1e-15
    # correlation: H = beta t^2 + O(t^4) at small t
    ks = math.sqrt(4 * kf / math.pi)
    t = 1e-3
    sigma = (t * 2 * ks * rho) ** 2
    c0 = fn.pbe_c_energy(np.array([rho]), np.array([0.0]))[0]
    c1 = fn.pbe_c_energy(np.array([rho]), np.array([sigma]))[0]
    assert abs((c1 - c0) / rho / t ** 2 - fn.PBE["beta"]) < 1e-6
    # rapidly varying limit: correlation vanishes (eps_c + H -> 0)
    assert abs(fn.pbe_c_energy(np.array([rho]), np.array([1e16]))[0]) < 1e-8 * abs(c0)


def test_complex_step_derivatives_against_differences():
    rng = np.random.default_rng(3)
    rho = rng.uniform(1e-3, 1.0, 20)
    sigma = rng.uniform(0.05, 1.0, 20) * rho ** (8 / 3)
    e, er, es = fn.complex_step(fn.pbe_energy, rho, sigma)
    h = 1e-5
    fr = (fn.pbe_energy(rho * (1 + h), sigma) - fn.pbe_energy(rho * (1 - h), sigma)) / (2 * h * rho)
    hs = 1e-4  # e_sigma sigma is a small part of e: a larger step against the cancellation
    fs = (fn.pbe_energy(rho, sigma * (1 + hs)) - fn.pbe_energy(rho, sigma * (1 - hs))) / (2 * hs * sigma)
    assert np.max(np.abs(er - fr) / np.abs(er)) < 1e-7
    assert np.max(np.abs(es - fs) / np.abs(es)) < 2e-6


def test_revapbek_limits_and_derivative():
    k, mu = fn.REVAPBEK["kappa"], fn.REVAPBEK["mu"]
    s = np.array([1e-4])
    assert abs((fn.revapbek_F(s)[0] - 1) / s[0] ** 2 - mu) < 1e-7
    assert abs(fn.revapbek_F(np.array([1e8]))[0] - (1 + k)) < 1e-12
    s = np.linspace(0.01, 6.0, 50)
    h = 1e-6
    fd = (fn.revapbek_F(s + h) - fn.revapbek_F(s - h)) / (2 * h)
    assert np.max(np.abs(fd - s * fn.revapbek_dF_over_s(s))) < 1e-8


@pytest.mark.parametrize("kinds", [dict(xc_kind="pbe", xc_nad="pbe", kin_nad="revapbek"),
                                   dict(xc_kind="lda", xc_nad="pbe", kin_nad="lc94"),
                                   dict(xc_kind="pbe", xc_nad="lda", kin_nad="revapbek")])
def test_gga_potentials_are_functional_derivatives(kinds):
    # V_eff^I = dE/drho_I (per grid point / dV) of the density-dependent energy, by
    # central differences at a few points: the gradient, divergence and e_sigma terms
    L, grid, ecut = (6.0, 6.0, 7.0), (12, 12, 15), 2.2
    cell = basis.Cell(L, grid)
    sph = basis.sphere(cell, ecut, (0.0, 0.0, 0.0))
    rs = []
    for I in range(2):
        c = fde_synth.random_complex(20 + I, (3, sph.npw)) / (1 + 2 * sph.kin)[None] ** 2
        from oracle import density, subspace
        rs.append(density.density(cell, sph, subspace.orthonormalise(c), np.full(3, 2.0)))
    rs = np.array(rs)
    vloc = fde_synth.random_real(5, cell.shape, -0.3, 0.3)
    veff, _ = embed.embed_potential(cell, ecut, rs, vloc, **kinds)
    rng = np.random.default_rng(9)
    for _ in range(3):
        I = int(rng.integers(0, 2))
        j = tuple(int(rng.integers(0, n)) for n in cell.shape)
        h = 1e-5 * rs[I][j]
        rp, rm = rs.copy(), rs.copy()
        rp[I][j] += h
        rm[I][j] -= h
        fd = (embed.potential_energy(cell, ecut, rp, vloc, **kinds)
              - embed.potential_energy(cell, ecut, rm, vloc, **kinds)) / (2 * h * cell.dV)
        assert abs(fd - veff[I][j]) < 1e-6 * max(1.0, abs(fd)), (kinds, fd, veff[I][j])
    # one subsystem with the same functional for xc and its nonadditive part: V_xc[rho]
    if kinds["xc_kind"] == kinds["xc_nad"]:
        v1, _ = embed.embed_potential(cell, ecut, rs, vloc, **kinds)
        ex, vx = embed.xc(rs.sum(0), cell, 1e-10, kinds["xc_kind"], ecut)
        Ek, vk = embed.kedf(cell, ecut, rs.sum(0), 1e-10, kinds["kin_nad"])
        VH, _ = embed.hartree(cell, ecut, rs.sum(0))
        for I in range(2):
            _, vkI = embed.kedf(cell, ecut, rs[I], 1e-10, kinds["kin_nad"])
            assert np.max(np.abs(v1[I] - (vloc + VH + vx + vk - vkI))) < 1e-12
