"""Pins of the oracle's pointwise functionals (CPU only)."""
import math

import numpy as np

from oracle import functionals as fn


def test_slater_and_tf_uniform_gas_via_kF():
    rho = np.array([1e-4, 0.01, 0.3, 2.0])
    kF = (3 * math.pi ** 2 * rho) ** (1 / 3)
    ex, vx = fn.slater(rho)
    assert np.allclose(ex, -3 * kF / (4 * math.pi), rtol=1e-14, atol=0)   # -3 k_F / 4 pi
    # Thomas-Fermi: kinetic energy per volume (3/5) rho eF with eF = kF^2/2
    assert np.allclose(fn.C_TF * rho ** (5 / 3), 0.6 * rho * kF ** 2 / 2, rtol=1e-14, atol=0)
    assert abs(fn.C_TF - 2.871234000188191) < 1e-12


def test_lda_potential_is_derivative_of_energy():
    rho = np.array([1e-3, 0.02, 0.07, 0.2387, 0.2388, 0.5, 3.0])
    h = 1e-6 * rho
    ep, _ = fn.lda(rho + h)
    em, _ = fn.lda(rho - h)
    _, v = fn.lda(rho)
    assert np.max(np.abs((ep - em) / (2 * h) - v) / np.abs(v)) < 1e-8


def test_pz81_branches_and_constants():
    p = fn.PZ
    # r_s = 1 is taken on the r_s >= 1 branch
    rho1 = 3 / (4 * math.pi)
    eps, _ = fn.pz81(np.array([rho1]))
    assert abs(eps[0] - p["g"] / (1 + p["b1"] + p["b2"])) < 1e-15
    lo = p["B"] + p["D"]
    hi = p["g"] / (1 + p["b1"] + p["b2"])
    assert abs(lo - hi) < 5e-5          # continuous by construction to ~3e-5
    # high-density coefficient equals the exact (1 - ln 2)/pi^2 to the printed digits
    assert abs(p["A"] - (1 - math.log(2)) / math.pi ** 2) < 1e-4
    assert fn.lda(np.array([1e-11]))[0][0] == 0.0


def test_lc94_limits_and_derivative():
    a = fn.LC94
    assert fn.lc94_F(np.array([0.0]))[0] == 1.0
    s = np.array([1e-4, 3e-4])
    coef = (fn.lc94_F(s) - 1) / s ** 2
    assert np.allclose(coef, a["a3"] - a["a4"], rtol=1e-3)
    assert abs((a["a3"] - a["a4"]) - 5 / 27) < 1e-4
    s = np.linspace(0.01, 8.0, 97)
    h = 1e-6
    fd = (fn.lc94_F(s + h) - fn.lc94_F(s - h)) / (2 * h)
    assert np.max(np.abs(fd - fn.lc94_dF(s))) < 1e-7
    assert abs(fn.lc94_dF_over_s(np.array([1e-7]))[0] - 2 * (a["a3"] - a["a4"])) < 1e-12
    assert abs(fn.lc94_dF_over_s(np.array([2e-6]))[0] - 2 * (a["a3"] - a["a4"])) < 1e-6


def test_reduced_gradient_constant_reproduces_gradient_expansion():
    # second-order gradient expansion of T_s: |grad rho|^2 / (72 rho). With
    # s = C_s |grad rho| / rho^{4/3} and F = 1 + (5/27) s^2 this holds only for
    # C_s = 1 / (2 (3 pi^2)^{1/3}); the (2 pi^2) constant printed in the paper's
    # appendix would be off by (3/2)^{2/3}.
    rho, g = 0.3, 1e-4
    s = fn.C_S * g / rho ** (4 / 3)
    t2 = fn.C_TF * rho ** (5 / 3) * (fn.lc94_F(np.array([s]))[0] - 1)
    assert abs(t2 / (g * g / (72 * rho)) - 1) < 1e-3
    cs_printed = 1 / (2 * (2 * math.pi ** 2) ** (1 / 3))
    s2 = cs_printed * g / rho ** (4 / 3)
    t2b = fn.C_TF * rho ** (5 / 3) * (fn.lc94_F(np.array([s2]))[0] - 1)
    assert abs(t2b / (g * g / (72 * rho)) - 1) > 0.2
