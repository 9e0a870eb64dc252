"""Pointwise density functionals (test infrastructure, FP64).

Exchange-correlation: LDA (below) and PBE, the paper's functional (Sec. 3;
see pbe_xc). Kinetic enhancement factors: LC94 and revAPBEK, the two
nonadditive kinetic functionals of Sec. 3.
LDA:
* Slater exchange  eps_x = -(3/4)(3/pi)^{1/3} rho^{1/3},  v_x = (4/3) eps_x.
* Perdew-Zunger 1981 correlation (unpolarised), r_s = (3/(4 pi rho))^{1/3}:
    r_s >= 1: eps_c = g / (1 + b1 sqrt(r_s) + b2 r_s),
              v_c = eps_c (1 + 7/6 b1 sqrt(r_s) + 4/3 b2 r_s) / (1 + b1 sqrt(r_s) + b2 r_s)
    r_s <  1: eps_c = A ln r_s + B + C r_s ln r_s + D r_s,
              v_c = A ln r_s + (B - A/3) + 2/3 C r_s ln r_s + (2D - C) r_s / 3
  with g = -0.1423, b1 = 1.0529, b2 = 0.3334, A = 0.0311, B = -0.048,
  C = 0.0020, D = -0.0116 (the published PZ81 values; the paper does not
  print them).

Kinetic energy (Appendix, kinetic energy functional and potential):
  T[X] = C_TF int X^{5/3} F(s),  s = C_s |grad X| / X^{4/3},
  C_TF = (3/10)(3 pi^2)^{2/3}.
  The appendix prints C_s = 1 / (2 (2 pi^2)^{1/3}); this is read as a typo for
  the standard reduced gradient C_s = 1 / (2 (3 pi^2)^{1/3}) on which LC94 is
  parametrised (s = |grad X| / (2 k_F X)).
  LC94 (Lembarki-Chermette 1994, cited in Sec. 3 as the nonadditive KEDF):
  F(s) = [1 + a1 s asinh(a2 s) + (a3 - a4 e^{-alpha s^2}) s^2]
         / [1 + a1 s asinh(a2 s) + a5 s^4]
  with a1 = 0.093907, a2 = 76.32, a3 = 0.26608, a4 = 0.0809615, a5 = 5.7767e-5,
  alpha = 100.

Low-density rule (paper silent): where X < rho_thr the functional's energy
density, its local potential and its gradient field are zero.

Pins: uniform-gas closed forms via k_F, the r_s = 1 branch values and the
continuity of v_c there (which fixes C to the printed precision), the
Gell-Mann-Brueckner coefficient (1 - ln 2)/pi^2 for A, the 5/27 gradient
coefficient of LC94 (a3 - a4), and finite differences of every energy against
its potential (tests/test_oracle_functionals.py, tests/test_oracle_pins.py).

Parity unpinned: published constants. The PZ81 values g, b1, b2, B, D and C
are checked only through their continuity relations at r_s = 1, and the LC94
values a1, a2, a5 and alpha (a3 and a4 only through their difference) have no
independent check here: they are taken from the cited publications as
printed, and a typo in them would change the oracle and the kernels alike.
"""
from __future__ import annotations

import math

import numpy as np

C_TF = 0.3 * (3.0 * math.pi ** 2) ** (2.0 / 3.0)
C_S = 1.0 / (2.0 * (3.0 * math.pi ** 2) ** (1.0 / 3.0))
C_X = 0.75 * (3.0 / math.pi) ** (1.0 / 3.0)

PZ = dict(g=-0.1423, b1=1.0529, b2=0.3334, A=0.0311, B=-0.048, C=0.0020, D=-0.0116)
LC94 = dict(a1=0.093907, a2=76.32, a3=0.26608, a4=0.0809615, a5=5.7767e-5, alpha=100.0)


def slater(rho):
    """(eps_x, v_x) per point."""
    rho = np.asarray(rho, dtype=np.float64)
    eps = -C_X * np.cbrt(rho)
    return eps, (4.0 / 3.0) * eps


def pz81(rho):
    """(eps_c, v_c) per point, r_s = 1 taken on the r_s >= 1 branch."""
    rho = np.asarray(rho, dtype=np.float64)
    rs = np.cbrt(3.0 / (4.0 * math.pi * rho))
    p = PZ
    hi = rs >= 1.0
    eps = np.empty_like(rs)
    v = np.empty_like(rs)
    r = rs[hi]
    sq = np.sqrt(r)
    den = 1.0 + p["b1"] * sq + p["b2"] * r
    eps[hi] = p["g"] / den
    v[hi] = eps[hi] * (1.0 + 7.0 / 6.0 * p["b1"] * sq + 4.0 / 3.0 * p["b2"] * r) / den
    r = rs[~hi]
    lr = np.log(r)
    eps[~hi] = p["A"] * lr + p["B"] + p["C"] * r * lr + p["D"] * r
    v[~hi] = p["A"] * lr + (p["B"] - p["A"] / 3.0) + 2.0 / 3.0 * p["C"] * r * lr \
        + (2.0 * p["D"] - p["C"]) * r / 3.0
    return eps, v


def lda(rho, thr=1e-10):
    """LDA energy density e = rho eps_xc and potential v_xc, zero below thr."""
    rho = np.asarray(rho, dtype=np.float64)
    ok = rho >= thr
    e = np.zeros_like(rho)
    v = np.zeros_like(rho)
    r = rho[ok]
    ex, vx = slater(r)
    ec, vc = pz81(r)
    e[ok] = r * (ex + ec)
    v[ok] = vx + vc
    return e, v


def lc94_F(s):
    p = LC94
    s = np.asarray(s, dtype=np.float64)
    t = p["a1"] * s * np.arcsinh(p["a2"] * s)
    num = 1.0 + t + (p["a3"] - p["a4"] * np.exp(-p["alpha"] * s * s)) * s * s
    den = 1.0 + t + p["a5"] * s ** 4
    return num / den


def lc94_dF(s):
    """dF/ds by the quotient rule."""
    p = LC94
    s = np.asarray(s, dtype=np.float64)
    a2s = p["a2"] * s
    t = p["a1"] * s * np.arcsinh(a2s)
    dt = p["a1"] * np.arcsinh(a2s) + p["a1"] * s * p["a2"] / np.sqrt(1.0 + a2s * a2s)
    ex = np.exp(-p["alpha"] * s * s)
    num = 1.0 + t + (p["a3"] - p["a4"] * ex) * s * s
    dnum = dt + 2.0 * s * (p["a3"] - p["a4"] * ex) + s * s * (2.0 * p["alpha"] * s * p["a4"] * ex)
    den = 1.0 + t + p["a5"] * s ** 4
    dden = dt + 4.0 * p["a5"] * s ** 3
    return (dnum * den - num * dden) / (den * den)


def lc94_dF_over_s(s):
    """F'(s)/s, with its s -> 0 limit 2 (a3 - a4) below s = 1e-6."""
    s = np.asarray(s, dtype=np.float64)
    small = s < 1e-6
    out = np.empty_like(s)
    out[small] = 2.0 * (LC94["a3"] - LC94["a4"])
    out[~small] = lc94_dF(s[~small]) / s[~small]
    return out


# ---------------------------------------------------------------------------
# PBE exchange-correlation (Perdew, Burke & Ernzerhof 1996; the functional of
# the paper's calculations, Sec. 3), spin-unpolarised, as an energy density
# e(rho, sigma) with sigma = |grad rho|^2:
#   exchange     e_x = -C_X rho^{4/3} F_x(s),  F_x = 1 + kappa - kappa/(1 + mu s^2/kappa),
#                s = C_S sqrt(sigma) / rho^{4/3}, kappa = 0.804, mu = beta pi^2 / 3;
#   correlation  e_c = rho [eps_c^PW92(r_s) + H(r_s, t)],
#                H = gamma ln(1 + (beta/gamma) t^2 (1 + A t^2)/(1 + A t^2 + A^2 t^4)),
#                A = (beta/gamma) / (exp(-eps_c/gamma) - 1), t = sqrt(sigma)/(2 k_s rho),
#                k_s = sqrt(4 k_F / pi), gamma = (1 - ln 2)/pi^2, beta = 0.06672455060314922;
#   PW92         eps_c = -2 a (1 + a1 r_s) ln(1 + 1/(2 a (b1 r_s^{1/2} + b2 r_s + b3 r_s^{3/2} + b4 r_s^2))).
# The derivatives e_rho, e_sigma are taken by the complex step (Im e(x + i h)/h, exact to
# rounding for these analytic forms), independently of any hand-derived formula.
# Parity unpinned: published constants -- PW92's a1, b1..b4 and PBE's kappa and beta
# (a and gamma are pinned by the Gell-Mann-Brueckner coefficient; mu = beta pi^2/3 by
# construction).
# ---------------------------------------------------------------------------
PW92 = dict(a=0.0310907, a1=0.21370, b1=7.5957, b2=3.5876, b3=1.6382, b4=0.49294)
PBE = dict(kappa=0.804, beta=0.06672455060314922, gamma=(1.0 - math.log(2.0)) / math.pi ** 2)
PBE["mu"] = PBE["beta"] * math.pi ** 2 / 3.0
# revAPBEK kinetic enhancement (APBEK's mu with revPBE's kappa; cited in Sec. 3)
REVAPBEK = dict(kappa=1.245, mu=0.23889)


def _cbrt(z):
    return z ** (1.0 / 3.0) if np.iscomplexobj(z) else np.cbrt(z)


def pw92_eps(rs):
    p = PW92
    q = 2.0 * p["a"] * (p["b1"] * np.sqrt(rs) + p["b2"] * rs + p["b3"] * rs ** 1.5 + p["b4"] * rs * rs)
    return -2.0 * p["a"] * (1.0 + p["a1"] * rs) * np.log(1.0 + 1.0 / q)


def pbe_x_energy(rho, sigma):
    k, mu = PBE["kappa"], PBE["mu"]
    r43 = rho * _cbrt(rho)
    s2 = C_S * C_S * sigma / (r43 * r43)
    return -C_X * r43 * (1.0 + k - k / (1.0 + mu * s2 / k))


def pbe_c_energy(rho, sigma):
    beta, gamma = PBE["beta"], PBE["gamma"]
    rs = _cbrt(3.0 / (4.0 * math.pi * rho))
    ec = pw92_eps(rs)
    kf = _cbrt(3.0 * math.pi ** 2 * rho)
    ks2 = 4.0 * kf / math.pi
    t2 = sigma / (4.0 * ks2 * rho * rho)
    A = (beta / gamma) / (np.exp(-ec / gamma) - 1.0)
    at2 = A * t2
    H = gamma * np.log(1.0 + (beta / gamma) * t2 * (1.0 + at2) / (1.0 + at2 + at2 * at2))
    return rho * (ec + H)


def pbe_energy(rho, sigma):
    return pbe_x_energy(rho, sigma) + pbe_c_energy(rho, sigma)


def complex_step(efun, rho, sigma):
    """(e, de/drho, de/dsigma) of an energy density by the complex step."""
    rho = np.asarray(rho, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    e = efun(rho, sigma)
    hr = 1e-30 * np.maximum(rho, 1e-300)
    hs = 1e-30 * np.maximum(sigma, 1e-200)
    dr = np.imag(efun(rho + 1j * hr, sigma.astype(np.complex128))) / hr
    ds = np.imag(efun(rho.astype(np.complex128), sigma + 1j * hs)) / hs
    return np.real(e), dr, ds


def revapbek_F(s):
    k, mu = REVAPBEK["kappa"], REVAPBEK["mu"]
    s = np.asarray(s, dtype=np.float64)
    return 1.0 + k - k / (1.0 + mu * s * s / k)


def revapbek_dF_over_s(s):
    """F'(s)/s = 2 mu / (1 + mu s^2/kappa)^2 (regular at s = 0)."""
    k, mu = REVAPBEK["kappa"], REVAPBEK["mu"]
    s = np.asarray(s, dtype=np.float64)
    return 2.0 * mu / (1.0 + mu * s * s / k) ** 2
