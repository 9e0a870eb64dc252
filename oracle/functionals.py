"""Pointwise density functionals (test infrastructure, FP64).

Exchange-correlation (LDA; the paper's runs use PBE, Sec. 3, which is a later
extension here):
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
