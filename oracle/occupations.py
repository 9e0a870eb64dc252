"""Occupations of one subsystem (test infrastructure, FP64).

Sec. 2 allows fractional occupations 0 <= n_jk <= 1 (f = 2n here) summing to
the subsystem's electrons; Sec. 3 smears only metallic subsystems and keeps
integer occupations for molecules. Reading used here: one Fermi level mu per
subsystem with the Brillouin-zone averaged constraint
sum_k w_k sum_n f_nk = N_I.

* integer: f = 2 on the lowest N_I/2 bands of every k (N_I must be even and
  whole: a singly occupied band is not part of this reading);
* fermi-dirac (width sigma): f = 1 - tanh((eps - mu) / (2 sigma)), the
  overflow-free form of 2 / (1 + e^{(eps-mu)/sigma}); mu by bisection on
  [min eps - 20 sigma, max eps + 20 sigma] until |sum w f - N| < 1e-13
  (at most 200 halvings);
* methfessel-paxton (first order, width sigma; Sec. 3 smears the metallic
  slabs this way): with x = (eps - mu) / sigma, f = 2 S_1(x),
  S_1(x) = erfc(x)/2 + A_1 H_1(x) e^{-x^2}, A_1 = -1/(4 sqrt(pi)), H_1 = 2x, i.e.
  f = erfc(x) - x e^{-x^2} / sqrt(pi); f may leave [0, 2] slightly. mu by the
  same bisection.

Pins: electron count; sigma -> 0 gives integer filling of a gapped spectrum;
mu lies in the gap (tests/test_oracle_solver.py); the Methfessel-Paxton
broadened delta -dS_1/dx has unit weight and zero second moment
(tests/test_oracle_mixing.py).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erfc


def fermi_dirac(eps, mu, sigma):
    return 1.0 - np.tanh((np.asarray(eps) - mu) / (2.0 * sigma))


def methfessel_paxton(eps, mu, sigma):
    """2 S_1((eps - mu) / sigma), first-order Methfessel-Paxton."""
    x = (np.asarray(eps, dtype=np.float64) - mu) / sigma
    return erfc(x) - x * np.exp(-x * x) / np.sqrt(np.pi)


def occupations(eps: np.ndarray, wk: np.ndarray, nelec: float, mode: str, sigma: float = 0.0):
    """(f [nk, nb], mu) for eigenvalues eps [nk, nb] ascending per k."""
    eps = np.asarray(eps, dtype=np.float64)
    wk = np.asarray(wk, dtype=np.float64)
    nk, nb = eps.shape
    if mode == "integer":
        if nelec < 0 or nelec != 2.0 * np.floor(nelec / 2.0):
            raise ValueError("integer occupations need an even, whole electron count")
        nocc = int(nelec // 2)
        if nocc > nb:
            raise ValueError("not enough bands")
        f = np.zeros_like(eps)
        f[:, :nocc] = 2.0
        mu = float(np.max(eps[:, nocc - 1])) if nocc > 0 else float(np.min(eps))
        return f, mu
    if mode not in ("fermi-dirac", "methfessel-paxton"):
        raise ValueError(mode)
    occ = fermi_dirac if mode == "fermi-dirac" else methfessel_paxton
    lo = float(eps.min()) - 20.0 * sigma
    hi = float(eps.max()) + 20.0 * sigma
    mu = 0.5 * (lo + hi)
    for _ in range(200):
        mu = 0.5 * (lo + hi)
        n = float(np.sum(wk[:, None] * occ(eps, mu, sigma)))
        if abs(n - nelec) < 1e-13:
            break
        if n < nelec:
            lo = mu
        else:
            hi = mu
    return occ(eps, mu, sigma), mu
