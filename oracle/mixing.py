"""Density mixing of the embedding cycle (test infrastructure, FP64).

The paper's cycle (Fig. 1b) rebuilds every subsystem density once per cycle
and leaves the mixing scheme to the host code; the readings used here are:

* linear:  rho_I^in <- rho_I^in + beta R_I, with R_I = rho_I^out - rho_I^in;
* Pulay (direct inversion in the iterative subspace) with a Kerker
  preconditioner: the densities of all subsystems form one vector x =
  (rho_1, ..., rho_ns) and its residual R = F(x) - x. From the last n pairs
  (x_i, R_i), the coefficients a minimise |sum_i a_i R_i|^2 (grid inner
  product) subject to sum_i a_i = 1, i.e. solve
      [B 1; 1^T 0] [a; lambda] = [0; 1],  B_ij = <R_i | R_j>,
  and the next input is  x = sum_i a_i x_i + beta K(sum_i a_i R_i), where K
  multiplies each subsystem's residual by |G|^2 / (|G|^2 + q0^2) on the whole
  FFT grid (q0 = 0: K = 1). K leaves the G = 0 term (the charge) unchanged
  only when q0 = 0; for q0 > 0 it removes it, so the input charge is kept.
  An exactly singular system (a repeated pair) falls back to the newest pair
  alone, i.e. linear mixing; a zero residual selects its own input. Nearly
  dependent residuals are kept: near a fixed point the minimising combination
  is exactly such a dependency.

Pins (tests/test_oracle_mixing.py): Pulay with K = 1 finds the fixed point of
an affine map on R^n in at most n + 1 evaluations (it is then GMRES on the
residual); one history entry reduces it to linear mixing; K acts on a single
plane wave as the scalar |G|^2 / (|G|^2 + q0^2) and keeps a uniform density.
"""
from __future__ import annotations

import numpy as np

from . import basis, dft


def kerker(cell: basis.Cell, R: np.ndarray, q0: float) -> np.ndarray:
    """K R per subsystem grid (R [..., N3, N2, N1] real)."""
    if q0 == 0.0:
        return np.array(R, dtype=np.float64, copy=True)
    g1, g2, g3 = basis.grid_g(cell)
    G2 = g1 * g1 + g2 * g2 + g3 * g3
    K = G2 / (G2 + q0 * q0)
    return dft.to_real(K * dft.to_reciprocal(R)).real


def pulay_coefficients(res_hist) -> np.ndarray:
    """a_i from the residual history (list of arrays): the bordered normal equations."""
    n = len(res_hist)
    B = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            B[i, j] = float(np.sum(res_hist[i] * res_hist[j]))
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = B
    M[:n, n] = 1.0
    M[n, :n] = 1.0
    rhs = np.zeros(n + 1)
    rhs[n] = 1.0
    d = np.sqrt(np.diag(B))
    if np.any(d == 0.0):
        # a zero residual: that input is the fixed point
        return np.eye(n)[int(np.nonzero(d == 0.0)[0][0])]
    try:
        a = np.linalg.solve(M, rhs)[:n]
    except np.linalg.LinAlgError:
        a = None
    if a is None or not np.all(np.isfinite(a)):
        # exactly singular (e.g. a repeated pair): the newest pair alone, linear mixing
        return np.eye(n)[n - 1]
    return a


def pulay(cell: basis.Cell, x_hist, res_hist, beta: float, q0: float) -> np.ndarray:
    """Next input x = sum a_i x_i + beta K(sum a_i R_i)."""
    a = pulay_coefficients(res_hist)
    xbar = sum(ai * xi for ai, xi in zip(a, x_hist))
    rbar = sum(ai * ri for ai, ri in zip(a, res_hist))
    return xbar + beta * kerker(cell, rbar, q0)


class Mixer:
    """State of the mixing across cycles: kind 'linear' or 'pulay' (history of nhist pairs)."""

    def __init__(self, cell: basis.Cell, kind: str = "linear", beta: float = 0.3, nhist: int = 6, q0: float = 0.0):
        if kind not in ("linear", "pulay"):
            raise ValueError(kind)
        self.cell, self.kind, self.beta, self.nhist, self.q0 = cell, kind, beta, nhist, q0
        self.x_hist, self.r_hist = [], []

    def reset(self):
        """Forget the Pulay history (the next call mixes with its own pair only)."""
        self.x_hist, self.r_hist = [], []

    def __call__(self, rho_in: np.ndarray, rho_out: np.ndarray) -> np.ndarray:
        R = rho_out - rho_in
        if self.kind == "linear":
            if self.q0 == 0.0:
                return (1.0 - self.beta) * rho_in + self.beta * rho_out
            return rho_in + self.beta * kerker(self.cell, R, self.q0)
        self.x_hist.append(np.array(rho_in, copy=True))
        self.r_hist.append(R)
        if len(self.x_hist) > self.nhist:
            self.x_hist.pop(0)
            self.r_hist.pop(0)
        return pulay(self.cell, self.x_hist, self.r_hist, self.beta, self.q0)
