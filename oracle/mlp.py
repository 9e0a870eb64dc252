"""Learned band-solver preconditioner: FP64 reference network (test infrastructure).

The paper leaves the band solver to Quantum ESPRESSO; the learned preconditioner
is this project's extension of the Davidson step (the Teter-Payne-Allan
preconditioner K_TPA stays as the fallback and as the baseline). Reading used
on both sides:

* per coefficient G of band n (plane-wave kinetic energy kin_G = |k+G|^2/2,
  band kinetic energy T_n = sum_G kin_G |x_nG|^2, residual r_n, Ritz value
  eps_n, mean effective potential vbar), four features
      u1 = log(1 + kin_G / T_n),  u2 = log T_n,
      u3 = log max(|r_nG| sqrt(npw) / ||r_n||, 1e-6),  u4 = (eps_n - vbar) / T_n;
* a 4 -> 64 -> 64 -> 1 network with tanh hidden layers,
      y = w3 . tanh(W2 tanh(W1 u + b1) + b2) + b3;
* the preconditioned residual T_nG = K_TPA(kin_G / T_n) exp(y_nG) r_nG, then
  normalised; y = 0 (w3 = 0, b3 = 0) is exactly TPA;
* training target: the Jacobi-Davidson correction delta_n solving
  (I - x x^H)(H - eps_n)(I - x x^H) delta = -r_n with delta _|_ x_n;
* loss per coefficient, with the per-band least-squares scale a_n of TPA
  (a_n = Re<K r, delta> / ||K r||^2, fixed from TPA) and the weight
  w_n = npw / ||delta_n||^2:
      l = w_n |a_n K exp(y) r_G - delta_G|^2 = A e^{2y} - 2 B e^y + C,
  A = w a^2 K^2 |r|^2, B = w a K Re(conj(r) delta), C = w |delta|^2; a sample
  is the row (u1, u2, u3, u4, A, B, C) and the loss is the mean over samples;
* Adam (Kingma & Ba 2015) on the flat parameter vector.

Parameter layout (flat, 4545 values): W1[64][4], b1[64], W2[64][64], b2[64],
w3[64], b3.

Pins: finite differences of the loss against the hand-written backward pass;
y = 0 reproduces TPA exactly; the correction satisfies its defining projected
equation; Adam's first steps against their closed form
(tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import numpy as np

from .subspace import ACTIVE_TOL, residual, tpa

HID = 64
NIN = 4
OFF_W1 = 0
OFF_B1 = OFF_W1 + HID * NIN
OFF_W2 = OFF_B1 + HID
OFF_B2 = OFF_W2 + HID * HID
OFF_W3 = OFF_B2 + HID
OFF_B3 = OFF_W3 + HID
NPARAM = OFF_B3 + 1
RHO_FLOOR = 1e-6


def unpack(theta: np.ndarray):
    t = np.asarray(theta, dtype=np.float64)
    return (t[OFF_W1:OFF_B1].reshape(HID, NIN), t[OFF_B1:OFF_W2], t[OFF_W2:OFF_B2].reshape(HID, HID),
            t[OFF_B2:OFF_W3], t[OFF_W3:OFF_B3], t[OFF_B3])


def features(kin: np.ndarray, X: np.ndarray, R: np.ndarray, eps: np.ndarray, vbar: float):
    """(U [nb, npw, 4], K_TPA [nb, npw]) for bands X with residuals R."""
    npw = X.shape[1]
    tkin = np.einsum("g,ng->n", kin, np.abs(X) ** 2)
    x = kin[None, :] / tkin[:, None]
    rn = np.linalg.norm(R, axis=1)
    rho = np.abs(R) * np.sqrt(npw) / np.where(rn > 0, rn, 1.0)[:, None]
    U = np.empty(X.shape + (NIN,))
    U[..., 0] = np.log1p(x)
    U[..., 1] = np.log(tkin)[:, None]
    U[..., 2] = np.log(np.maximum(rho, RHO_FLOOR))
    U[..., 3] = ((np.asarray(eps) - vbar) / tkin)[:, None]
    return U, tpa(x)


def forward(theta: np.ndarray, U: np.ndarray):
    """y for feature rows U [..., 4], and the activations for the backward pass."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    h1 = np.tanh(U @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ w3 + b3, (U, h1, h2)


def loss(theta: np.ndarray, S: np.ndarray) -> float:
    y, _ = forward(theta, S[:, :NIN])
    A, B, C = S[:, 4], S[:, 5], S[:, 6]
    e = np.exp(y)
    return float(np.mean(A * e * e - 2.0 * B * e + C))


def loss_grad(theta: np.ndarray, S: np.ndarray):
    """(loss, d loss / d theta) by explicit backpropagation."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    y, (U, h1, h2) = forward(theta, S[:, :NIN])
    A, B, C = S[:, 4], S[:, 5], S[:, 6]
    n = S.shape[0]
    e = np.exp(y)
    L = float(np.mean(A * e * e - 2.0 * B * e + C))
    gy = (2.0 * A * e * e - 2.0 * B * e) / n
    g = np.zeros(NPARAM)
    g[OFF_W3:OFF_B3] = h2.T @ gy
    g[OFF_B3] = gy.sum()
    gz2 = gy[:, None] * w3[None, :] * (1.0 - h2 * h2)
    g[OFF_W2:OFF_B2] = (gz2.T @ h1).ravel()
    g[OFF_B2:OFF_W3] = gz2.sum(axis=0)
    gz1 = (gz2 @ W2) * (1.0 - h1 * h1)
    g[OFF_W1:OFF_B1] = (gz1.T @ U).ravel()
    g[OFF_B1:OFF_W2] = gz1.sum(axis=0)
    return L, g


def adam(theta, g, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def exact_correction(Hm: np.ndarray, x: np.ndarray, eps: float, r: np.ndarray) -> np.ndarray:
    """delta _|_ x with (I - x x^H)(H - eps)(I - x x^H) delta = -r (bordered solve; ||x|| = 1)."""
    n = Hm.shape[0]
    K = np.zeros((n + 1, n + 1), dtype=np.complex128)
    K[:n, :n] = Hm - eps * np.eye(n)
    K[:n, n] = x
    K[n, :n] = x.conj()
    rhs = np.concatenate([-r, [0.0]])
    sol = np.linalg.solve(K, rhs)
    return sol[:n]


def samples(kin, X, R, eps, vbar, D) -> np.ndarray:
    """Training rows (u1, u2, u3, u4, A, B, C) of every coefficient of the given bands."""
    U, K = features(kin, X, R, eps, vbar)
    npw = X.shape[1]
    KR = K * R
    a = np.real(np.sum(KR.conj() * D, axis=1)) / np.sum(np.abs(KR) ** 2, axis=1)
    w = npw / np.sum(np.abs(D) ** 2, axis=1)
    Arow = (w * a * a)[:, None] * K * K * np.abs(R) ** 2
    Brow = (w * a)[:, None] * K * np.real(R.conj() * D)
    Crow = w[:, None] * np.abs(D) ** 2
    S = np.concatenate([U.reshape(-1, NIN), Arow.reshape(-1, 1), Brow.reshape(-1, 1), Crow.reshape(-1, 1)], axis=1)
    return S


def precondition(theta, X, HX, lam, kin, vbar):
    """Like subspace.precondition with T = K_TPA exp(y) R: (T, active, ||R||)."""
    R = residual(X, HX, lam)
    rn = np.linalg.norm(R, axis=1)
    active = rn > ACTIVE_TOL
    U, K = features(kin, X, R, lam, vbar)
    y, _ = forward(theta, U)
    T = K * np.exp(y) * R
    tn = np.linalg.norm(T, axis=1)
    T = np.where(active[:, None], T / np.where(tn > 0, tn, 1.0)[:, None], 0.0)
    return T, active, rn
