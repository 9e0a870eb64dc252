"""Band solver steps: residual, preconditioner, Rayleigh-Ritz (test infrastructure, FP64).

The paper solves Eq. KS per subsystem with Quantum ESPRESSO's solver and
states nothing about it; the block-Davidson scheme below is this project's
reading, identical on the CPU and GPU sides:

* residual R_n = H x_n - lambda_n x_n, active_n = ||R_n|| > 1e-10;
* Teter-Payne-Allan preconditioner: T_n = K(x) R_n with
  x = (|k+G|^2/2) / T_n^kin, T_n^kin = sum_G |k+G|^2/2 |x_nG|^2 and
  K(x) = (27 + 18x + 12x^2 + 8x^3) / (27 + 18x + 12x^2 + 8x^3 + 16x^4);
  T_n is normalised, and set to zero when inactive;
* Rayleigh-Ritz on V = [X | T]: S = V^H V, A = V^H H V; inactive columns get
  S = e_j, A = 1e6 e_j (static shapes); S = L L^H by a column-by-column
  Cholesky that also masks a T column whose pivot falls below 1e-10 S_jj
  (a direction already in the span; without this the factor breaks down once
  several residuals share one error direction); A~ = L^{-1} A L^{-H}
  made Hermitian; A~ W = W Theta ascending; C = L^{-H} W[:, :nb];
  X = V C, HX = HV C, Lambda = Theta[:nb].

Pins: at a fixed potential the Ritz values converge to the lowest eigenvalues
of the dense matrix and never increase from one iteration to the next;
C^H S C = I (tests/test_oracle_solver.py).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

INACTIVE_DIAG = 1.0e6
DROP_TOL = 1.0e-10
ACTIVE_TOL = 1.0e-10


def tpa(x: np.ndarray) -> np.ndarray:
    """Teter-Payne-Allan polynomial ratio K(x).

    Pinned: K(0) = 1 and K ~ 1/(2x) for large x (the 27, 8 and 16). Parity
    unpinned: published constants -- the middle coefficients 18 and 12 are taken
    from Teter, Payne & Allan (1989) as printed.
    """
    p = 27.0 + 18.0 * x + 12.0 * x ** 2 + 8.0 * x ** 3
    return p / (p + 16.0 * x ** 4)


def residual(X: np.ndarray, HX: np.ndarray, lam: np.ndarray) -> np.ndarray:
    return HX - np.asarray(lam)[:, None] * X


def precondition(X: np.ndarray, HX: np.ndarray, lam: np.ndarray, kin: np.ndarray):
    """(T [nb, npw], active [nb] bool, ||R|| [nb])."""
    R = residual(X, HX, lam)
    rn = np.linalg.norm(R, axis=1)
    active = rn > ACTIVE_TOL
    tkin = np.einsum("g,ng->n", kin, np.abs(X) ** 2)
    x = kin[None, :] / tkin[:, None]
    T = tpa(x) * R
    tn = np.linalg.norm(T, axis=1)
    T = np.where(active[:, None], T / np.where(tn > 0, tn, 1.0)[:, None], 0.0)
    return T, active, rn


def subspace_rr(V: np.ndarray, HV: np.ndarray, nb: int, active=None, drop_tol=DROP_TOL):
    """Rayleigh-Ritz on the rows of V [m, npw]: (X [nb, npw], HX, Lambda [nb]).

    Masked columns (inactive, or dropped by the Cholesky) take no part: the
    projected problem is solved on the kept columns only, which is what the
    static-shape form (S = e_j, A = 1e6 e_j) computes in exact arithmetic.
    """
    V = np.asarray(V, dtype=np.complex128)
    HV = np.asarray(HV, dtype=np.complex128)
    m = V.shape[0]
    S = V.conj() @ V.T
    A = V.conj() @ HV.T
    keep = np.ones(m, dtype=bool) if active is None else np.asarray(active, dtype=bool).copy()
    for j in np.nonzero(~keep)[0]:
        S[j, :] = 0.0
        S[:, j] = 0.0
        S[j, j] = 1.0
    _, dropped = cholesky_drop(S, first_droppable=nb, tol=drop_tol)
    keep[dropped] = False
    idx = np.nonzero(keep)[0]
    Sk = S[np.ix_(idx, idx)]
    Ak = A[np.ix_(idx, idx)]
    L = np.linalg.cholesky(Sk)
    B = sla.solve_triangular(L, Ak, lower=True)
    At = sla.solve_triangular(L, B.conj().T, lower=True)
    At = 0.5 * (At + At.conj().T)
    theta, W = np.linalg.eigh(At)
    Ck = sla.solve_triangular(L.conj().T, W[:, :nb], lower=False)
    C = np.zeros((m, nb), dtype=np.complex128)
    C[idx] = Ck
    return C.T @ V, C.T @ HV, theta[:nb].copy()


def cholesky_drop(S: np.ndarray, first_droppable: int, tol: float):
    """Lower Cholesky factor of S, column by column, dropping near-dependent columns.

    Column j >= first_droppable whose pivot S_jj - sum_k |L_jk|^2 falls below
    tol * S_jj is treated as masked: its row and column become e_j (exactly the
    factor of S with row/column j replaced by e_j). A band column (j <
    first_droppable) with such a pivot is an error. Returns (L, dropped).
    """
    m = S.shape[0]
    L = np.zeros_like(S)
    dropped = []
    for j in range(m):
        d = S[j, j].real - np.sum(np.abs(L[j, :j]) ** 2)
        if j >= first_droppable and d < tol * S[j, j].real:
            L[j, :j] = 0.0
            L[j, j] = 1.0
            dropped.append(j)
            continue
        if not d >= tol * S[j, j].real:
            raise np.linalg.LinAlgError(f"band column {j} is linearly dependent (pivot {d:.3e})")
        L[j, j] = np.sqrt(d)
        for i in range(j + 1, m):
            L[i, j] = (S[i, j] - np.sum(L[i, :j] * L[j, :j].conj())) / L[j, j]
    return L, dropped


def orthonormalise(V: np.ndarray) -> np.ndarray:
    """Cholesky-QR: V <- L^{-1} V with V V^H = L L^H (rows orthonormal)."""
    V = np.asarray(V, dtype=np.complex128)
    S = V.conj() @ V.T
    L = np.linalg.cholesky(S)
    # rows x_n = sum_j C[j,n] v_j with C = L^{-H}
    C = sla.solve_triangular(L.conj().T, np.eye(len(S)), lower=False)
    return C.T @ V
