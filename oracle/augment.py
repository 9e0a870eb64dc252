"""Subsystem-specific augmentation: overlap operator, generalised Rayleigh-Ritz and
augmentation charge (test infrastructure, FP64).

Appendix, non-local pseudopotentials: with PAW or ultrasoft pseudopotentials the
smooth orbitals of subsystem I are tied to the true ones by T^I = 1 + sum over the
atoms a of I of sum_i (|phi_i^a> - |phi~_i^a>) <p~_i^a|, with projectors of the
subsystem's own atoms only. The smooth orbitals then solve the generalised problem
H psi = eps S^I psi with the overlap S^I = (T^I)^H T^I = 1 + sum_{a in I} sum_ij
|p~_i^a> q_ij^a <p~_j^a| (q_ij^a = <phi_i|phi_j> - <phi~_i|phi~_j>), are
S^I-orthonormal, and the density gains the augmentation charge
sum_a sum_ij rho_ij^a Q_ij^a(r), rho_ij^a = sum_n f_n <psi_n|p~_i^a><p~_j^a|psi_n>,
with int Q_ij^a = q_ij^a.

Synthetic reading (no PAW data sets are available): the projectors p~ are the
Gaussian s and p projectors of `pseudo.kb_projectors`; q^a is an Hermitian positive
semi-definite block per atom (nproj x nproj overall, zero between atoms) given by
the caller; Q_ij^a(r) = q_ij^a g_a(r) with g_a a unit-normalised Gaussian of width
w_a at the atom, so the augmentation charge of atom a is c_a g_a(r) with
c_a = sum_{i,j in a} q_ij rho_ij^a.

The Rayleigh-Ritz step is the one of `subspace` with S = V^H (S^I V).

Pins (tests/test_oracle_augment.py): q = 0 gives the standard step; the
generalised Ritz values equal scipy.linalg.eigh(A, S) of the projected matrices;
X^H S X = I; the Davidson iteration converges to the dense generalised
eigenvalues of (H_GG', S_GG'); the augmented density integrates to sum_n f_n.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import basis, subspace

DROP_TOL = subspace.DROP_TOL


def projections(beta: np.ndarray, X: np.ndarray) -> np.ndarray:
    """P[i, n] = <beta_i | x_n> (beta [nproj, npw], X [nb, npw])."""
    return np.asarray(beta).conj() @ np.asarray(X).T


def apply_s(X: np.ndarray, beta: np.ndarray, q: np.ndarray) -> np.ndarray:
    """S X = X + sum_ij beta_i q_ij <beta_j|X> (rows of X)."""
    X = np.asarray(X, dtype=np.complex128)
    if beta is None or len(beta) == 0:
        return X.copy()
    return X + (np.asarray(q) @ projections(beta, X)).T @ np.asarray(beta)


def subspace_rr_gen(V, HV, SV, nb, active=None, drop_tol=DROP_TOL):
    """Generalised Rayleigh-Ritz on the rows of V: (X, HX, SX, Lambda), with
    S = V^H (S V) in place of V^H V, otherwise exactly `subspace.subspace_rr`
    (masks, dropping, Cholesky reduction, ascending eigenpairs)."""
    V = np.asarray(V, dtype=np.complex128)
    HV = np.asarray(HV, dtype=np.complex128)
    SV = np.asarray(SV, dtype=np.complex128)
    m = V.shape[0]
    S = V.conj() @ SV.T
    A = V.conj() @ HV.T
    keep = np.ones(m, dtype=bool) if active is None else np.asarray(active, dtype=bool).copy()
    for j in np.nonzero(~keep)[0]:
        S[j, :] = 0.0
        S[:, j] = 0.0
        S[j, j] = 1.0
    _, dropped = subspace.cholesky_drop(S, first_droppable=nb, tol=drop_tol)
    keep[dropped] = False
    idx = np.nonzero(keep)[0]
    Sk = 0.5 * (S[np.ix_(idx, idx)] + S[np.ix_(idx, idx)].conj().T)
    Ak = A[np.ix_(idx, idx)]
    L = np.linalg.cholesky(Sk)
    B = sla.solve_triangular(L, Ak, lower=True)
    At = sla.solve_triangular(L, B.conj().T, lower=True)
    At = 0.5 * (At + At.conj().T)
    theta, W = np.linalg.eigh(At)
    Ck = sla.solve_triangular(L.conj().T, W[:, :nb], lower=False)
    C = np.zeros((m, nb), dtype=np.complex128)
    C[idx] = Ck
    return C.T @ V, C.T @ HV, C.T @ SV, theta[:nb].copy()


def precondition_gen(X, HX, SX, lam, kin):
    """The TPA preconditioner of `subspace.precondition` on the generalised residual
    R_n = H x_n - lambda_n S x_n: (T, active, ||R||)."""
    R = np.asarray(HX) - np.asarray(lam)[:, None] * np.asarray(SX)
    rn = np.linalg.norm(R, axis=1)
    active = rn > subspace.ACTIVE_TOL
    tkin = np.einsum("g,ng->n", kin, np.abs(X) ** 2)
    x = kin[None, :] / tkin[:, None]
    T = subspace.tpa(x) * R
    tn = np.linalg.norm(T, axis=1)
    T = np.where(active[:, None], T / np.where(tn > 0, tn, 1.0)[:, None], 0.0)
    return T, active, rn


def davidson_gen(H, S, X0, n_iter, kin):
    """Block Davidson at a fixed potential for H x = eps S x (H, S: callables on rows):
    Rayleigh-Ritz on X0, then n_iter iterations of the generalised residual, TPA,
    and Rayleigh-Ritz on [X | T]. Returns the Ritz values after every step."""
    nb = X0.shape[0]
    X, HX, SX, lam = subspace_rr_gen(X0, H(X0), S(X0), nb)
    hist = [lam.copy()]
    for _ in range(n_iter):
        T, active, _ = precondition_gen(X, HX, SX, lam, kin)
        act = np.concatenate([np.ones(nb, dtype=bool), active])
        X, HX, SX, lam = subspace_rr_gen(np.vstack([X, T]), np.vstack([HX, H(T)]), np.vstack([SX, S(T)]), nb, act)
        hist.append(lam.copy())
    return X, HX, SX, hist


def atom_charges(beta, X, occw, q, atom_of):
    """c_a = sum_n f_n sum_{i,j in a} conj(P_in) q_ij P_jn (atom_of[i]: the atom of
    projector i; q zero between atoms)."""
    P = projections(beta, X)
    natom = int(np.max(atom_of)) + 1 if len(atom_of) else 0
    c = np.zeros(natom)
    for a in range(natom):
        idx = np.nonzero(np.asarray(atom_of) == a)[0]
        Pa = P[idx]
        c[a] = float(np.real(np.einsum("n,in,ij,jn->", occw, Pa.conj(), np.asarray(q)[np.ix_(idx, idx)], Pa)))
    return c


def augmentation_density(cell: basis.Cell, ecut: float, pos, width, charges) -> np.ndarray:
    """sum_a c_a g_a(r) on the grid [N3, N2, N1], g_a the unit-normalised Gaussian of
    width w_a at R_a: c_a exp(-G^2 w_a^2 / 2) e^{-iG.R_a} / Omega on the density
    sphere D, then the inverse transform (the construction of `pseudo.local_potential`)."""
    from . import dft
    g1, g2, g3 = basis.grid_g(cell)
    G2 = g1 * g1 + g2 * g2 + g3 * g3
    mask = basis.density_mask(cell, ecut)
    F = np.zeros(cell.shape, dtype=np.complex128)
    for R, w, ca in zip(pos, width, charges):
        R = np.asarray(R, dtype=np.float64)
        phase = np.exp(-1j * (g1[mask] * R[0] + g2[mask] * R[1] + g3[mask] * R[2]))
        F[mask] += ca * np.exp(-0.5 * G2[mask] * w * w) * phase
    return dft.to_real(F / cell.omega).real
