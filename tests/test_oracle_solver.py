"""Pins of the oracle's band solver and occupations (CPU only)."""
import numpy as np

import fde_synth
from oracle import basis, hamiltonian as ham, occupations as occ, pseudo, subspace


def _problem(kf=(0.25, 0.0, -0.25)):
    cell = basis.Cell((6.0, 6.5, 7.0), (12, 12, 14))
    sph = basis.sphere(cell, 2.5, kf)
    atoms = [fde_synth.Atom((1.0, 2.0, 3.0), 2.0, 0.6, lmax=1, rbeta=0.7, d_s=0.8, d_p=0.4),
             fde_synth.Atom((4.0, 4.5, 5.0), 1.0, 0.6, lmax=0, rbeta=0.7, d_s=1.1)]
    v = pseudo.local_potential(cell, 2.5, atoms)
    beta, dkb = pseudo.kb_projectors(cell, sph, atoms)
    return cell, sph, v, beta, dkb


def test_tpa_closed_form():
    assert subspace.tpa(np.array([0.0]))[0] == 1.0
    x = np.array([1e3])
    assert abs(subspace.tpa(x)[0] * 2 * x[0] - 1) < 2e-3   # K ~ 1/(2x) for large x


def test_davidson_converges_to_dense_eigenvalues_monotonically():
    cell, sph, v, beta, dkb = _problem()
    H = ham.explicit_h(cell, sph, v, beta, dkb)
    exact = np.linalg.eigvalsh(H)
    nb = 4
    X = fde_synth.random_coefficients(9, 0, 0, 0, nb, sph.npw) / (1 + 2 * sph.kin)[None]
    HX = ham.apply_h(cell, sph, X, v, beta, dkb)
    X, HX, lam = subspace.subspace_rr(X, HX, nb)
    prev = lam
    for it in range(80):
        T, active, rn = subspace.precondition(X, HX, lam, sph.kin)
        HT = ham.apply_h(cell, sph, T, v, beta, dkb)
        act = np.concatenate([np.ones(nb, bool), active])
        X, HX, lam = subspace.subspace_rr(np.vstack([X, T]), np.vstack([HX, HT]), nb, act)
        assert np.all(lam <= prev + 1e-11)      # X is inside span[X|T]: Ritz values never rise
        prev = lam
    assert np.max(np.abs(lam - exact[:nb])) < 1e-10
    assert np.max(np.abs(X.conj() @ X.T - np.eye(nb))) < 1e-12
    assert np.max(np.abs(HX - ham.apply_h(cell, sph, X, v, beta, dkb))) < 1e-10


def test_inactive_columns_are_ignored():
    cell, sph, v, beta, dkb = _problem()
    nb = 3
    X = subspace.orthonormalise(fde_synth.random_complex(40, (nb, sph.npw)))
    HX = ham.apply_h(cell, sph, X, v, beta, dkb)
    X, HX, lam = subspace.subspace_rr(X, HX, nb)
    T, active, _ = subspace.precondition(X, HX, lam, sph.kin)
    HT = ham.apply_h(cell, sph, T, v, beta, dkb)
    act = np.array([True] * nb + [True, False, True])
    T2 = T.copy(); T2[1] = 0.0
    HT2 = HT.copy(); HT2[1] = 0.0
    a = subspace.subspace_rr(np.vstack([X, T2]), np.vstack([HX, HT2]), nb, act)
    keep = [0, 1, 2, 3, 5]
    b = subspace.subspace_rr(np.vstack([X, T])[keep], np.vstack([HX, HT])[keep], nb)
    assert np.max(np.abs(a[2] - b[2])) < 1e-12


def test_occupations():
    eps = np.array([[-0.5, -0.3, -0.1, 0.2, 0.4], [-0.45, -0.28, -0.05, 0.25, 0.5]])
    wk = np.array([0.5, 0.5])
    f, mu = occ.occupations(eps, wk, 6.0, "fermi-dirac", 0.01)
    assert abs(np.sum(wk[:, None] * f) - 6.0) < 1e-13
    assert -0.05 < mu < 0.2                       # in the gap
    assert np.max(np.abs(f - np.array([[2, 2, 2, 0, 0]] * 2))) < 1e-5   # sigma -> 0: integer
    f2, _ = occ.occupations(eps, wk, 5.0, "fermi-dirac", 0.05)
    assert abs(np.sum(wk[:, None] * f2) - 5.0) < 1e-13
    assert np.all((f2 >= 0) & (f2 <= 2))
    fi, _ = occ.occupations(eps, wk, 4.0, "integer")
    assert np.array_equal(fi, np.array([[2, 2, 0, 0, 0]] * 2, float))
