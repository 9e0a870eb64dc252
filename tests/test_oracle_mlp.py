"""Pins of the oracle's learned-preconditioner network (CPU only)."""
import numpy as np

import fde_synth
from oracle import basis, hamiltonian as ham, mlp, pseudo, subspace


def _samples(n, seed):
    rng = np.random.default_rng(seed)
    U = rng.normal(0.0, 1.0, (n, 4))
    A = rng.uniform(0.1, 2.0, n)
    B = rng.uniform(-1.0, 1.0, n) * np.sqrt(A)
    C = B * B / A + rng.uniform(0.0, 1.0, n)
    return np.concatenate([U, A[:, None], B[:, None], C[:, None]], axis=1)


def _theta(seed):
    t = fde_synth.mlp_init(seed)
    rng = np.random.default_rng(seed + 1)
    t[mlp.OFF_W3:mlp.OFF_B3] = rng.normal(0.0, 0.3, mlp.HID)
    t[mlp.OFF_B3] = 0.1
    t[mlp.OFF_B1:mlp.OFF_W2] = rng.normal(0.0, 0.1, mlp.HID)
    t[mlp.OFF_B2:mlp.OFF_W3] = rng.normal(0.0, 0.1, mlp.HID)
    return t


def test_layout_size():
    assert mlp.NPARAM == 4545 and fde_synth.mlp_init(0).size == mlp.NPARAM


def test_gradient_matches_central_differences():
    S = _samples(50, 3)
    th = _theta(4)
    L, g = mlp.loss_grad(th, S)
    assert abs(L - mlp.loss(th, S)) < 1e-14 * abs(L)
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(np.arange(mlp.OFF_W1, mlp.OFF_B1), 6), rng.choice(np.arange(mlp.OFF_B1, mlp.OFF_W2), 4),
                          rng.choice(np.arange(mlp.OFF_W2, mlp.OFF_B2), 10), rng.choice(np.arange(mlp.OFF_B2, mlp.OFF_W3), 4),
                          rng.choice(np.arange(mlp.OFF_W3, mlp.OFF_B3), 4), [mlp.OFF_B3]])
    h = 1e-5
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, S) - mlp.loss(tm, S)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_loss_minimum_per_sample():
    # one sample: the loss A e^{2y} - 2 B e^y + C is stationary at e^y = B / A
    S = _samples(1, 7)
    S[0, 5] = abs(S[0, 5]) + 0.1
    th = np.zeros(mlp.NPARAM)
    th[mlp.OFF_B3] = np.log(S[0, 5] / S[0, 4])
    L, g = mlp.loss_grad(th, S)
    assert abs(g[mlp.OFF_B3]) < 1e-12
    assert abs(L - (S[0, 6] - S[0, 5] ** 2 / S[0, 4])) < 1e-12


def _small():
    cell = basis.Cell((6.0, 6.5, 7.0), (12, 12, 14))
    sph = basis.sphere(cell, 2.5, (0.25, 0.0, -0.25))
    atoms = [fde_synth.Atom((1.0, 2.0, 3.0), 2.0, 0.6), fde_synth.Atom((4.0, 4.5, 5.0), 1.0, 0.6)]
    v = pseudo.local_potential(cell, 2.5, atoms)
    return cell, sph, v


def test_zero_network_is_tpa():
    cell, sph, v = _small()
    nb = 3
    X = subspace.orthonormalise(fde_synth.random_complex(41, (nb, sph.npw)))
    HX = ham.apply_h(cell, sph, X, v)
    lam = np.real(np.sum(X.conj() * HX, axis=1))
    th = fde_synth.mlp_init(0)           # output layer zero
    T1, a1, r1 = subspace.precondition(X, HX, lam, sph.kin)
    T2, a2, r2 = mlp.precondition(th, X, HX, lam, sph.kin, float(np.mean(v)))
    assert np.array_equal(T1, T2) and np.array_equal(a1, a2) and np.array_equal(r1, r2)


def test_exact_correction_solves_projected_equation():
    cell, sph, v = _small()
    Hm = ham.explicit_h(cell, sph, v)
    X = subspace.orthonormalise(fde_synth.random_complex(42, (1, sph.npw)) / (1 + 2 * sph.kin)[None])
    x = X[0]
    eps = float(np.real(x.conj() @ Hm @ x))
    r = Hm @ x - eps * x
    d = mlp.exact_correction(Hm, x, eps, r)
    assert abs(x.conj() @ d) < 1e-12 * np.linalg.norm(d)
    P = np.eye(sph.npw) - np.outer(x, x.conj())
    res = P @ (Hm - eps * np.eye(sph.npw)) @ P @ d + r
    assert np.linalg.norm(res) < 1e-10 * np.linalg.norm(r)


def test_sample_rows_reproduce_the_band_loss():
    cell, sph, v = _small()
    Hm = ham.explicit_h(cell, sph, v)
    nb = 2
    X = subspace.orthonormalise(fde_synth.random_complex(43, (nb, sph.npw)) / (1 + 2 * sph.kin)[None])
    HX = X @ Hm.T
    lam = np.real(np.sum(X.conj() * HX, axis=1))
    R = HX - lam[:, None] * X
    D = np.stack([mlp.exact_correction(Hm, X[n], lam[n], R[n]) for n in range(nb)])
    vbar = float(np.mean(v))
    S = mlp.samples(sph.kin, X, R, lam, vbar, D)
    th = np.zeros(mlp.NPARAM)
    _, K = mlp.features(sph.kin, X, R, lam, vbar)
    direct = 0.0
    for n in range(nb):
        kr = K[n] * R[n]
        a = np.real(np.vdot(kr, D[n])) / np.vdot(kr, kr).real
        direct += sph.npw / np.vdot(D[n], D[n]).real * np.sum(np.abs(a * kr - D[n]) ** 2)
    assert abs(mlp.loss(th, S) - direct / S.shape[0]) < 1e-12 * direct / S.shape[0]


def test_adam_first_steps_closed_form():
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 2.0])
    m = np.zeros(3)
    v = np.zeros(3)
    t1, m, v = mlp.adam(th, g, m, v, 1, 0.01)
    # bias-corrected moments equal g and g^2 after the first step
    assert np.allclose(t1, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    t2, m, v = mlp.adam(t1, g, m, v, 2, 0.01)
    assert np.allclose(t2, t1 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-14)
