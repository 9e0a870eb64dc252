"""Pins of the oracle's density mixing and Methfessel-Paxton smearing (CPU only)."""
import math

import numpy as np
import pytest

import fde_synth
from oracle import basis, dft, mixing, occupations as occ, scf


def test_pulay_solves_an_affine_fixed_point_in_n_plus_one_steps():
    # F(x) = A x + b on R^6, not a contraction (simple iteration diverges); with K = 1
    # and the whole history Pulay is GMRES on the residual: exact after n + 1 evaluations
    rng = np.random.default_rng(7)
    n = 6
    A = rng.normal(0.0, 0.6, (n, n))
    assert np.max(np.abs(np.linalg.eigvals(A))) > 1.0
    b = rng.normal(0.0, 1.0, n)
    xs = np.linalg.solve(np.eye(n) - A, b)
    cell = basis.Cell((1.0, 1.0, 1.0), (2, 2, 2))
    m = mixing.Mixer(cell, "pulay", beta=0.5, nhist=n + 2, q0=0.0)
    x = np.zeros(n)
    for _ in range(n + 1):
        x = m(x, A @ x + b)
    # exact in exact arithmetic; the bordered normal equations square the condition
    # number of the residual basis, so FP64 keeps about half its digits here
    assert np.max(np.abs(x - xs)) < 1e-6 * np.max(np.abs(xs))
    for _ in range(2):
        x = m(x, A @ x + b)
    assert np.max(np.abs(x - xs)) < 1e-11 * np.max(np.abs(xs))


def test_pulay_with_one_entry_is_linear_mixing():
    rng = np.random.default_rng(8)
    cell = basis.Cell((5.0, 5.0, 5.0), (6, 6, 6))
    x, y = rng.uniform(0, 1, (2,) + cell.shape)
    got = mixing.pulay(cell, [x], [y - x], 0.3, 0.0)
    assert np.max(np.abs(got - (x + 0.3 * (y - x)))) < 1e-15
    lin = mixing.Mixer(cell, "linear", 0.3)(x, y)
    assert np.max(np.abs(got - lin)) < 1e-15


def test_kerker_on_a_plane_wave_and_a_uniform_density():
    cell = basis.Cell((6.0, 7.0, 8.0), (8, 10, 12))
    N1, N2, N3 = cell.grid
    z, y, x = np.meshgrid(np.arange(N3) / N3, np.arange(N2) / N2, np.arange(N1) / N1, indexing="ij")
    m = (2, -1, 3)
    G = np.array(m) * cell.b
    wave = np.cos(2 * np.pi * (m[0] * x + m[1] * y + m[2] * z))
    q0 = 0.8
    k = G @ G / (G @ G + q0 * q0)
    assert np.max(np.abs(mixing.kerker(cell, wave, q0) - k * wave)) < 1e-13
    ones = np.ones(cell.shape)
    assert np.max(np.abs(mixing.kerker(cell, ones, q0))) < 1e-14      # the charge is not moved
    assert np.max(np.abs(mixing.kerker(cell, ones, 0.0) - ones)) == 0.0


def test_methfessel_paxton_delta_has_unit_weight_and_zero_second_moment():
    x = np.linspace(-8.0, 8.0, 16001)
    h = 1e-5
    # S_1 = f / 2 at mu = 0, sigma = 1; the broadened delta is -dS_1/dx
    d = -(occ.methfessel_paxton(x + h, 0.0, 1.0) - occ.methfessel_paxton(x - h, 0.0, 1.0)) / (4 * h)
    w0 = np.trapezoid(d, x)
    w2 = np.trapezoid(x * x * d, x)
    assert abs(w0 - 1.0) < 1e-8
    assert abs(w2) < 1e-8
    # closed form of the delta: (3/2 - x^2) e^{-x^2} / sqrt(pi)
    assert np.max(np.abs(d - (1.5 - x * x) * np.exp(-x * x) / math.sqrt(math.pi))) < 1e-7
    assert occ.methfessel_paxton(np.array([-7.0]), 0.0, 1.0)[0] == pytest.approx(2.0, abs=1e-15)
    assert occ.methfessel_paxton(np.array([7.0]), 0.0, 1.0)[0] == pytest.approx(0.0, abs=1e-15)


def test_methfessel_paxton_occupations_count_electrons():
    eps = np.array([[-0.5, -0.3, -0.12, -0.1, 0.2, 0.4], [-0.45, -0.28, -0.11, -0.05, 0.25, 0.5]])
    wk = np.array([0.5, 0.5])
    for ne, sig in ((6.0, 0.01), (5.0, 0.05), (7.3, 0.02)):
        f, mu = occ.occupations(eps, wk, ne, "methfessel-paxton", sig)
        assert abs(np.sum(wk[:, None] * f) - ne) < 1e-13
    f, mu = occ.occupations(eps, wk, 6.0, "methfessel-paxton", 0.001)
    assert np.max(np.abs(f - np.array([[2, 2, 2, 0, 0, 0]] * 2))) < 1e-6   # sigma -> 0: integer


def test_pulay_reaches_a_self_consistent_solution():
    # on the two-subsystem cube Pulay + Kerker converges to a fixed point of the cycle
    # (input = output density, bands the lowest eigenvectors of their potential, both
    # E_FDE routes equal). It is not the one linear mixing reaches: this cell has two
    # self-consistent solutions (E_FDE -1.7540 and -1.9040 Ha), and the mixing decides
    # which one the cycle finds.
    from oracle import hamiltonian as ham
    s = fde_synth.config1()
    st = scf.setup(s)
    recs, X, _ = scf.run(s, n_cycles=60, st=st, mixer=mixing.Mixer(st.cell, "pulay", 0.5, 6, 0.5))
    r = recs[-1]
    ef = []
    for I, sub in enumerate(s.subsystems):
        assert np.sum(np.abs(r.rho_out[I] - r.rho_in[I])) * st.cell.dV < 1e-7
        dense = np.linalg.eigvalsh(ham.explicit_h(st.cell, st.spheres[0], r.veff[I]))
        assert np.max(np.abs(r.eps[I][0] - dense[:sub.nbands])) < 1e-8
        ef.append((r.eps[I], occ.occupations(r.eps[I], sub.kweight, sub.nelec, sub.smearing, sub.sigma)[0]))
    E = scf.energies(st, X, ef, r.veff, r.rho_out)
    assert abs(E["E_FDE"] - E["E_FDE_fragments"]) < 1e-10
    assert E["E_FDE"] == pytest.approx(-1.7540267, abs=1e-6)
