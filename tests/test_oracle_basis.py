"""Pins of the oracle's transforms, plane-wave sets and density (CPU only)."""
import itertools
import math

import numpy as np
import pytest

import fde_synth
from oracle import basis, density, dft


def test_dft_equals_direct_sum():
    # brute-force triple sum on a ragged 5 x 3 x 4 grid (N1, N2, N3)
    f = fde_synth.random_complex(1, (4, 3, 5))
    N3, N2, N1 = f.shape
    F = dft.to_reciprocal(f)
    for m3, m2, m1 in [(0, 0, 0), (1, 2, 3), (3, 1, 4), (2, 0, 1)]:
        acc = 0j
        for j3, j2, j1 in itertools.product(range(N3), range(N2), range(N1)):
            acc += f[j3, j2, j1] * np.exp(-2j * math.pi * (m1 * j1 / N1 + m2 * j2 / N2 + m3 * j3 / N3))
        assert abs(F[m3, m2, m1] - acc / (N1 * N2 * N3)) < 1e-14
    g = dft.to_real(F)
    assert np.max(np.abs(g - f)) < 1e-14


def test_parseval_and_plane_wave():
    cell = basis.Cell((6.0, 7.0, 8.0), (10, 12, 15))
    sph = basis.sphere(cell, 2.0, (0.25, -0.25, 0.0))
    c = fde_synth.random_complex(2, (sph.npw,))
    c /= np.linalg.norm(c)
    u = dft.to_real(basis.to_grid(cell, sph, c)) / math.sqrt(cell.omega)
    assert abs(np.sum(np.abs(u) ** 2) * cell.dV - 1.0) < 1e-14
    # a single plane wave is a delta in G and a uniform |u|^2 = 1/Omega in r
    e = np.zeros(sph.npw, complex)
    e[sph.npw // 3] = 1.0
    rho = density.density(cell, sph, e[None], np.array([2.0]))
    assert np.max(np.abs(rho - 2.0 / cell.omega)) < 1e-15
    back = basis.from_grid(sph, dft.to_reciprocal(dft.to_real(basis.to_grid(cell, sph, e))))
    assert np.max(np.abs(back - e)) < 1e-15


def test_sphere_brute_force_count_and_order():
    cell = basis.Cell((10.0, 10.0, 10.0), (24, 24, 24))
    kf = np.array([0.25, 0.0, -0.25])
    sph = basis.sphere(cell, 7.0, kf)
    # independent enumeration: every grid Miller index, vectorised test
    m = np.array(list(itertools.product(range(-12, 12), repeat=3)))
    q = (m + kf) * cell.b
    inside = m[0.5 * np.sum(q * q, axis=1) <= 7.0]
    assert len(inside) == sph.npw
    assert sorted(map(tuple, inside)) == list(map(tuple, sph.miller))  # lexicographic
    assert np.all(sph.kin <= 7.0)
    # Gamma-point set of the 24^3 test cell: symmetric under G -> -G
    g0 = basis.sphere(cell, 7.0, (0, 0, 0))
    assert set(map(tuple, g0.miller)) == set(map(tuple, -g0.miller))


def test_density_charge_conservation():
    cell = basis.Cell((8.0, 8.0, 9.0), (12, 12, 15))
    sph = basis.sphere(cell, 2.5, (0.0, 0.25, 0.0))
    from oracle import subspace
    X = subspace.orthonormalise(fde_synth.random_complex(3, (5, sph.npw)))
    occw = np.array([2.0, 2.0, 1.5, 0.25, 0.0]) * 0.5
    rho = density.density(cell, sph, X, occw)
    assert rho.min() >= 0.0
    assert abs(rho.sum() * cell.dV - occw.sum()) < 1e-13


def test_grid_condition():
    with pytest.raises(ValueError):
        basis.check_grid(basis.Cell((10.0, 10.0, 10.0), (20, 24, 24)), 7.0)
    basis.check_grid(basis.Cell((10.0, 10.0, 10.0), (24, 24, 24)), 7.0)


def test_fft_mode_equals_the_dense_dft():
    import fde_synth
    from oracle import dft
    for shape in ((24, 24, 24), (9, 12, 10)):
        f = fde_synth.random_complex(3, shape)
        a, b = dft.to_reciprocal(f), dft.to_real(f)
        dft.set_mode("fft", 2)
        try:
            c, d = dft.to_reciprocal(f), dft.to_real(f)
        finally:
            dft.set_mode("naive")
        assert np.max(np.abs(a - c)) < 1e-13 * np.max(np.abs(a))
        assert np.max(np.abs(b - d)) < 1e-13 * np.max(np.abs(b))
