"""Pins of the oracle's H application (CPU only)."""
import math

import numpy as np

import fde_synth
from oracle import basis, dft, hamiltonian as ham, pseudo


def _small(kf=(0.25, -0.25, 0.0), grid=(10, 12, 9), L=(6.0, 7.0, 5.5), ecut=3.0):
    cell = basis.Cell(L, grid)
    return cell, basis.sphere(cell, ecut, kf)


def test_free_electrons_exact():
    cell, sph = _small()
    V0 = -0.37
    veff = np.full(cell.shape, V0)
    H = ham.explicit_h(cell, sph, veff)
    ev = np.linalg.eigvalsh(H)
    assert np.max(np.abs(ev - np.sort(sph.kin + V0))) < 1e-13
    # matrix-free on the plane waves themselves
    E = np.eye(sph.npw, dtype=complex)[:7]
    y = ham.apply_h(cell, sph, E, veff)
    assert np.max(np.abs(y - (sph.kin[:7, None] + V0) * E)) < 1e-13


def test_matrix_free_equals_explicit_with_projectors():
    cell, sph = _small()
    veff = fde_synth.random_real(4, cell.shape)
    atoms = [fde_synth.Atom((1.0, 2.0, 3.0), 1.0, 0.7, lmax=1, rbeta=0.8, d_s=0.9, d_p=-0.3),
             fde_synth.Atom((4.0, 5.5, 1.0), 1.0, 0.7, lmax=0, rbeta=0.6, d_s=1.3)]
    beta, dkb = pseudo.kb_projectors(cell, sph, atoms)
    assert beta.shape == (5, sph.npw)
    H = ham.explicit_h(cell, sph, veff, beta, dkb)
    assert np.max(np.abs(H - H.conj().T)) < 1e-14
    psi = fde_synth.random_complex(5, (4, sph.npw))
    y = ham.apply_h(cell, sph, psi, veff, beta, dkb)
    assert np.max(np.abs(y - psi @ H.T)) < 1e-12


def test_hermiticity_matrix_free():
    cell, sph = _small()
    veff = fde_synth.random_real(6, cell.shape)
    phi, psi = fde_synth.random_complex(7, (2, sph.npw))
    a = np.vdot(phi, ham.apply_h(cell, sph, psi[None], veff)[0])
    b = np.vdot(ham.apply_h(cell, sph, phi[None], veff)[0], psi)
    assert abs(a - b) < 1e-12 * abs(a)


def test_rank_one_projector_energy():
    cell, sph = _small()
    veff = fde_synth.random_real(8, cell.shape)
    atoms = [fde_synth.Atom((2.0, 2.0, 2.0), 1.0, 0.7, lmax=0, rbeta=0.7, d_s=0.75)]
    beta, dkb = pseudo.kb_projectors(cell, sph, atoms)
    psi = fde_synth.random_complex(9, (1, sph.npw))
    e0 = np.vdot(psi[0], ham.apply_h(cell, sph, psi, veff)[0]).real
    e1 = np.vdot(psi[0], ham.apply_h(cell, sph, psi, veff, beta, dkb)[0]).real
    assert abs((e1 - e0) - 0.75 * abs(np.vdot(beta[0], psi[0])) ** 2) < 1e-12


def test_projector_normalisation_continuum():
    # sum_G |beta(G)|^2 -> 1 once the sphere holds the Gaussian's transform
    cell = basis.Cell((9.0, 9.0, 9.0), (40, 40, 40))
    sph = basis.sphere(cell, 30.0, (0.0, 0.0, 0.0))
    atoms = [fde_synth.Atom((1.0, 2.0, 3.0), 1.0, 1.0, lmax=1, rbeta=1.0)]
    beta, _ = pseudo.kb_projectors(cell, sph, atoms)
    n = np.sum(np.abs(beta) ** 2, axis=1)
    assert np.max(np.abs(n - 1.0)) < 1e-6
    # p channels are orthogonal to s and to each other
    ov = beta.conj() @ beta.T
    assert np.max(np.abs(ov - np.diag(np.diag(ov)))) < 1e-6


def test_translation_by_grid_vector_keeps_spectrum():
    cell, sph = _small(kf=(0.0, 0.25, 0.0))
    N1, N2, N3 = cell.grid
    a = [fde_synth.Atom((1.1, 2.2, 0.7), 1.5, 0.6, lmax=0, rbeta=0.7)]
    shift = np.array([2 * cell.L[0] / N1, 3 * cell.L[1] / N2, 1 * cell.L[2] / N3])
    b = [fde_synth.Atom(tuple(np.array(a[0].pos) + shift), 1.5, 0.6, lmax=0, rbeta=0.7)]
    ev = []
    for atoms in (a, b):
        v = pseudo.local_potential(cell, 3.0, atoms)
        beta, dkb = pseudo.kb_projectors(cell, sph, atoms)
        ev.append(np.linalg.eigvalsh(ham.explicit_h(cell, sph, v, beta, dkb)))
    assert np.max(np.abs(ev[0] - ev[1])) < 1e-12


def test_local_potential_matches_erf_far_field():
    # single Gaussian ion in a big box: V(r) ~ -Z erf(r/(sqrt2 s))/r + const
    cell = basis.Cell((16.0, 16.0, 16.0), (48, 48, 48))
    ecut = 9.0
    Z, s = 2.0, 0.9
    c = np.array([8.0, 8.0, 8.0])
    v = pseudo.local_potential(cell, ecut, [fde_synth.Atom(tuple(c), Z, s)])
    x, y, z = cell.positions()
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    from scipy.special import erf
    ref = np.where(r > 0, -Z * erf(r / (math.sqrt(2) * s)) / np.where(r > 0, r, 1), -Z * math.sqrt(2 / math.pi) / s)
    # compare differences between two inner points (periodic images and G=0 shift cancel
    # to the quadrupole order for points near the ion)
    i1 = (24, 24, 24)
    i2 = (24, 24, 27)
    d_or = v[i1] - v[i2]
    d_ref = ref[i1] - ref[i2]
    assert abs(d_or - d_ref) < 2e-3
