"""Pins of the oracle's augmentation: overlap operator, generalised Rayleigh-Ritz and
augmentation charge (CPU only)."""
import numpy as np
import pytest
import scipy.linalg as sla

import fde_synth
from oracle import augment as oaug, basis, density as dens, hamiltonian as ham, pseudo, subspace


def _cell(with_kb=True):
    s = fde_synth.tiny(3, with_kb=with_kb, nbands=4)
    cell = basis.Cell(s.L, s.grid)
    sph = basis.sphere(cell, s.ecut, s.subsystems[0].kfrac[0])
    atoms = [a for sub in s.subsystems for a in sub.atoms]
    v = pseudo.local_potential(cell, s.ecut, atoms)
    own = s.subsystems[0].atoms
    beta, dkb = pseudo.kb_projectors(cell, sph, own)
    q, atom_of = fde_synth.augmentation_q(own)
    return s, cell, sph, v, beta, dkb, q, atom_of, own


def test_overlap_of_one_projector_closed_form():
    """S = 1 + q |b><b|: S b = (1 + q <b|b>) b, and S x = x for x orthogonal to b."""
    _, cell, sph, _, beta, _, _, _, _ = _cell()
    b = beta[:1]
    q = np.array([[0.7]])
    nb2 = float(np.real(np.vdot(b[0], b[0])))
    assert abs(nb2 - 1.0) < 0.1  # unit-normalised in the continuum, truncated by the sphere
    Sb = oaug.apply_s(b, b, q)
    assert np.max(np.abs(Sb - (1.0 + 0.7 * nb2) * b)) < 1e-14
    x = fde_synth.random_complex(5, (1, sph.npw))
    x = x - (np.vdot(b[0], x[0]) / nb2) * b
    assert np.max(np.abs(oaug.apply_s(x, b, q) - x)) < 1e-14


def test_zero_overlap_is_the_standard_step():
    _, cell, sph, v, beta, dkb, q, _, _ = _cell()
    V = subspace.orthonormalise(fde_synth.random_complex(6, (8, sph.npw)))
    HV = ham.apply_h(cell, sph, V, v, beta, dkb)
    X, HX, SX, lam = oaug.subspace_rr_gen(V, HV, oaug.apply_s(V, beta, 0.0 * q), 4)
    X0, HX0, lam0 = subspace.subspace_rr(V, HV, 4)
    assert np.max(np.abs(lam - lam0)) < 1e-12
    assert np.max(np.abs(X.T @ X.conj() - X0.T @ X0.conj())) < 1e-11
    assert np.max(np.abs(SX - X)) < 1e-13


def test_generalised_davidson_reaches_the_dense_generalised_eigenvalues():
    """H x = eps S x: the Davidson iterates converge to scipy's dense generalised
    eigenvalues of (H_GG', S_GG'), and the bands come out S-orthonormal."""
    s, cell, sph, v, beta, dkb, q, _, _ = _cell()
    H = ham.explicit_h(cell, sph, v, beta, dkb)
    Sd = np.eye(sph.npw) + beta.T @ q @ beta.conj()
    ev = sla.eigh(H, Sd, eigvals_only=True)[:6]
    X0 = fde_synth.random_complex(7, (6, sph.npw)) / (1 + sph.kin)[None]
    Hf = lambda Y: ham.apply_h(cell, sph, Y, v, beta, dkb)  # noqa: E731
    Sf = lambda Y: oaug.apply_s(Y, beta, q)  # noqa: E731
    X, HX, SX, hist = oaug.davidson_gen(Hf, Sf, X0, 60, sph.kin)
    # the lowest four of a six-band block
    assert np.max(np.abs(hist[-1][:4] - ev[:4])) < 1e-9, np.max(np.abs(hist[-1][:4] - ev[:4]))
    assert np.all(np.diff([h.sum() for h in hist]) <= 1e-10)  # Ritz values never rise
    assert np.all(hist[-1] >= ev - 1e-12)                     # and bound the exact ones from above
    assert np.max(np.abs(X.conj() @ SX.T - np.eye(6))) < 1e-10
    # and they are not the standard eigenvalues
    assert np.max(np.abs(ev - np.linalg.eigvalsh(H)[:6])) > 1e-3


def test_augmented_density_carries_the_missing_charge():
    """For S-orthonormal bands, int (rho + rho_aug) = sum_n f_n: the atom charges from the
    projections equal <psi|S - 1|psi>, and the Gaussian charges integrate to c_a."""
    s, cell, sph, v, beta, dkb, q, atom_of, own = _cell()
    Hf = lambda Y: ham.apply_h(cell, sph, Y, v, beta, dkb)  # noqa: E731
    Sf = lambda Y: oaug.apply_s(Y, beta, q)  # noqa: E731
    X, HX, SX, _ = oaug.davidson_gen(Hf, Sf, fde_synth.random_complex(8, (4, sph.npw)), 5, sph.kin)
    occw = np.array([2.0, 2.0, 1.5, 0.25])
    c = oaug.atom_charges(beta, X, occw, q, atom_of)
    extra = float(np.real(np.sum(occw * np.einsum("ng,ng->n", X.conj(), SX - X))))
    assert abs(c.sum() - extra) < 1e-12
    rho = dens.density(cell, sph, X, occw)
    rho_aug = oaug.augmentation_density(cell, s.ecut, [a.pos for a in own], [a.rbeta for a in own], c)
    assert abs((rho.sum() + rho_aug.sum()) * cell.dV - occw.sum()) < 1e-11
    # the Gaussian shape: a direct sum over periodic images at a few points
    N1, N2, N3 = cell.grid
    for (i3, i2, i1) in [(0, 0, 0), (3, 5, 7), (N3 - 1, 2, N1 // 2)]:
        r = np.array([i1 * cell.L[0] / N1, i2 * cell.L[1] / N2, i3 * cell.L[2] / N3])
        val = 0.0
        for a, ca in zip(own, c):
            w = a.rbeta
            for n in np.ndindex(5, 5, 5):
                d = r - np.asarray(a.pos) - (np.array(n) - 2) * np.asarray(cell.L)
                val += ca * (2 * np.pi * w * w) ** -1.5 * np.exp(-d @ d / (2 * w * w))
        assert abs(rho_aug[i3, i2, i1] - val) < 2e-3 * max(1.0, abs(c).max()), (val, rho_aug[i3, i2, i1])


def _aug_system():
    s = fde_synth.tiny(4, with_kb=True, nbands=3)
    s.subsystems[0].aug = True  # subsystem-specific: only the first one is augmented
    return s


def test_augmented_cycle_conserves_charge_and_solves_the_generalised_problem():
    """Every cycle's rho_I (bands plus augmentation) holds N_I electrons, and after the
    cycle settles the augmented subsystem's eigenvalues are the dense generalised ones of
    its last potential, the other subsystem's the standard ones."""
    from oracle import scf
    s = _aug_system()
    recs, X, st = scf.run(s, n_cycles=30, n_david=4)
    for r in recs:
        for I, sub in enumerate(s.subsystems):
            assert abs(r.rho_out[I].sum() * st.cell.dV - sub.nelec) < 1e-11
    d = [np.max(np.abs(r.rho_out - r.rho_in)) for r in recs]
    assert d[-1] < 1e-5 and d[-1] < 1e-3 * d[0]
    last = recs[-1]
    sph = st.spheres[0]
    for I, sub in enumerate(s.subsystems):
        beta, dkb = st.proj[(I, 0)]
        H = ham.explicit_h(st.cell, sph, last.veff[I], beta, dkb)
        if I == 0:
            q, _ = fde_synth.augmentation_q(sub.atoms)
            Sd = np.eye(sph.npw) + beta.T @ q @ beta.conj()
            ev = sla.eigh(H, Sd, eigvals_only=True)[:2]
        else:
            ev = np.linalg.eigvalsh(H)[:2]
        assert np.max(np.abs(last.eps[I][0][:2] - ev)) < 1e-8, (I, last.eps[I][0][:2], ev)


def test_energies_of_augmented_subsystems_are_rejected():
    """The augmented energy needs one-centre terms the synthetic overlaps do not define."""
    from oracle import scf
    s = _aug_system()
    recs, X, st = scf.run(s, n_cycles=1, n_david=1)
    with pytest.raises(ValueError, match="augmented"):
        scf.energies(st, X, [], recs[-1].veff, recs[-1].rho_out)
