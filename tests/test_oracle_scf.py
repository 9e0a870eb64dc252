"""Pins of the oracle's embedding cycle and energies (CPU only)."""
import numpy as np

import fde_synth
from oracle import basis, density as dens, embed, hamiltonian as ham, occupations as occ, scf


def test_band_energy_identity_and_two_energy_routes():
    s = fde_synth.tiny(0, with_kb=True, kfrac=[(0.25, 0.0, 0.0), (-0.25, 0.0, 0.0)])
    recs, X, st = scf.run(s, n_cycles=3, n_david=3)
    last = recs[-1]
    eps_f = []
    for I, sub in enumerate(s.subsystems):
        f, _ = occ.occupations(last.eps[I], sub.kweight, sub.nelec, sub.smearing, sub.sigma)
        eps_f.append((last.eps[I], f))
    E = scf.energies(st, X, eps_f, last.veff, last.rho_out)
    for lhs, rhs in E["identity"]:      # sum eps + V_K rho_K = T_J + E_eN + E_NL
        assert abs(lhs - rhs) < 1e-12 * max(1, abs(rhs))
    assert abs(E["E_FDE"] - E["E_FDE_fragments"]) < 1e-12 * abs(E["E_FDE"])
    # charges
    for I, sub in enumerate(s.subsystems):
        assert abs(last.rho_out[I].sum() * st.cell.dV - sub.nelec) < 1e-12


def test_converged_cycle_matches_dense_diagonalisation():
    s = fde_synth.tiny(1, nsub=2, nbands=2)
    recs, X, st = scf.run(s, n_cycles=40, n_david=4)
    last = recs[-1]
    # the cycle contracts towards the fixed point rho_out = rho_in
    d = [np.max(np.abs(r.rho_out - r.rho_in)) for r in recs]
    assert d[-1] < 1e-4 and d[-1] < 1e-2 * d[0]
    # and every cycle's bands solve Eq. KS for that cycle's potential
    sph = st.spheres[0]
    for I in range(2):
        H = ham.explicit_h(st.cell, sph, last.veff[I])
        exact = np.linalg.eigvalsh(H)[:2]
        assert np.max(np.abs(last.eps[I][0] - exact)) < 1e-9


def test_single_subsystem_equals_kohn_sham():
    s = fde_synth.tiny(2, nsub=1, nbands=2)
    recs, X, st = scf.run(s, n_cycles=2, n_david=2)
    v = recs[-1].veff[0]
    rho = recs[-2].rho_in[0]
    VH, _ = embed.hartree(st.cell, s.ecut, rho)
    _, vxc = embed.xc(rho, st.cell)
    assert np.max(np.abs(v - (st.vloc + VH + vxc))) < 1e-13


def test_freeze_thaw_with_one_inner_cycle_is_the_jacobi_cycle():
    """env_I + rho_I = rho: with one inner cycle per broadcast the two schemes see the same
    potentials (up to the summation order of rho)."""
    s = fde_synth.tiny(1, nsub=2, nbands=2)
    ra, _, _ = scf.run(s, n_cycles=3, n_david=3)
    rb, _, _ = scf.run(s, n_cycles=3, n_david=3, scheme="freeze-thaw", n_inner=1)
    assert len(rb) == 3
    for a, b in zip(ra, rb):
        assert np.max(np.abs(a.veff - b.veff)) < 1e-12
        assert np.max(np.abs(a.rho_in - b.rho_in)) < 1e-12
        for I in range(2):
            assert np.max(np.abs(a.eps[I] - b.eps[I])) < 1e-12


def test_freeze_thaw_of_one_subsystem_is_the_plain_cycle():
    """A single subsystem has an empty environment: 2 outer x 3 inner cycles are 6 cycles."""
    s = fde_synth.tiny(2, nsub=1, nbands=2)
    ra, _, _ = scf.run(s, n_cycles=6, n_david=2)
    rb, _, _ = scf.run(s, n_cycles=2, n_david=2, scheme="freeze-thaw", n_inner=3)
    assert len(rb) == 6
    for a, b in zip(ra, rb):
        assert np.max(np.abs(a.rho_in - b.rho_in)) < 1e-13
        assert np.max(np.abs(a.eps[0] - b.eps[0])) < 1e-12


def test_freeze_thaw_inner_cycles_reach_the_frozen_environment_ground_state():
    """One outer cycle of many inner ones: each rho_I converges to the ground state of
    subsystem I in the environment frozen at the start (dense diagonalisation of H_I with
    V_eff^I from rho_I and that environment, occupations of its eigenvalues), and not to the
    one of the environment that moved meanwhile."""
    s = fde_synth.tiny(1, nsub=2, nbands=2)
    recs, X, st = scf.run(s, n_cycles=1, n_david=4, scheme="freeze-thaw", n_inner=40)
    rho0 = scf.initial_density(st, scf.initial_bands(st))
    env0 = scf.environment(rho0)
    assert np.max(np.abs(env0 - (rho0.sum(axis=0)[None] - rho0))) < 1e-14
    last = recs[-1]
    d = [np.max(np.abs(r.rho_out - r.rho_in)) for r in recs]
    assert d[-1] < 1e-5 and d[-1] < 1e-3 * d[0]
    sph = st.spheres[0]
    moved = np.max(np.abs(last.rho_in - rho0))
    assert moved > 1e-3  # the densities did change, so a moving environment would differ
    for I, sub in enumerate(s.subsystems):
        v = scf.frozen_potentials(st, last.rho_in, env0)[I]
        w, U = np.linalg.eigh(ham.explicit_h(st.cell, sph, v))
        C = U[:, :sub.nbands].T
        f, _ = occ.occupations(w[None, :sub.nbands], sub.kweight, sub.nelec, sub.smearing, sub.sigma)
        rho = dens.density(st.cell, sph, C, sub.kweight[0] * f[0])
        assert np.max(np.abs(rho - last.rho_in[I])) < 1e-4, np.max(np.abs(rho - last.rho_in[I]))
        # the moving environment's potential is not the one it converged in
        v_now = scf.frozen_potentials(st, last.rho_in, scf.environment(last.rho_in))[I]
        assert np.max(np.abs(v_now - v)) > 1e-4
