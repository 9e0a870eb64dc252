"""Pins of the oracle's embedding cycle and energies (CPU only)."""
import numpy as np

import fde_synth
from oracle import basis, embed, hamiltonian as ham, occupations as occ, scf


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
