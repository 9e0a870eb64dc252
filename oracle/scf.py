"""Embedding cycle and energies (test infrastructure, FP64).

Fig. 1b and Sec. 2: the subsystem SCF step is executed once per embedding
cycle and the total density is rebuilt every cycle, so all subsystem
densities become self-consistent together. (The freeze-and-thaw scheme the
Fig. 1b caption recovers, with every subsystem iterated against a frozen
environment before the densities are broadcast, is the option
scheme="freeze-thaw" of ``run``.) One cycle,
with every subsystem seeing the densities of the cycle start (Jacobi order):

  1. V_eff^I for all I (recast effective potential, Appendix);
  2. per subsystem and k-point: HX = H X, Rayleigh-Ritz on X, then n_david
     block-Davidson iterations (see ``subspace``);
  3. occupations and mu_I (``occupations``); rho_I^out (``density``);
  4. mixing: linear rho_I^in <- (1 - beta) rho_I^in + beta rho_I^out
     (beta = 0.3; the paper does not state its mixing), or Pulay with a Kerker
     preconditioner (``mixing``);
  5. rho = sum_I rho_I^in (Eq. int1).

Cycle 0 starts from the density of the initial bands c = r / (1 + |k+G|^2)
(r: seeded normal draws) with uniform occupations N_I / nb, which does not
depend on the basis chosen for their span.

Energies (Sec. 2, E_FDE; Appendix, recast of the total energy), V_NN
excluded (a constant of the geometry):
  E_FDE = sum_I {T_J + E_NL + int V_loc rho_I + E_xc[rho_I]} + E_H[rho]
          + (T~[rho] - sum T~[rho_I]) + (E~xc[rho] - sum E~xc[rho_I])
  and through fragment energies E_K = sum eps + V_K rho_K + E_xc[rho_K]
  + 1/2 int V_H[rho] rho_K, E_FDE = sum E_K + T^nad + E_xc^nad, where
  V_K rho_K = -int (V_eff^K - V_loc) rho_K. Reading: E_H[rho_K] inside E_K is
  the share 1/2 int V_H[rho] rho_K, so that summing over K gives E_H[rho].

Pins: N_S = 1 gives plain Kohn-Sham with V_emb = 0; the band-energy identity
sum eps + V_K rho_K = T_J + E_eN + E_NL; both E_FDE expressions agree; the
converged cycle equals dense diagonalisation at the self-consistent
potential (tests/test_oracle_scf.py).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List

import numpy as np

import fde_synth

from . import basis, density as dens, embed, hamiltonian as ham, mixing, occupations as occ, pseudo
from . import subspace


@dataclass
class Setup:
    system: object
    cell: basis.Cell
    spheres: List[basis.Sphere]           # per distinct k-point
    vloc: np.ndarray
    proj: Dict[tuple, tuple]              # (isub, ik) -> (beta, dkb)
    kinds: dict = field(default_factory=lambda: dict(xc_kind="lda", xc_nad="lda", kin_nad="lc94"))


def setup(system, kinds=None) -> Setup:
    cell = basis.Cell(system.L, system.grid)
    basis.check_grid(cell, system.ecut)
    spheres = [basis.sphere(cell, system.ecut, k) for k in system.all_kfrac]
    atoms = [a for s in system.subsystems for a in s.atoms]
    vloc = pseudo.local_potential(cell, system.ecut, atoms)
    proj = {}
    for I, s in enumerate(system.subsystems):
        for ik in system.k_index(I):
            proj[(I, ik)] = pseudo.kb_projectors(cell, spheres[ik], s.atoms)
    st = Setup(system, cell, spheres, vloc, proj)
    if kinds:
        st.kinds.update(kinds)
    return st


def initial_bands(st: Setup):
    """X[I][j] for the j-th k-point of subsystem I (not orthonormal)."""
    sysm = st.system
    X = []
    for I, s in enumerate(sysm.subsystems):
        xs = []
        for ik in sysm.k_index(I):
            sph = st.spheres[ik]
            raw = fde_synth.random_coefficients(sysm.cfg, sysm.geometry, I, ik, s.nbands, sph.npw)
            xs.append(raw / (1.0 + 2.0 * sph.kin)[None, :])
        X.append(xs)
    return X


def orthonormal_start(st: Setup, I: int, ik: int, X: np.ndarray) -> np.ndarray:
    """Orthonormal (S^I-orthonormal when augmented) rows spanning X."""
    ag = aug_of(st, I)
    if ag is None:
        return subspace.orthonormalise(X)
    from . import augment
    SX = augment.apply_s(X, st.proj[(I, ik)][0], ag[0])
    return augment.subspace_rr_gen(X, SX, SX, X.shape[0])[0]


def subsystem_density(st: Setup, I: int, Xs, occws) -> np.ndarray:
    """rho_I from the bands of every k-point of subsystem I, plus, when augmented, the
    augmentation density of its atoms' charges (summed over k)."""
    sysm = st.system
    s = sysm.subsystems[I]
    rho = np.zeros(st.cell.shape)
    ag = aug_of(st, I)
    charges = None
    for j, ik in enumerate(sysm.k_index(I)):
        rho += dens.density(st.cell, st.spheres[ik], Xs[j], occws[j])
        if ag is not None:
            from . import augment
            c = augment.atom_charges(st.proj[(I, ik)][0], Xs[j], occws[j], ag[0], ag[1])
            charges = c if charges is None else charges + c
    if ag is not None:
        from . import augment
        owners = [a for a in s.atoms if a.lmax >= 0]
        rho += augment.augmentation_density(st.cell, sysm.ecut, [a.pos for a in owners], [a.rbeta for a in owners],
                                            charges)
    return rho


def initial_density(st: Setup, X) -> np.ndarray:
    sysm = st.system
    rho = np.zeros((len(sysm.subsystems),) + st.cell.shape)
    for I, s in enumerate(sysm.subsystems):
        Xs, occws = [], []
        for j, ik in enumerate(sysm.k_index(I)):
            Xs.append(orthonormal_start(st, I, ik, X[I][j]))
            occws.append(np.full(s.nbands, s.kweight[j] * s.nelec / s.nbands))
        rho[I] = subsystem_density(st, I, Xs, occws)
    return rho


def aug_of(st: Setup, I: int):
    """(q, atom_of) of an augmented subsystem (the Appendix's subsystem-specific
    projectors), else None."""
    sub = st.system.subsystems[I]
    if not getattr(sub, "aug", False):
        return None
    return fde_synth.augmentation_q(sub.atoms)


def davidson(st: Setup, I: int, ik: int, X: np.ndarray, veff: np.ndarray, n_david: int,
             history=None):
    """Per-cycle solve of one (subsystem, k): RR on X, then n_david iterations (the
    generalised problem H x = e S^I x for an augmented subsystem)."""
    sph = st.spheres[ik]
    beta, dkb = st.proj[(I, ik)]
    nb = X.shape[0]
    H = lambda Y: ham.apply_h(st.cell, sph, Y, veff, beta, dkb)  # noqa: E731
    ag = aug_of(st, I)
    if ag is not None:
        from . import augment
        S = lambda Y: augment.apply_s(Y, beta, ag[0])  # noqa: E731
        X, HX, SX, lam = augment.subspace_rr_gen(X, H(X), S(X), nb)
        if history is not None:
            history.append(lam.copy())
        for _ in range(n_david):
            T, active, _ = augment.precondition_gen(X, HX, SX, lam, sph.kin)
            act = np.concatenate([np.ones(nb, dtype=bool), active])
            X, HX, SX, lam = augment.subspace_rr_gen(np.vstack([X, T]), np.vstack([HX, H(T)]),
                                                     np.vstack([SX, S(T)]), nb, act)
            if history is not None:
                history.append(lam.copy())
        return X, HX, lam
    HX = H(X)
    X, HX, lam = subspace.subspace_rr(X, HX, nb)
    if history is not None:
        history.append(lam.copy())
    for _ in range(n_david):
        T, active, _ = subspace.precondition(X, HX, lam, sph.kin)
        HT = H(T)
        act = np.concatenate([np.ones(nb, dtype=bool), active])
        X, HX, lam = subspace.subspace_rr(np.vstack([X, T]), np.vstack([HX, HT]), nb, act)
        if history is not None:
            history.append(lam.copy())
    return X, HX, lam


@dataclass
class CycleRecord:
    eps: List[np.ndarray]        # per subsystem [nk, nb]
    mu: List[float]
    rho_out: np.ndarray          # [ns, N3, N2, N1]
    rho_in: np.ndarray           # after mixing
    veff: np.ndarray             # used in this cycle
    energies: np.ndarray         # embed energies of the input densities


def environment(rho_in):
    """env_I = sum_{J != I} rho_J (ascending J; zero for a single subsystem)."""
    env = np.zeros_like(rho_in)
    for I in range(rho_in.shape[0]):
        for J in range(rho_in.shape[0]):
            if J != I:
                env[I] += rho_in[J]
    return env


def frozen_potentials(st: Setup, rho_in, env):
    """V_eff^I with the environment of subsystem I frozen at env[I] (Fig. 1b caption:
    each subsystem iterates against the densities of the last broadcast). The
    recast V_eff^I depends only on rho = rho_I + env_I and on rho_I, so it is the
    first potential of the two-density set {rho_I, env_I}."""
    sysm = st.system
    veff = np.zeros_like(rho_in)
    for I in range(rho_in.shape[0]):
        v2, _ = embed.embed_potential(st.cell, sysm.ecut, np.stack([rho_in[I], env[I]]), st.vloc, sysm.rho_thr,
                                      **st.kinds)
        veff[I] = v2[0]
    return veff


def run(system, n_cycles=None, n_david=None, kinds=None, st: Setup = None, callback=None, mixer=None,
        scheme="jacobi", n_inner=1):
    """Run the embedding cycle; returns (records, final bands, setup). mixer: None for
    the linear mixing of the system (beta = system.mix_beta), else a
    mixing.Mixer (e.g. Pulay with a Kerker preconditioner).

    scheme "jacobi": the cycle above, the total density rebuilt every cycle.
    scheme "freeze-thaw" (Fig. 1b caption; Sec. 2 on the freeze-and-thaw
    procedure): each of the n_cycles outer cycles freezes every subsystem's
    environment env_I = sum_{J != I} rho_J^in at its start and runs n_inner
    subsystem SCF cycles against it (V_eff^I from rho_I + env_I and rho_I, steps
    2-4 above for all I); only then is the total density rebuilt. A Pulay mixer
    restarts its history at every outer cycle. One record per inner cycle.
    n_inner = 1 is the Jacobi cycle up to the summation order of rho."""
    if scheme not in ("jacobi", "freeze-thaw"):
        raise ValueError("scheme must be 'jacobi' or 'freeze-thaw'")
    st = st or setup(system, kinds)
    mix = mixer or mixing.Mixer(st.cell, "linear", system.mix_beta)
    n_cycles = system.n_cycles if n_cycles is None else n_cycles
    n_david = system.n_david if n_david is None else n_david
    X = initial_bands(st)
    rho_in = initial_density(st, X)
    for I in range(len(X)):
        X[I] = [orthonormal_start(st, I, ik, x) for ik, x in zip(system.k_index(I), X[I])]
    records = []
    inner = n_inner if scheme == "freeze-thaw" else 1
    for c in range(n_cycles * inner):
        if scheme == "jacobi":
            veff, en = embed.embed_potential(st.cell, system.ecut, rho_in, st.vloc, system.rho_thr,
                                             **st.kinds)
        else:
            if c % inner == 0:
                env = environment(rho_in)
                if c > 0:
                    mix.reset()
            veff = frozen_potentials(st, rho_in, env)
            _, en = embed.embed_potential(st.cell, system.ecut, rho_in, st.vloc, system.rho_thr, **st.kinds)
        rho_out = np.zeros_like(rho_in)
        eps_all, mus = [], []
        for I, s in enumerate(system.subsystems):
            ks = system.k_index(I)
            eps = np.zeros((len(ks), s.nbands))
            for j, ik in enumerate(ks):
                X[I][j], _, eps[j] = davidson(st, I, ik, X[I][j], veff[I], n_david)
            f, mu = occ.occupations(eps, s.kweight, s.nelec, s.smearing, s.sigma)
            rho_out[I] = subsystem_density(st, I, X[I], [s.kweight[j] * f[j] for j in range(len(ks))])
            eps_all.append(eps)
            mus.append(mu)
        rho_in = mix(rho_in, rho_out)
        rec = CycleRecord(eps_all, mus, rho_out, rho_in.copy(), veff, en)
        records.append(rec)
        if callback:
            callback(c, rec)
    return records, X, st


def band_terms(st: Setup, X, eps_f):
    """Per subsystem (T_J, E_NL, sum w f eps) from bands X and (eps, f) per k."""
    out = []
    sysm = st.system
    for I, s in enumerate(sysm.subsystems):
        tj = enl = be = 0.0
        for j, ik in enumerate(sysm.k_index(I)):
            eps, f = eps_f[I]
            w = s.kweight[j] * f[j]
            beta, dkb = st.proj[(I, ik)]
            tj += float(np.sum(w * ham.kinetic_band(st.spheres[ik], X[I][j])))
            enl += float(np.sum(w * ham.nonlocal_band(X[I][j], beta, dkb)))
            be += float(np.sum(w * eps[j]))
        out.append((tj, enl, be))
    return out


def energies(st: Setup, X, eps_f, veff_in, rho_out):
    """E_FDE both ways plus the band-energy identity terms (see module docstring)."""
    sysm = st.system
    if any(aug_of(st, I) is not None for I in range(len(sysm.subsystems))):
        # an augmented subsystem's energy needs the one-centre terms of its augmentation
        # spheres, which the synthetic overlaps do not define
        raise ValueError("energies of augmented subsystems are not defined")
    cell = st.cell
    _, en = embed.embed_potential(cell, sysm.ecut, rho_out, st.vloc, sysm.rho_thr, **st.kinds)
    ns = len(sysm.subsystems)
    bt = band_terms(st, X, eps_f)
    dV = cell.dV
    tnad = en[ns, embed.E_KIN] - sum(en[I, embed.E_KIN] for I in range(ns))
    xnad = en[ns, embed.E_XCT] - sum(en[I, embed.E_XCT] for I in range(ns))
    e142 = en[ns, embed.E_HSELF] + tnad + xnad
    e419 = tnad + xnad
    ident = []
    for I in range(ns):
        tj, enl, be = bt[I]
        eloc = en[I, embed.E_LOC]
        e142 += tj + enl + eloc + en[I, embed.E_XC]
        deband = -float(np.sum((veff_in[I] - st.vloc) * rho_out[I])) * dV
        e419 += be + deband + en[I, embed.E_XC] + 0.5 * en[I, embed.E_HEMB]
        ident.append((be + deband, tj + eloc + enl))
    return dict(E_FDE=e142, E_FDE_fragments=e419, identity=ident, embed=en)
