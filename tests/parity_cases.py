"""Parity cases shared by the host-emulation tests and the GPU tests.

Each case builds the same seeded inputs for the CPU oracle and for the
library (through the C ABI), and compares element by element. Tolerances:
FP64 plans to 1e-12 relative (rounding-order differences only), FP32 plans
to a few 1e-6 relative (single-precision FFTs: about log2(N) * 6e-8 per
transform, with FP64 accumulation of every reduction).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import fde_synth
from oracle import mlp as omlp
from oracle import basis, dft, density as odens, embed as oembed, hamiltonian as oham, occupations as oocc
from oracle import pseudo as opseudo, scf as oscf, subspace as osub
from paper_1406_7803_amd import driver, fde

TOL = {fde.F64: 1e-12, fde.F32: 5e-6}


def to_dev(plan, a, kind):
    dt = plan.cdtype if kind == "c" else (plan.rdtype if kind == "r" else torch.float64)
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dt, device=plan.be.device)


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


SMALL = dict(L=(6.0, 7.0, 5.5), grid=(10, 12, 9), ecut=3.0, kf=[(0.25, -0.25, 0.0), (0.0, 0.0, 0.0)])
KB_ATOMS = [fde_synth.Atom((1.0, 2.0, 3.0), 1.0, 0.7, lmax=1, rbeta=0.8, d_s=0.9, d_p=-0.3),
            fde_synth.Atom((4.0, 5.5, 1.0), 1.0, 0.7, lmax=0, rbeta=0.6, d_s=1.3)]


def small_plan(be, prec, max_nb=4, max_nproj=8, case=SMALL):
    return fde.Plan(case["L"], case["grid"], case["ecut"], case["kf"], prec=prec, max_nb=max_nb,
                    max_nproj=max_nproj, backend=be)


def check_plan_sets(be, prec):
    plan = small_plan(be, prec)
    cell = basis.Cell(SMALL["L"], SMALL["grid"])
    for ik, kf in enumerate(SMALL["kf"]):
        sph = basis.sphere(cell, SMALL["ecut"], kf)
        assert plan.npw(ik) == sph.npw
        assert np.array_equal(plan.miller(ik), sph.miller)


def check_apply_h(be, prec, nb=9, with_kb=True):
    """nb > max_nb exercises the band chunking; ncol is not a multiple of the stick group."""
    plan = small_plan(be, prec)
    cell = basis.Cell(SMALL["L"], SMALL["grid"])
    veff = fde_synth.random_real(4, cell.shape)
    for ik, kf in enumerate(SMALL["kf"]):
        sph = basis.sphere(cell, SMALL["ecut"], kf)
        psi = fde_synth.random_complex(5 + ik, (nb, sph.npw))
        beta = dkb = None
        tb = tdkb = None
        if with_kb:
            beta, dkb = opseudo.kb_projectors(cell, sph, KB_ATOMS)
            tb = plan.kb_projectors(ik, [a.pos for a in KB_ATOMS], [a.lmax for a in KB_ATOMS],
                                    [a.rbeta for a in KB_ATOMS])
            assert rel(host(tb), beta) < TOL[prec]
            tdkb = to_dev(plan, dkb, "d")
        ref = oham.apply_h(cell, sph, psi, veff, beta, dkb)
        out = plan.apply_h(ik, to_dev(plan, psi, "c"), to_dev(plan, veff, "r"), tb, tdkb)
        be.sync()
        assert rel(host(out), ref) < TOL[prec], rel(host(out), ref)


def check_apply_h_many_projectors(be, prec, nb=70, natoms=24):
    """More projectors than one LDS chunk and more bands than one band chunk of the
    projector update; npw is not a multiple of the plane-wave tile."""
    case = MEDIUM
    plan = small_plan(be, prec, max_nb=nb, max_nproj=4 * natoms, case=case)
    cell = basis.Cell(case["L"], case["grid"])
    rng = np.random.default_rng(5150)
    atoms = [fde_synth.Atom(tuple(rng.uniform(0, 1, 3) * np.array(case["L"])), 1.0, 0.7, lmax=int(i % 3 != 0),
                            rbeta=0.7 + 0.01 * i, d_s=0.5 + 0.05 * i, d_p=-0.2 + 0.03 * i) for i in range(natoms)]
    sph = basis.sphere(cell, case["ecut"], case["kf"][0])
    assert sph.npw % 64 != 0
    veff = fde_synth.random_real(6, cell.shape)
    psi = fde_synth.random_complex(7, (nb, sph.npw))
    beta, dkb = opseudo.kb_projectors(cell, sph, atoms)
    assert beta.shape[0] > 64
    tb = plan.kb_projectors(0, [a.pos for a in atoms], [a.lmax for a in atoms], [a.rbeta for a in atoms])
    ref = oham.apply_h(cell, sph, psi, veff, beta, dkb)
    out = plan.apply_h(0, to_dev(plan, psi, "c"), to_dev(plan, veff, "r"), tb, to_dev(plan, dkb, "d"))
    be.sync()
    assert rel(host(out), ref) < TOL[prec], rel(host(out), ref)


def check_density(be, prec, nb=7):
    plan = small_plan(be, prec)
    cell = basis.Cell(SMALL["L"], SMALL["grid"])
    rho = plan.zeros_grid()
    ref = np.zeros(cell.shape)
    for ik, kf in enumerate(SMALL["kf"]):
        sph = basis.sphere(cell, SMALL["ecut"], kf)
        psi = osub.orthonormalise(fde_synth.random_complex(11 + ik, (nb, sph.npw)))
        occw = np.linspace(1.0, 0.0, nb) * 0.5
        ref += odens.density(cell, sph, psi, occw)
        plan.density(ik, to_dev(plan, psi, "c"), to_dev(plan, occw, "d"), rho)
    be.sync()
    assert rel(host(rho), ref) < TOL[prec]
    # charge conservation
    assert abs(float(host(rho).sum()) * cell.dV - np.linspace(1.0, 0.0, nb).sum()) < 50 * TOL[prec]


def _smooth_densities(cell, ecut, ns=2, nb=3, seed=20):
    sph = basis.sphere(cell, ecut, (0.0, 0.0, 0.0))
    out = []
    for I in range(ns):
        c = fde_synth.random_complex(seed + I, (nb, sph.npw)) / (1 + 2 * sph.kin)[None] ** 2
        out.append(odens.density(cell, sph, osub.orthonormalise(c), np.full(nb, 2.0)))
    return np.array(out)


KIN_NAMES = {fde.KIN_LC94: "lc94", fde.KIN_TF: "tf", fde.KIN_NONE: "none", fde.KIN_REVAPBEK: "revapbek"}
XC_NAMES = {fde.XC_LDA: "lda", fde.XC_PBE: "pbe", fde.XC_NONE: "none"}


def check_embed(be, prec, kin=fde.KIN_LC94, grid=(12, 12, 15), L=(6.0, 6.0, 7.0), ecut=2.2, ns=2, xc=fde.XC_LDA,
                xc_nad=fde.XC_LDA):
    cell = basis.Cell(L, grid)
    rs = _smooth_densities(cell, ecut, ns=ns)
    vloc = fde_synth.random_real(5, cell.shape, -0.3, 0.3)
    vref, eref = oembed.embed_potential(cell, ecut, rs, vloc, kin_nad=KIN_NAMES[kin], xc_kind=XC_NAMES[xc],
                                        xc_nad=XC_NAMES[xc_nad])
    plan = fde.Plan(L, grid, ecut, [(0, 0, 0)], prec=prec, max_nb=4, backend=be)
    veff, en, info = plan.embed_potential(to_dev(plan, rs, "r"), to_dev(plan, vloc, "r"), kin_nad=kin, xc=xc,
                                          xc_nad=xc_nad)
    be.sync()
    assert int(host(info)[0]) == 0
    assert rel(host(veff), vref) < TOL[prec]
    assert np.max(np.abs(host(en) - eref)) < 10 * TOL[prec] * max(1.0, np.max(np.abs(eref)))


def check_local_potential(be, prec):
    L, grid, ecut = (6.0, 6.0, 7.0), (12, 12, 15), 2.2
    cell = basis.Cell(L, grid)
    atoms = [fde_synth.Atom((1.0, 2.0, 3.0), 2.0, 0.6), fde_synth.Atom((4.0, 4.5, 5.0), 1.0, 0.7)]
    ref = opseudo.local_potential(cell, ecut, atoms)
    plan = fde.Plan(L, grid, ecut, [(0, 0, 0)], prec=prec, max_nb=4, backend=be)
    v = plan.local_potential([a.pos for a in atoms], [a.Z for a in atoms], [a.width for a in atoms])
    be.sync()
    assert rel(host(v), ref) < TOL[prec]


MEDIUM = dict(L=(8.0, 8.0, 9.0), grid=(18, 18, 20), ecut=5.0, kf=[(0.25, 0.0, -0.25)])
# 1877 plane waves: room for m = 600 (the global solver with its inverse-iteration factors in global memory)
LARGE = dict(L=(12.0, 12.0, 12.0), grid=(32, 32, 32), ecut=8.0, kf=[(0.25, 0.0, -0.25)])


# Ritz values / projector tolerances per subspace-product mode (FP32 plans); BF16x3
# keeps about 16 significant bits per product.
GEMM_TOL = {fde.GEMM_FP64: (2e-5, 1e-4), fde.GEMM_BF16X6: (2e-5, 1e-4), fde.GEMM_BF16X3: (3e-4, 3e-3)}


def _rr_inputs(case, nb, drop_case, ik=0, seed=21):
    """[X; T] and [HX; HT] of a Davidson step (m = 2 nb) with its column flags, and the oracle's
    Rayleigh-Ritz result on them."""
    cell = basis.Cell(case["L"], case["grid"])
    sph = basis.sphere(cell, case["ecut"], case["kf"][ik])
    v = opseudo.local_potential(cell, case["ecut"], KB_ATOMS)
    beta, dkb = opseudo.kb_projectors(cell, sph, KB_ATOMS)
    X = osub.orthonormalise(fde_synth.random_complex(seed, (nb, sph.npw)))
    HX = oham.apply_h(cell, sph, X, v, beta, dkb)
    X, HX, lam = osub.subspace_rr(X, HX, nb)
    T, active, _ = osub.precondition(X, HX, lam, sph.kin)
    act = np.concatenate([np.ones(nb, bool), active])
    if drop_case:
        act[nb + 1] = False          # an inactive column
        T[1] = 0.0
        T[2] = X[0] + 1e-7 * T[3]     # nearly dependent: dropped by the pivot test
    HT = oham.apply_h(cell, sph, T, v, beta, dkb)
    Xr, HXr, lr = osub.subspace_rr(np.vstack([X, T]), np.vstack([HX, HT]), nb, act)
    H = lambda Y: oham.apply_h(cell, sph, Y, v, beta, dkb)  # noqa: E731
    return np.vstack([X, T]), np.vstack([HX, HT]), act, Xr, lr, H


def _rr_compare(prec, gemm, nb, V, HV, ev, info, Xr, lr, H):
    assert int(host(info)[0]) == 0
    tol, ptol = (1e-11, 1e-10) if prec == fde.F64 else GEMM_TOL[gemm]
    assert np.max(np.abs(host(ev) - lr)) < tol, np.max(np.abs(host(ev) - lr))
    Xg = host(V)[:nb]
    # eigenvectors are unique up to a phase: compare projectors and Ritz values
    assert np.max(np.abs(Xg.conj() @ Xg.T - np.eye(nb))) < (1e-12 if prec == fde.F64 else 10 * ptol / 100)
    P_gpu = Xg.T @ Xg.conj()
    P_ref = Xr.T @ Xr.conj()
    assert np.max(np.abs(P_gpu - P_ref)) < ptol, np.max(np.abs(P_gpu - P_ref))
    # HX rows are H applied to the new X
    assert rel(host(HV)[:nb], H(Xg)) < (1e-10 if prec == fde.F64 else 1e-4)


def check_subspace_rr(be, prec, drop_case=False, nb=4, case=SMALL, gemm=fde.GEMM_FP64, split=None):
    """nb = 45 (m = 90) and nb = 140 (m = 280) exercise the tridiagonal solver with its matrices in
    global memory, smaller m the LDS ones; from m = 256 on (or from m = split) the eigensolver runs
    as multi-workgroup phase launches."""
    plan = small_plan(be, prec, max_nb=max(4, nb), case=case)
    if gemm != fde.GEMM_FP64:
        plan.set_gemm_mode(gemm)
    if split is not None:
        plan.set_tuning(fde.TUNE_RR_SPLIT, split)
    ik = 0
    VT, HVT, act, Xr, lr, H = _rr_inputs(case, nb, drop_case, ik)
    V = to_dev(plan, VT, "c")
    HV = to_dev(plan, HVT, "c")
    ev, info = plan.subspace_rr(ik, V, HV, nb, active=torch.from_numpy(act.astype(np.uint8)).to(plan.be.device))
    be.sync()
    _rr_compare(prec, gemm, nb, V, HV, ev, info, Xr, lr, H)


def check_subspace_rr_clustered(be, prec, m, nb, split=None, case=MEDIUM):
    """A Rayleigh-Ritz problem with a designed spectrum: orthonormal V and HV = M V with
    M = U diag(lam) U^H (U random unitary), lam holding a chain of 40 values 2e-5 apart
    (one cluster for the eigenvector phase), an exactly degenerate pair inside the chain, a
    triple 1e-12 apart, and a gap of 0.5 above band nb so the wanted subspace is well defined."""
    plan = small_plan(be, prec, max_nb=max(4, nb, (m + 1) // 2), case=case)
    if split is not None:
        plan.set_tuning(fde.TUNE_RR_SPLIT, split)
    npw = plan.npw(0)
    assert npw >= m
    rng = np.random.default_rng(77)
    lam = np.sort(rng.uniform(-2.0, 1.0, m))
    lam[5:45] = -1.0 + 2e-5 * np.arange(40)
    lam[20] = lam[21]
    lam[nb - 3:nb] = 0.3 + 1e-12 * np.arange(3)
    lam[nb:] = np.sort(rng.uniform(0.8, 3.0, m - nb))
    lam[:nb] = np.sort(lam[:nb])
    Z = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    U, _ = np.linalg.qr(Z)
    M = (U * lam) @ U.conj().T
    M = 0.5 * (M + M.conj().T)
    V = osub.orthonormalise(fde_synth.random_complex(23, (m, npw)))
    HV = M.T @ V  # hv_j = sum_k M_kj v_k: <v_i|H v_j> = M_ij
    Xr, HXr, lr = osub.subspace_rr(V, HV, nb)
    assert np.max(np.abs(lr - lam[:nb])) < 1e-10  # the oracle sees the designed spectrum
    Vd, HVd = to_dev(plan, V, "c"), to_dev(plan, HV, "c")
    ev, info = plan.subspace_rr(0, Vd, HVd, nb)
    be.sync()
    assert int(host(info)[0]) == 0
    tol, ptol, otol = (1e-11, 1e-10, 1e-12) if prec == fde.F64 else (2e-5, 1e-4, 1e-5)
    assert np.max(np.abs(host(ev) - lr)) < tol, np.max(np.abs(host(ev) - lr))
    Xg = host(Vd)[:nb]
    assert np.max(np.abs(Xg.conj() @ Xg.T - np.eye(nb))) < otol, np.max(np.abs(Xg.conj() @ Xg.T - np.eye(nb)))
    P = Xg.T @ Xg.conj() - Xr.T @ Xr.conj()
    assert np.max(np.abs(P)) < ptol, np.max(np.abs(P))


def check_subspace_rr_batched_split(be, prec, split):
    """One batch of blocks of different m through the split eigensolver (split = smallest m that
    takes it): m = 90, m = 60 with an inactive and a dropped column, and m = 3 with two equal band
    columns (info = 3, its X left unchanged, the other blocks unaffected)."""
    case = MEDIUM
    plan = fde.Plan(case["L"], case["grid"], case["ecut"], case["kf"], prec=prec, max_nb=45, max_nproj=8,
                    max_batch=3, backend=be)
    plan.set_tuning(fde.TUNE_RR_SPLIT, split)
    dev = plan.be.device
    blocks, want = [], []
    for nb, drop, seed in [(45, False, 21), (30, True, 22)]:
        VT, HVT, act, Xr, lr, H = _rr_inputs(case, nb, drop, 0, seed)
        V, HV = to_dev(plan, VT, "c"), to_dev(plan, HVT, "c")
        a = torch.from_numpy(act.astype(np.uint8)).to(dev)
        ev = torch.zeros(nb, dtype=torch.float64, device=dev)
        info = torch.full((1,), -7, dtype=torch.int32, device=dev)
        blocks.append(plan.make_block(0, nb, 2 * nb, V, HV, active=a, eval=ev, info=info))
        want.append((nb, V, HV, ev, info, Xr, lr, H, a))
    Xs = fde_synth.random_complex(31, (3, plan.npw(0)))
    Xs[2] = Xs[1]
    Vs = to_dev(plan, Xs, "c")
    HVs = Vs.clone()
    evs = torch.zeros(3, dtype=torch.float64, device=dev)
    infos = torch.zeros(1, dtype=torch.int32, device=dev)
    blocks.insert(1, plan.make_block(0, 3, 3, Vs, HVs, eval=evs, info=infos))
    plan.subspace_rr_batched(blocks)
    be.sync()
    for nb, V, HV, ev, info, Xr, lr, H, a in want:
        _rr_compare(prec, fde.GEMM_FP64, nb, V, HV, ev, info, Xr, lr, H)
    assert int(host(infos)[0]) == 3
    assert np.array_equal(host(Vs), Xs.astype(host(Vs).dtype))


def check_singular_gram(be, prec):
    """Two identical X columns (j < nb cannot be dropped): info = column + 1, X left unchanged."""
    plan = small_plan(be, prec)
    sph_npw = plan.npw(0)
    X = fde_synth.random_complex(31, (3, sph_npw))
    X[2] = X[1]
    V = to_dev(plan, X, "c")
    HV = V.clone()
    ev, info = plan.subspace_rr(0, V, HV, 3)
    be.sync()
    assert int(host(info)[0]) == 3
    assert np.array_equal(host(V), X.astype(host(V).dtype))


def check_precondition(be, prec):
    plan = small_plan(be, prec)
    cell = basis.Cell(SMALL["L"], SMALL["grid"])
    ik = 0
    sph = basis.sphere(cell, SMALL["ecut"], SMALL["kf"][ik])
    X = fde_synth.random_complex(41, (4, sph.npw))
    HX = fde_synth.random_complex(42, (4, sph.npw))
    lam = np.array([0.1, -0.2, 0.3, 0.5])
    HX[3] = lam[3] * X[3]      # zero residual -> inactive, T = 0
    T, active, rn = osub.precondition(X, HX, lam, sph.kin)
    t = plan.zeros_bands(4, ik)
    act = torch.zeros(4, dtype=torch.uint8, device=plan.be.device)
    rnorm = torch.zeros(4, dtype=torch.float64, device=plan.be.device)
    plan.precondition(ik, to_dev(plan, X, "c"), to_dev(plan, HX, "c"), to_dev(plan, lam, "d"), t, act, rnorm)
    be.sync()
    assert np.array_equal(host(act).astype(bool), active)
    assert rel(host(t), T) < TOL[prec] * 10
    assert rel(host(rnorm)[:3], rn[:3]) < TOL[prec] * 10


def check_precondition_batched(be, prec):
    """Three blocks over two k-points with max_batch 2 (two launches), ragged nb, a zero-residual row;
    T lands in rows nb..2nb-1 of each block's v."""
    plan = fde.Plan(SMALL["L"], SMALL["grid"], SMALL["ecut"], SMALL["kf"], prec=prec, max_nb=5, max_nproj=8,
                    max_batch=2, backend=be)
    cell = basis.Cell(SMALL["L"], SMALL["grid"])
    blocks, keep, want = [], [], []
    for j, (ik, nb) in enumerate([(0, 5), (1, 3), (0, 2)]):
        sph = basis.sphere(cell, SMALL["ecut"], SMALL["kf"][ik])
        X = fde_synth.random_complex(60 + j, (nb, sph.npw))
        HX = fde_synth.random_complex(70 + j, (nb, sph.npw))
        lam = fde_synth.random_real(80 + j, (nb,))
        if j == 1:
            lam[1] = 0.5  # exact in FP32 too, so the residual is zero there as well
            HX[1] = lam[1] * X[1]
        T, active, rn = osub.precondition(X, HX, lam, sph.kin)
        v = plan.zeros_bands(2 * nb, ik)
        v[:nb] = to_dev(plan, X, "c")
        hv = plan.zeros_bands(2 * nb, ik)
        hv[:nb] = to_dev(plan, HX, "c")
        ev = to_dev(plan, lam, "d")
        act = torch.full((nb,), 7, dtype=torch.uint8, device=plan.be.device)
        rnorm = torch.zeros(nb, dtype=torch.float64, device=plan.be.device)
        blocks.append(plan.make_block(ik, nb, 2 * nb, v, hv, t_active=act, eval=ev, rnorm=rnorm))
        keep.append((v, hv, ev, act, rnorm))
        want.append((nb, T, active, rn))
    plan.precondition_batched(blocks)
    be.sync()
    for (v, _, _, act, rnorm), (nb, T, active, rn) in zip(keep, want):
        assert np.array_equal(host(act).astype(bool), active)
        assert rel(host(v)[nb:], T) < TOL[prec] * 10
        on = active
        assert rel(host(rnorm)[on], rn[on]) < TOL[prec] * 10


def check_occupations(be):
    dev = be.device
    eps = np.array([[-0.5, -0.3, -0.1, 0.2, 0.4], [-0.45, -0.28, -0.05, 0.25, 0.5]])
    wk = np.array([0.5, 0.5])
    modes = {"integer": fde.OCC_INTEGER, "fermi-dirac": fde.OCC_FERMI_DIRAC,
             "methfessel-paxton": fde.OCC_METHFESSEL_PAXTON}
    for nel, mode, sig in [(6.0, "fermi-dirac", 0.01), (5.0, "fermi-dirac", 0.05), (4.0, "integer", 0.0),
                           (6.0, "methfessel-paxton", 0.01), (5.0, "methfessel-paxton", 0.05),
                           (7.3, "methfessel-paxton", 0.02)]:
        f, mu = oocc.occupations(eps, wk, nel, mode, sig)
        m = modes[mode]
        occw, tmu, info = fde.occupations(be, torch.tensor(eps, device=dev), torch.tensor(wk, device=dev), nel, m,
                                          max(sig, 1e-300))
        be.sync()
        assert int(host(info)[0]) == 0
        assert np.max(np.abs(host(occw) - wk[:, None] * f)) < 1e-10
        assert abs(float(host(occw).sum()) - nel) < 1e-12
    # odd or fractional counts cannot fill whole bands
    for nel in (5.0, 3.5):
        with pytest.raises(fde.FdeError):
            fde.occupations(be, torch.tensor(eps, device=dev), torch.tensor(wk, device=dev), nel, fde.OCC_INTEGER,
                            1e-300)


_ORACLE_RUNS = {}


def oracle_run(system, n_cycles):
    """oracle.scf.run, kept per (config, geometry, cycles) for the tests of one session."""
    key = (system.cfg, system.geometry, tuple(system.grid), len(system.subsystems), n_cycles)
    if key not in _ORACLE_RUNS:
        _ORACLE_RUNS[key] = oscf.run(system, n_cycles=n_cycles)
    return _ORACLE_RUNS[key]


def check_trajectory(be, prec, system, n_cycles, eps_tol, drho_tol, gemm=fde.GEMM_FP64):
    recs, _, st = oracle_run(system, n_cycles)
    eng = driver.Engine(system, prec=prec, backend=be, gemm=gemm)
    worst = (0.0, 0.0)
    for c in range(n_cycles):
        eng.cycle()
        be.sync()
        for I in range(len(system.subsystems)):
            e = np.max(np.abs(host(eng.eps[I]) - recs[c].eps[I]))
            d = float(np.sum(np.abs(host(eng.rho_out[I]) - recs[c].rho_out[I]))) * st.cell.dV
            worst = (max(worst[0], e), max(worst[1], d))
    assert all(int(host(b.info)[0]) == 0 for row in eng.blocks for b in row)
    assert worst[0] < eps_tol and worst[1] < drho_tol, worst
    return worst


def check_apply_h_grid(be, prec, grid, spacing=0.3, ecut=3.0, nb=2, kf=(0.25, -0.25, 0.0)):
    """H application and density on a grid of the given FFT lengths (the
    specialised in-LDS FFT lengths of the configured cells)."""
    L = tuple(n * spacing for n in grid)
    cell = basis.Cell(L, grid)
    sph = basis.sphere(cell, ecut, kf)
    plan = fde.Plan(L, grid, ecut, [kf], prec=prec, max_nb=nb, backend=be)
    assert plan.npw(0) == sph.npw
    veff = fde_synth.random_real(50, cell.shape)
    psi = fde_synth.random_complex(51, (nb, sph.npw)) / (1 + 2 * sph.kin)[None]
    ref = oham.apply_h(cell, sph, psi, veff)
    out = plan.apply_h(0, to_dev(plan, psi, "c"), to_dev(plan, veff, "r"))
    occw = np.linspace(1.0, 0.5, nb)
    rho = plan.zeros_grid()
    plan.density(0, to_dev(plan, psi, "c"), to_dev(plan, occw, "d"), rho)
    be.sync()
    assert rel(host(out), ref) < TOL[prec], rel(host(out), ref)
    rref = odens.density(cell, sph, psi, occw)
    assert rel(host(rho), rref) < TOL[prec]
    # every in-plane pass that applies (the others fall back to the automatic choice),
    # and the two-factor pass with small row batches
    for kind, rows in ((fde.PLANE_REG, 0), (fde.PLANE_LDS, 0), (fde.PLANE_TWO_FACTOR, 0),
                       (fde.PLANE_TWO_FACTOR, 7)):
        plan.set_tuning(fde.TUNE_PLANE_KIND, kind)
        plan.set_tuning(fde.TUNE_PLANE_ROWS, rows)
        outk = plan.apply_h(0, to_dev(plan, psi, "c"), to_dev(plan, veff, "r"))
        rhok = plan.zeros_grid()
        plan.density(0, to_dev(plan, psi, "c"), to_dev(plan, occw, "d"), rhok)
        be.sync()
        assert rel(host(outk), ref) < TOL[prec], (kind, rows, rel(host(outk), ref))
        assert rel(host(rhok), rref) < TOL[prec], (kind, rows)
    plan.set_tuning(fde.TUNE_PLANE_KIND, 0)
    plan.set_tuning(fde.TUNE_PLANE_ROWS, 0)
    # z-passes through LDS instead of the four-step register FFT (where one exists)
    plan.set_tuning(fde.TUNE_Z_REGISTER, 1)
    out2 = plan.apply_h(0, to_dev(plan, psi, "c"), to_dev(plan, veff, "r"))
    rho2 = plan.zeros_grid()
    plan.density(0, to_dev(plan, psi, "c"), to_dev(plan, occw, "d"), rho2)
    be.sync()
    plan.set_tuning(fde.TUNE_Z_REGISTER, 0)
    assert rel(host(out2), ref) < TOL[prec]
    assert rel(host(rho2), rref) < TOL[prec]



# ---------------------------------------------------------------------------
# Learned preconditioner network
# ---------------------------------------------------------------------------
def bf16_round(a):
    """Round float values to the nearest BF16 value (ties to even), as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def mlp_params(seed):
    """Parameters with a nonzero output layer, BF16-representable weights."""
    t = fde_synth.mlp_init(seed)
    rng = np.random.default_rng(seed + 1)
    t[omlp.OFF_W3:omlp.OFF_B3] = rng.normal(0.0, 0.3, omlp.HID)
    t[omlp.OFF_B3] = 0.1
    t[omlp.OFF_B1:omlp.OFF_W2] = rng.normal(0.0, 0.1, omlp.HID)
    t[omlp.OFF_B2:omlp.OFF_W3] = rng.normal(0.0, 0.1, omlp.HID)
    return bf16_round(t)


def mlp_samples(n, seed):
    rng = np.random.default_rng(seed)
    U = np.stack([rng.uniform(0.0, 3.0, n), rng.normal(0.0, 1.0, n), rng.normal(-1.0, 1.5, n),
                  rng.normal(0.0, 1.0, n)], axis=1)
    A = rng.uniform(0.1, 2.0, n)
    B = rng.uniform(-1.0, 1.0, n) * np.sqrt(A)
    C = B * B / A + rng.uniform(0.0, 1.0, n)
    return np.concatenate([U, A[:, None], B[:, None], C[:, None]], axis=1)


def fdev(be, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(be.device)


def check_mlp_forward(be, n=1000):
    """BF16 weights and first hidden layer, FP32 accumulation, against the FP64 network."""
    th = mlp_params(11)
    U = mlp_samples(n, 12)[:, :4].astype(np.float32).astype(np.float64)
    ref, _ = omlp.forward(th, U)
    y = fde.mlp_forward(be, fdev(be, U), fdev(be, th))
    be.sync()
    err = np.abs(host(y) - ref)
    assert err.max() < 0.03 and err.mean() < 0.005, (err.max(), err.mean())


def check_mlp_loss_grad(be, n=3000):
    th = mlp_params(13)
    S = mlp_samples(n, 14).astype(np.float32).astype(np.float64)
    L, g = omlp.loss_grad(th, S)
    tr = fde.MlpTrainer(be, fdev(be, S), fdev(be, th))
    loss, grad = tr.loss_grad()
    be.sync()
    gg = host(grad).astype(np.float64)
    assert abs(float(host(loss)[0]) - L) < 1e-2 * abs(L)
    cos = gg @ g / (np.linalg.norm(gg) * np.linalg.norm(g))
    assert cos > 0.999, cos
    assert np.linalg.norm(gg - g) < 3e-2 * np.linalg.norm(g)
    # every block of the parameter vector carries gradient
    for a, b in [(omlp.OFF_W1, omlp.OFF_B1), (omlp.OFF_B1, omlp.OFF_W2), (omlp.OFF_W2, omlp.OFF_B2),
                 (omlp.OFF_B2, omlp.OFF_W3), (omlp.OFF_W3, omlp.OFF_B3), (omlp.OFF_B3, omlp.NPARAM)]:
        assert np.linalg.norm(gg[a:b] - g[a:b]) < 5e-2 * np.linalg.norm(g[a:b]) + 1e-9, (a, b)


def check_mlp_adam(be):
    th = mlp_params(15)
    rng = np.random.default_rng(16)
    g = rng.normal(0.0, 1.0, omlp.NPARAM)
    m = np.zeros(omlp.NPARAM)
    v = np.zeros(omlp.NPARAM)
    p = fdev(be, th)
    gm = torch.zeros_like(p)
    gv = torch.zeros_like(p)
    gd = fdev(be, g)
    ref = th.copy()
    for t in range(1, 4):
        ref, m, v = omlp.adam(ref, g, m, v, t, 1e-3)
        st = be.lib.fde_mlp_adam(gd.data_ptr(), p.data_ptr(), gm.data_ptr(), gv.data_ptr(), t, 1e-3, 0.9, 0.999,
                                 1e-8, be.stream())
        assert st == 0
    be.sync()
    assert np.max(np.abs(host(p) - ref)) < 1e-6


def check_precondition_mlp(be, prec):
    plan = small_plan(be, prec)
    cell = basis.Cell(SMALL["L"], SMALL["grid"])
    ik = 0
    sph = basis.sphere(cell, SMALL["ecut"], SMALL["kf"][ik])
    X = osub.orthonormalise(fde_synth.random_complex(51, (4, sph.npw)))
    HX = fde_synth.random_complex(52, (4, sph.npw)) * 0.3 + X
    lam = np.array([0.9, 1.1, 0.95, 0.5])  # 0.5: HX = lam X is exact in FP32 too
    HX[3] = lam[3] * X[3]      # zero residual -> inactive, T = 0
    vbar = 0.37
    th = mlp_params(17)
    T, active, rn = omlp.precondition(th, X, HX, lam, sph.kin, vbar)
    dev = plan.be.device
    V = to_dev(plan, np.vstack([X, np.zeros_like(X)]), "c")
    HV = to_dev(plan, np.vstack([HX, np.zeros_like(HX)]), "c")
    ev = to_dev(plan, lam, "d")
    act = torch.zeros(4, dtype=torch.uint8, device=dev)
    rnorm = torch.zeros(4, dtype=torch.float64, device=dev)
    blk = plan.make_block(ik, 4, 4, V, HV, t_active=act, eval=ev, rnorm=rnorm)
    plan.precondition_mlp_batched([blk], fdev(be, th), torch.tensor([vbar], dtype=torch.float64, device=dev))
    be.sync()
    assert np.array_equal(host(act).astype(bool), active)
    got = host(V)[4:]
    assert rel(got, T) < 2e-2, rel(got, T)
    assert rel(host(rnorm)[:3], rn[:3]) < TOL[prec] * 10
    # zero output layer: exactly the TPA preconditioner
    th0 = fde_synth.mlp_init(3)
    T0, _, _ = osub.precondition(X, HX, lam, sph.kin)
    plan.precondition_mlp_batched([blk], fdev(be, th0), torch.tensor([vbar], dtype=torch.float64, device=dev))
    be.sync()
    assert rel(host(V)[4:], T0) < TOL[prec] * 10


def check_mlp_training_reduces_loss(be, n=4096, steps=150):
    """A target the network can represent: y* = 0.5 tanh(u1) - 0.3 u4 (through B/A)."""
    rng = np.random.default_rng(21)
    U = np.stack([rng.uniform(0.0, 3.0, n), rng.normal(0.0, 1.0, n), rng.normal(-1.0, 1.5, n),
                  rng.normal(0.0, 1.0, n)], axis=1)
    ystar = 0.5 * np.tanh(U[:, 0]) - 0.3 * U[:, 3]
    A = rng.uniform(0.5, 1.5, n)
    B = A * np.exp(ystar)
    C = B * B / A
    S = np.concatenate([U, A[:, None], B[:, None], C[:, None]], axis=1)
    th = fde_synth.mlp_init(5)
    tr = fde.MlpTrainer(be, fdev(be, S), fdev(be, th), lr=3e-3)
    l0 = float(host(tr.loss_grad()[0])[0])
    for _ in range(steps):
        tr.step()
    l1 = float(host(tr.loss_grad()[0])[0])
    be.sync()
    assert l1 < 0.1 * l0, (l0, l1)
    # the oracle agrees on the trained parameters' loss
    Lo = omlp.loss(host(tr.params).astype(np.float64), S.astype(np.float32).astype(np.float64))
    assert abs(Lo - l1) < 0.05 * l0, (Lo, l1)


def check_engine_mlp_zero_output_is_tpa(be):
    """The cycle with a network whose output layer is zero reproduces the TPA cycle."""
    from paper_1406_7803_amd import driver
    s = fde_synth.config1()
    e1 = driver.Engine(s, prec=fde.F64, backend=be)
    e2 = driver.Engine(s, prec=fde.F64, backend=be, mlp_params=fdev(be, fde_synth.mlp_init(0)))
    for _ in range(2):
        e1.cycle()
        e2.cycle()
    be.sync()
    for a, b in zip(e1.eps, e2.eps):
        assert np.max(np.abs(host(a) - host(b))) < 1e-12


def check_tuning_keeps_results(be, prec):
    """The bands-per-plane-workgroup launch shape does not change fde_apply_h's result."""
    plan = small_plan(be, prec, max_nb=9)
    cell = basis.Cell(SMALL["L"], SMALL["grid"])
    sph = basis.sphere(cell, SMALL["ecut"], SMALL["kf"][0])
    veff = to_dev(plan, fde_synth.random_real(4, cell.shape), "r")
    psi = to_dev(plan, fde_synth.random_complex(5, (9, sph.npw)), "c")
    ref = host(plan.apply_h(0, psi, veff)).copy()
    for bpw in (1, 2, 3, 9):
        plan.set_tuning(fde.TUNE_APPLY_BPW, bpw)
        out = host(plan.apply_h(0, psi, veff))
        be.sync()
        assert np.max(np.abs(out - ref)) <= 1e-14 * np.max(np.abs(ref)), bpw
    plan.set_tuning(fde.TUNE_APPLY_BPW, 0)
    occw = to_dev(plan, np.linspace(0.1, 0.9, 9), "d")
    rho = plan.zeros_grid()
    plan.density(0, psi, occw, rho)
    rho_ref = host(rho).copy()
    for sz in (1, 2, 4, 8, 16):  # every z-stick is transformed on its own: results identical
        plan.set_tuning(fde.TUNE_STICK_GROUP, sz)
        out = host(plan.apply_h(0, psi, veff))
        rho.zero_()
        plan.density(0, psi, occw, rho)
        be.sync()
        assert np.array_equal(out, ref), sz
        assert np.array_equal(host(rho), rho_ref), sz
    plan.set_tuning(fde.TUNE_STICK_GROUP, 0)
    with pytest.raises(fde.FdeError):
        plan.set_tuning(fde.TUNE_STICK_GROUP, 3)


# ---------------------------------------------------------------------------
# Energy terms (row a13): band energies, grid dots, E_FDE by both routes
# ---------------------------------------------------------------------------
def check_band_energies(be, prec, nb=5):
    """T_J, E_NL and sum w eps at two k-points with s + p projectors, accumulated."""
    plan = small_plan(be, prec, max_nb=nb)
    cell = basis.Cell(SMALL["L"], SMALL["grid"])
    out = torch.zeros(3, dtype=torch.float64, device=plan.be.device)
    ref = np.zeros(3)
    for ik, kf in enumerate(SMALL["kf"]):
        sph = basis.sphere(cell, SMALL["ecut"], kf)
        psi = osub.orthonormalise(fde_synth.random_complex(90 + ik, (nb, sph.npw)))
        beta, dkb = opseudo.kb_projectors(cell, sph, KB_ATOMS)
        occw = np.linspace(0.9, 0.1, nb) * (0.5 + ik)
        eps = fde_synth.random_real(95 + ik, (nb,))
        ref += [np.sum(occw * oham.kinetic_band(sph, psi)), np.sum(occw * oham.nonlocal_band(psi, beta, dkb)),
                np.sum(occw * eps)]
        tb = plan.kb_projectors(ik, [a.pos for a in KB_ATOMS], [a.lmax for a in KB_ATOMS],
                                [a.rbeta for a in KB_ATOMS])
        plan.band_energies(ik, to_dev(plan, psi, "c"), to_dev(plan, occw, "d"), tb, to_dev(plan, dkb, "d"),
                           out=out, eval=to_dev(plan, eps, "d"))
    be.sync()
    tol = 1e-12 if prec == fde.F64 else 2e-6
    assert np.max(np.abs(host(out) - ref) / np.abs(ref)) < tol, (host(out), ref)
    # without projectors: only the kinetic and band sums
    out2 = plan.band_energies(1, to_dev(plan, psi, "c"), to_dev(plan, occw, "d"))
    be.sync()
    assert abs(float(host(out2)[1])) == 0.0


def check_grid_dot(be, prec):
    L, grid = (6.0, 6.0, 7.0), (12, 12, 15)
    cell = basis.Cell(L, grid)
    plan = fde.Plan(L, grid, 2.2, [(0, 0, 0)], prec=prec, max_nb=4, backend=be)
    a = fde_synth.random_real(61, cell.shape)
    b = fde_synth.random_real(62, cell.shape, 0.0, 2.0)
    out = plan.grid_dot(to_dev(plan, a, "r"), to_dev(plan, b, "r"))
    out = plan.grid_dot(to_dev(plan, a, "r"), to_dev(plan, b, "r"), out=out)   # accumulates
    one = plan.grid_dot(to_dev(plan, b, "r"), None)
    be.sync()
    if prec == fde.F32:
        a, b = a.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
    ref = float(np.sum(a * b)) * cell.dV
    assert abs(float(host(out)[0]) - 2 * ref) < 1e-12 * np.sum(np.abs(a * b)) * cell.dV * 2
    assert abs(float(host(one)[0]) - float(np.sum(b)) * cell.dV) < 1e-12 * float(np.sum(b)) * cell.dV


def check_energies(be, prec, system, n_cycles, tol):
    """E_FDE of the last cycle's bands and output densities, from the library's energy
    terms (Engine.total_energies) against the oracle's direct and fragment expressions."""
    recs, X, st = oracle_run(system, n_cycles)
    eps_f = []
    for I, sub in enumerate(system.subsystems):
        f, _ = oocc.occupations(recs[-1].eps[I], sub.kweight, sub.nelec, sub.smearing, sub.sigma)
        eps_f.append((recs[-1].eps[I], f))
    ref = oscf.energies(st, X, eps_f, recs[-1].veff, recs[-1].rho_out)
    assert abs(ref["E_FDE"] - ref["E_FDE_fragments"]) < 1e-10
    eng = driver.Engine(system, prec=prec, backend=be)
    for _ in range(n_cycles):
        eng.cycle()
    out = host(eng.total_energies())
    be.sync()
    ns = len(system.subsystems)
    assert abs(out[ns + 2] - ref["E_FDE"]) < tol, (out[ns + 2], ref["E_FDE"])
    assert abs(out[ns + 3] - ref["E_FDE_fragments"]) < tol, (out[ns + 3], ref["E_FDE_fragments"])
    assert abs(out[ns + 2] - out[ns + 3]) < tol
    en = ref["embed"]
    tnad = en[ns, oembed.E_KIN] - sum(en[I, oembed.E_KIN] for I in range(ns))
    assert abs(out[ns] - tnad) < tol
    return out, ref


def _vacuum_densities(cell, ns):
    """rho_A: Gaussian blobs with regions below the density threshold; rho_B = 0."""
    N1, N2, N3 = cell.grid
    L = np.array(cell.L)
    z, y, x = np.meshgrid(np.arange(N3) * L[2] / N3, np.arange(N2) * L[1] / N2, np.arange(N1) * L[0] / N1,
                          indexing="ij")
    g = (x, y, z)
    rho = np.zeros((ns,) + cell.shape)
    for c, q, s in [((0.3, 0.4, 0.5), 2.0, 0.55), ((0.6, 0.5, 0.3), 1.0, 0.45)]:
        d2 = 0.0
        for i in range(3):
            d = g[i] - c[i] * L[i]
            d -= L[i] * np.round(d / L[i])
            d2 = d2 + d * d
        rho[0] += q * (2 * np.pi * s * s) ** -1.5 * np.exp(-0.5 * d2 / (s * s))
    return rho


def check_embed_grid(be, prec, grid, spacing, kin=fde.KIN_LC94, ecut=3.0, xc=fde.XC_LDA, xc_nad=fde.XC_LDA):
    """The embedding potential on a grid of compile-time FFT lengths, with a vacuum
    region below rho_thr (reading 11) and a second subsystem of zero density
    (T^nad[rho_A, 0] = 0 and V^nad = 0 exactly)."""
    L = tuple(n * spacing for n in grid)
    cell = basis.Cell(L, grid)
    rs = _vacuum_densities(cell, 2)
    assert np.mean(rs[0] < 1e-10) > 0.05          # part of the cell is vacuum
    vloc = fde_synth.random_real(7, cell.shape, -0.3, 0.3)
    vref, eref = oembed.embed_potential(cell, ecut, rs, vloc, kin_nad=KIN_NAMES[kin], xc_kind=XC_NAMES[xc],
                                        xc_nad=XC_NAMES[xc_nad])
    plan = fde.Plan(L, grid, ecut, [(0, 0, 0)], prec=prec, max_nb=2, backend=be)
    veff, en, info = plan.embed_potential(to_dev(plan, rs, "r"), to_dev(plan, vloc, "r"), kin_nad=kin, xc=xc,
                                          xc_nad=xc_nad)
    be.sync()
    assert int(host(info)[0]) == 0
    v = host(veff)
    scale = np.max(np.abs(vref))
    assert np.max(np.abs(v - vref)) < 2 * TOL[prec] * scale, np.max(np.abs(v - vref)) / scale
    e = host(en)
    assert np.max(np.abs(e - eref)) < 10 * TOL[prec] * max(1.0, np.max(np.abs(eref)))
    # rho_B = 0: no nonadditive kinetic or xc energy
    assert abs(e[2, fde.E_KIN] - e[0, fde.E_KIN]) <= 1e-12 * max(1.0, abs(e[0, fde.E_KIN]))
    assert e[1, fde.E_KIN] == 0.0 and e[1, fde.E_XC] == 0.0 and e[1, fde.E_CHARGE] == 0.0


def check_trajectory_uneven(be, prec, n_cycles=3):
    """Six uneven subsystems (4-48 bands, 1-4 k-points) in one cycle: the LDS
    (m <= 80) and the global (m = 96) eigensolvers run in the same cycle, in
    ragged batches over several solver groups.

    FP64: 1e-10 Ha and 1e-10 in int |d rho_I|. FP32: the rounding of an FP32 FFT
    sandwich is relative (about log2(N) 2^-24 per element), so the bound scales
    with the size of what is compared: 1e-6 Ha per Ha of the largest |eps|, and
    2.5e-6 per electron in int |d rho_I| (an L1 norm: per-point rounding does not
    cancel). For the 4-electron subsystems of the two-subsystem cube these are
    the 1e-6 Ha / 1e-5 targets; the 76-electron subsystem here gets 1.9e-4."""
    s = fde_synth.config3_reduced()
    ms = sorted({2 * sub.nbands for sub in s.subsystems})
    assert ms[0] <= 80 < ms[-1]
    if prec == fde.F64:
        return check_trajectory(be, prec, s, n_cycles, 1e-10, 1e-10)
    recs, _, st = oracle_run(s, n_cycles)
    eng = driver.Engine(s, prec=prec, backend=be)
    emax = max(float(np.max(np.abs(e))) for r in recs for e in r.eps)
    worst_e, worst_d = 0.0, 0.0
    for c in range(n_cycles):
        eng.cycle()
        be.sync()
        for I, sub in enumerate(s.subsystems):
            worst_e = max(worst_e, float(np.max(np.abs(host(eng.eps[I]) - recs[c].eps[I]))))
            d = float(np.sum(np.abs(host(eng.rho_out[I]) - recs[c].rho_out[I]))) * st.cell.dV
            worst_d = max(worst_d, d / sub.nelec)
    assert all(int(host(b.info)[0]) == 0 for row in eng.blocks for b in row)
    assert worst_e < 1e-6 * max(1.0, emax), (worst_e, emax)
    assert worst_d < 2.5e-6, worst_d
    return worst_e, worst_d


# ---------------------------------------------------------------------------
# Pulay mixing with a Kerker preconditioner; cycles with it and with
# Methfessel-Paxton smearing
# ---------------------------------------------------------------------------
def check_mix_pulay(be, prec, q0, nhmax=4, ncalls=7, ns=2):
    """A sequence of calls with the history wrapping around, against oracle.mixing."""
    from oracle import mixing as omix
    L, grid = (6.0, 6.0, 7.0), (12, 12, 15)
    cell = basis.Cell(L, grid)
    plan = fde.Plan(L, grid, 2.2, [(0, 0, 0)], prec=prec, max_nb=2, backend=be)
    ref = omix.Mixer(cell, "pulay", beta=0.4, nhist=nhmax, q0=q0)
    dev = plan.be.device
    state = torch.zeros(3, dtype=torch.int32, device=dev)
    xh = torch.zeros((nhmax, ns) + plan.shape, dtype=plan.rdtype, device=dev)
    rh = torch.zeros_like(xh)
    x = fde_synth.random_real(70, (ns,) + cell.shape, 0.0, 1.0)
    if prec == fde.F32:
        x = x.astype(np.float32).astype(np.float64)
    rho_in = to_dev(plan, x, "r")
    for k in range(ncalls):
        # a smooth nonlinear map of the input, so the residuals stay independent
        y = 0.5 * np.tanh(x + 0.3 * np.roll(x, 1, axis=-1)) + fde_synth.random_real(71 + k, x.shape, 0.0, 0.05)
        if prec == fde.F32:
            y = y.astype(np.float32).astype(np.float64)
        want = ref(x, y)
        got, info = plan.mix_pulay(state, xh, rh, rho_in, to_dev(plan, y, "r"), 0.4, q0)
        be.sync()
        assert int(host(info)[0]) == 0
        g = host(got).astype(np.float64)
        tol = 1e-11 if prec == fde.F64 else 5e-5
        assert rel(g, want) < tol, (k, rel(g, want))
        assert list(host(state)) [:2] == [min(k + 1, nhmax), (k + 1) % nhmax]
        x = g  # continue from what the library produced (rounding stays in step)


def check_trajectory_pulay(be, prec, system, n_cycles, eps_tol, drho_tol, mixer):
    from oracle import mixing as omix
    st = oscf.setup(system)
    recs, _, _ = oscf.run(system, n_cycles=n_cycles, st=st,
                          mixer=omix.Mixer(st.cell, "pulay", mixer["beta"], mixer["nhist"], mixer["q0"]))
    eng = driver.Engine(system, prec=prec, backend=be, mixer=mixer)
    worst = (0.0, 0.0)
    for c in range(n_cycles):
        eng.cycle()
        be.sync()
        for I in range(len(system.subsystems)):
            e = np.max(np.abs(host(eng.eps[I]) - recs[c].eps[I]))
            d = float(np.sum(np.abs(host(eng.rho_out[I]) - recs[c].rho_out[I]))) * st.cell.dV
            worst = (max(worst[0], e), max(worst[1], d))
    assert int(host(eng.mix_info)[0]) == 0
    assert worst[0] < eps_tol and worst[1] < drho_tol, worst
    return worst


def check_trajectory_freeze_thaw(be, prec, n_outer, n_inner, eps_tol, drho_tol, mixer=None):
    """The two-subsystem cube in the freeze-and-thaw scheme: n_outer frozen environments,
    n_inner cycles each (linear mixing, or Pulay restarted per environment)."""
    from oracle import mixing as omix
    s = fde_synth.config1()
    st = oscf.setup(s)
    om = None if mixer is None else omix.Mixer(st.cell, "pulay", mixer["beta"], mixer["nhist"], mixer["q0"])
    recs, _, _ = oscf.run(s, n_cycles=n_outer, st=st, mixer=om, scheme="freeze-thaw", n_inner=n_inner)
    eng = driver.Engine(s, prec=prec, backend=be, mixer=mixer, scheme="freeze-thaw", n_inner=n_inner)
    worst = (0.0, 0.0, 0.0)
    for c in range(n_outer * n_inner):
        eng.cycle()
        be.sync()
        for I in range(len(s.subsystems)):
            e = np.max(np.abs(host(eng.eps[I]) - recs[c].eps[I]))
            d = float(np.sum(np.abs(host(eng.rho_out[I]) - recs[c].rho_out[I]))) * st.cell.dV
            v = float(np.max(np.abs(host(eng.veff[I]) - recs[c].veff[I])))
            worst = (max(worst[0], e), max(worst[1], d), max(worst[2], v))
    assert all(int(host(b.info)[0]) == 0 for row in eng.blocks for b in row)
    assert worst[0] < eps_tol and worst[1] < drho_tol, worst
    return worst


def check_frozen_environment(be, prec):
    """env_I = sum_{J != I} rho_J for three subsystems, into [ns][N] and into the pairs'
    second slot (first slot untouched); one subsystem gives zero."""
    plan = small_plan(be, prec)
    n = int(np.prod(plan.shape))
    rho = fde_synth.random_real(91, (3,) + plan.shape)
    want = oscf.environment(rho)
    got = plan.frozen_environment(to_dev(plan, rho, "r"), plan.zeros_grid(3))
    be.sync()
    tol = 1e-15 if prec == fde.F64 else 1e-6
    assert np.max(np.abs(host(got) - want)) < tol
    pairs = torch.full((3, 2) + plan.shape, 7.0, dtype=plan.rdtype, device=plan.be.device)
    plan.frozen_environment(to_dev(plan, rho, "r"), pairs)
    be.sync()
    assert np.max(np.abs(host(pairs)[:, 1] - want)) < tol
    assert np.all(host(pairs)[:, 0] == 7.0)
    one = plan.frozen_environment(to_dev(plan, rho[:1], "r"), plan.zeros_grid(1) + 5.0)
    be.sync()
    assert np.all(host(one) == 0.0)
    assert n == rho[0].size


def check_trajectory_gga(be, prec, n_cycles, eps_tol, drho_tol):
    """The two-subsystem cube with the paper's functionals: PBE xc both ways, revAPBEK."""
    s = fde_synth.config1()
    st = oscf.setup(s, dict(xc_kind="pbe", xc_nad="pbe", kin_nad="revapbek"))
    recs, _, _ = oscf.run(s, n_cycles=n_cycles, st=st)
    eng = driver.Engine(s, prec=prec, backend=be,
                        kinds=dict(xc=fde.XC_PBE, xc_nad=fde.XC_PBE, kin_nad=fde.KIN_REVAPBEK))
    worst = (0.0, 0.0)
    for c in range(n_cycles):
        eng.cycle()
        be.sync()
        for I in range(len(s.subsystems)):
            e = np.max(np.abs(host(eng.eps[I]) - recs[c].eps[I]))
            d = float(np.sum(np.abs(host(eng.rho_out[I]) - recs[c].rho_out[I]))) * st.cell.dV
            worst = (max(worst[0], e), max(worst[1], d))
    assert worst[0] < eps_tol and worst[1] < drho_tol, worst
    return worst


def oracle_supersystem_comparison(system, kinds, mixer, n_cycles):
    """The Table 1 quantities from the oracle alone, after a fixed number of cycles."""
    from oracle import mixing as omix
    okinds = dict(xc_kind=XC_NAMES[kinds["xc"]], xc_nad=XC_NAMES[kinds["xc_nad"]], kin_nad=KIN_NAMES[kinds["kin_nad"]])

    def run(sysm):
        st = oscf.setup(sysm, okinds)
        recs, X, _ = oscf.run(sysm, n_cycles=n_cycles, st=st,
                              mixer=omix.Mixer(st.cell, "pulay", mixer["beta"], mixer["nhist"], mixer["q0"]))
        r = recs[-1]
        ef = [(r.eps[I], oocc.occupations(r.eps[I], sub.kweight, sub.nelec, sub.smearing, sub.sigma)[0])
              for I, sub in enumerate(sysm.subsystems)]
        return r, oscf.energies(st, X, ef, r.veff, r.rho_out)["E_FDE"], st

    rks, eks, st = run(fde_synth.supersystem(system))
    rfde, efde, _ = run(system)
    efrag = [run(fde_synth.fragment(system, I))[1] for I in range(len(system.subsystems))]
    dd = 0.5 * float(np.sum(np.abs(rfde.rho_out.sum(0) - rks.rho_out[0]))) * st.cell.dV
    return dict(dens_diff=dd, E_KS=eks, E_FDE=efde, E_frag=efrag, int_KS=eks - sum(efrag), int_FDE=efde - sum(efrag))


def check_supersystem_comparison(be, prec, kinds, n_cycles=6, tol=1e-9):
    s = fde_synth.tiny(0, with_kb=True, kfrac=[(0.25, 0.0, 0.0), (-0.25, 0.0, 0.0)], grid=(12, 12, 15))
    mixer = dict(kind="pulay", nhist=4, beta=0.5, q0=0.6)
    ref = oracle_supersystem_comparison(s, kinds, mixer, n_cycles)
    got = driver.supersystem_comparison(s, prec=prec, backend=be, kinds=kinds, mixer=mixer, fixed_cycles=n_cycles)
    for k in ("dens_diff", "E_KS", "E_FDE", "int_KS", "int_FDE"):
        assert abs(got[k] - ref[k]) < tol * max(1.0, abs(ref[k])), (k, got[k], ref[k])
    assert ref["dens_diff"] > 1e-4    # FDE and KS densities do differ
    return got, ref


# ---------------------------------------------------------------------------
# Subsystem-specific augmentation: overlap S^I, generalised Rayleigh-Ritz and
# Davidson, augmentation charge (Appendix, non-local pseudopotentials)
# ---------------------------------------------------------------------------
def _aug_setup(be, prec, nb, natoms=3, case=None, max_nb=None):
    from oracle import augment as oaug  # noqa: F401
    case = case or MEDIUM
    plan = small_plan(be, prec, max_nb=max_nb or max(4, nb), max_nproj=4 * natoms, case=case)
    cell = basis.Cell(case["L"], case["grid"])
    rng = np.random.default_rng(4242)
    atoms = [fde_synth.Atom(tuple(rng.uniform(0, 1, 3) * np.array(case["L"])), 1.0, 0.7, lmax=1,
                            rbeta=0.8 + 0.05 * i, d_s=0.6, d_p=-0.25) for i in range(natoms)]
    sph = basis.sphere(cell, case["ecut"], case["kf"][0])
    beta, dkb = opseudo.kb_projectors(cell, sph, atoms)
    q, atom_of = fde_synth.augmentation_q(atoms)
    v = opseudo.local_potential(cell, case["ecut"], atoms)
    tb = plan.kb_projectors(0, [a.pos for a in atoms], [a.lmax for a in atoms], [a.rbeta for a in atoms])
    dev = plan.be.device
    tq = torch.from_numpy(q).to(device=dev)
    return plan, cell, sph, atoms, beta, dkb, q, atom_of, v, tb, tq


def check_apply_s(be, prec, nb=9, natoms=3):
    """S psi against the oracle; nb above max_nb exercises the band chunks, 20 atoms (80
    projectors) the tiled projection."""
    from oracle import augment as oaug
    plan, cell, sph, atoms, beta, dkb, q, atom_of, v, tb, tq = _aug_setup(be, prec, nb, natoms, max_nb=4)
    psi = fde_synth.random_complex(61, (nb, sph.npw))
    out = plan.apply_s(0, to_dev(plan, psi, "c"), tb, tq)
    be.sync()
    ref = oaug.apply_s(psi, beta, q)
    assert rel(host(out), ref) < TOL[prec], rel(host(out), ref)
    # no projectors: a copy
    out0 = plan.apply_s(0, to_dev(plan, psi, "c"), None, None)
    be.sync()
    assert np.array_equal(host(out0), psi.astype(host(out0).dtype))


def check_subspace_rr_gen(be, prec, nb=12):
    """Rayleigh-Ritz of the generalised problem on [X | T]-like rows (m = 2 nb) with an
    inactive column: Ritz values, projectors X X^H, and S X = S applied to the new X."""
    from oracle import augment as oaug
    from oracle import hamiltonian as oh
    plan, cell, sph, atoms, beta, dkb, q, atom_of, v, tb, tq = _aug_setup(be, prec, 2 * nb)
    V = fde_synth.random_complex(62, (2 * nb, sph.npw)) / (1 + sph.kin)[None]
    HV = oh.apply_h(cell, sph, V, v, beta, dkb)
    SV = oaug.apply_s(V, beta, q)
    act = np.ones(2 * nb, bool)
    act[nb + 2] = False
    Xr, HXr, SXr, lr = oaug.subspace_rr_gen(V, HV, SV, nb, act)
    dev = plan.be.device
    tV, tHV, tSV = to_dev(plan, V, "c"), to_dev(plan, HV, "c"), to_dev(plan, SV, "c")
    ev = torch.zeros(nb, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    # a standard problem in the same batch (no S V rows: the third rotation skips it)
    W = fde_synth.random_complex(65, (2 * nb, sph.npw)) / (1 + sph.kin)[None]
    HW = oh.apply_h(cell, sph, W, v, beta, dkb)
    Xw, _, lw = osub.subspace_rr(W, HW, nb)
    tW, tHW = to_dev(plan, W, "c"), to_dev(plan, HW, "c")
    ev2 = torch.zeros(nb, dtype=torch.float64, device=dev)
    info2 = torch.zeros(1, dtype=torch.int32, device=dev)
    plan.subspace_rr_batched([plan.make_block(0, nb, 2 * nb, tV, tHV, active=torch.from_numpy(act.astype(np.uint8)).to(dev),
                                              eval=ev, info=info, sv=tSV),
                              plan.make_block(0, nb, 2 * nb, tW, tHW, eval=ev2, info=info2)])
    be.sync()
    assert int(host(info)[0]) == 0 and int(host(info2)[0]) == 0
    tol, ptol = (1e-10, 1e-9) if prec == fde.F64 else (2e-5, 1e-4)
    assert np.max(np.abs(host(ev2) - lw)) < tol * max(1.0, np.max(np.abs(lw)))
    Wg = host(tW)[:nb].astype(np.complex128)
    assert np.max(np.abs(Wg.T @ Wg.conj() - Xw.T @ Xw.conj())) < ptol
    assert np.max(np.abs(host(ev) - lr)) < tol * max(1.0, np.max(np.abs(lr))), np.max(np.abs(host(ev) - lr))
    Xg = host(tV)[:nb].astype(np.complex128)
    assert np.max(np.abs(Xg.T @ Xg.conj() - Xr.T @ Xr.conj())) < ptol
    assert rel(host(tSV)[:nb].astype(np.complex128), oaug.apply_s(Xg, beta, q)) < (1e-10 if prec == fde.F64 else 1e-4)
    assert np.max(np.abs(Xg.conj() @ host(tSV)[:nb].T - np.eye(nb))) < (1e-10 if prec == fde.F64 else 1e-4)


def check_davidson_gen(be, prec, nb=6, n_iter=8):
    """The generalised band solver at a fixed potential, iteration by iteration against
    the oracle's Davidson with the same start."""
    from oracle import augment as oaug
    from oracle import hamiltonian as oh
    from paper_1406_7803_amd import driver
    plan, cell, sph, atoms, beta, dkb, q, atom_of, v, tb, tq = _aug_setup(be, prec, nb)
    X0 = fde_synth.random_complex(63, (nb, sph.npw)) / (1 + sph.kin)[None]
    Hf = lambda Y: oh.apply_h(cell, sph, Y, v, beta, dkb)  # noqa: E731
    Sf = lambda Y: oaug.apply_s(Y, beta, q)  # noqa: E731
    _, _, _, hist = oaug.davidson_gen(Hf, Sf, X0, n_iter, sph.kin)
    g = driver.davidson_fixed(plan, 0, to_dev(plan, X0, "c"), to_dev(plan, v, "r"), n_iter, beta=tb,
                              dkb=to_dev(plan, dkb, "d"), aug=(tb, tq))
    ghist, info, X, SX = g
    be.sync()
    assert int(host(info)[0]) == 0
    tol = 1e-10 if prec == fde.F64 else 2e-5
    for it, (a, b) in enumerate(zip(ghist, hist[1:])):
        assert np.max(np.abs(host(a) - b)) < tol * max(1.0, np.max(np.abs(b))), (it, np.max(np.abs(host(a) - b)))
    Xg = host(X).astype(np.complex128)
    assert np.max(np.abs(Xg.conj() @ host(SX).T - np.eye(nb))) < (1e-10 if prec == fde.F64 else 1e-4)


def check_aug_density(be, prec, nb=5):
    """Atom charges from the projections and the augmentation density on the grid."""
    from oracle import augment as oaug
    plan, cell, sph, atoms, beta, dkb, q, atom_of, v, tb, tq = _aug_setup(be, prec, nb)
    X = fde_synth.random_complex(64, (nb, sph.npw)) / (1 + sph.kin)[None]
    occw = np.linspace(2.0, 0.5, nb)
    dev = plan.be.device
    ch = torch.full((len(atoms),), 0.25, dtype=torch.float64, device=dev)  # accumulates
    plan.aug_charges(0, to_dev(plan, X, "c"), to_dev(plan, occw, "d"), tb, tq,
                     torch.from_numpy(atom_of).to(dev), ch)
    be.sync()
    ref = oaug.atom_charges(beta, X, occw, q, atom_of)
    assert np.max(np.abs(host(ch) - 0.25 - ref)) < (1e-11 if prec == fde.F64 else 1e-5) * max(1.0, np.max(np.abs(ref)))
    at = torch.tensor([[*a.pos, a.rbeta] for a in atoms], dtype=torch.float64, device=dev)
    rho = plan.zeros_grid() + 0.125
    plan.aug_density(at, to_dev(plan, ref, "d"), rho)
    be.sync()
    want = oaug.augmentation_density(cell, MEDIUM["ecut"], [a.pos for a in atoms], [a.rbeta for a in atoms], ref)
    assert rel(host(rho).astype(np.float64) - 0.125, want) < TOL[prec], rel(host(rho).astype(np.float64) - 0.125, want)


def check_trajectory_aug(be, prec, n_cycles, eps_tol, drho_tol):
    """A k-point cell with projectors whose first subsystem is augmented (generalised band
    solver, augmentation density) and whose second is not, against the oracle cycle."""
    s = fde_synth.tiny(4, with_kb=True, nbands=3, kfrac=[(0.25, 0.0, 0.0), (-0.25, 0.0, 0.0)], grid=(12, 12, 15))
    s.subsystems[0].aug = True
    recs, _, st = oscf.run(s, n_cycles=n_cycles)
    eng = driver.Engine(s, prec=prec, backend=be)
    worst = (0.0, 0.0)
    for c in range(n_cycles):
        eng.cycle()
        be.sync()
        for I, sub in enumerate(s.subsystems):
            e = np.max(np.abs(host(eng.eps[I]) - recs[c].eps[I]))
            d = float(np.sum(np.abs(host(eng.rho_out[I]) - recs[c].rho_out[I]))) * st.cell.dV
            q = float(host(eng.rho_out[I]).astype(np.float64).sum()) * st.cell.dV
            assert abs(q - sub.nelec) < (1e-10 if prec == fde.F64 else 1e-4), (c, I, q)
            worst = (max(worst[0], e), max(worst[1], d))
    assert all(int(host(b.info)[0]) == 0 for row in eng.blocks for b in row)
    assert worst[0] < eps_tol and worst[1] < drho_tol, worst
    with pytest.raises(fde.FdeError, match="augmented"):
        eng.total_energies()
    return worst
