"""Embedding-cycle driver over the C ABI (orchestration only).

One cycle (Fig. 1b of the paper: the subsystem SCF step runs once per cycle
and the total density is rebuilt every cycle; all subsystems see the densities
of the cycle start):
  1. fde_embed_potential: V_eff^I of every subsystem (recast form, Appendix);
  2. per subsystem and k-point: fde_apply_h + fde_subspace_rr on X, then
     n_david iterations of fde_precondition, fde_apply_h, fde_subspace_rr on [X|T];
  3. fde_occupations, fde_density;
  4. fde_mix (linear, beta = 0.3) or fde_mix_pulay (Pulay with a Kerker preconditioner);
     the next fde_embed_potential sums rho = sum rho_I.
Every arithmetic step runs in the library's kernels; this module only owns
buffers (PyTorch tensors) and the order of the calls.
"""
from __future__ import annotations

import contextlib
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

import fde_synth

from . import fde


@dataclass
class BandBlock:
    isub: int
    ik: int              # plan k index
    j: int               # k index within the subsystem
    V: torch.Tensor      # [2 nb][npw]: rows 0..nb-1 = X, nb..2nb-1 = T
    HV: torch.Tensor
    beta: Optional[torch.Tensor]
    dkb: Optional[torch.Tensor]
    eval: torch.Tensor   # [nb] float64
    active: torch.Tensor  # [2 nb] uint8
    rnorm: torch.Tensor  # [nb] float64
    info: torch.Tensor   # [1] int32
    nb: int
    SV: Optional[torch.Tensor] = None   # [2 nb][npw] S V of an augmented subsystem
    aug_q: Optional[torch.Tensor] = None  # [nproj][nproj] float64 augmentation overlaps


@dataclass
class SolverGroup:
    """Band blocks solved together: their own plan (workspace) and HIP stream, so that
    one group's Rayleigh-Ritz solve (a few CUs) overlaps another group's H applications."""
    plan: "fde.Plan"
    blocks: List[BandBlock]
    stream: Optional[torch.cuda.Stream]
    vbar: Optional[torch.Tensor] = None


# Blocks this large (nb npw) fill the GPU on their own: concurrent solver groups then only
# contend (large metal-surface cell, 320 x 158 149: one group 508 ms per cycle, three
# 605 ms), while smaller blocks gain from them (slab + molecule cell, 40 x 50 300: three
# groups 11.9 ms, one 13.9 ms; 64-subsystem cube: 272 against 370 ms).
AUTO_ONE_STREAM_LOAD = 10_000_000


@dataclass
class Engine:
    system: object
    prec: int = fde.F64
    backend: Optional[fde.Backend] = None
    kinds: dict = field(default_factory=lambda: dict(xc=fde.XC_LDA, xc_nad=fde.XC_LDA, kin_nad=fde.KIN_LC94))
    mlp_params: Optional[torch.Tensor] = None   # learned preconditioner (FP32, FDE_MLP_NPARAM); None = TPA
    gemm: int = fde.GEMM_FP64                   # arithmetic of the Rayleigh-Ritz subspace products
    streams: int = 3                            # band-solver groups run concurrently (GPU backend);
                                                # 0: one group when a block alone fills the GPU
                                                # (nb npw >= AUTO_ONE_STREAM_LOAD), else three
    mixer: Optional[dict] = None                # None: linear (system.mix_beta); or dict(kind="pulay",
                                                # nhist=6, beta=0.5, q0=0.5) for fde_mix_pulay
    scheme: str = "jacobi"                      # or "freeze-thaw": n_inner cycles per frozen environment
    n_inner: int = 1

    def __post_init__(self):
        s = self.system
        self.be = self.backend or fde.gpu_backend()
        max_nb = max(sub.nbands for sub in s.subsystems)
        nproj_max = max([self._nproj(sub) for sub in s.subsystems] + [0])
        nblocks = sum(len(sub.kfrac) for sub in s.subsystems)
        self.plan = fde.Plan(s.L, s.grid, s.ecut, s.all_kfrac, prec=self.prec, max_nb=max_nb, max_nproj=nproj_max,
                             max_batch=min(16, nblocks), backend=self.be)
        p = self.plan
        if self.gemm != fde.GEMM_FP64:
            p.set_gemm_mode(self.gemm)
        dev = self.be.device
        atoms = [a for sub in s.subsystems for a in sub.atoms]
        self.vloc = p.local_potential([a.pos for a in atoms], [a.Z for a in atoms], [a.width for a in atoms])
        self.blocks: List[List[BandBlock]] = []
        for I, sub in enumerate(s.subsystems):
            row = []
            for j, ik in enumerate(s.k_index(I)):
                nb = sub.nbands
                npw = p.npw(ik)
                beta = dkb = None
                if self._nproj(sub):
                    beta = p.kb_projectors(ik, [a.pos for a in sub.atoms], [a.lmax for a in sub.atoms],
                                           [a.rbeta for a in sub.atoms]).contiguous()
                    d = []
                    for a in sub.atoms:
                        if a.lmax >= 0:
                            d.append(a.d_s)
                        if a.lmax >= 1:
                            d += [a.d_p] * 3
                    dkb = torch.tensor(d, dtype=torch.float64, device=dev)
                V = torch.zeros((2 * nb, npw), dtype=p.cdtype, device=dev)
                raw = torch.from_numpy(fde_synth.random_coefficients(s.cfg, s.geometry, I, ik, nb, npw)).to(
                    dtype=p.cdtype, device=dev)
                p.init_bands(ik, raw, out=V[:nb])
                SV = aq = None
                if getattr(sub, "aug", False):
                    if beta is None:
                        raise fde.FdeError("an augmented subsystem needs projectors")
                    if self.mlp_params is not None:
                        raise fde.FdeError("the learned preconditioner takes standard problems only")
                    SV = torch.zeros_like(V)
                    aq = torch.from_numpy(fde_synth.augmentation_q(sub.atoms)[0]).to(device=dev)
                row.append(BandBlock(I, ik, j, V, torch.zeros_like(V), beta, dkb,
                                     torch.zeros(nb, dtype=torch.float64, device=dev),
                                     torch.ones(2 * nb, dtype=torch.uint8, device=dev),
                                     torch.zeros(nb, dtype=torch.float64, device=dev),
                                     torch.zeros(1, dtype=torch.int32, device=dev), nb, SV, aq))
            self.blocks.append(row)
        # augmentation charges and atoms (x, y, z, width) of the augmented subsystems
        self.aug = {}
        for I, sub in enumerate(s.subsystems):
            if getattr(sub, "aug", False):
                owners = [a for a in sub.atoms if a.lmax >= 0]
                _, atom_of = fde_synth.augmentation_q(sub.atoms)
                self.aug[I] = dict(
                    atom_of=torch.from_numpy(atom_of).to(device=dev),
                    atoms=torch.tensor([[*a.pos, a.rbeta] for a in owners], dtype=torch.float64, device=dev),
                    charges=torch.zeros(len(owners), dtype=torch.float64, device=dev))
        ns = len(s.subsystems)
        self.rho_in = p.zeros_grid(ns)
        self.rho_out = p.zeros_grid(ns)
        self.veff = p.zeros_grid(ns)
        self.energies = torch.zeros((ns + 1, fde.NE), dtype=torch.float64, device=dev)
        self.einfo = torch.zeros(1, dtype=torch.int32, device=dev)
        self.wk = [torch.tensor(sub.kweight, dtype=torch.float64, device=dev) for sub in s.subsystems]
        self.eps = [torch.zeros((len(sub.kfrac), sub.nbands), dtype=torch.float64, device=dev) for sub in s.subsystems]
        self.occw = [torch.zeros_like(e) for e in self.eps]
        self.mu = [torch.zeros(1, dtype=torch.float64, device=dev) for _ in s.subsystems]
        self.oinfo = [torch.zeros(1, dtype=torch.int32, device=dev) for _ in s.subsystems]
        self._make_groups(max_nb, nproj_max, nblocks)
        if self.mixer is not None:
            if self.mixer.get("kind", "pulay") != "pulay":
                raise fde.FdeError("mixer kind must be 'pulay' (None for linear mixing)")
            nh = int(self.mixer.get("nhist", 6))
            self.mix_state = torch.zeros(3, dtype=torch.int32, device=dev)
            self.mix_info = torch.zeros(1, dtype=torch.int32, device=dev)
            self.x_hist = torch.zeros((nh, ns) + p.shape, dtype=p.rdtype, device=dev)
            self.r_hist = torch.zeros_like(self.x_hist)
        if self.scheme not in ("jacobi", "freeze-thaw") or self.n_inner < 1:
            raise fde.FdeError("scheme must be 'jacobi' or 'freeze-thaw' with n_inner >= 1")
        if self.scheme == "freeze-thaw":
            # {rho_I, env_I} pairs and their two potentials, per subsystem
            self.pairs = torch.zeros((ns, 2) + p.shape, dtype=p.rdtype, device=dev)
            self.pair_veff = torch.zeros_like(self.pairs)
            self.pair_en = torch.zeros((ns, 3, fde.NE), dtype=torch.float64, device=dev)
            self.inner = 0
        self._initial_density()

    def _make_groups(self, max_nb, nproj_max, nblocks):
        """Split the band blocks into `streams` groups of about equal nb * npw."""
        s, p = self.system, self.plan
        blocks = [b for row in self.blocks for b in row]
        streams = self.streams
        if streams <= 0:
            big = max(b.nb * p.npw(b.ik) for b in blocks)
            streams = 1 if big >= AUTO_ONE_STREAM_LOAD else 3
        self.n_groups = 1 if self.be.emulated else max(1, min(streams, len(blocks)))
        ng = self.n_groups
        loads, members = [0] * ng, [[] for _ in range(ng)]
        for b in sorted(blocks, key=lambda b: -b.nb * p.npw(b.ik)):
            g = loads.index(min(loads))
            members[g].append(b)
            loads[g] += b.nb * p.npw(b.ik)
        self.groups = []
        for g in range(ng):
            plan = p
            if g > 0:
                plan = fde.Plan(s.L, s.grid, s.ecut, s.all_kfrac, prec=self.prec, max_nb=max_nb,
                                max_nproj=nproj_max, max_batch=min(16, nblocks), backend=self.be)
                if self.gemm != fde.GEMM_FP64:
                    plan.set_gemm_mode(self.gemm)
            stream = torch.cuda.Stream(self.be.device) if ng > 1 else None
            vbar = torch.zeros(len(members[g]), dtype=torch.float64, device=self.be.device)
            self.groups.append(SolverGroup(plan, members[g], stream, vbar))

    def set_tuning(self, key: int, value: int):
        for g in self.groups:
            g.plan.set_tuning(key, value)

    @staticmethod
    def _nproj(sub) -> int:
        return sum(0 if a.lmax < 0 else (1 if a.lmax == 0 else 4) for a in sub.atoms)

    def _initial_density(self):
        """Orthonormalise the initial bands and take their density with f = N_I / nb."""
        p = self.plan
        for I, sub in enumerate(self.system.subsystems):
            occws = []
            for b in self.blocks[I]:
                X = b.V[:b.nb]
                HX = b.HV[:b.nb]
                w = float(sub.kweight[b.j]) * sub.nelec / sub.nbands
                occw = torch.full((b.nb,), w, dtype=torch.float64, device=self.be.device)
                occws.append(occw)
                if b.SV is None:
                    HX.copy_(X)                   # A = S: the Rayleigh-Ritz step only orthonormalises
                    p.subspace_rr(b.ik, X, HX, b.nb, eval=b.eval, info=b.info)
                else:                             # S-orthonormal: A = S = X^H S X
                    p.apply_s(b.ik, X, b.beta, b.aug_q, out=b.SV[:b.nb])
                    HX.copy_(b.SV[:b.nb])
                    p.subspace_rr_batched([p.make_block(b.ik, b.nb, b.nb, b.V, b.HV, eval=b.eval, info=b.info,
                                                        sv=b.SV)])
            self._subsystem_density(I, occws, self.rho_in[I])

    @staticmethod
    def _rr_blocks(g: SolverGroup, m_of):
        return [g.plan.make_block(b.ik, b.nb, m_of(b), b.V, b.HV, active=b.active, eval=b.eval, info=b.info,
                                  sv=b.SV) for b in g.blocks]

    @staticmethod
    def _pc_blocks(g: SolverGroup):
        return [g.plan.make_block(b.ik, b.nb, b.nb, b.V, b.HV, t_active=b.active[b.nb:], eval=b.eval,
                                  rnorm=b.rnorm, sv=b.SV) for b in g.blocks]

    def solve(self, n_david: int):
        """Every band block in lockstep within its group: H X and Rayleigh-Ritz on X, then
        n_david block-Davidson iterations; the solver calls are batched over a group's
        blocks, and the groups run on their own streams (forked from and joined back to
        the current stream)."""
        main = None if self.be.emulated else torch.cuda.current_stream(self.be.device)

        def on(g):
            return torch.cuda.stream(g.stream) if g.stream is not None else contextlib.nullcontext()

        for g in self.groups:
            if g.stream is not None:
                g.stream.wait_stream(main)
        for g in self.groups:
            with on(g):
                p = g.plan
                for b in g.blocks:
                    p.apply_h(b.ik, b.V[:b.nb], self.veff[b.isub], b.beta, b.dkb, out=b.HV[:b.nb])
                p.subspace_rr_batched(self._rr_blocks(g, lambda b: b.nb))
                if self.mlp_params is not None:
                    for i, b in enumerate(g.blocks):
                        p.grid_mean(self.veff[b.isub], out=g.vbar[i:i + 1])
        for _ in range(n_david):
            for g in self.groups:
                with on(g):
                    p = g.plan
                    if self.mlp_params is None:
                        p.precondition_batched(self._pc_blocks(g))
                    else:
                        p.precondition_mlp_batched(self._pc_blocks(g), self.mlp_params, g.vbar)
                    for b in g.blocks:
                        p.apply_h(b.ik, b.V[b.nb:], self.veff[b.isub], b.beta, b.dkb, out=b.HV[b.nb:])
                        if b.SV is not None:
                            p.apply_s(b.ik, b.V[b.nb:], b.beta, b.aug_q, out=b.SV[b.nb:])
                    p.subspace_rr_batched(self._rr_blocks(g, lambda b: 2 * b.nb))
        for g in self.groups:
            if g.stream is not None:
                main.wait_stream(g.stream)

    def _subsystem_density(self, I: int, occws, rho):
        """rho += the density of subsystem I's bands over its k-points and, when the
        subsystem is augmented, the augmentation density of its atoms' charges."""
        p = self.plan
        for b, occw in zip(self.blocks[I], occws):
            p.density(b.ik, b.V[:b.nb], occw, rho)
        if I in self.aug:
            a = self.aug[I]
            a["charges"].zero_()
            for b, occw in zip(self.blocks[I], occws):
                p.aug_charges(b.ik, b.V[:b.nb], occw, b.beta, b.aug_q, a["atom_of"], a["charges"])
            p.aug_density(a["atoms"], a["charges"], rho)

    def _frozen_potentials(self):
        """Freeze-and-thaw (Fig. 1b caption: each subsystem iterated against the densities
        of the last broadcast): at the first of n_inner cycles the environments
        env_I = sum_{J != I} rho_J are frozen (and a Pulay history restarts); every cycle
        V_eff^I is the first potential of the pair {rho_I, env_I}."""
        s, p = self.system, self.plan
        if self.inner == 0:
            p.frozen_environment(self.rho_in, self.pairs)
            if self.mixer is not None:
                self.mix_state.zero_()
        self.inner = (self.inner + 1) % self.n_inner
        for I in range(len(s.subsystems)):
            self.pairs[I, 0].copy_(self.rho_in[I])
            p.embed_potential(self.pairs[I], self.vloc, rho_thr=s.rho_thr, veff=self.pair_veff[I],
                              energies=self.pair_en[I], info=self.einfo, **self.kinds)
            self.veff[I].copy_(self.pair_veff[I, 0])

    def cycle(self, n_david: Optional[int] = None):
        """One embedding cycle (Jacobi), or one inner cycle of the freeze-and-thaw scheme."""
        s = self.system
        p = self.plan
        n_david = s.n_david if n_david is None else n_david
        if self.scheme == "jacobi":
            p.embed_potential(self.rho_in, self.vloc, rho_thr=s.rho_thr, veff=self.veff, energies=self.energies,
                              info=self.einfo, **self.kinds)
        else:
            self._frozen_potentials()
        self.solve(n_david)
        for I, sub in enumerate(s.subsystems):
            for b in self.blocks[I]:
                self.eps[I][b.j].copy_(b.eval)
            mode = {"integer": fde.OCC_INTEGER, "fermi-dirac": fde.OCC_FERMI_DIRAC,
                    "methfessel-paxton": fde.OCC_METHFESSEL_PAXTON}[sub.smearing]
            fde.occupations(self.be, self.eps[I], self.wk[I], sub.nelec, mode, max(sub.sigma, 1e-300),
                            occw=self.occw[I], mu=self.mu[I], info=self.oinfo[I])
            self.rho_out[I].zero_()
            self._subsystem_density(I, [self.occw[I][b.j] for b in self.blocks[I]], self.rho_out[I])
        if self.mixer is None:
            fde.mix(self.be, self.rho_in, self.rho_out, s.mix_beta)
        else:
            p.mix_pulay(self.mix_state, self.x_hist, self.r_hist, self.rho_in, self.rho_out,
                        float(self.mixer.get("beta", 0.5)), float(self.mixer.get("q0", 0.0)), info=self.mix_info)

    # ---- energies ----------------------------------------------------------------
    def total_energies(self) -> torch.Tensor:
        """Energies of the last cycle's bands and output densities (Sec. 2, E_FDE; the
        Appendix recast through fragment energies), all terms from the library's
        kernels: fde_embed_potential at the output densities, fde_band_energies per
        block, fde_grid_dot of the cycle's V_eff^I and V_loc with rho_I, combined by
        fde_energy_total. Returns the device tensor [ns + 4] of fde_energy_total
        (E_K per subsystem, T^nad, E_xc^nad, E_FDE directly, E_FDE via fragments)."""
        s, p = self.system, self.plan
        if self.aug:
            # the augmented energy needs the one-centre terms of each atom's augmentation
            # sphere (Appendix, non-local pseudopotentials), which the synthetic q blocks
            # do not define
            raise fde.FdeError("energies of augmented subsystems are not defined")
        ns = len(s.subsystems)
        dev = self.be.device
        if not hasattr(self, "_e_buf"):
            self._e_buf = dict(veff=p.zeros_grid(ns),
                               en=torch.zeros((ns + 1, fde.NE), dtype=torch.float64, device=dev),
                               info=torch.zeros(1, dtype=torch.int32, device=dev),
                               band=torch.zeros((ns, 3), dtype=torch.float64, device=dev),
                               dots=torch.zeros((ns, 2), dtype=torch.float64, device=dev),
                               out=torch.zeros(ns + 4, dtype=torch.float64, device=dev))
        e = self._e_buf
        p.embed_potential(self.rho_out, self.vloc, rho_thr=s.rho_thr, veff=e["veff"], energies=e["en"],
                          info=e["info"], **self.kinds)
        e["band"].zero_()
        e["dots"].zero_()
        for I, sub in enumerate(s.subsystems):
            for b in self.blocks[I]:
                p.band_energies(b.ik, b.V[:b.nb], self.occw[I][b.j], b.beta, b.dkb, out=e["band"][I],
                                eval=self.eps[I][b.j])
            p.grid_dot(self.veff[I], self.rho_out[I], out=e["dots"][I, 0:1])
            p.grid_dot(self.vloc, self.rho_out[I], out=e["dots"][I, 1:2])
        return fde.energy_total(self.be, e["en"], e["band"], e["dots"], out=e["out"])

    # ---- one HIP graph per cycle ------------------------------------------------
    def capture(self, n_david: Optional[int] = None):
        """Run one cycle eagerly (first-use set-up of every kernel), then record the
        next cycle into a HIP graph; replay() runs the recorded cycle. The state
        tensors are fixed, so every replay advances the same engine by one cycle."""
        if self.be.emulated:
            raise fde.FdeError("graph capture needs the GPU backend")
        if self.scheme != "jacobi":
            raise fde.FdeError("graph capture records the Jacobi cycle only")
        self.cycle(n_david)
        torch.cuda.synchronize(self.be.device)
        self._graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self._graph):
            self.cycle(n_david)
        torch.cuda.synchronize(self.be.device)

    def replay(self):
        self._graph.replay()

    # ---- launch-shape autotuning ----------------------------------------------
    def autotune(self, candidates=(1, 2, 4, 8, 16), sz_candidates=None, reps: int = 5):
        """Time fde_apply_h of the largest band block with each in-plane pass kind
        (and, for the two-factor pass, each row-batch size), then with each
        bands-per-plane-workgroup value, then, where a register z-FFT exists, with
        it and with the LDS z-passes, then (for the LDS z-passes) with each
        z-sticks-per-workgroup value, and keep the fastest of each (launch shapes and
        FFT factorisations only). A value replaces the automatic choice (0) only when
        it is more than 1 % faster. Returns the best value and the timings in ms of
        every search: {"plane", "plane_ms", "rows", "rows_ms", "bpw", "bpw_ms",
        "zlds", "zlds_ms", "sz", "sz_ms"}."""
        if self.be.emulated:
            return None
        b = max((b for row in self.blocks for b in row), key=lambda b: b.nb * self.plan.npw(b.ik))
        X = b.V[:b.nb]
        HX = b.HV[b.nb:2 * b.nb] if b.HV.shape[0] >= 2 * b.nb else torch.empty_like(X)
        veff = self.veff[b.isub]

        def timed():
            self.plan.apply_h(b.ik, X, veff, b.beta, b.dkb, out=HX)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                self.plan.apply_h(b.ik, X, veff, b.beta, b.dkb, out=HX)
            e1.record()
            torch.cuda.synchronize(self.be.device)
            return e0.elapsed_time(e1) / reps

        def search(key, values):
            times = {}
            for v in values:
                self.plan.set_tuning(key, v)
                times[v] = timed()
            best = min(times, key=times.get)
            if 0 in times and times[best] > 0.99 * times[0]:
                best = 0
            self.set_tuning(key, best)
            return best, times

        kind, kind_ms = search(fde.TUNE_PLANE_KIND, (0, fde.PLANE_REG, fde.PLANE_LDS, fde.PLANE_TWO_FACTOR))
        rows, rows_ms = (None, {})
        if kind in (0, fde.PLANE_TWO_FACTOR):
            rows, rows_ms = search(fde.TUNE_PLANE_ROWS, [0] + [r for r in (4, 8, 12, 16, 20)
                                                           if r < self.system.grid[1]])
        bpw, bpw_ms = search(fde.TUNE_APPLY_BPW, [0] + [v for v in candidates if v <= b.nb])
        n3 = self.system.grid[2]
        zreg = n3 in (240, 120) or (n3 == 432 and self.prec == fde.F32)
        zlds, zlds_ms = search(fde.TUNE_Z_REGISTER, (0, 1)) if zreg else (None, {})
        if sz_candidates is None:  # the stick group only shapes the LDS z-passes
            sz_candidates = () if zreg and zlds == 0 else (1, 2, 4, 8, 16)
        sz, sz_ms = search(fde.TUNE_STICK_GROUP, sz_candidates) if sz_candidates else (None, {})
        return {"plane": kind, "plane_ms": kind_ms, "rows": rows, "rows_ms": rows_ms, "bpw": bpw, "bpw_ms": bpw_ms,
                "zlds": zlds, "zlds_ms": zlds_ms, "sz": sz, "sz_ms": sz_ms}

    def band_applies_per_cycle(self, n_david: Optional[int] = None) -> int:
        n_david = self.system.n_david if n_david is None else n_david
        return sum(b.nb * (1 + n_david) for row in self.blocks for b in row)


def davidson_fixed(plan: fde.Plan, ik: int, X0: torch.Tensor, veff: torch.Tensor, n_iter: int, beta=None, dkb=None,
                   mlp_params: Optional[torch.Tensor] = None, aug=None):
    """Block Davidson at a fixed potential (the band solver of one cycle, iterated):
    H X and Rayleigh-Ritz on X, then n_iter iterations of preconditioner (TPA, or
    the learned network when mlp_params is given), H T and Rayleigh-Ritz on [X | T].
    aug = (beta_aug, q): the generalised problem H x = e S x with the subsystem's
    augmentation overlap S (fde_apply_s), its rows S V kept beside V and HV.
    Returns the Ritz values after every iteration (list of float64 tensors [nb]);
    with aug also (X, S X) at the end."""
    nb, npw = X0.shape
    dev = plan.be.device
    V = torch.zeros((2 * nb, npw), dtype=plan.cdtype, device=dev)
    HV = torch.zeros_like(V)
    SV = torch.zeros_like(V) if aug is not None else None
    V[:nb].copy_(X0)
    eval_ = torch.zeros(nb, dtype=torch.float64, device=dev)
    active = torch.ones(2 * nb, dtype=torch.uint8, device=dev)
    rnorm = torch.zeros(nb, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    vbar = plan.grid_mean(veff) if mlp_params is not None else None
    plan.apply_h(ik, V[:nb], veff, beta, dkb, out=HV[:nb])
    if aug is not None:
        plan.apply_s(ik, V[:nb], aug[0], aug[1], out=SV[:nb])
    plan.subspace_rr_batched([plan.make_block(ik, nb, nb, V, HV, active=active, eval=eval_, info=info, sv=SV)])
    hist = []
    for _ in range(n_iter):
        pcb = [plan.make_block(ik, nb, nb, V, HV, t_active=active[nb:], eval=eval_, rnorm=rnorm, sv=SV)]
        if mlp_params is None:
            plan.precondition_batched(pcb)
        else:
            plan.precondition_mlp_batched(pcb, mlp_params, vbar)
        plan.apply_h(ik, V[nb:], veff, beta, dkb, out=HV[nb:])
        if aug is not None:
            plan.apply_s(ik, V[nb:], aug[0], aug[1], out=SV[nb:])
        plan.subspace_rr_batched([plan.make_block(ik, nb, 2 * nb, V, HV, active=active, eval=eval_, info=info,
                                                  sv=SV)])
        hist.append(eval_.clone())
    if aug is not None:
        return hist, info, V[:nb], SV[:nb]
    return hist, info


# ---------------------------------------------------------------------------
# Convergence and the supersystem comparison (Sec. 4, Table 1)
# ---------------------------------------------------------------------------
def converge(eng: "Engine", tol: float = 1e-6, max_cycles: int = 200, n_david: Optional[int] = None):
    """Cycle until int |rho_out - rho_in| summed over subsystems is below tol (electrons).
    Returns (cycles, last residual). The residual is read back each cycle."""
    p = eng.plan
    rin = torch.empty_like(eng.rho_in)
    acc = torch.zeros(1, dtype=torch.float64, device=eng.be.device)
    resid = float("inf")
    for c in range(max_cycles):
        rin.copy_(eng.rho_in)
        eng.cycle(n_david)
        acc.zero_()
        for I in range(len(eng.system.subsystems)):
            p.density_l1(eng.rho_out[I], rin[I], out=acc)
        resid = float(acc.item())
        if resid < tol:
            return c + 1, resid
    return max_cycles, resid


def supersystem_comparison(system, prec=fde.F64, backend=None, kinds=None, tol=1e-6, max_cycles=300,
                           mixer=None, n_david: Optional[int] = None, fixed_cycles: Optional[int] = None):
    """The quantities of Table 1 for one geometry: Kohn-Sham of the supersystem, FDE of the
    subsystems, and each fragment alone, every one converged with the same cycle and
    functionals. Returns a dict with
      dens_diff   <Delta rho> = 1/2 int |rho_FDE - rho_KS| (Sec. 4, the density error);
      E_KS, E_FDE, E_frag    energies (ion-ion terms excluded);
      int_KS, int_FDE        E_AB - sum_I E_I of the supersystem and of FDE, without the
                             inter-fragment ion-ion term (the same constant in both);
      cycles, residuals      of every run.
    fixed_cycles: run exactly that many cycles instead of converging to tol.
    The densities and energies come from the library's kernels; only the final
    scalars (integrals already reduced on the device) are combined here."""
    import fde_synth
    kinds = kinds or dict(xc=fde.XC_PBE, xc_nad=fde.XC_PBE, kin_nad=fde.KIN_LC94)
    mixer = mixer or dict(kind="pulay", nhist=8, beta=0.5, q0=0.8)
    out = {"cycles": {}, "residuals": {}}

    def run(sysm, name):
        eng = Engine(sysm, prec=prec, backend=backend, kinds=kinds, mixer=mixer, streams=1)
        if fixed_cycles is None:
            cyc, res = converge(eng, tol, max_cycles, n_david)
        else:
            cyc, res = converge(eng, 0.0, fixed_cycles, n_david)
        e = eng.total_energies()
        ns = len(sysm.subsystems)
        out["cycles"][name] = cyc
        out["residuals"][name] = res
        return eng, float(e[ns + 2].item())

    ks, e_ks = run(fde_synth.supersystem(system), "KS")
    rho_ks = ks.rho_out[0].clone()
    del ks
    fdeng, e_fde = run(system, "FDE")
    # 1/2 int |sum_I rho_I - rho_KS| through the library's grid reduction
    diff = fdeng.plan.density_l1(fdeng.rho_out, rho_ks)
    del fdeng
    e_frag = []
    for I in range(len(system.subsystems)):
        eng, e = run(fde_synth.fragment(system, I), f"fragment{I}")
        e_frag.append(e)
        del eng
    out.update(dens_diff=0.5 * float(diff.item()), E_KS=e_ks, E_FDE=e_fde, E_frag=e_frag,
               int_KS=e_ks - sum(e_frag), int_FDE=e_fde - sum(e_frag))
    return out
