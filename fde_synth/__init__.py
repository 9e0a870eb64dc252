"""Seeded synthetic inputs for periodic frozen-density embedding runs.

This module only draws random numbers and lays out geometries, k-meshes and
run settings. It contains none of the method's arithmetic (no reciprocal
lattice, no transforms, no potentials): both the CPU reference in ``oracle/``
and the GPU library consume what it returns, each computing everything else on
its own.

The paper's benchmark systems (molecules on Pt/Au slabs, Sec. 4 and Table 1)
need pseudopotential files and geometries that are not available, so these
synthetic cells keep their shape instead: one metallic slab sampled with a
2x2x1 Monkhorst-Pack mesh (Sec. 3), molecules treated at Gamma with integer
occupations (Sec. 3), and many fragments (the 13-fragment water bilayer of
Sec. 4 motivates the batched cell).

Random streams: numpy PCG64 seeded with ``SeedSequence([base + 1000*cfg +
geometry, *tags])`` where ``base = 14067803``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

SEED_BASE = 14067803


def rng_for(cfg: int, geometry: int = 0, *tags: int) -> np.random.Generator:
    """Independent PCG64 stream for (config, geometry, tags...)."""
    ss = np.random.SeedSequence([SEED_BASE + 1000 * cfg + geometry, *[int(t) for t in tags]])
    return np.random.Generator(np.random.PCG64(ss))


@dataclass
class Atom:
    pos: Tuple[float, float, float]  # bohr, Cartesian, inside the cell
    Z: float                          # ionic charge of the Gaussian ion
    width: float                      # Gaussian width sigma (bohr)
    lmax: int = -1                    # -1: no projector, 0: s, 1: s + p_x,p_y,p_z
    rbeta: float = 1.0                # projector Gaussian radius (bohr)
    d_s: float = 1.0                  # KB energy of the s channel (Ha)
    d_p: float = 0.5                  # KB energy of each p channel (Ha)


@dataclass
class Subsystem:
    name: str
    atoms: List[Atom]
    nbands: int
    nelec: float                      # electrons (occupations f in [0, 2])
    kfrac: np.ndarray                 # [nk, 3] reduced k (units of b_i)
    kweight: np.ndarray               # [nk], sums to 1
    smearing: str                     # "integer" | "fermi-dirac"
    sigma: float = 0.0                # smearing width (Ha)
    aug: bool = False                 # augmentation overlap on the subsystem's own projectors
                                      # (augmentation_q; Gaussian augmentation of width rbeta)


@dataclass
class System:
    cfg: int
    geometry: int
    L: Tuple[float, float, float]
    grid: Tuple[int, int, int]        # (N1, N2, N3); arrays are C-order [N3][N2][N1]
    ecut: float                       # wavefunction kinetic cutoff (Ha)
    subsystems: List[Subsystem]
    n_cycles: int = 10
    n_david: int = 4
    mix_beta: float = 0.3
    rho_thr: float = 1e-10

    @property
    def all_kfrac(self) -> np.ndarray:
        """Distinct k-points over all subsystems, in first-seen order."""
        out: List[Tuple[float, float, float]] = []
        for s in self.subsystems:
            for k in s.kfrac:
                t = tuple(float(x) for x in k)
                if t not in out:
                    out.append(t)
        return np.array(out, dtype=np.float64).reshape(-1, 3)

    def k_index(self, isub: int) -> List[int]:
        allk = [tuple(k) for k in self.all_kfrac.tolist()]
        return [allk.index(tuple(float(x) for x in k)) for k in self.subsystems[isub].kfrac]


# ----------------------------------------------------------------------------
# k meshes (unshifted-standard Monkhorst-Pack with q=2 gives +-1/4)
# ----------------------------------------------------------------------------
def mp_mesh(n1: int, n2: int, n3: int) -> Tuple[np.ndarray, np.ndarray]:
    def axis(n):
        return [0.0] if n == 1 else [(2 * r - n - 1) / (2.0 * n) for r in range(1, n + 1)]
    ks = [(a, b, c) for a in axis(n1) for b in axis(n2) for c in axis(n3)]
    k = np.array(ks, dtype=np.float64)
    w = np.full(len(ks), 1.0 / len(ks))
    return k, w


GAMMA = (np.zeros((1, 3)), np.ones(1))


def _min_image_dist(a, b, L):
    d = np.asarray(a, float) - np.asarray(b, float)
    L = np.asarray(L, float)
    d -= L * np.round(d / L)
    return float(np.sqrt(np.dot(d, d)))


def _place_uniform(rng, n, L, dmin, existing, lo=None, hi=None, ball=None, max_tries=200000):
    """Random sequential addition with a minimum-image distance constraint."""
    pts = []
    L = np.asarray(L, float)
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place atoms")
        if ball is not None:
            c, r = ball
            while True:
                v = rng.uniform(-r, r, 3)
                if np.dot(v, v) <= r * r:
                    break
            p = np.asarray(c, float) + v
        else:
            l0 = np.zeros(3) if lo is None else np.asarray(lo, float)
            h0 = L if hi is None else np.asarray(hi, float)
            p = l0 + rng.uniform(0.0, 1.0, 3) * (h0 - l0)
        p = np.mod(p, L)
        others = existing + pts
        if others:
            d = np.asarray(others, float) - p
            d -= L * np.round(d / L)
            if np.min(np.einsum('ij,ij->i', d, d)) < dmin * dmin:
                continue
        pts.append(p)
    return pts


# ----------------------------------------------------------------------------
# Building blocks
# ----------------------------------------------------------------------------
def slab_positions(nrep: int = 1, a: float = 3.4) -> List[Tuple[float, float, float]]:
    """4 layers of 3x3 square nets with ABCA registry shifts, repeated nrep x nrep."""
    shifts = [(0.0, 0.0), (a / 3, a / 3), (2 * a / 3, 2 * a / 3), (0.0, 0.0)]
    zs = [4.0, 6.2, 8.4, 10.6]
    side = 3 * a
    out = []
    for (sx, sy), z in zip(shifts, zs):
        for rx in range(nrep):
            for ry in range(nrep):
                for i in range(3):
                    for j in range(3):
                        x = (i * a + sx + rx * side) % (side * nrep)
                        y = (j * a + sy + ry * side) % (side * nrep)
                        out.append((x, y, z))
    return out


def molecule(rng, centre, L, existing, natoms=6, radius=2.5, dmin=1.5, width=0.8):
    """Seeded molecule: Z in 1..4 resampled until the total is even and <= 16."""
    while True:
        Z = rng.integers(1, 5, natoms)
        if Z.sum() % 2 == 0 and Z.sum() <= 16:
            break
    pos = _place_uniform(rng, natoms, L, dmin, existing, ball=(centre, radius))
    return [Atom(tuple(map(float, p)), float(z), width) for p, z in zip(pos, Z)]


# ----------------------------------------------------------------------------
# Configurations
# ----------------------------------------------------------------------------
def config1(geometry: int = 0) -> System:
    """Two 2-atom subsystems in a 10 bohr cube, 24^3 grid, Gamma, FP64 plain method."""
    rng = rng_for(1, geometry)
    L = (10.0, 10.0, 10.0)
    pos = _place_uniform(rng, 4, L, 3.0, [])
    subs = []
    for i in range(2):
        atoms = [Atom(tuple(map(float, p)), 2.0, 0.8) for p in pos[2 * i:2 * i + 2]]
        subs.append(Subsystem(f"frag{i}", atoms, nbands=2, nelec=4.0,
                              kfrac=GAMMA[0].copy(), kweight=GAMMA[1].copy(), smearing="integer"))
    return System(1, geometry, L, (24, 24, 24), 7.0, subs, n_cycles=10, n_david=4)


def config2(geometry: int = 0, jitter: float = 0.0) -> System:
    """Slab (36 atoms, s projectors, 4 k) + 6-atom molecule (Gamma) in 10.2x10.2x40."""
    rng = rng_for(2, geometry)
    L = (10.2, 10.2, 40.0)
    sp = slab_positions(1)
    if jitter > 0:
        sp = [tuple(float(c) for c in np.mod(np.asarray(p) + rng.normal(0, jitter, 3), L)) for p in sp]
    slab = [Atom(p, 1.0, 1.0, lmax=0) for p in sp]
    k, w = mp_mesh(2, 2, 1)
    A = Subsystem("slab", slab, nbands=40, nelec=36.0, kfrac=k, kweight=w,
                  smearing="fermi-dirac", sigma=0.01)
    mol = molecule(rng, (5.1, 5.1, 16.6), L, [a.pos for a in slab])
    B = Subsystem("molecule", mol, nbands=8, nelec=float(sum(a.Z for a in mol)),
                  kfrac=GAMMA[0].copy(), kweight=GAMMA[1].copy(), smearing="integer")
    return System(2, geometry, L, (60, 60, 240), 40.0, [A, B], n_cycles=10, n_david=4)


_C3_MESH = {1: (1, 1, 1), 2: (1, 1, 2), 4: (2, 2, 1), 8: (2, 2, 2)}


def config3(geometry: int = 0, nsub: int = 64) -> System:
    """64 uneven subsystems in a 20 bohr cube on a 72^3 grid (batched cycle)."""
    rng = rng_for(3, geometry)
    L = (20.0, 20.0, 20.0)
    existing: List[np.ndarray] = []
    subs = []
    for i in range(nsub):
        nb = int(round(math.exp(rng.uniform(math.log(4), math.log(128)))))
        nk = int(rng.choice([1, 2, 4, 8]))
        nat = int(rng.integers(1, 25))
        ne = 2.0 * math.floor(0.8 * nb)
        pos = _place_uniform(rng, nat, L, 1.6, existing)
        existing.extend(pos)
        atoms = [Atom(tuple(map(float, p)), ne / nat, 0.8) for p in pos]
        k, w = mp_mesh(*_C3_MESH[nk])
        subs.append(Subsystem(f"s{i}", atoms, nbands=nb, nelec=ne, kfrac=k, kweight=w,
                              smearing="fermi-dirac", sigma=0.01))
    return System(3, geometry, L, (72, 72, 72), 15.0, subs, n_cycles=10, n_david=4)


def config3_reduced(geometry: int = 0) -> System:
    """Six uneven subsystems in a 12 bohr cube on a 30^3 grid (E_cut 5 Ha): a cell the
    CPU reference can follow for a few cycles, with the unevenness of the 64-subsystem
    cube -- 4 to 48 bands, 1 to 4 k-points, Fermi-Dirac 0.01 Ha, 2 floor(0.8 nb)
    electrons on ceil(N_e / 4) Gaussian ions each (width 0.8, >= 1.6 bohr apart)."""
    rng = rng_for(6, geometry)
    L = (12.0, 12.0, 12.0)
    existing: List[np.ndarray] = []
    subs = []
    for i, (nb, nk) in enumerate([(4, 1), (6, 2), (10, 4), (16, 1), (30, 2), (48, 1)]):
        ne = 2.0 * math.floor(0.8 * nb)
        nat = max(1, int(math.ceil(ne / 4.0)))
        pos = _place_uniform(rng, nat, L, 1.6, existing)
        existing.extend(pos)
        atoms = [Atom(tuple(map(float, p)), ne / nat, 0.8) for p in pos]
        k, w = mp_mesh(*_C3_MESH[nk])
        subs.append(Subsystem(f"u{i}", atoms, nbands=nb, nelec=ne, kfrac=k, kweight=w,
                              smearing="fermi-dirac", sigma=0.01))
    return System(6, geometry, L, (30, 30, 30), 5.0, subs, n_cycles=3, n_david=4)


def config4(geometry: int = 0) -> System:
    """144-atom slab (s+p projectors, 2 k, 320 bands) + 4 molecules, 144x144x432 grid."""
    rng = rng_for(4, geometry)
    L = (20.4, 20.4, 60.0)
    slab = [Atom(p, 1.0, 1.0, lmax=1) for p in slab_positions(2)]
    k = np.array([[0.25, 0.0, 0.0], [-0.25, 0.0, 0.0]])
    w = np.array([0.5, 0.5])
    subs = [Subsystem("slab", slab, nbands=320, nelec=144.0, kfrac=k, kweight=w,
                      smearing="fermi-dirac", sigma=0.01)]
    existing = [a.pos for a in slab]
    for q, (cx, cy) in enumerate([(5.1, 5.1), (15.3, 5.1), (5.1, 15.3), (15.3, 15.3)]):
        mol = molecule(rng, (cx, cy, 16.6), L, existing)
        existing += [a.pos for a in mol]
        subs.append(Subsystem(f"mol{q}", mol, nbands=8, nelec=float(sum(a.Z for a in mol)),
                              kfrac=GAMMA[0].copy(), kweight=GAMMA[1].copy(), smearing="integer"))
    return System(4, geometry, L, (144, 144, 432), 26.0, subs, n_cycles=3, n_david=4)


def config5(geometry: int) -> System:
    """Config-2 cell with the molecule redrawn and the slab jittered (learned preconditioner set)."""
    s = config2(geometry, jitter=0.05)
    s.cfg = 5
    return s


def tiny(geometry: int = 0, grid=(12, 12, 12), L=(6.0, 6.0, 6.0), ecut=3.0, nbands=3,
         kfrac=None, with_kb=False, nsub=2) -> System:
    """Small cells for dense-matrix checks (8^3-12^3 grids)."""
    rng = rng_for(9, geometry)
    pos = _place_uniform(rng, 2 * nsub, L, 1.5, [])
    if kfrac is None:
        k, w = GAMMA[0].copy(), GAMMA[1].copy()
    else:
        k = np.asarray(kfrac, float).reshape(-1, 3)
        w = np.full(len(k), 1.0 / len(k))
    subs = []
    for i in range(nsub):
        atoms = [Atom(tuple(map(float, p)), 1.0, 0.7, lmax=(1 if with_kb else -1), rbeta=0.8)
                 for p in pos[2 * i:2 * i + 2]]
        subs.append(Subsystem(f"t{i}", atoms, nbands=nbands, nelec=2.0, kfrac=k.copy(),
                              kweight=w.copy(), smearing="fermi-dirac", sigma=0.05))
    return System(9, geometry, tuple(L), tuple(grid), ecut, subs, n_cycles=3, n_david=3)


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4}


def augmentation_q(atoms, q_s: float = 0.4, q_p: float = 0.15, q_sp: float = 0.05):
    """Synthetic augmentation overlaps for the projectors of `atoms` (channel order s,
    p_x, p_y, p_z as the projectors): a real symmetric positive definite block per atom
    (s and p diagonal, an s-p_x coupling), zero between atoms; and the atom of every
    projector. Returns (q [nproj, nproj], atom_of [nproj])."""
    blocks, owner = [], []
    for a_i, a in enumerate(atoms):
        if a.lmax < 0:
            continue
        n = 1 if a.lmax == 0 else 4
        b = np.zeros((n, n))
        b[0, 0] = q_s
        for i in range(1, n):
            b[i, i] = q_p
        if n > 1:
            b[0, 1] = b[1, 0] = q_sp
        blocks.append(b)
        owner += [a_i] * n
    nproj = len(owner)
    q = np.zeros((nproj, nproj))
    o = 0
    for b in blocks:
        n = b.shape[0]
        q[o:o + n, o:o + n] = b
        o += n
    return q, np.array(owner, dtype=np.int32)


# ----------------------------------------------------------------------------
# Partitions of one geometry (layout only): the supersystem and the fragments
# ----------------------------------------------------------------------------
def supersystem(system: System, sigma: float = 0.01) -> System:
    """All atoms, bands and electrons of `system` in one subsystem (Kohn-Sham of the
    whole: N_S = 1), on the k-mesh of the subsystem with the most k-points, Fermi-Dirac
    smearing of width sigma (the slab is metallic)."""
    kmain = max(system.subsystems, key=lambda s: len(s.kfrac))
    atoms = [a for s in system.subsystems for a in s.atoms]
    sub = Subsystem("supersystem", atoms, nbands=sum(s.nbands for s in system.subsystems),
                    nelec=sum(s.nelec for s in system.subsystems), kfrac=kmain.kfrac.copy(),
                    kweight=kmain.kweight.copy(), smearing="fermi-dirac", sigma=sigma)
    return System(system.cfg, system.geometry, system.L, system.grid, system.ecut, [sub],
                  n_cycles=system.n_cycles, n_david=system.n_david, mix_beta=system.mix_beta,
                  rho_thr=system.rho_thr)


def fragment(system: System, isub: int) -> System:
    """Subsystem isub alone in the same cell (its own atoms, bands, electrons and k-points)."""
    s = system.subsystems[isub]
    sub = Subsystem(s.name, list(s.atoms), s.nbands, s.nelec, s.kfrac.copy(), s.kweight.copy(), s.smearing,
                    s.sigma)
    return System(system.cfg, system.geometry, system.L, system.grid, system.ecut, [sub],
                  n_cycles=system.n_cycles, n_david=system.n_david, mix_beta=system.mix_beta,
                  rho_thr=system.rho_thr)


# ----------------------------------------------------------------------------
# Random numbers consumed by the method
# ----------------------------------------------------------------------------
def random_coefficients(cfg: int, geometry: int, isub: int, ik: int, nb: int, npw: int,
                        dtype=np.complex128) -> np.ndarray:
    """Raw complex normal draws u1 + i u2, shape [nb][npw] (band-major).

    The initial bands are these numbers damped by a function of |k+G|; the
    damping is computed by each side from its own plane-wave set.
    """
    rng = rng_for(cfg, geometry, 7, isub, ik)
    z = rng.standard_normal((nb, npw, 2))
    return (z[..., 0] + 1j * z[..., 1]).astype(dtype)


def random_grid(seed: int, grid: Sequence[int], lo=0.0, hi=1.0, dtype=np.float64) -> np.ndarray:
    """Uniform random real field [N3][N2][N1]."""
    rng = rng_for(0, 0, 11, seed)
    N1, N2, N3 = grid
    return rng.uniform(lo, hi, (N3, N2, N1)).astype(dtype)


def random_complex(seed: int, shape, dtype=np.complex128) -> np.ndarray:
    rng = rng_for(0, 0, 13, seed)
    z = rng.standard_normal(tuple(shape) + (2,))
    return (z[..., 0] + 1j * z[..., 1]).astype(dtype)


def random_real(seed: int, shape, lo=-1.0, hi=1.0, dtype=np.float64) -> np.ndarray:
    rng = rng_for(0, 0, 17, seed)
    return rng.uniform(lo, hi, tuple(shape)).astype(dtype)


def mlp_init(seed: int = 0) -> np.ndarray:
    """Initial parameters of the 4 -> 64 -> 64 -> 1 preconditioner network, flat
    [W1 (64x4), b1, W2 (64x64), b2, w3, b3]: normal hidden weights scaled by
    1/sqrt(fan-in), zero biases, zero output layer (so the network starts at 0)."""
    rng = rng_for(5, 0, 23, seed)
    w1 = rng.normal(0.0, 0.5, 64 * 4)
    w2 = rng.normal(0.0, 0.125, 64 * 64)
    return np.concatenate([w1, np.zeros(64), w2, np.zeros(64), np.zeros(64), np.zeros(1)])
