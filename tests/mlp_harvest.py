"""Training and evaluation data for the learned preconditioner, from FP64 oracle
solves (test infrastructure: calls only oracle/ and fde_synth).

Cells: 8 x 8 x 9 bohr, 18 x 18 x 20 grid, E_cut = 5 Ha, k = (1/4, 0, -1/4);
four Gaussian ions per geometry (Z in {1, 2}, width 0.7-0.9 bohr, >= 1.5 bohr
apart, seeded by the geometry index); the potential is the ions' local
potential. For each training geometry the oracle runs TPA-preconditioned
Davidson from seeded bands and, after every Rayleigh-Ritz step, solves the
Jacobi-Davidson correction equation exactly against the dense H; every
coefficient of every active band becomes one training row.
"""
import numpy as np

import fde_synth
from oracle import basis, hamiltonian as ham, mlp, pseudo, subspace

L = (8.0, 8.0, 9.0)
GRID = (18, 18, 20)
ECUT = 5.0
KF = (0.25, 0.0, -0.25)
NB = 6


def case(geometry: int):
    rng = fde_synth.rng_for(5, geometry, 31)
    cell = basis.Cell(L, GRID)
    sph = basis.sphere(cell, ECUT, KF)
    pos = []
    while len(pos) < 4:
        p = rng.uniform(0.0, 1.0, 3) * np.array(L)
        if all(np.linalg.norm((p - q + 0.5 * np.array(L)) % np.array(L) - 0.5 * np.array(L)) >= 1.5 for q in pos):
            pos.append(p)
    atoms = [fde_synth.Atom(tuple(map(float, p)), float(rng.integers(1, 3)), float(rng.uniform(0.7, 0.9)))
             for p in pos]
    veff = pseudo.local_potential(cell, ECUT, atoms)
    X0 = fde_synth.random_coefficients(5, geometry, 0, 0, NB, sph.npw) / (1 + 2 * sph.kin)[None]
    return cell, sph, veff, X0


def harvest(geometries, n_iter=8):
    rows = []
    for g in geometries:
        cell, sph, veff, X0 = case(g)
        Hm = ham.explicit_h(cell, sph, veff)
        vbar = float(np.mean(veff))
        X = subspace.orthonormalise(X0)
        HX = X @ Hm.T
        X, HX, lam = subspace.subspace_rr(X, HX, NB)
        for _ in range(n_iter):
            R = HX - lam[:, None] * X
            act = np.linalg.norm(R, axis=1) > 1e-8
            if act.any():
                D = np.stack([mlp.exact_correction(Hm, X[n], lam[n], R[n]) for n in np.nonzero(act)[0]])
                rows.append(mlp.samples(sph.kin, X[act], R[act], lam[act], vbar, D))
            T, active, _ = subspace.precondition(X, HX, lam, sph.kin)
            HT = T @ Hm.T
            X, HX, lam = subspace.subspace_rr(np.vstack([X, T]), np.vstack([HX, HT]), NB,
                                              np.concatenate([np.ones(NB, bool), active]))
    return np.concatenate(rows).astype(np.float32)


def exact_eigenvalues(geometry: int):
    cell, sph, veff, _ = case(geometry)
    return np.linalg.eigvalsh(ham.explicit_h(cell, sph, veff))[:NB]
