"""Gaussian local ions and Kleinman-Bylander projectors (test infrastructure, FP64).

The paper uses ultrasoft pseudopotentials (Sec. 3) whose files are not
available; synthetic Gaussian ions and Gaussian projectors stand in.

* Local part (electron-nuclear attraction E_eN of Sec. 2; the recast
  effective potential of the Appendix groups all nuclei of all subsystems in
  V_eN). Ion potential -Z erf(r / (sqrt(2) sigma)) / r, whose transform is
  -4 pi Z exp(-G^2 sigma^2 / 2) / G^2. On D without G = 0:
      V_loc(G) = (1/Omega) sum_a [-4 pi Z_a e^{-G^2 s_a^2/2} / G^2] e^{-i G.R_a}
  and at G = 0 the regular part sum_a 2 pi Z_a s_a^2 / Omega (the divergent
  -4 pi Z / G^2 is cancelled by the neutralising background).
* Nonlocal part (Appendix, handling of non-local pseudopotentials): only the
  projectors of the subsystem's own atoms enter H_I. With q = k + G,
      s:   beta(q) = Omega^{-1/2} 2^{3/2} pi^{3/4} r^{3/2} e^{-q^2 r^2/2} e^{-i q.R}
      p_x: beta(q) = Omega^{-1/2} 4 pi^{3/4} r^{5/2} q_x e^{-q^2 r^2/2} e^{-i q.R}
  (continuum-normalised Gaussians), V_NL = sum_i |beta_i> D_i <beta_i|.

Pins: the sum over G of |beta|^2 tends to 1 (normalisation); the potential of
a single ion agrees with the erf form in real space away from the cutoff
(tests/test_oracle_hamiltonian.py); the G = 0 value equals a radial quadrature
of the regular part -Z erf(r/(sqrt 2 sigma))/r + Z/r (tests/test_oracle_pins.py).
"""
from __future__ import annotations

import math

import numpy as np

from . import basis, dft


def local_potential_G(cell: basis.Cell, ecut: float, atoms) -> np.ndarray:
    """V_loc(G) on the grid [N3, N2, N1] (zero outside D)."""
    g1, g2, g3 = basis.grid_g(cell)
    G2 = g1 * g1 + g2 * g2 + g3 * g3
    mask = basis.density_mask(cell, ecut)
    V = np.zeros(cell.shape, dtype=np.complex128)
    nz = mask & (G2 > 0)
    for a in atoms:
        R = np.asarray(a.pos, dtype=np.float64)
        phase = np.exp(-1j * (g1[nz] * R[0] + g2[nz] * R[1] + g3[nz] * R[2]))
        V[nz] += (-4.0 * math.pi * a.Z * np.exp(-0.5 * G2[nz] * a.width ** 2) / G2[nz]) * phase
    V[0, 0, 0] = sum(2.0 * math.pi * a.Z * a.width ** 2 for a in atoms)
    return V / cell.omega


def local_potential(cell: basis.Cell, ecut: float, atoms) -> np.ndarray:
    """V_loc(r) on the grid [N3, N2, N1] (real)."""
    return dft.to_real(local_potential_G(cell, ecut, atoms)).real


def kb_projectors(cell: basis.Cell, sph: basis.Sphere, atoms):
    """Projectors beta [nproj, npw] and energies D [nproj] of the given atoms.

    Channel order per atom: s, then p_x, p_y, p_z when lmax >= 1.
    """
    betas, ds = [], []
    q = sph.q
    q2 = np.einsum("gi,gi->g", q, q)
    pref = 1.0 / math.sqrt(cell.omega)
    for a in atoms:
        if a.lmax < 0:
            continue
        R = np.asarray(a.pos, dtype=np.float64)
        r = a.rbeta
        phase = np.exp(-1j * (q @ R))
        gauss = np.exp(-0.5 * q2 * r * r)
        betas.append(pref * 2.0 ** 1.5 * math.pi ** 0.75 * r ** 1.5 * gauss * phase)
        ds.append(a.d_s)
        if a.lmax >= 1:
            for i in range(3):
                betas.append(pref * 4.0 * math.pi ** 0.75 * r ** 2.5 * q[:, i] * gauss * phase)
                ds.append(a.d_p)
    if not betas:
        return np.zeros((0, sph.npw), dtype=np.complex128), np.zeros(0)
    return np.array(betas), np.array(ds, dtype=np.float64)
