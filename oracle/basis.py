"""Cell, plane-wave sets and reciprocal-space grids (test infrastructure, FP64).

The paper expands the periodic parts u_{j,k} of the Bloch orbitals and the
density in plane waves (Sec. 1 and Sec. 3; the Kohn-Sham-like equation Eq. KS
acts on u with -(nabla + ik)^2/2). Conventions used here:

* orthorhombic cell L1 x L2 x L3, Omega = L1 L2 L3, b_i = 2 pi / L_i;
* centred Miller indices m_i; grid index j_i = m_i mod N_i;
* wavefunction sphere S_k = {G : |k+G|^2 / 2 <= E_cut} with
  q_i = (m_i + kf_i) * b_i and the test 0.5*(q1*q1 + q2*q2 + q3*q3) <= E_cut
  evaluated in that order in FP64;
* S_k is ordered lexicographically on (m1, m2, m3), m3 fastest, so every
  z-stick (fixed m1, m2) is contiguous;
* density sphere D = {G : g1*g1 + g2*g2 + g3*g3 <= 8 E_cut}, g_i = m_i * b_i,
  i.e. |G| <= 2 sqrt(2 E_cut), which holds every component of a product of
  two orbitals;
* u(r) = Omega^{-1/2} sum_{G in S_k} c(G) e^{i G.r}, so sum |c|^2 = 1 for a
  normalised orbital.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Cell:
    L: np.ndarray
    grid: tuple  # (N1, N2, N3)

    def __init__(self, L, grid):
        self.L = np.asarray(L, dtype=np.float64).reshape(3)
        self.grid = tuple(int(n) for n in grid)

    @property
    def b(self) -> np.ndarray:
        return 2.0 * np.pi / self.L

    @property
    def omega(self) -> float:
        return float(self.L[0] * self.L[1] * self.L[2])

    @property
    def npts(self) -> int:
        N1, N2, N3 = self.grid
        return N1 * N2 * N3

    @property
    def dV(self) -> float:
        return self.omega / self.npts

    @property
    def shape(self) -> tuple:
        """Array shape of a grid, C-order [N3, N2, N1]."""
        N1, N2, N3 = self.grid
        return (N3, N2, N1)

    def positions(self):
        """Cartesian coordinates of the grid points, three arrays [N3, N2, N1]."""
        N1, N2, N3 = self.grid
        z, y, x = np.meshgrid(np.arange(N3) * self.L[2] / N3, np.arange(N2) * self.L[1] / N2,
                              np.arange(N1) * self.L[0] / N1, indexing="ij")
        return x, y, z


def centred(n: int) -> np.ndarray:
    """Centred Miller index of each grid index 0..n-1 (Nyquist -> +n/2)."""
    j = np.arange(n)
    return np.where(j <= n // 2, j, j - n)


def grid_g(cell: Cell):
    """Cartesian G components on the FFT grid, three arrays [N3, N2, N1]."""
    N1, N2, N3 = cell.grid
    b = cell.b
    m3, m2, m1 = np.meshgrid(centred(N3), centred(N2), centred(N1), indexing="ij")
    return m1 * b[0], m2 * b[1], m3 * b[2]


def density_mask(cell: Cell, ecut: float) -> np.ndarray:
    """Boolean [N3, N2, N1]: grid point's G lies in D (|G|^2 <= 8 E_cut)."""
    g1, g2, g3 = grid_g(cell)
    return (g1 * g1 + g2 * g2 + g3 * g3) <= 8.0 * ecut


def check_grid(cell: Cell, ecut: float) -> None:
    """Products of two orbitals must not alias: N_i > 4 sqrt(2 E_cut) / b_i."""
    gmax = math.sqrt(2.0 * ecut)
    for n, b in zip(cell.grid, cell.b):
        if not n > 4.0 * gmax / b:
            raise ValueError(f"grid {n} too small for E_cut {ecut} (needs > {4 * gmax / b:.2f})")


@dataclass
class Sphere:
    """Plane-wave set S_k of one k-point."""
    kfrac: np.ndarray    # [3] reduced
    miller: np.ndarray   # [npw, 3] int (m1, m2, m3), lexicographic
    q: np.ndarray        # [npw, 3] Cartesian k+G
    kin: np.ndarray      # [npw] |k+G|^2 / 2
    index: tuple         # (iz, iy, ix) grid indices of each G

    @property
    def npw(self) -> int:
        return len(self.kin)


def sphere(cell: Cell, ecut: float, kfrac) -> Sphere:
    """S_k = {G : |k+G|^2/2 <= E_cut}, lexicographic on (m1, m2, m3)."""
    kf = np.asarray(kfrac, dtype=np.float64).reshape(3)
    b = cell.b
    gmax = math.sqrt(2.0 * ecut)
    lim = [int(math.ceil(gmax / b[i] + abs(kf[i]))) + 1 for i in range(3)]
    rows = []
    for m1 in range(-lim[0], lim[0] + 1):
        q1 = (m1 + kf[0]) * b[0]
        for m2 in range(-lim[1], lim[1] + 1):
            q2 = (m2 + kf[1]) * b[1]
            for m3 in range(-lim[2], lim[2] + 1):
                q3 = (m3 + kf[2]) * b[2]
                if 0.5 * (q1 * q1 + q2 * q2 + q3 * q3) <= ecut:
                    rows.append((m1, m2, m3))
    mill = np.array(rows, dtype=np.int64).reshape(-1, 3)
    for i in range(3):
        if mill.size and 2 * np.max(np.abs(mill[:, i])) >= cell.grid[i]:
            raise ValueError("sphere does not fit the grid")
    q = (mill + kf[None, :]) * b[None, :]
    kin = 0.5 * (q[:, 0] * q[:, 0] + q[:, 1] * q[:, 1] + q[:, 2] * q[:, 2])
    N1, N2, N3 = cell.grid
    index = (np.mod(mill[:, 2], N3), np.mod(mill[:, 1], N2), np.mod(mill[:, 0], N1))
    return Sphere(kf, mill, q, kin, index)


def to_grid(cell: Cell, sph: Sphere, c: np.ndarray) -> np.ndarray:
    """Place sphere coefficients [..., npw] on a zero reciprocal grid [..., N3, N2, N1]."""
    c = np.asarray(c)
    out = np.zeros(c.shape[:-1] + cell.shape, dtype=np.complex128)
    out[(...,) + sph.index] = c
    return out


def from_grid(sph: Sphere, F: np.ndarray) -> np.ndarray:
    """Read the sphere coefficients [..., npw] back from a reciprocal grid."""
    return F[(...,) + sph.index]
