"""Further pins of the oracle (CPU only): the G = 0 term of the local potential,
the dropped-column branch of the Rayleigh-Ritz Cholesky, the continuity of the
published Perdew-Zunger correlation across r_s = 1, and the integer-occupation
electron-count rule."""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as ss

import fde_synth
from oracle import basis, hamiltonian as ham, occupations as occ, pseudo, subspace
from oracle import functionals as fn


@pytest.mark.parametrize("Z,width", [(1.0, 0.7), (2.0, 0.8), (3.5, 1.3)])
def test_vloc_g0_is_the_regular_part_of_the_erf_ion(Z, width):
    # V_loc(G=0) Omega = int [-Z erf(r / (sqrt 2 w)) / r + Z / r] d^3r, by radial quadrature
    # (independent of the closed form 2 pi Z w^2 the oracle uses)
    f = lambda r: 4.0 * math.pi * r * r * Z * ss.erfc(r / (math.sqrt(2.0) * width)) / r  # noqa: E731
    ref, err = si.quad(f, 0.0, 60.0 * width, epsabs=1e-13, epsrel=1e-13, limit=400)
    assert err < 1e-10
    cell = basis.Cell((7.0, 8.0, 9.0), (12, 12, 14))
    atoms = [fde_synth.Atom((1.0, 2.0, 3.0), Z, width)]
    VG = pseudo.local_potential_G(cell, 2.0, atoms)
    assert abs(VG[0, 0, 0].real * cell.omega - ref) < 1e-10 * ref
    # two ions add
    atoms2 = atoms + [fde_synth.Atom((4.0, 5.0, 6.0), 2 * Z, 0.5 * width)]
    VG2 = pseudo.local_potential_G(cell, 2.0, atoms2)
    ref2, _ = si.quad(lambda r: 4.0 * math.pi * r * 2 * Z * ss.erfc(r / (math.sqrt(2.0) * 0.5 * width)),
                      0.0, 60.0 * width, epsabs=1e-13, epsrel=1e-13, limit=400)
    assert abs(VG2[0, 0, 0].real * cell.omega - (ref + ref2)) < 1e-10 * (ref + ref2)


def _block(nb=3, seed=41):
    cell = basis.Cell((6.0, 6.5, 7.0), (12, 12, 14))
    sph = basis.sphere(cell, 2.5, (0.25, 0.0, -0.25))
    atoms = [fde_synth.Atom((1.0, 2.0, 3.0), 2.0, 0.6, lmax=1, rbeta=0.7, d_s=0.8, d_p=0.4)]
    v = pseudo.local_potential(cell, 2.5, atoms)
    beta, dkb = pseudo.kb_projectors(cell, sph, atoms)
    X = subspace.orthonormalise(fde_synth.random_complex(seed, (nb, sph.npw)))
    H = lambda Y: ham.apply_h(cell, sph, Y, v, beta, dkb)  # noqa: E731
    HX = H(X)
    X, HX, lam = subspace.subspace_rr(X, HX, nb)
    T, _, _ = subspace.precondition(X, HX, lam, sph.kin)
    return X, HX, T, H(T), H


def _proj(X):
    return X.T @ X.conj()


def test_duplicated_correction_column_is_dropped_exactly():
    nb = 3
    X, HX, T, HT, _ = _block(nb)
    # column 5 = a copy of column 3 (T_0): its pivot is exactly rounding-level
    Td = np.vstack([T, T[:1]])
    HTd = np.vstack([HT, HT[:1]])
    S = np.vstack([X, Td]).conj() @ np.vstack([X, Td]).T
    _, dropped = subspace.cholesky_drop(S, first_droppable=nb, tol=subspace.DROP_TOL)
    assert dropped == [2 * nb]
    a = subspace.subspace_rr(np.vstack([X, Td]), np.vstack([HX, HTd]), nb)
    b = subspace.subspace_rr(np.vstack([X, T]), np.vstack([HX, HT]), nb)
    assert np.max(np.abs(a[2] - b[2])) < 1e-12
    assert np.max(np.abs(_proj(a[0]) - _proj(b[0]))) < 1e-11
    # a dependent combination of two earlier corrections is dropped as well
    Tc = np.vstack([T, 0.6 * T[1] - 0.8j * T[2]])
    HTc = np.vstack([HT, 0.6 * HT[1] - 0.8j * HT[2]])
    c = subspace.subspace_rr(np.vstack([X, Tc]), np.vstack([HX, HTc]), nb)
    assert np.max(np.abs(c[2] - b[2])) < 1e-12


def test_dropped_column_factor_is_the_factor_of_the_masked_gram():
    nb = 3
    X, _, T, _, _ = _block(nb, seed=43)
    V = np.vstack([X, T, T[2:3]])
    S = V.conj() @ V.T
    L, dropped = subspace.cholesky_drop(S, first_droppable=nb, tol=subspace.DROP_TOL)
    j = dropped[0]
    Sm = S.copy()
    Sm[j, :] = 0.0
    Sm[:, j] = 0.0
    Sm[j, j] = 1.0
    assert np.max(np.abs(L - np.linalg.cholesky(Sm))) < 1e-12


def test_dependent_band_column_is_an_error():
    nb = 3
    X, _, _, _, _ = _block(nb)
    V = np.vstack([X[:2], X[1:2]])
    with pytest.raises(np.linalg.LinAlgError):
        subspace.cholesky_drop(V.conj() @ V.T, first_droppable=nb, tol=subspace.DROP_TOL)


def test_pz81_potential_continuous_at_rs_1():
    # the published C and D were chosen so that eps_c and v_c are continuous at
    # r_s = 1; the C r_s ln r_s term vanishes there in eps_c but not in v_c, so this
    # pins C (to the printed precision of the constants, about 3e-5 Ha)
    p = fn.PZ
    hi = p["g"] / (1 + p["b1"] + p["b2"])
    vhi = hi * (1 + 7.0 / 6.0 * p["b1"] + 4.0 / 3.0 * p["b2"]) / (1 + p["b1"] + p["b2"])
    vlo = (p["B"] - p["A"] / 3.0) + (2.0 * p["D"] - p["C"]) / 3.0
    assert abs(vhi - vlo) < 5e-5
    rho1 = 3 / (4 * math.pi)
    e_a, v_a = fn.pz81(np.array([rho1 * (1 + 1e-12), rho1 * (1 - 1e-12)]))
    assert abs(v_a[0] - v_a[1]) < 5e-5 and abs(e_a[0] - e_a[1]) < 5e-5


def test_integer_occupations_reject_odd_or_fractional_counts():
    eps = np.array([[-0.5, -0.3, -0.1, 0.2]])
    wk = np.array([1.0])
    for ne in (1.0, 5.0, 3.5):
        with pytest.raises(ValueError):
            occ.occupations(eps, wk, ne, "integer")
    f, _ = occ.occupations(eps, wk, 6.0, "integer")
    assert np.array_equal(f, np.array([[2.0, 2.0, 2.0, 0.0]]))
