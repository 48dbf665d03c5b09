"""Pins for the oracle's scalar -> spinor transformation (Eq. 33 with the
matrices of Eq. 14, the coupling of Eq. 10 / App. A and the complex harmonics
of Eq. 13).  Each test fixes part of it by something other than the oracle:

  * C_alpha, C_beta (Eq. 10)                 -> sympy's Clebsch-Gordan coefficients
  * complex harmonics from App. B real ones  -> scipy's sph_harm_y (Condon-Shortley)
  * pairing of large spinors with small shells, phases of both components
                                             -> (sigma . r) Upsilon_kappa = -Upsilon_-kappa
  * completeness / normalisation             -> G^L unitary, G^S columns orthonormal
  * the transform itself                     -> one atom in a spherical potential:
                                                H+ and S+ diagonal in (kappa, m_j), m_j-independent
"""
import math

import numpy as np
import pytest
from scipy.special import erf, sph_harm_y

import oracle
import workload as W

SIG = (np.array([[0, 1], [1, 0]], dtype=complex), np.array([[0, -1j], [1j, 0]]),
       np.array([[1, 0], [0, -1]], dtype=complex))


def test_cg_half_matches_sympy():
    from sympy import S
    from sympy.physics.quantum.cg import CG
    for l in range(5):
        for j2 in ((2 * l + 1, 2 * l - 1) if l else (1,)):
            for mj2 in range(-j2, j2 + 1, 2):
                for spin, ms2 in ((0, 1), (1, -1)):
                    ml2 = mj2 - ms2
                    ref = 0.0
                    if abs(ml2) <= 2 * l:
                        ref = float(CG(S(l), S(ml2) / 2, S(1) / 2, S(ms2) / 2, S(j2) / 2, S(mj2) / 2).doit())
                    assert abs(oracle.cg_half(l, j2, mj2, spin) - ref) < 1e-14, (l, j2, mj2, spin)


def test_complex_harmonics_match_scipy():
    rng = np.random.default_rng(8001)
    for l in range(5):
        for m in range(-l, l + 1):
            for _ in range(5):
                p = rng.standard_normal(3)
                r = np.linalg.norm(p)
                got = sum(z * oracle.solid_harmonic(l, mp, *p)[0] / r ** l
                          for mp, z in oracle.complex_harmonic_coefs(l, m))
                ref = complex(sph_harm_y(l, m, math.acos(p[2] / r), math.atan2(p[1], p[0])))
                assert abs(got - ref) < 1e-13, (l, m)


@pytest.fixture(scope="module")
def pair_bases():
    # one atom with shells s..f (and a second p, d) so every kappa of l <= 3 occurs;
    # its small component has l~ up to 4
    shells = [(0, [0.6, 2.5, 9.0], [0.4, 0.9, 0.3]), (1, [0.5, 1.7, 6.0], [0.7, 0.6, 0.4]),
              (2, [0.55, 2.0, 8.0], [0.5, 0.5, 0.5]), (3, [0.7, 3.0, 10.0], [0.6, 0.4, 0.9]),
              (1, [0.9, 4.0, 15.0], [0.3, 1.0, 0.2]), (2, [0.8, 2.6, 11.0], [0.4, 0.7, 0.2])]
    v = lambda x, y, z: -82.0 * erf(np.sqrt(x * x + y * y + z * z) / 0.5) / np.maximum(
        np.sqrt(x * x + y * y + z * z), 1e-300)
    wl = W.pin_workload([82], [[0.0, 0.0, 0.0]], [shells], nrad=200, ntheta=14, nphi=28, nint=1024, v=v)
    wl = W.ket_tables(wl, np.array([-1.3, -0.4, -0.75, -0.2, -0.05, -0.9]))
    ws = W.small_component(wl, 8002)
    return wl, ws


def test_sigma_r_maps_large_to_small_spin_angular(pair_bases):
    """For every spinor function, the angular parts built from G^L and G^S
    (with the real harmonics of App. B) satisfy (sigma . r^) U_L = -U_S: the
    small component carries Upsilon_{-kappa, m_j} of the same j, m_j."""
    wl, ws = pair_bases
    GL, GS = oracle.spinor_G(wl, ws)
    rng = np.random.default_rng(8003)

    def real_Y(w, p):
        vals = []
        for s in range(w.atom_shell_off[0], w.atom_shell_off[1]):
            l = int(w.shell_l[s])
            vals.extend(oracle.solid_harmonic(l, m, *p)[0] for m in range(-l, l + 1))
        return np.array(vals)

    worst = 0.0
    for _ in range(12):
        p = rng.standard_normal(3)
        p /= np.linalg.norm(p)  # unit sphere: solid harmonics = Y_lm
        yl, ys = real_Y(wl, p), real_Y(ws, p)
        UL = np.stack([yl @ GL[0][sp] for sp in range(2)])  # [spin, spinor]
        US = np.stack([ys @ GS[0][sp] for sp in range(2)])
        sr = sum(p[c] * SIG[c] for c in range(3))
        worst = max(worst, float(np.max(np.abs(sr @ UL + US))))
    assert worst < 1e-13, worst


def test_G_unitary_and_isometric(pair_bases):
    wl, ws = pair_bases
    GL, GS = oracle.spinor_G(wl, ws)
    for gl, gs in zip(GL, GS):
        ML = np.concatenate([gl[0], gl[1]])
        MS = np.concatenate([gs[0], gs[1]])
        assert ML.shape[0] == ML.shape[1]
        assert np.max(np.abs(ML.conj().T @ ML - np.eye(ML.shape[1]))) < 1e-14
        assert np.max(np.abs(ML @ ML.conj().T - np.eye(ML.shape[0]))) < 1e-14
        assert np.max(np.abs(MS.conj().T @ MS - np.eye(MS.shape[1]))) < 1e-14


def test_spherical_atom_is_diagonal_in_kappa_mj(pair_bases):
    """One atom, spherical v and u: H+ and S+ couple only spinors with the same
    (kappa, m_j), with values independent of m_j; both Hermitian, S+ positive."""
    wl, ws = pair_bases
    pairs = np.array([[0, 0]])
    bl = oracle.pair_blocks_hs(wl, pairs)
    bs = oracle.pair_blocks_hs(ws, pairs)
    GL, GS = oracle.spinor_G(wl, ws)
    X = oracle.spinor_transform(pairs, bl, bs, GL, GS)[0]
    lab = oracle.spinor_labels(wl)[0]
    for q in range(2):
        M = X[q]
        sc = np.max(np.abs(M))
        assert np.max(np.abs(M - M.conj().T)) < 1e-13 * sc
        for i, (s1, l1, k1, m1) in enumerate(lab):
            for j, (s2, l2, k2, m2) in enumerate(lab):
                if k1 != k2 or m1 != m2:
                    assert abs(M[i, j]) < 5e-9 * sc, (q, lab[i], lab[j], M[i, j])
                else:
                    # same (kappa, m_j): equal to the m_j = first value of that pair of shells
                    i0 = next(t for t, L in enumerate(lab) if L[0] == s1 and L[2] == k1)
                    j0 = next(t for t, L in enumerate(lab) if L[0] == s2 and L[2] == k2)
                    assert abs(M[i, j] - M[i0, j0]) < 5e-9 * sc
    assert np.min(np.linalg.eigvalsh(X[1])) > 0.0
