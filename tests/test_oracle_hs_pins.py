"""Pins for the oracle's H and S of one component (the paper's Q4C integrand,
Sec. II Eq. 19 in the scalar form of Eq. 29, symmetrised):

    H_ij = sum_g w phi_i phi_j (v + (u_i + u_j) / 2),   S_ij = sum_g w phi_i phi_j

Each test fixes part of the result by something other than the oracle itself.
Coverage map (a plausible mistake and the pin that catches it):
  * ket-potential table evaluation, the (u_i + u_j)/2 average, l = 4 (g)
    functions of the small component                    -> test_single_centre_closed_form
  * u taken from the wrong centre / not symmetrised      -> test_two_centre_constant_ket
  * v term, weights, S part                              -> test_ket_zero_reduces_to_v_integral,
                                                             test_two_centre_overlap_s_part
  * ket table of the smeared-nucleus potential           -> test_smeared_nucleus_ket_table
  * screening                                             -> test_screened_equals_bruteforce_hs
  * l~ = l +- 1 small-component shells and eps per parent -> test_small_component_recipe
"""
import math

import numpy as np
import pytest
from scipy.special import erf

import oracle
import workload as W


def I_rad(n, p):
    """int_0^inf s^(2n) exp(-p s^2) ds = Gamma(n + 1/2) / (2 p^(n + 1/2))."""
    return math.gamma(n + 0.5) / (2.0 * p ** (n + 0.5))


def _moment_1c(l, a1, c1, a2, c2, extra):
    """int R1 R2 s^(2l+2+2 extra) ds for R = sum_k c_k exp(-a_k s^2) (times s^l each)."""
    return sum(x1 * x2 * I_rad(l + 1 + extra, b1 + b2) for b1, x1 in zip(a1, c1) for b2, x2 in zip(a2, c2))


def _fn_index(wl, atom, shell_local, m):
    f = 0
    for a in range(atom):
        f += int(np.sum(2 * wl.shell_l[wl.atom_shell_off[a]:wl.atom_shell_off[a + 1]] + 1))
    s0 = wl.atom_shell_off[atom]
    for s in range(s0, s0 + shell_local):
        f += 2 * int(wl.shell_l[s]) + 1
    return f + m + int(wl.shell_l[s0 + shell_local])


# shells up to l = 4 (a g shell as in the small component of an f shell); alpha >= 0.5,
# where the cutoff taper is below 1e-16
SHELLS_1C = [(0, [0.6, 2.5, 9.0], [0.4, 0.9, 0.3]), (1, [0.5, 1.7, 6.0], [0.7, 0.6, 0.4]),
             (2, [0.55, 2.0, 8.0], [0.5, 0.5, 0.5]), (3, [0.7, 3.0, 10.0], [0.6, 0.4, 0.9]),
             (4, [0.6, 2.2, 7.0], [0.5, 0.8, 0.3]), (4, [0.9, 3.5, 12.0], [0.3, 0.6, 0.7]),
             (2, [0.8, 2.6, 11.0], [0.4, 0.7, 0.2])]
EPS_1C = [-1.3, -0.4, -0.75, -0.2, -0.05, -0.9, -0.6]
KQ_1C = [0.3, 0.05, 0.12, 0.0, 0.2, 0.07, 0.4]
V0 = 0.7


@pytest.fixture(scope="module")
def one_centre():
    wl = W.pin_workload([82], [[0.0, 0.0, 0.0]], [SHELLS_1C], nrad=300, ntheta=14, nphi=28,
                        v=lambda x, y, z: np.full_like(x, V0))
    wl = W.poly_ket_tables(wl, EPS_1C, KQ_1C)
    return wl, oracle.pair_blocks_hs(wl, np.array([[0, 0]]))[0]


def test_single_centre_closed_form(one_centre):
    """One centre, v = V0, u_s = eps_s + k_s r^2:
    H_ij = delta_ll' delta_mm' [(V0 + (eps_i + eps_j)/2) I0 + (k_i + k_j)/2 I2],
    S_ij = delta_ll' delta_mm' I0, I_n = int R_i R_j r^(2l+2+n) dr (Gamma closed form)."""
    wl, blk = one_centre
    H, S = blk
    n = H.shape[0]
    Hr, Sr = np.zeros((n, n)), np.zeros((n, n))
    for s1 in range(wl.n_shells):
        for s2 in range(wl.n_shells):
            l1, l2 = int(wl.shell_l[s1]), int(wl.shell_l[s2])
            if l1 != l2:
                continue
            args = (wl.shell_alpha[s1], wl.shell_gcoef[s1], wl.shell_alpha[s2], wl.shell_gcoef[s2])
            i0 = _moment_1c(l1, *args, 0)
            i2 = _moment_1c(l1, *args, 1)
            h = (V0 + 0.5 * (EPS_1C[s1] + EPS_1C[s2])) * i0 + 0.5 * (KQ_1C[s1] + KQ_1C[s2]) * i2
            for m in range(-l1, l1 + 1):
                Hr[_fn_index(wl, 0, s1, m), _fn_index(wl, 0, s2, m)] = h
                Sr[_fn_index(wl, 0, s1, m), _fn_index(wl, 0, s2, m)] = i0
    assert np.max(np.abs(np.diag(Sr) - 1.0)) < 1e-12
    assert np.max(np.abs(S - Sr)) < 2e-9
    assert np.max(np.abs(H - Hr)) < 2e-9 * np.max(np.abs(Hr))


def test_hs_symmetric(one_centre):
    _, (H, S) = one_centre
    assert np.max(np.abs(H - H.T)) <= 1e-15 * np.max(np.abs(H)) * 10
    assert np.max(np.abs(S - S.T)) <= 1e-15 * np.max(np.abs(S)) * 10


@pytest.fixture(scope="module")
def two_centre():
    sa = [(0, [0.7, 2.0, 6.0], [0.6, 0.5, 0.4]), (1, [0.6, 1.5, 5.0], [0.5, 0.7, 0.3])]
    sb = [(0, [0.9, 3.0, 8.0], [0.3, 0.9, 0.5]), (1, [0.5, 2.5, 7.0], [0.8, 0.4, 0.6])]
    RA, RB = [0.0, 0.0, 0.0], [1.3, -0.8, 1.9]
    wl = W.pin_workload([53, 6], [RA, RB], [sa, sb], nrad=200, ntheta=40, nphi=80,
                        v=lambda x, y, z: np.zeros_like(x))
    return wl, np.array(RA), np.array(RB)


def _gpt(RA, RB, aa, ca, ab, cb, comp_a, comp_b):
    """int phi_a phi_b of s/p Gaussian sums (Gaussian product theorem); comp =
    None for s, 0/1/2 for the x/y/z factor."""
    tot = 0.0
    for a1, x1 in zip(aa, ca):
        for b1, x2 in zip(ab, cb):
            p = a1 + b1
            P = (a1 * RA + b1 * RB) / p
            K = math.exp(-a1 * b1 / p * np.sum((RA - RB) ** 2)) * (math.pi / p) ** 1.5
            if comp_a is None and comp_b is None:
                f = 1.0
            elif comp_b is None:
                f = P[comp_a] - RA[comp_a]
            elif comp_a is None:
                f = P[comp_b] - RB[comp_b]
            else:
                f = (P[comp_a] - RA[comp_a]) * (P[comp_b] - RB[comp_b]) + (0.5 / p if comp_a == comp_b else 0.0)
            tot += x1 * x2 * K * f
    return tot


def _two_centre_overlap(wl, RA, RB):
    kp = -math.sqrt(3 / (4 * math.pi))
    ks = 1.0 / math.sqrt(4 * math.pi)
    comp_of_m = {-1: (1, kp), 0: (2, -kp), 1: (0, kp)}

    def desc(atom):
        out = []
        for s in range(wl.atom_shell_off[atom], wl.atom_shell_off[atom + 1]):
            if int(wl.shell_l[s]) == 0:
                out.append((s, None, ks))
            else:
                for m in (-1, 0, 1):
                    out.append((s,) + comp_of_m[m])
        return out

    da, db = desc(0), desc(1)
    ref = np.zeros((len(da), len(db)))
    for i, (sa, ca_, ka) in enumerate(da):
        for j, (sb, cb_, kb) in enumerate(db):
            ref[i, j] = ka * kb * _gpt(RA, RB, wl.shell_alpha[sa], wl.shell_gcoef[sa], wl.shell_alpha[sb],
                                       wl.shell_gcoef[sb], ca_, cb_)
    return ref, [d[0] for d in da], [d[0] for d in db]


def test_two_centre_overlap_s_part(two_centre):
    wl, RA, RB = two_centre
    wl = W.poly_ket_tables(wl, [0.0] * wl.n_shells, [0.0] * wl.n_shells)
    H, S = oracle.pair_blocks_hs(wl, np.array([[0, 1]]))[0]
    ref, _, _ = _two_centre_overlap(wl, RA, RB)
    assert np.max(np.abs(S - ref)) < 2e-7
    assert np.max(np.abs(H)) == 0.0  # v = 0, u = 0


def test_two_centre_constant_ket(two_centre):
    """v = 0, u_s = eps_s constant per shell, different on every shell of both
    centres: H_ij = (eps_i + eps_j)/2 S_ij with S from the Gaussian product theorem."""
    wl, RA, RB = two_centre
    eps = [-1.7, -0.3, 0.45, -0.9]
    wl = W.poly_ket_tables(wl, eps, [0.0] * wl.n_shells)
    H, S = oracle.pair_blocks_hs(wl, np.array([[0, 1]]))[0]
    ref, sha, shb = _two_centre_overlap(wl, RA, RB)
    href = np.array([[0.5 * (eps[a] + eps[b]) * ref[i, j] for j, b in enumerate(shb)] for i, a in enumerate(sha)])
    assert np.max(np.abs(H - href)) < 2e-7


@pytest.fixture(scope="module")
def small_sub():
    wl = W.with_ket(W.config_small(nint=512, nrad=16, nang=50), 7001)
    return wl, W.atom_pairs(wl)


def test_ket_zero_reduces_to_v_integral(small_sub):
    """u = 0: H = V of the W-path oracle (the v integral, pinned by its own closed
    forms) term by term, and S = V at v = 1."""
    wl, pairs = small_sub
    w0 = W.poly_ket_tables(wl, [0.0] * wl.n_shells, [0.0] * wl.n_shells)
    hs = oracle.pair_blocks_hs(w0, pairs)
    ref = oracle.pair_blocks(wl, pairs)
    ref1 = oracle.pair_blocks(wl, pairs, v=np.ones_like(wl.v))
    for k in range(len(pairs)):
        sc = np.max(np.abs(ref[k][0])) + 1e-300
        assert np.max(np.abs(hs[k][0] - ref[k][0])) <= 1e-13 * sc
        assert np.max(np.abs(hs[k][1] - ref1[k][0])) <= 1e-13 * np.max(np.abs(ref1[k][0]))


def test_smeared_nucleus_ket_table(small_sub):
    """The tabulated u = eps + Z erf(r/0.5)/r against scipy's erf, including the
    finite limit 2Z/(0.5 sqrt(pi)) + eps at the nucleus."""
    wl, _ = small_sub
    rng = np.random.default_rng(7003)
    for a in range(wl.n_atoms):
        s = wl.atom_shell_off[a]
        Z, eps, rc, ni = float(wl.Z[a]), float(wl.shell_eps[s]), float(wl.shell_rcut[s]), int(wl.shell_nint[s])
        tab = wl.u_coef[wl.shell_u_off[s]:wl.shell_u_off[s] + 4 * ni].reshape(ni, 4)
        val0, _ = oracle.radial(tab, rc, 0.0)
        assert abs(val0 - (eps + 2.0 * Z / (0.5 * math.sqrt(math.pi)))) < 1e-12 * Z
        for r in rng.uniform(1e-3, rc, 50):
            val, _ = oracle.radial(tab, rc, r)
            assert abs(val - (eps + Z * erf(r / 0.5) / r)) < 1e-6


def test_screened_equals_bruteforce_hs(small_sub):
    wl, pairs = small_sub
    sub = wl.subset_points(np.arange(0, wl.n_points, 7))
    a = oracle.pair_blocks_hs(sub, pairs, screened=True)
    b = oracle.pair_blocks_hs(sub, pairs, screened=False)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_small_component_recipe(small_sub):
    """l~ = l + 1 for every large shell and l - 1 for l >= 1, with the parent's eps."""
    wl, _ = small_sub
    ws = W.small_component(wl, 7002)
    for a in range(wl.n_atoms):
        big = [(int(wl.shell_l[s]), float(wl.shell_eps[s])) for s in range(wl.atom_shell_off[a], wl.atom_shell_off[a + 1])]
        want = []
        for l, e in big:
            want.append((l + 1, e))
            if l >= 1:
                want.append((l - 1, e))
        got = [(int(ws.shell_l[s]), float(ws.shell_eps[s])) for s in range(ws.atom_shell_off[a], ws.atom_shell_off[a + 1])]
        assert got == want
    # normalised small-component radials (closed form, untapered)
    for s in range(ws.n_shells):
        l = int(ws.shell_l[s])
        a, c = ws.shell_alpha[s], ws.shell_gcoef[s]
        assert abs(_moment_1c(l, a, c, a, c, 0) - 1.0) < 1e-13
