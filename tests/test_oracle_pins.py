"""Pins for the FP64 oracle: each test fixes part of the oracle's result by
something other than the oracle itself (closed-form Gaussian integrals, a
library routine, invariants, brute force).  No GPU needed.

Coverage map (a plausible mistake and the pin that catches it):
  * real Y_lm sign / normalisation / gradient  -> test_solid_harmonics_*
  * radial spline evaluation / derivative        -> test_radial_table_*
  * V integrand, weights, grid                    -> test_single_centre_overlap, test_two_centre_overlap_sp
  * grad phi (radial-derivative term) and c'      -> test_single_centre_kinetic, test_two_centre_kinetic_ss
  * spin-orbit parts: cross-product sign/index    -> test_so_sign_spherical_potential, test_so_vanishes_constant_v
  * screening                                      -> test_screened_equals_bruteforce
  * density / adjoint and the A <= B doubling     -> test_adjoint_dot_product_*, test_electron_count
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import erf, sph_harm_y

import oracle
import workload as W

C = W.C_LIGHT
CP = 1.0 / (4.0 * C * C)


# ---------------------------------------------------------------------------
# helpers: closed-form Gaussian integrals (written from the mathematics)
# ---------------------------------------------------------------------------

def I_rad(n, p):
    """int_0^inf s^(2n) exp(-p s^2) ds = Gamma(n + 1/2) / (2 p^(n + 1/2))."""
    return math.gamma(n + 0.5) / (2.0 * p ** (n + 0.5))


def overlap_1c(l, a1, c1, a2, c2):
    """<R1 Y_lm | R2 Y_lm> for R = sum_k c_k exp(-a_k s^2) s^l."""
    return sum(x1 * x2 * I_rad(l + 1, b1 + b2) for b1, x1 in zip(a1, c1) for b2, x2 in zip(a2, c2))


def gradgrad_1c(l, a1, c1, a2, c2):
    """int grad phi1 . grad phi2 for phi = g(s) S_lm, g = sum c exp(-a s^2):
    -lap(g S) = -(g'' + (2l+2) g'/s) S, and for g = exp(-b s^2) that is
    (2b(2l+3) - 4b^2 s^2) exp(-b s^2) S."""
    tot = 0.0
    for b1, x1 in zip(a1, c1):
        for b2, x2 in zip(a2, c2):
            p = b1 + b2
            tot += x1 * x2 * (2.0 * b2 * (2 * l + 3) * I_rad(l + 1, p) - 4.0 * b2 * b2 * I_rad(l + 2, p))
    return tot


def _fn_index(wl, atom, shell_local, m):
    """Global function index (atom-major, shell order, m = -l..l)."""
    f = 0
    for a in range(atom):
        f += int(np.sum(2 * wl.shell_l[wl.atom_shell_off[a]:wl.atom_shell_off[a + 1]] + 1))
    s0 = wl.atom_shell_off[atom]
    for s in range(s0, s0 + shell_local):
        f += 2 * int(wl.shell_l[s]) + 1
    return f + m + int(wl.shell_l[s0 + shell_local])


# ---------------------------------------------------------------------------
# Y_lm (App. B) and radial tables
# ---------------------------------------------------------------------------

def test_solid_harmonics_match_scipy_app_b_convention():
    """Real Y_lm of App. B equal sqrt2 Re / Im of the complex (Condon-Shortley)
    harmonics of scipy: Y_l^m = sqrt2 Re Y_l^|m| (m>0), Y_l^0, sqrt2 Im Y_l^|m| (m<0)."""
    rng = np.random.default_rng(11)
    for l in range(5):
        for m in range(-l, l + 1):
            for _ in range(6):
                p = rng.standard_normal(3)
                r = np.linalg.norm(p)
                th, ph = math.acos(p[2] / r), math.atan2(p[1], p[0])
                S, _ = oracle.solid_harmonic(l, m, *p)
                Yc = sph_harm_y(l, abs(m), th, ph)
                ref = math.sqrt(2) * Yc.real if m > 0 else (Yc.real if m == 0 else math.sqrt(2) * Yc.imag)
                assert abs(S / r ** l - ref) < 1e-13


def test_solid_harmonics_explicit_low_order():
    """App. B read literally gives negative p_x and p_y: Y_11 = -sqrt(3/4pi) x/r,
    Y_1-1 = -sqrt(3/4pi) y/r, Y_10 = +sqrt(3/4pi) z/r; Y_00 = 1/sqrt(4 pi)."""
    k = math.sqrt(3.0 / (4.0 * math.pi))
    x, y, z = 0.3, -1.1, 0.7
    assert abs(oracle.solid_harmonic(1, 1, x, y, z)[0] + k * x) < 1e-15
    assert abs(oracle.solid_harmonic(1, -1, x, y, z)[0] + k * y) < 1e-15
    assert abs(oracle.solid_harmonic(1, 0, x, y, z)[0] - k * z) < 1e-15
    assert abs(oracle.solid_harmonic(0, 0, x, y, z)[0] - 1.0 / math.sqrt(4 * math.pi)) < 1e-15
    # d_xy: m=-2 -> (-1)^2 sqrt2 K sin(2 phi) P_2^2, P_2^2 = 3 sin^2 -> sqrt(15/4pi) x y
    assert abs(oracle.solid_harmonic(2, -2, x, y, z)[0] - math.sqrt(15 / (4 * math.pi)) * x * y) < 1e-14


def test_solid_harmonics_gradient_finite_difference():
    rng = np.random.default_rng(12)
    h = 1e-5
    for l in range(5):
        for m in range(-l, l + 1):
            p = rng.standard_normal(3)
            _, g = oracle.solid_harmonic(l, m, *p)
            fd = np.array([(oracle.solid_harmonic(l, m, *(p + h * e))[0] -
                            oracle.solid_harmonic(l, m, *(p - h * e))[0]) / (2 * h) for e in np.eye(3)])
            assert np.max(np.abs(fd - g)) < 1e-8


def test_solid_harmonics_orthonormal_on_product_grid():
    u, wu = W.product_sphere(10, 20)
    Y = np.array([[oracle.solid_harmonic(l, m, *p)[0] for p in u] for l in range(5) for m in range(-l, l + 1)])
    G = (Y * wu[None, :]) @ Y.T
    assert np.max(np.abs(G - np.eye(25))) < 1e-13


def test_radial_table_reproduces_analytic_function():
    alpha, c = np.array([0.3, 2.0, 15.0]), np.array([0.5, 0.8, 0.3])
    rcut = 6.0 * W.ANGSTROM
    tab = W.spline_table(alpha, c, rcut, 2048)
    rng = np.random.default_rng(3)
    for s in np.concatenate([rng.uniform(0, rcut, 200), [0.0, 1e-9, rcut - 1e-9, rcut, rcut + 1.0]]):
        val, der = oracle.radial(tab, rcut, s)
        ref, dref = W.radial_values(np.array([s]), alpha, c, rcut)
        assert abs(val - ref[0]) < 2e-9
        assert abs(der - dref[0]) < 2e-6
    assert oracle.radial(tab, rcut, rcut) == (0.0, 0.0)


def test_radial_table_exact_on_cubic_intervals():
    """Hermite coefficients reproduce knot values/derivatives exactly."""
    rcut = 10.0
    alpha, c = np.array([0.7, 1.5, 3.0]), np.array([1.0, -0.4, 0.2])
    tab = W.spline_table(alpha, c, rcut, 64)
    knots = rcut * (np.arange(64) / 64.0) ** 2
    f, d = W.radial_values(knots, alpha, c, rcut)
    for k, s in enumerate(knots):
        val, der = oracle.radial(tab, rcut, s)
        assert abs(val - f[k]) <= 1e-15 * max(1.0, abs(f[k]))
        assert abs(der - d[k]) <= 1e-12 * max(1.0, abs(d[k]))


# ---------------------------------------------------------------------------
# Closed-form integrals
# ---------------------------------------------------------------------------

SHELLS_1C = [(0, [0.6, 2.5, 9.0], [0.4, 0.9, 0.3]), (0, [0.8, 3.0, 12.0], [1.0, 0.2, 0.5]),
             (1, [0.5, 1.7, 6.0], [0.7, 0.6, 0.4]), (1, [0.9, 4.0, 15.0], [0.3, 1.0, 0.2]),
             (2, [0.55, 2.0, 8.0], [0.5, 0.5, 0.5]), (3, [0.7, 3.0, 10.0], [0.6, 0.4, 0.9])]


@pytest.fixture(scope="module")
def one_centre():
    wl = W.pin_workload([82], [[0.0, 0.0, 0.0]], [SHELLS_1C], nrad=300, ntheta=12, nphi=24)
    blk = oracle.pair_blocks(wl, np.array([[0, 0]]))[0]
    return wl, blk


def _shell_norm_coefs(wl, s):
    return wl.shell_alpha[s], wl.shell_gcoef[s]


def test_single_centre_overlap(one_centre):
    """v = 1: V = S with S_ij = delta_ll' delta_mm' int R_i R_j r^2 dr (Gamma closed form)."""
    wl, blk = one_centre
    V = blk[0]
    n = V.shape[0]
    S = np.zeros((n, n))
    for s1 in range(wl.n_shells):
        for s2 in range(wl.n_shells):
            l1, l2 = wl.shell_l[s1], wl.shell_l[s2]
            if l1 != l2:
                continue
            a1, c1 = _shell_norm_coefs(wl, s1)
            a2, c2 = _shell_norm_coefs(wl, s2)
            val = overlap_1c(int(l1), a1, c1, a2, c2)
            for m in range(-l1, l1 + 1):
                S[_fn_index(wl, 0, s1, m), _fn_index(wl, 0, s2, m)] = val
    assert np.max(np.abs(np.diag(S) - 1.0)) < 1e-12  # normalised radials
    assert np.max(np.abs(V - S)) < 2e-9


def test_single_centre_kinetic(one_centre):
    """v = 1: 4c^2 Ws = int grad phi_i . grad phi_j = 2T (closed form)."""
    wl, blk = one_centre
    G = blk[1] / CP
    n = G.shape[0]
    T2 = np.zeros((n, n))
    for s1 in range(wl.n_shells):
        for s2 in range(wl.n_shells):
            l1, l2 = wl.shell_l[s1], wl.shell_l[s2]
            if l1 != l2:
                continue
            val = gradgrad_1c(int(l1), *_shell_norm_coefs(wl, s1), *_shell_norm_coefs(wl, s2))
            for m in range(-l1, l1 + 1):
                T2[_fn_index(wl, 0, s1, m), _fn_index(wl, 0, s2, m)] = val
    assert np.max(np.abs(G - T2)) < 5e-7 * np.max(np.abs(T2))


def test_so_vanishes_constant_v(one_centre):
    """int grad phi_i x grad phi_j = int curl(phi_i grad phi_j) = 0."""
    wl, blk = one_centre
    for q in (2, 3, 4):
        assert np.max(np.abs(blk[q])) < 1e-12


def test_symmetries(one_centre):
    wl, blk = one_centre
    assert np.max(np.abs(blk[0] - blk[0].T)) < 1e-14
    assert np.max(np.abs(blk[1] - blk[1].T)) < 1e-14 * np.max(np.abs(blk[1])) * 10
    # SO antisymmetric (nonzero v needed to make it nonzero)
    wl2 = wl.with_v(-82.0 * erf(np.sqrt(wl.x ** 2 + wl.y ** 2 + wl.z ** 2) / 0.5) /
                    np.maximum(np.sqrt(wl.x ** 2 + wl.y ** 2 + wl.z ** 2), 1e-300))
    b2 = oracle.pair_blocks(wl2, np.array([[0, 0]]))[0]
    for q in (2, 3, 4):
        A = b2[q]
        assert np.max(np.abs(A + A.T)) < 1e-15 * max(1.0, np.max(np.abs(A))) * 10


def test_so_sign_spherical_potential():
    """One atom, spherical v, phi_x ~ -sqrt(3/4pi) Rt x, phi_y ~ -sqrt(3/4pi) Rt y:
    4c^2 Wso_z[x, y] = int v (grad phi_x x grad phi_y)_z = -int v'(r) Rt^2 r^3 dr."""
    Z = 82.0
    a = 0.5
    sh = [(1, [0.6, 2.0, 9.0], [0.5, 0.7, 0.4])]
    wl = W.pin_workload([82], [[0.0, 0.0, 0.0]], [sh], nrad=400, ntheta=12, nphi=24,
                        v=lambda x, y, z: -Z * erf(np.sqrt(x * x + y * y + z * z) / a) /
                        np.sqrt(x * x + y * y + z * z))
    blk = oracle.pair_blocks(wl, np.array([[0, 0]]))[0]
    alpha, c = wl.shell_alpha[0], wl.shell_gcoef[0]

    def vprime(r):
        return Z * erf(r / a) / r ** 2 - Z * 2.0 / (a * math.sqrt(math.pi)) * math.exp(-(r / a) ** 2) / r

    def integrand(r):
        g = sum(ck * math.exp(-ak * r * r) for ak, ck in zip(alpha, c))
        return vprime(r) * g * g * r ** 3

    ref = -integrate.quad(integrand, 1e-12, 40.0, limit=400, epsabs=1e-14, epsrel=1e-13)[0]
    # function order m = -1 (y), 0 (z), 1 (x): element [x, y] = [2, 0]
    got = blk[4][2, 0] / CP
    assert abs(got - ref) < 1e-8 * abs(ref)
    assert abs(blk[4][0, 2] / CP + ref) < 1e-8 * abs(ref)
    # x and y components vanish for this pair by symmetry
    assert abs(blk[2][2, 0]) < 1e-10 * abs(got * CP) and abs(blk[3][2, 0]) < 1e-10 * abs(got * CP)


def _s_p_two_centre(RA, RB, la, aa, ca, lb, ab, cb, comp_a=None, comp_b=None):
    """int phi_a phi_b for s or p primitives sums via the Gaussian product
    theorem.  comp = None for s, or 0/1/2 for the x/y/z factor."""
    tot = 0.0
    RA, RB = np.asarray(RA), np.asarray(RB)
    for a1, x1 in zip(aa, ca):
        for b1, x2 in zip(ab, cb):
            p = a1 + b1
            mu = a1 * b1 / p
            P = (a1 * RA + b1 * RB) / p
            K = math.exp(-mu * np.sum((RA - RB) ** 2)) * (math.pi / p) ** 1.5
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


@pytest.fixture(scope="module")
def two_centre():
    sa = [(0, [0.7, 2.0, 6.0], [0.6, 0.5, 0.4]), (1, [0.6, 1.5, 5.0], [0.5, 0.7, 0.3])]
    sb = [(0, [0.9, 3.0, 8.0], [0.3, 0.9, 0.5]), (1, [0.5, 2.5, 7.0], [0.8, 0.4, 0.6])]
    RA, RB = [0.0, 0.0, 0.0], [1.3, -0.8, 1.9]
    wl = W.pin_workload([53, 6], [RA, RB], [sa, sb], nrad=200, ntheta=40, nphi=80)
    blocks = oracle.pair_blocks(wl, np.array([[0, 1]]))
    return wl, blocks[0], np.array(RA), np.array(RB)


def test_two_centre_overlap_sp(two_centre):
    """Becke-partitioned two-centre overlap of s and p functions against the
    Gaussian product theorem (p factor -sqrt(3/4pi){y, z, x} for m = -1, 0, 1)."""
    wl, blk, RA, RB = two_centre
    V = blk[0]
    kp = -math.sqrt(3 / (4 * math.pi))
    ks = 1.0 / math.sqrt(4 * math.pi)
    comp_of_m = {-1: (1, kp), 0: (2, -kp), 1: (0, kp)}

    def fn_desc(atom):
        out = []
        s0 = wl.atom_shell_off[atom]
        for s in range(s0, wl.atom_shell_off[atom + 1]):
            l = int(wl.shell_l[s])
            if l == 0:
                out.append((s, None, ks))
            else:
                for m in (-1, 0, 1):
                    cmp_, k = comp_of_m[m]
                    out.append((s, cmp_, k))
        return out

    da, db = fn_desc(0), fn_desc(1)
    ref = np.zeros_like(V)
    for i, (sa, ca_, ka) in enumerate(da):
        for j, (sb, cb_, kb) in enumerate(db):
            ref[i, j] = ka * kb * _s_p_two_centre(RA, RB, 0, wl.shell_alpha[sa], wl.shell_gcoef[sa], 0,
                                                  wl.shell_alpha[sb], wl.shell_gcoef[sb], ca_, cb_)
    assert np.max(np.abs(V - ref)) < 2e-7


def test_two_centre_kinetic_ss(two_centre):
    """s-s: int grad phi_a . grad phi_b = 2 mu (3 - 2 mu R^2) S_ab per primitive pair."""
    wl, blk, RA, RB = two_centre
    G = blk[1] / CP
    sa, sb = wl.atom_shell_off[0], wl.atom_shell_off[1]
    R2 = float(np.sum((RA - RB) ** 2))
    tot = 0.0
    for a1, x1 in zip(wl.shell_alpha[sa], wl.shell_gcoef[sa]):
        for b1, x2 in zip(wl.shell_alpha[sb], wl.shell_gcoef[sb]):
            p = a1 + b1
            mu = a1 * b1 / p
            S = math.exp(-mu * R2) * (math.pi / p) ** 1.5
            tot += x1 * x2 * 2.0 * mu * (3.0 - 2.0 * mu * R2) * S
    tot /= 4.0 * math.pi
    assert abs(G[0, 0] - tot) < 2e-6 * max(1.0, abs(tot))


def test_two_centre_so_vanishes_constant_v(two_centre):
    wl, blk, _, _ = two_centre
    for q in (2, 3, 4):
        assert np.max(np.abs(blk[q] / CP)) < 5e-6


# ---------------------------------------------------------------------------
# Invariants and brute force
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small_sub():
    wl = W.config_small(nint=512, nrad=16, nang=50)
    return wl


def test_linearity_in_v(small_sub):
    wl = small_sub
    pairs = W.atom_pairs(wl)
    b1 = oracle.pair_blocks(wl.with_v(np.ones(wl.n_points)), pairs)
    b3 = oracle.pair_blocks(wl.with_v(np.full(wl.n_points, 3.0)), pairs)
    for x, y in zip(b1, b3):
        assert np.max(np.abs(3.0 * x - y)) <= 1e-14 * max(1.0, np.max(np.abs(y)))


def test_screened_equals_bruteforce(small_sub):
    wl = small_sub
    pairs = np.array([[a, b] for a in range(wl.n_atoms) for b in range(a, wl.n_atoms)], dtype=np.int32)
    s = oracle.pair_blocks(wl, pairs, screened=True)
    b = oracle.pair_blocks(wl, pairs, screened=False)
    for x, y in zip(s, b):
        assert np.array_equal(x, y)


def test_pair_blocks_equal_dense_tabulation(small_sub):
    """The pair-block sums equal Phi^T diag(w v) Phi built from the dense
    tabulation (a different route to the same definition)."""
    wl = small_sub
    phi, grad = oracle.tabulate(wl, wl.x, wl.y, wl.z)
    om = wl.w * wl.v
    V = phi.T @ (om[:, None] * phi)
    Gs = sum(grad[:, :, a].T @ (om[:, None] * grad[:, :, a]) for a in range(3))
    Mx = grad[:, :, 1].T @ (om[:, None] * grad[:, :, 2])
    pairs = W.atom_pairs(wl)
    nfn = wl.atom_nfn()
    off = np.concatenate([[0], np.cumsum(nfn)])
    blocks = oracle.pair_blocks(wl, pairs)
    for (a, b), blk in zip(pairs, blocks):
        sa, sb = slice(off[a], off[a + 1]), slice(off[b], off[b + 1])
        sc = np.max(np.abs(V)) + 1.0
        assert np.max(np.abs(blk[0] - V[sa, sb])) < 1e-11 * sc
        assert np.max(np.abs(blk[1] - CP * Gs[sa, sb])) < 1e-11 * CP * (np.max(np.abs(Gs)) + 1)
        assert np.max(np.abs(blk[2] - CP * (Mx - Mx.T)[sa, sb])) < 1e-11 * CP * (np.max(np.abs(Mx)) + 1)


def test_translation_invariance(small_sub):
    wl = small_sub
    pairs = W.atom_pairs(wl)
    b0 = oracle.pair_blocks(wl, pairs)
    b1 = oracle.pair_blocks(wl.translated([3.7, -1.2, 0.4]), pairs)
    for x, y in zip(b0, b1):
        for q in range(5):
            assert np.max(np.abs(x[q] - y[q])) < 1e-10 * (np.max(np.abs(x[q])) + 1e-30)


# ---------------------------------------------------------------------------
# Density and adjoint
# ---------------------------------------------------------------------------

def test_adjoint_dot_product_real_parts(small_sub):
    """sum_g dL/dv_g dv_g = sum_p <C_p, H_p(dv)>: the density in weight mode 1
    is the transpose of the integration on the stored elements."""
    wl = small_sub
    pairs = W.atom_pairs(wl)
    rng = np.random.default_rng(5)
    nfn = wl.atom_nfn()
    coef = [rng.standard_normal((5, nfn[a], nfn[b])) for a, b in pairs]
    grad = oracle.density(wl, pairs, coef, weight_mode=1)
    dv = rng.standard_normal(wl.n_points)
    H = oracle.pair_blocks(wl, pairs, v=dv)
    rhs = sum(float(np.sum(c * h)) for c, h in zip(coef, H))
    lhs = float(np.dot(grad, dv))
    scale = sum(float(np.sum(np.abs(c * h))) for c, h in zip(coef, H))
    assert abs(lhs - rhs) < 1e-12 * scale


def test_adjoint_dot_product_spinor_density(small_sub):
    """L(v) = Re Tr(D H(v)) with the full Hermitian spinor matrices rebuilt
    from the A <= B blocks; dL/dv from the stored-element coefficients
    (doubling of off-diagonal pair blocks) satisfies <dL/dv, dv> = L(dv)."""
    wl = small_sub
    pairs = W.atom_pairs(wl)
    D = W.spinor_density(wl, pairs, 5001)
    coef = oracle.coef_from_spinor_density(pairs, D)
    grad = oracle.density(wl, pairs, coef, weight_mode=1)
    rng = np.random.default_rng(9)
    dv = rng.standard_normal(wl.n_points)
    L = oracle.loss_re_tr(pairs, D, oracle.pair_blocks(wl, pairs, v=dv))
    assert abs(float(np.dot(grad, dv)) - L) < 1e-11 * (abs(L) + np.sum(np.abs(grad * dv)))


def test_spinor_blocks_hermitian(small_sub):
    wl = small_sub
    pairs = W.atom_pairs(wl)
    blocks = oracle.pair_blocks(wl, pairs)
    for (a, b), blk in zip(pairs, blocks):
        Wsp = oracle.spinor_W(blk)
        n = blk.shape[1]
        # spin sub-blocks: uu = Ws + i Wz, ud = Wy + i Wx, du = -Wy + i Wx, dd = Ws - i Wz
        assert np.allclose(Wsp[:n, :blk.shape[2]], blk[1] + 1j * blk[4], rtol=0, atol=0)
        assert np.allclose(Wsp[:n, blk.shape[2]:], blk[3] + 1j * blk[2], rtol=0, atol=0)
        assert np.allclose(Wsp[n:, :blk.shape[2]], -blk[3] + 1j * blk[2], rtol=0, atol=0)
        assert np.allclose(Wsp[n:, blk.shape[2]:], blk[1] - 1j * blk[4], rtol=0, atol=0)
        if a == b:
            assert np.max(np.abs(Wsp - Wsp.conj().T)) < 1e-12 * (np.max(np.abs(Wsp)) + 1e-30)


def test_electron_count(small_sub):
    """sum_g w_g nL_g = sum_ij d_ij S_grid,ij with S_grid the v = 1 integrals."""
    wl = small_sub
    pairs = W.atom_pairs(wl)
    rng = np.random.default_rng(6)
    nfn = wl.atom_nfn()
    coef = []
    for a, b in pairs:
        c = np.zeros((5, nfn[a], nfn[b]))
        c[0] = rng.standard_normal((nfn[a], nfn[b]))
        coef.append(c)
    n, parts = oracle.density(wl, pairs, coef, weight_mode=0, with_parts=True)
    S = oracle.pair_blocks(wl.with_v(np.ones(wl.n_points)), pairs)
    lhs = float(np.sum(wl.w * parts[:, 0]))
    rhs = sum(float(np.sum(c[0] * s[0])) for c, s in zip(coef, S))
    assert abs(lhs - rhs) < 1e-12 * sum(float(np.sum(np.abs(c[0] * s[0]))) for c, s in zip(coef, S))
