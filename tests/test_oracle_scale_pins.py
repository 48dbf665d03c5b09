"""Pins for the oracle's per-value error scales: the magnitudes against which
single tabulated values (Eq. 12a, App. B) and the density / adjoint at one
point (Eq. 39) are compared element by element.

A scale is the sum, over the terms a value is summed from, of their
magnitudes; rounding in any summation order stays within a small multiple of
unit roundoff times it.  Pinned here:

  * exactness where nothing cancels: a radial table with only the constant
    coefficient per interval, s and p_0 functions (S_00 = const, S_10 = K z),
    and one nonzero coefficient: every scale equals the magnitude of the value
  * a scale never undercuts its value (random coefficients, l <= 2)
  * |C| enters, not C: sign flips leave the scale unchanged, scaling by k
    scales it by |k|
  * part selection: each part's scale depends only on its own coefficients
  * nodal planes: a d function whose value cancels to ~0 keeps a scale of
    the size of its terms
"""
import dataclasses

import numpy as np
import pytest

import oracle
import workload as W


def _const_table_workload(nint=8, rc=8.0):
    """One atom, an s shell and a p shell, each radial table piecewise
    constant (c1 = c2 = c3 = 0), on a small seeded grid."""
    base = W.config_small(nrad=12, nang=26)
    coef = np.zeros(2 * 4 * nint)
    coef[0:4 * nint:4] = np.linspace(0.9, 0.2, nint)          # s: Rt = c0 per interval
    coef[4 * nint::4] = np.linspace(0.7, 0.1, nint)           # p
    rng = np.random.default_rng(9101)
    n = 40
    r = rng.uniform(0.3, 0.9 * rc, n)
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    pts = r[:, None] * u
    return dataclasses.replace(
        base, Z=np.array([82], np.int32), R=np.zeros((1, 3)), atom_shell_off=np.array([0, 2], np.int32),
        shell_l=np.array([0, 1], np.int32), shell_rcut=np.array([rc, rc]), shell_nint=np.array([nint, nint], np.int32),
        shell_coef_off=np.array([0, 4 * nint], np.int64), coef=coef, shell_alpha=np.ones((2, 3)),
        shell_gcoef=np.ones((2, 3)), x=pts[:, 0].copy(), y=pts[:, 1].copy(), z=pts[:, 2].copy(),
        w=rng.uniform(0.1, 1.0, n), pt_atom=np.zeros(n, np.int32), v=np.ones(n), molecule=None, meta={})


def test_tabulation_scale_exact_without_cancellation():
    wl = _const_table_workload()
    phi, grad, aphi, agrad = oracle.tabulate(wl, wl.x, wl.y, wl.z, with_abs=True)
    # functions: s (0), p_-1 (1), p_0 (2), p_1 (3)
    for f in (0, 2):
        assert np.array_equal(aphi[:, f], np.abs(phi[:, f])), f
    # grad of s is 0 (constant radial, S_00 constant); grad p_0 = Rt (0, 0, K)
    assert np.all(agrad[:, 0, :] == 0.0)
    assert np.allclose(agrad[:, 2, :], np.abs(grad[:, 2, :]), rtol=0, atol=0)


def test_tabulation_scale_bounds_values_and_nodal_planes():
    wl = W.config_small(nrad=12, nang=26)
    phi, grad, aphi, agrad = oracle.tabulate(wl, wl.x, wl.y, wl.z, with_abs=True)
    assert np.all(aphi >= np.abs(phi))
    assert np.all(agrad >= np.abs(grad) * (1 - 1e-15))
    # a d_xy function (l = 2, m = -2: S ~ x y) on the plane y = R_y of its
    # atom: the value is 0 while its terms are not
    nfn = wl.atom_nfn()
    f0 = 0
    a = 0
    sh = [s for s in range(wl.atom_shell_off[a], wl.atom_shell_off[a + 1]) if wl.shell_l[s] == 2][0]
    for s in range(wl.atom_shell_off[a], sh):
        f0 += 2 * int(wl.shell_l[s]) + 1
    x = np.array([wl.R[a, 0] + 0.7]); y = np.array([wl.R[a, 1]]); z = np.array([wl.R[a, 2] + 0.2])
    p1, _, a1, _ = oracle.tabulate(wl, x, y, z, with_abs=True)
    assert p1[0, f0] == 0.0 and a1[0, f0] > 0.0
    assert int(nfn[a]) > f0


def _one_pair_coef(wl, e, q, c):
    """Coefficient blocks for the single pair (0, 0): value c at element e of part q."""
    nf = int(wl.atom_nfn()[0])
    blk = np.zeros((5, nf, nf))
    blk[q][e] = c
    return [blk]


def test_density_scale_exact_without_cancellation():
    wl = _const_table_workload()
    pairs = np.array([[0, 0]])
    cp = 1.0 / (4.0 * wl.c_light ** 2)
    phi, grad = oracle.tabulate(wl, wl.x, wl.y, wl.z)
    # LL term on (s, s): n = C phi_s^2
    out, parts, sc = oracle.density(wl, pairs, _one_pair_coef(wl, (0, 0), 0, -1.7), with_parts=True,
                                    with_scale=True)
    assert np.allclose(sc[:, 0], np.abs(parts[:, 0]), rtol=1e-15, atol=0)
    assert np.allclose(parts[:, 0], -1.7 * phi[:, 0] ** 2, rtol=1e-14, atol=0)
    assert np.all(sc[:, 1:] == 0.0)
    # SS scalar term on (p0, p0): n = c' C |grad p0|^2, all terms of one sign
    out, parts, sc = oracle.density(wl, pairs, _one_pair_coef(wl, (2, 2), 1, 0.6), with_parts=True,
                                    with_scale=True)
    assert np.allclose(sc[:, 1], np.abs(parts[:, 1]), rtol=1e-15, atol=0)
    assert np.allclose(parts[:, 1], cp * 0.6 * np.sum(grad[:, 2, :] ** 2, axis=1), rtol=1e-14, atol=0)
    # gradient of n on (s, p0): dn/dz = C (d_z s p0 + s d_z p0) = C s d_z p0 (d_z s = 0)
    nf = int(wl.atom_nfn()[0])
    c = np.zeros((nf, nf)); c[0, 2] = 2.5
    g, gs = oracle.density_grad(wl, pairs, [c], with_scale=True)
    assert np.allclose(gs, np.abs(g), rtol=1e-15, atol=0)


@pytest.fixture(scope="module")
def small():
    wl = W.config_small(nrad=16, nang=38)
    pairs = W.atom_pairs(wl)
    nfn = wl.atom_nfn()
    rng = np.random.default_rng(9102)
    blocks = [rng.standard_normal((5, nfn[a], nfn[b])) for a, b in pairs]
    idx = np.sort(rng.choice(wl.n_points, size=300, replace=False))
    return wl, pairs, blocks, idx


def test_density_scale_bounds_and_uses_abs_coefficients(small):
    wl, pairs, blocks, idx = small
    out, parts, sc = oracle.density(wl, pairs, blocks, idx=idx, with_parts=True, with_scale=True)
    assert np.all(sc >= np.abs(parts))
    assert np.all(oracle.density_scale(sc) >= np.abs(out))
    flipped = [(-1.0) ** p * b for p, b in enumerate(blocks)]
    _, sc2 = oracle.density(wl, pairs, flipped, idx=idx, with_scale=True)
    assert np.array_equal(sc, sc2)
    _, sc3 = oracle.density(wl, pairs, [-3.0 * b for b in blocks], idx=idx, with_scale=True)
    assert np.allclose(sc3, 3.0 * sc, rtol=1e-13, atol=0)
    # weighted form: |w| times the unweighted scale
    outw = oracle.density(wl, pairs, blocks, idx=idx, weight_mode=1)
    assert np.all(oracle.density_scale(sc, wl.w[idx]) >= np.abs(outw))


def test_density_scale_parts_follow_their_coefficients(small):
    wl, pairs, blocks, idx = small
    _, sc = oracle.density(wl, pairs, blocks, idx=idx, with_scale=True)
    for q, k in ((0, 0), (1, 1), (2, 2), (3, 2), (4, 2)):
        zeroed = [b.copy() for b in blocks]
        for b in zeroed:
            b[q] = 0.0
        _, scz = oracle.density(wl, pairs, zeroed, idx=idx, with_scale=True)
        for kk in range(3):
            if kk != k:
                assert np.array_equal(scz[:, kk], sc[:, kk]), (q, kk)
        assert np.all(scz[:, k] <= sc[:, k]) and np.any(scz[:, k] < sc[:, k]), q


def test_density_grad_scale_bounds(small):
    wl, pairs, blocks, idx = small
    g, gs = oracle.density_grad(wl, pairs, [b[0] for b in blocks], idx=idx, with_scale=True)
    assert np.all(gs >= np.abs(g))
    _, gs2 = oracle.density_grad(wl, pairs, [-b[0] for b in blocks], idx=idx, with_scale=True)
    assert np.array_equal(gs, gs2)
    # n's scale equals the LL scale of the adjoint oracle for the same coefficients
    _, sc = oracle.density(wl, pairs, [np.stack([b[0]] + [0 * b[0]] * 4) for b in blocks], idx=idx,
                           with_scale=True)
    assert np.allclose(gs[:, 0], sc[:, 0], rtol=1e-13, atol=0)


def test_tabulation_scale_covers_distance_rounding():
    """Moving a point away from an atom by a relative eps changes each of that
    atom's values by about eps s |dvalue/ds|; the scale carries this
    sensitivity (needed in the steep tails of tight functions, where a
    one-ulp difference in s moves the value far more than one ulp).  The
    move also scales S_lm ~ s^l (l <= 4 here), hence the factor l + 2.5."""
    wl = W.small_component(W.with_ket(W.config_small(nrad=16, nang=26), 7001), 7002)
    a = 0
    rng = np.random.default_rng(9103)
    n = 400
    r = rng.uniform(0.05, 0.99 * float(wl.shell_rcut.max()), n)
    u = rng.standard_normal((n, 3))
    u /= np.linalg.norm(u, axis=1)[:, None]
    eps = 1e-9
    p0 = wl.R[a] + r[:, None] * u
    p1 = wl.R[a] + (r * (1 + eps))[:, None] * u
    f0 = int(np.sum([2 * int(wl.shell_l[s]) + 1 for s in range(wl.atom_shell_off[a])]))
    f1 = f0 + int(wl.atom_nfn()[a])
    phi0, g0, aphi, agrad = oracle.tabulate(wl, p0[:, 0], p0[:, 1], p0[:, 2], with_abs=True)
    phi1, g1 = oracle.tabulate(wl, p1[:, 0], p1[:, 1], p1[:, 2])
    sl = slice(f0, f1)
    nz = aphi[:, sl] > 1e-250
    assert np.all(np.abs(phi1[:, sl] - phi0[:, sl])[nz] <= 6.5 * eps * aphi[:, sl][nz])
    nzg = agrad[:, sl, :] > 1e-250
    assert np.all(np.abs(g1[:, sl, :] - g0[:, sl, :])[nzg] <= 6.5 * eps * agrad[:, sl, :][nzg])
    # without the sensitivity term the plain term magnitudes would not cover it
    # somewhere in the tails: the largest relative change exceeds eps there
    rel = np.max(np.abs(phi1[:, sl] - phi0[:, sl])[nz] / (np.abs(phi0[:, sl])[nz] + 1e-300))
    assert rel > 10 * eps
