"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (FP64 path): per element |GPU - oracle| <= 1e-12 * A_ij with
A_ij = sum_g |term_g| (the oracle's own scale of the element).  Split-FP32
path: |GPU - oracle| <= 1e-8 Ha per element and part.  Integer work (batches,
pairs) is compared bit for bit."""
import numpy as np
import pytest

import oracle
import workload as W
from helpers import (blocks_to_store, gamma, gpu_available, per_point_worst, spinor_to_blocks, split_bound_worst,
                     store_to_blocks)

pytestmark = pytest.mark.gpu

FP64_REL = 1e-12
SPLIT_ABS = 1e-8


def _torch():
    import torch
    return torch


@pytest.fixture(scope="module")
def q():
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_2608_00773_amd as q4c
    return q4c


def _run(q, wl, precision=0, assemble=True, p_max=None, staging_bytes=0):
    torch = _torch()
    plan = q.Plan(wl, p_max=p_max, staging_bytes=staging_bytes)
    v = torch.from_numpy(wl.v).cuda()
    store = q.new_store(plan)
    spin_w = q.new_spinor(plan)
    spin_v = q.new_spinor(plan)
    flags = (q.ASSEMBLE_W | q.ASSEMBLE_V) if assemble else 0
    q.q4c_integrate_H(plan, v, precision, flags, store, spin_w, spin_v)
    torch.cuda.synchronize()
    return plan, store.cpu().numpy(), spin_w.cpu().numpy(), spin_v.cpu().numpy()


@pytest.fixture(scope="module")
def small(q):
    wl = W.config_small()
    pairs = W.atom_pairs(wl)
    ref, scale = oracle.pair_blocks(wl, pairs, with_abs=True)
    return wl, pairs, ref, scale


def _compare_f64(got_blocks, ref, scale, tol=FP64_REL):
    worst, where = 0.0, None
    for p, (g, r, s) in enumerate(zip(got_blocks, ref, scale)):
        # elements whose terms are all exact zeros must come out exactly zero
        err = np.abs(g - r)
        ok_zero = np.all(err[s == 0] == 0)
        assert ok_zero
        nz = s > 0
        if np.any(nz):
            rel = np.where(nz, err / np.where(nz, s, 1.0), 0.0)
            k = np.unravel_index(np.argmax(rel), rel.shape)
            if rel[k] > worst:
                worst, where = float(rel[k]), (p, k, float(g[k]), float(r[k]), float(s[k]), float(np.max(s[k[0]])))
    assert worst <= tol, (worst, where)
    return worst


def test_plan_pairs_and_batches_bitexact(q, small):
    wl, pairs, _, _ = small
    plan = q.Plan(wl)
    p, _ = plan.pairs()
    assert np.array_equal(p, pairs)
    pt_off, pidx, fn_off, fidx = plan.batches()
    # every active point exactly once; inactive points have no function in range
    assert len(np.unique(pidx)) == len(pidx) == plan.info["n_active"]
    rc = wl.atom_rcut()
    d = np.sqrt((wl.x[:, None] - wl.R[None, :, 0]) ** 2 + (wl.y[:, None] - wl.R[None, :, 1]) ** 2 +
                (wl.z[:, None] - wl.R[None, :, 2]) ** 2)
    active = np.nonzero(np.any(d < rc[None, :], axis=1))[0]
    assert np.array_equal(np.sort(pidx), active)
    # relevant functions of each batch = all functions of atoms with a point of the batch inside the cutoff
    aoff = np.concatenate([[0], np.cumsum(wl.atom_nfn())])
    for b in range(plan.info["n_batches"]):
        pts = pidx[pt_off[b]:pt_off[b + 1]]
        atoms = np.nonzero(np.any(d[pts] < rc[None, :], axis=0))[0]
        want = np.concatenate([np.arange(aoff[a], aoff[a + 1]) for a in atoms])
        assert np.array_equal(fidx[fn_off[b]:fn_off[b + 1]], want)
        assert pt_off[b + 1] - pt_off[b] <= 128


def test_nao_tabulate_matches_oracle(q, small):
    torch = _torch()
    wl = small[0]
    plan = q.Plan(wl)
    nb = plan.info["n_batches"]
    n = plan.tabulate_size(0, nb, 1)
    out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    q.nao_tabulate(plan, 0, nb, 1, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    pt_off, pidx, fn_off, fidx = plan.batches()
    phi, grad, aphi, agrad = oracle.tabulate(wl, wl.x[pidx], wl.y[pidx], wl.z[pidx], with_abs=True)
    o = 0
    worst = 0.0
    for b in range(nb):
        P = pt_off[b + 1] - pt_off[b]
        fns = fidx[fn_off[b]:fn_off[b + 1]]
        nf = len(fns)
        blk = got[o:o + 4 * P * nf].reshape(4, P, nf)
        o += 4 * P * nf
        rows = slice(pt_off[b], pt_off[b + 1])
        ref = np.concatenate([phi[rows][:, fns][None], np.moveaxis(grad[rows][:, fns, :], 2, 0)], axis=0)
        sref = np.concatenate([aphi[rows][:, fns][None], np.moveaxis(agrad[rows][:, fns, :], 2, 0)], axis=0)
        # every value against the magnitude of its own terms
        worst = max(worst, per_point_worst(blk, ref, sref, floor=1e-300))
    assert o == n
    print("nao_tabulate: worst |d| / (own scale + 1e-300) %.3g" % worst)
    assert worst <= 1e-12, worst
    # FP32 hi + lo output: per batch [4][2][P][n] floats, hi = fl32(x) and
    # lo = fl32(x - hi) of the FP64 values, bit for bit
    hl = torch.full((2 * n,), float("nan"), dtype=torch.float32, device="cuda")
    q.nao_tabulate(plan, 0, nb, 1, hl, q.DTYPE_F32_HILO)
    torch.cuda.synchronize()
    hl = hl.cpu().numpy()
    o = 0
    for b in range(nb):
        m = (pt_off[b + 1] - pt_off[b]) * (fn_off[b + 1] - fn_off[b])
        x = got[o:o + 4 * m].reshape(4, m)
        h = hl[2 * o:2 * o + 8 * m].reshape(4, 2, m)
        hi = x.astype(np.float32)
        assert np.array_equal(h[:, 0], hi) and np.array_equal(h[:, 1], (x - hi.astype(np.float64)).astype(np.float32))
        o += 4 * m


def test_tabulate_values_only_and_size_errors(q, small):
    torch = _torch()
    wl = small[0]
    plan = q.Plan(wl)
    n1 = plan.tabulate_size(3, 7, 0)
    n4 = plan.tabulate_size(3, 7, 1)
    assert n4 == 4 * n1
    full = torch.zeros(n4, dtype=torch.float64, device="cuda")
    q.nao_tabulate(plan, 3, 7, 1, full)
    vals = torch.zeros(n1, dtype=torch.float64, device="cuda")
    q.nao_tabulate(plan, 3, 7, 0, vals)
    torch.cuda.synchronize()
    # values-only output equals the phi planes of the full output
    f = full.cpu().numpy()
    pt_off, _, fn_off, _ = plan.batches()
    o4 = o1 = 0
    for b in range(3, 7):
        m = (pt_off[b + 1] - pt_off[b]) * (fn_off[b + 1] - fn_off[b])
        assert np.array_equal(vals.cpu().numpy()[o1:o1 + m], f[o4:o4 + m])
        o1 += m
        o4 += 4 * m
    small_buf = torch.zeros(n1 - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(q.Q4CError) as e:
        q.nao_tabulate(plan, 3, 7, 0, small_buf)
    assert e.value.status == q.Q4C_ESIZE


@pytest.mark.parametrize("prec", [0, 4])
def test_integrate_f64_small(q, small, prec):
    """FP64 on the matrix cores and the plain FP64 baseline on the vector ALU:
    every element within 1e-12 A_ij of the oracle."""
    wl, pairs, ref, scale = small
    plan, store, spin_w, spin_v = _run(q, wl, precision=prec)
    _, po = plan.pairs()
    got = store_to_blocks(store, pairs, po, wl.atom_nfn())
    _compare_f64(got, ref, scale)


def test_integrate_f64_valu_multitile(q, medium):
    """The plain FP64 baseline on the multi-tile case (diagonal, edge and
    ragged tiles, batches of up to 300 points): the FP64 bar on every element."""
    wl, pairs, ref, scale = medium
    plan, store, _, _ = _run(q, wl, precision=4, assemble=False)
    _, po = plan.pairs()
    got = store_to_blocks(store, pairs, po, wl.atom_nfn())
    _compare_f64(got, ref, scale)


def test_spinor_assembly_small(q, small):
    wl, pairs, ref, scale = small
    plan, store, spin_w, spin_v = _run(q, wl)
    _, po = plan.pairs()
    nfn = wl.atom_nfn()
    got_parts = store_to_blocks(store, pairs, po, nfn)
    gw = spinor_to_blocks(spin_w, pairs, po, nfn)
    gv = spinor_to_blocks(spin_v, pairs, po, nfn)
    for p in range(len(pairs)):
        # assembly is exact given the parts
        assert np.array_equal(gw[p], oracle.spinor_W(got_parts[p]))
        assert np.array_equal(gv[p], oracle.spinor_V(got_parts[p]))
        # and matches the oracle's spinor blocks within the parity bar
        wref = oracle.spinor_W(ref[p])
        sc = oracle.spinor_W(scale[p]).real + np.abs(oracle.spinor_W(scale[p]).imag) + 1e-300
        assert np.max(np.abs(gw[p] - wref) / sc) < 1e-11


def test_integrate_repeatable_bitwise(q, small):
    torch = _torch()
    wl = small[0]
    plan = q.Plan(wl)
    v = torch.from_numpy(wl.v).cuda()
    a = q.new_store(plan)
    b = q.new_store(plan)
    q.q4c_integrate_H(plan, v, 0, 0, a)
    q.q4c_integrate_H(plan, v, 0, 0, b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_integrate_accumulate(q, small):
    torch = _torch()
    wl = small[0]
    plan = q.Plan(wl)
    v = torch.from_numpy(wl.v).cuda()
    a = q.new_store(plan)
    q.q4c_integrate_H(plan, v, 0, 0, a)
    b = a.clone()
    q.q4c_integrate_H(plan, v, 0, q.ACCUMULATE, b)
    torch.cuda.synchronize()
    # b adds the same staged blocks onto a one by one: it differs from 2a only
    # by the rounding of that chain (a few ulps of the part's largest element)
    scale = torch.amax(torch.abs(a), dim=1, keepdim=True)
    assert torch.all(torch.abs(b - 2 * a) <= 1e-14 * scale)
    assert not torch.equal(b, a)


@pytest.mark.parametrize("prec", [1, 3])
def test_integrate_split_small(q, small, prec):
    wl, pairs, ref, scale = small
    plan, store, _, _ = _run(q, wl, precision=prec)
    _, po = plan.pairs()
    got = store_to_blocks(store, pairs, po, wl.atom_nfn())
    err = [np.max(np.abs(g[k] - r[k])) for g, r in zip(got, ref) for k in range(5)]
    assert max(err) <= SPLIT_ABS, max(err)
    assert split_bound_worst(got, ref, scale, prec) <= 1.0
    # V stays on FP64 MFMA: FP64 bar
    worst = 0.0
    for g, r, s in zip(got, ref, scale):
        nz = s[0] > 0
        worst = max(worst, float(np.max(np.abs(g[0][nz] - r[0][nz]) / s[0][nz])))
    assert worst <= FP64_REL


def test_density_matches_oracle(q, small):
    torch = _torch()
    wl, pairs, _, _ = small
    plan = q.Plan(wl)
    _, po = plan.pairs()
    nfn = wl.atom_nfn()
    rng = np.random.default_rng(77)
    coef_blocks = [rng.standard_normal((5, nfn[a], nfn[b])) for a, b in pairs]
    from helpers import blocks_to_store
    coef = torch.from_numpy(blocks_to_store(coef_blocks, po)).cuda()
    for mode in (0, 1):
        out = torch.full((wl.n_points,), float("nan"), dtype=torch.float64, device="cuda")
        q.density_on_grid(plan, coef, q.TERM_ALL, mode, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref, sc = oracle.density(wl, pairs, coef_blocks, weight_mode=mode, with_scale=True)
        # every point against its own scale (R15 applied to Eq. 39)
        worst = per_point_worst(got, ref, oracle.density_scale(sc, wl.w if mode else None))
        assert worst <= 1e-12, (mode, worst)


def test_density_f32_stated_bound(q, small):
    """density_on_grid in FP32 (SS and SO terms on FP32 MFMA): every point
    within gamma_98 (u = 2^-24) of the magnitudes of its SS and SO terms plus
    the FP64 bar on all terms; the LL term alone (it stays FP64) within the
    FP64 bar in both precisions."""
    torch = _torch()
    wl, pairs, _, _ = small
    plan = q.Plan(wl)
    _, po = plan.pairs()
    nfn = wl.atom_nfn()
    rng = np.random.default_rng(79)
    coef_blocks = [rng.standard_normal((5, nfn[a], nfn[b])) for a, b in pairs]
    from helpers import blocks_to_store
    coef = torch.from_numpy(blocks_to_store(coef_blocks, po)).cuda()
    for mode in (0, 1):
        out = torch.full((wl.n_points,), float("nan"), dtype=torch.float64, device="cuda")
        q.density_on_grid(plan, coef, q.TERM_ALL, mode, out, precision=q.PREC_F32)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref, sc = oracle.density(wl, pairs, coef_blocks, weight_mode=mode, with_scale=True)
        w = wl.w if mode else None
        bound = gamma(98) * oracle.density_scale(sc, w, terms=6) + 1e-12 * oracle.density_scale(sc, w)
        worst = per_point_worst(got, ref, bound, floor=1e-30)
        print("F32 adjoint, weight mode %d: worst |d| / bound %.3g" % (mode, worst), flush=True)
        assert worst <= 1.0, (mode, worst)
    ll = {}
    for prec in (q.PREC_F64, q.PREC_F32):
        ll[prec] = torch.empty(wl.n_points, dtype=torch.float64, device="cuda")
        q.density_on_grid(plan, coef, q.TERM_LL, 1, ll[prec], precision=prec)
    torch.cuda.synchronize()
    ref, sc = oracle.density(wl, pairs, coef_blocks, weight_mode=1, with_scale=True)
    ref_ll = oracle.density(wl, pairs, [np.concatenate([c[:1], 0 * c[1:]]) for c in coef_blocks], weight_mode=1,
                            with_scale=True)[0]
    sc_ll = oracle.density_scale(sc, wl.w, terms=1)
    for prec in (q.PREC_F64, q.PREC_F32):
        assert per_point_worst(ll[prec].cpu().numpy(), ref_ll, sc_ll) <= 1e-12, prec


def test_density_terms_and_dot_product(q, small):
    """Adjoint identity through the library alone: <density(C, weighted), dv> = <C, H(dv)>."""
    torch = _torch()
    wl, pairs, _, _ = small
    plan = q.Plan(wl)
    L = plan.info["store_len"]
    rng = np.random.default_rng(78)
    coef = torch.from_numpy(rng.standard_normal((5, L))).cuda()
    dv = torch.from_numpy(rng.standard_normal(wl.n_points)).cuda()
    grad = torch.zeros(wl.n_points, dtype=torch.float64, device="cuda")
    q.density_on_grid(plan, coef, q.TERM_ALL, 1, grad)
    H = q.new_store(plan)
    q.q4c_integrate_H(plan, dv, 0, 0, H)
    torch.cuda.synchronize()
    lhs = float(torch.dot(grad, dv))
    rhs = float(torch.sum(coef * H))
    scale = float(torch.sum(torch.abs(coef * H)))
    assert abs(lhs - rhs) <= 1e-12 * scale
    # term selection adds up
    parts = []
    for t in (q.TERM_LL, q.TERM_SS, q.TERM_SO):
        o = torch.zeros_like(grad)
        q.density_on_grid(plan, coef, t, 1, o)
        parts.append(o)
    torch.cuda.synchronize()
    assert torch.allclose(parts[0] + parts[1] + parts[2], grad, rtol=1e-12, atol=1e-12 * float(grad.abs().max()))


def test_coef_from_spinor_matches_oracle(q, small):
    torch = _torch()
    wl, pairs, _, _ = small
    plan = q.Plan(wl)
    _, po = plan.pairs()
    D = W.spinor_density(wl, pairs, 5001)
    from helpers import blocks_to_store, spinor_coef_scale, spinor_from_blocks
    spin = torch.from_numpy(spinor_from_blocks(D, po)).cuda()
    out = q.new_store(plan)
    q.q4c_coef_from_spinor(plan, spin, out)
    torch.cuda.synchronize()
    ref = blocks_to_store(oracle.coef_from_spinor_density(pairs, D), po)
    scale = blocks_to_store(spinor_coef_scale(pairs, D), po)
    assert per_point_worst(out.cpu().numpy(), ref, 1e-15 * scale) <= 1.0


# ---------------------------------------------------------------------------
# Multi-tile case: 24 atoms in a 9 angstrom cube, 119..372 functions per batch
# (up to 6 x 6 tiles of 64), so off-diagonal tiles and atom blocks split over
# tiles are exercised; also run with small batches and a tiny staging budget
# (many passes).
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def medium(q):
    wl = W.config_cluster(n_atoms=24, nrad=24, nang=50, box_ang=9.0, k=7)
    pairs = W.atom_pairs(wl)
    ref, scale = oracle.pair_blocks(wl, pairs, with_abs=True)
    return wl, pairs, ref, scale


@pytest.mark.parametrize("p_max,staging", [(300, 0), (64, 1 << 20)])
def test_integrate_f64_multitile(q, medium, p_max, staging):
    wl, pairs, ref, scale = medium
    plan, store, spin_w, _ = _run(q, wl, p_max=p_max, staging_bytes=staging)
    if staging:
        assert plan.info["n_passes"] > 1
    assert plan.info["max_batch_fn"] > 2 * 64
    _, po = plan.pairs()
    nfn = wl.atom_nfn()
    got = store_to_blocks(store, pairs, po, nfn)
    _compare_f64(got, ref, scale)
    gw = spinor_to_blocks(spin_w, pairs, po, nfn)
    for p in range(len(pairs)):
        assert np.array_equal(gw[p], oracle.spinor_W(got[p]))


def test_integrate_split_multitile(q, medium):
    wl, pairs, ref, scale = medium
    for prec in (1, 2, 3):
        plan, store, _, _ = _run(q, wl, precision=prec, assemble=False)
        _, po = plan.pairs()
        got = store_to_blocks(store, pairs, po, wl.atom_nfn())
        err = max(float(np.max(np.abs(g[k] - r[k]))) for g, r in zip(got, ref) for k in range(1, 5))
        assert err <= SPLIT_ABS, (prec, err)
        _compare_f64([g[:1] for g in got], [r[:1] for r in ref], [s[:1] for s in scale])


def test_density_multitile(q, medium):
    torch = _torch()
    wl, pairs, _, _ = medium
    nfn = wl.atom_nfn()
    rng = np.random.default_rng(79)
    coef_blocks = [rng.standard_normal((5, nfn[a], nfn[b])) for a, b in pairs]
    idx = np.sort(rng.choice(wl.n_points, size=1500, replace=False))
    ref, scp = oracle.density(wl, pairs, coef_blocks, idx=idx, weight_mode=1, with_scale=True)
    sc = oracle.density_scale(scp, wl.w[idx])
    bound32 = gamma(98) * oracle.density_scale(scp, wl.w[idx], terms=6) + 1e-12 * sc
    from helpers import blocks_to_store
    for p_max, staging in ((300, 0), (64, 1 << 20)):
        plan = q.Plan(wl, p_max=p_max, staging_bytes=staging)
        _, po = plan.pairs()
        coef = torch.from_numpy(blocks_to_store(coef_blocks, po)).cuda()
        for prec in (q.PREC_F64, q.PREC_F32):
            out = torch.full((wl.n_points,), float("nan"), dtype=torch.float64, device="cuda")
            q.density_on_grid(plan, coef, q.TERM_ALL, 1, out, precision=prec)
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            assert np.all(np.isfinite(got))
            if prec == q.PREC_F64:
                assert per_point_worst(got[idx], ref, sc) <= 1e-12, (p_max, staging)
            else:
                assert per_point_worst(got[idx], ref, bound32, floor=1e-30) <= 1.0, (p_max, staging)


def test_staging_passes_do_not_change_results(q, medium):
    """The batch-to-global sums are one sequential chain per element in batch
    order, so splitting the batches into many staging passes gives bitwise the
    same store and the same adjoint."""
    torch = _torch()
    wl = medium[0]
    v = torch.from_numpy(wl.v).cuda()
    rng = np.random.default_rng(7301)
    outs = []
    for budget in (0, 1 << 20):
        plan = q.Plan(wl, staging_bytes=budget)
        print("passes:", plan.info["n_passes"], flush=True)
        coef = torch.from_numpy(np.random.default_rng(7301).standard_normal((5, plan.info["store_len"]))).cuda()
        res = []
        for prec in (q.PREC_F64, q.PREC_SPLIT_F32, q.PREC_BF16X3):
            st = q.new_store(plan)
            q.q4c_integrate_H(plan, v, prec, 0, st)
            res.append(st)
        out = torch.empty(wl.n_points, dtype=torch.float64, device="cuda")
        q.density_on_grid(plan, coef, q.TERM_ALL, 1, out)
        res.append(out)
        torch.cuda.synchronize()
        outs.append((plan.info["n_passes"], res))
    assert outs[0][0] == 1 and outs[1][0] > 3
    for x, y in zip(outs[0][1], outs[1][1]):
        assert torch.equal(x, y)


def test_split_precisions_stated_bound_and_long_batches(q, medium):
    """The split precisions (FP32 W parts, FP64 V) against the oracle on every
    element of the multi-tile case, with batches of at most 300 and of at
    most 1,024 points: each W element within the stated bound (gamma of the
    16-point FP32 partial sums times the magnitudes of its terms, plus the
    FP32 underflow floor), within 1e-8 Ha, and V bitwise equal to the FP64
    path's."""
    torch = _torch()
    wl, pairs, ref, scale = medium
    v = torch.from_numpy(wl.v).cuda()
    for p_max in (300, 1024):
        plan = q.Plan(wl, p_max=p_max)
        print("p_max %d: largest batch %d points" % (p_max, plan.info["max_batch_points"]), flush=True)
        _, po = plan.pairs()
        f64 = q.new_store(plan)
        q.q4c_integrate_H(plan, v, q.PREC_F64, 0, f64)
        for prec in (q.PREC_SPLIT_F32, q.PREC_F32, q.PREC_BF16X3):
            st = q.new_store(plan)
            q.q4c_integrate_H(plan, v, prec, 0, st)
            torch.cuda.synchronize()
            assert torch.equal(st[0], f64[0]), (p_max, prec)
            got = store_to_blocks(st.cpu().numpy(), pairs, po, wl.atom_nfn())
            worst = split_bound_worst(got, ref, scale, prec)
            err = max(float(np.max(np.abs(g[1:] - r[1:]))) for g, r in zip(got, ref))
            print("  precision %d: max |W - oracle| %.3g Ha, worst / bound %.3g" % (prec, err, worst), flush=True)
            assert worst <= 1.0 and err <= SPLIT_ABS, (p_max, prec, worst, err)


def test_parts_mask(q, medium):
    """Selected parts equal the all-parts call bit for bit; parts not selected
    keep what the store held; V-only and W-only calls in every precision."""
    torch = _torch()
    wl, pairs, _, scale = medium
    plan = q.Plan(wl)
    v = torch.from_numpy(wl.v).cuda()
    # the oracle's per-element scale of V (sum of the magnitudes of its terms)
    sv = torch.from_numpy(blocks_to_store(scale, plan.pairs()[1])[0]).cuda()
    rows = {"V": [0], "WS": [1], "WSO": [2, 3, 4]}
    bits = {"V": q.PART_V, "WS": q.PART_WS, "WSO": q.PART_WSO}
    for prec in (q.PREC_F64, q.PREC_F32, q.PREC_SPLIT_F32, q.PREC_BF16X3):
        full = q.new_store(plan)
        q.q4c_integrate_H(plan, v, prec, 0, full)
        for sel in (("V",), ("WS",), ("WSO",), ("V", "WS"), ("WS", "WSO")):
            parts = sum(bits[k] for k in sel)
            st = torch.full_like(full, 7.0)
            q.q4c_integrate_H(plan, v, prec, 0, st, parts=parts)
            torch.cuda.synchronize()
            on = sorted(r for k in sel for r in rows[k])
            off = [r for r in range(5) if r not in on]
            assert torch.equal(st[on], full[on]), (prec, sel)
            assert bool(torch.all(st[off] == 7.0)), (prec, sel)
        # accumulate one part onto another call's result
        acc = full.clone()
        q.q4c_integrate_H(plan, v, prec, q.ACCUMULATE, acc, parts=q.PART_V)
        torch.cuda.synchronize()
        assert torch.equal(acc[1:], full[1:])
        # the batch sums are added one by one onto the stored value: within
        # 1e-13 of each element's scale (twice the scale of one call)
        d = torch.abs(acc[0] - 2 * full[0])
        assert bool(torch.all(d[sv == 0] == 0)) and bool(torch.all(d <= 2e-13 * sv)), (prec, float(torch.max(d / (sv + 1e-300))))
    with pytest.raises(q.Q4CError):
        q.q4c_integrate_H(plan, v, q.PREC_F64, q.ASSEMBLE_W, q.new_store(plan), q.new_spinor(plan), parts=q.PART_WS)


def test_adjoint_reuses_resident_panels_bitwise(q, medium):
    """density_on_grid after q4c_integrate_H takes the operand panels the
    forward call left resident for its last staging pass instead of
    tabulating them again, and runs the passes from the last one down.  Its
    output must be bitwise that of a call that tabulates every pass (after
    q4c_integrate_HS has replaced the panels), with one pass and with many,
    eagerly and under graph replay."""
    torch = _torch()
    wl = W.with_ket(medium[0], 7011)
    rng = np.random.default_rng(83)
    v = torch.from_numpy(wl.v).cuda()
    for staging in (0, 1 << 20):
        plan = q.Plan(wl, staging_bytes=staging)
        plan.set_ket_potential(wl)
        print("passes:", plan.info["n_passes"], flush=True)
        coef = torch.from_numpy(rng.standard_normal((5, plan.info["store_len"]))).cuda()
        st, hs = q.new_store(plan), q.new_hs(plan)
        fresh = torch.empty(wl.n_points, dtype=torch.float64, device="cuda")
        q.q4c_integrate_HS(plan, v, 0, hs)  # panels now hold H/S values: every pass tabulates
        q.density_on_grid(plan, coef, q.TERM_ALL, 1, fresh)
        for graphs in (False, True):
            plan.set_graphs(graphs)
            for rep in range(3):
                reused = torch.full_like(fresh, float("nan"))
                q.q4c_integrate_H(plan, v, q.PREC_F64, 0, st)
                q.density_on_grid(plan, coef, q.TERM_ALL, 1, reused)
                again = torch.full_like(fresh, float("nan"))
                q.density_on_grid(plan, coef, q.TERM_ALL, 1, again)  # pass 0 resident now
                q.q4c_integrate_HS(plan, v, 0, hs)
                after_hs = torch.full_like(fresh, float("nan"))
                q.density_on_grid(plan, coef, q.TERM_ALL, 1, after_hs)
                torch.cuda.synchronize()
                assert torch.equal(reused, fresh), (staging, graphs, rep)
                assert torch.equal(again, fresh), (staging, graphs, rep)
                assert torch.equal(after_hs, fresh), (staging, graphs, rep)
        plan.set_graphs(False)
