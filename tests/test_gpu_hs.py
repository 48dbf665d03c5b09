"""GPU parity of q4c_integrate_HS (the paper's ket-dependent Q4C H and S of one
component, Eq. 19 in the scalar form of Eq. 29, symmetrised) against the FP64
oracle, through the C ABI.

Bar: per element |GPU - oracle| <= 1e-12 * A_ij, A_ij the oracle's own error
scale of the element (sum over points of the magnitudes of its terms); elements
whose terms are all exact zeros must be exactly zero.

Workloads: the 3-atom case (Pb, 2 I) and the 24-atom multi-tile cluster, each
with seeded ket potentials u = eps + Z erf(r/0.5)/r, for the large component
and for its small component (l~ = l +- 1: the 24-atom case has g functions and
up to ~800 functions per batch, several 64-function tiles)."""
import numpy as np
import pytest

import oracle
import workload as W
from helpers import gpu_available, per_point_worst

pytestmark = pytest.mark.gpu

FP64_REL = 1e-12


@pytest.fixture(scope="module")
def q():
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_2608_00773_amd as q4c
    return q4c


def _hs_blocks(hs, pairs, po, nfn):
    return [hs[:, po[p]:po[p + 1]].reshape(2, int(nfn[a]), int(nfn[b])) for p, (a, b) in enumerate(pairs)]


def _run_hs(q, wl, p_max=None, staging_bytes=0, launch=None, flags=0, hs0=None):
    import torch
    plan = q.Plan(wl, p_max=p_max, staging_bytes=staging_bytes)
    plan.set_ket_potential(wl)
    if launch is not None:
        plan.set_launch(q.KERNEL_HS, *launch)
    v = torch.from_numpy(wl.v).cuda()
    hs = q.new_hs(plan) if hs0 is None else torch.from_numpy(hs0).cuda()
    if hs0 is None:
        hs.fill_(float("nan"))
    q.q4c_integrate_HS(plan, v, flags, hs)
    torch.cuda.synchronize()
    return plan, hs.cpu().numpy()


def _compare(got, ref, scale, tol=FP64_REL, floor=1e-300):
    """Per element |got - ref| <= tol A + floor.  The floor covers subnormal
    rounding (each operation may lose up to 2^-1074 absolutely): the small
    component's tight Gaussians carry products near 1e-320 in their tails,
    where a relative bar cannot hold.  The worst element is reported."""
    worst, where, n_big = 0.0, None, 0
    for p, (g, r, s) in enumerate(zip(got, ref, scale)):
        err = np.abs(g - r)
        bad = err > tol * s + floor
        n_big += int(np.count_nonzero(bad & (s > 1e-290)))
        rel = err / (tol * s + floor)
        k = np.unravel_index(np.argmax(rel), rel.shape)
        if rel[k] > worst:
            worst, where = float(rel[k]), (p, k, float(g[k]), float(r[k]), float(s[k]))
    print("worst (|d| / (tol A + floor)) %.3g at pair %s element %s: got %.6g ref %.6g A %.6g; "
          "elements over the bar with A > 1e-290: %d" % ((worst,) + (where[0], where[1]) + where[2:] + (n_big,)),
          flush=True)
    assert worst <= 1.0, (worst, where)
    return worst


@pytest.fixture(scope="module")
def small_lc(q):
    wl = W.with_ket(W.config_small(), 7001)
    pairs = W.atom_pairs(wl)
    ref, sc = oracle.pair_blocks_hs(wl, pairs, with_abs=True)
    return wl, pairs, ref, sc


@pytest.fixture(scope="module")
def small_sc(q, small_lc):
    ws = W.small_component(small_lc[0], 7002)
    pairs = W.atom_pairs(ws)
    ref, sc = oracle.pair_blocks_hs(ws, pairs, with_abs=True)
    return ws, pairs, ref, sc


@pytest.fixture(scope="module")
def medium_lc(q):
    wl = W.with_ket(W.config_cluster(n_atoms=24, nrad=24, nang=50, box_ang=9.0, k=7), 7011)
    pairs = W.atom_pairs(wl)
    ref, sc = oracle.pair_blocks_hs(wl, pairs, with_abs=True)
    return wl, pairs, ref, sc


@pytest.fixture(scope="module")
def medium_sc(q, medium_lc):
    ws = W.small_component(medium_lc[0], 7012)
    pairs = W.atom_pairs(ws)
    ref, sc = oracle.pair_blocks_hs(ws, pairs, with_abs=True)
    return ws, pairs, ref, sc


@pytest.mark.parametrize("case", ["small_lc", "small_sc"])
def test_hs_small(q, case, request):
    wl, pairs, ref, sc = request.getfixturevalue(case)
    plan, hs = _run_hs(q, wl)
    p, po = plan.pairs()
    assert np.array_equal(p, pairs)
    _compare(_hs_blocks(hs, pairs, po, wl.atom_nfn()), ref, sc)


@pytest.mark.parametrize("case,p_max,staging", [("medium_lc", 300, 0), ("medium_sc", 300, 0),
                                                ("medium_sc", 64, 1 << 20)])
def test_hs_multitile(q, case, p_max, staging, request):
    wl, pairs, ref, sc = request.getfixturevalue(case)
    print("case %s p_max %d staging %d" % (case, p_max, staging), flush=True)
    plan, hs = _run_hs(q, wl, p_max=p_max, staging_bytes=staging)
    if staging:
        assert plan.info["n_passes"] > 1
    assert plan.info["max_batch_fn"] > 64
    _, po = plan.pairs()
    _compare(_hs_blocks(hs, pairs, po, wl.atom_nfn()), ref, sc)


def test_hs_repeatable_accumulate_and_launch_shapes(q, medium_sc):
    """Bitwise repeatable; ACCUMULATE adds onto the given values in FP64; every
    launch shape of k_contract_hs gives the same bits."""
    wl = medium_sc[0]
    _, a = _run_hs(q, wl)
    _, b = _run_hs(q, wl)
    assert np.array_equal(a, b)
    for launch in ((1, 0), (0, 512), (1, 512)):
        print("launch", launch, flush=True)
        _, c = _run_hs(q, wl, launch=launch)
        assert np.array_equal(a, c), launch
    # onto a copy of the result: the staged blocks are added one by one, so the
    # sum differs from 2a only by the rounding of that chain
    _, acc = _run_hs(q, wl, flags=q.ACCUMULATE, hs0=a)
    scale = np.max(np.abs(a), axis=1, keepdims=True)
    assert np.all(np.abs(acc - 2 * a) <= 1e-14 * scale)
    assert not np.array_equal(acc, a)


def test_hs_graph_replay_bitwise(q, medium_sc):
    """q4c_integrate_HS captured in a HIP graph and replayed several times,
    with eager torch work and synchronisations between the replays, and
    after a new ket potential (the captured graph is dropped): every replay
    equals the eager result bit for bit."""
    import torch
    wl = medium_sc[0]
    _, ref = _run_hs(q, wl)
    plan = q.Plan(wl)
    plan.set_ket_potential(wl)
    plan.set_graphs(True)
    v = torch.from_numpy(wl.v).cuda()
    hs = q.new_hs(plan)
    for rep in range(4):
        hs.fill_(float("nan"))
        q.q4c_integrate_HS(plan, v, 0, hs)
        junk = torch.randn(1 << 16, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        assert np.array_equal(hs.cpu().numpy(), ref), rep
        del junk
    plan.set_ket_potential(wl)  # the same table again: new device copies, graphs dropped
    hs.fill_(float("nan"))
    q.q4c_integrate_HS(plan, v, 0, hs)
    torch.cuda.synchronize()
    assert np.array_equal(hs.cpu().numpy(), ref)
    plan.set_graphs(False)


def test_hs_requires_ket_potential(q, small_lc):
    import torch
    wl = small_lc[0]
    plan = q.Plan(wl)
    hs = q.new_hs(plan)
    with pytest.raises(q.Q4CError) as e:
        q.q4c_integrate_HS(plan, torch.from_numpy(wl.v).cuda(), 0, hs)
    assert e.value.status == q.Q4C_EINVAL


def test_g_functions_tabulate_and_integrate_H(q, medium_sc):
    """l = 4 (g) functions on the existing paths: nao_tabulate (values and
    gradients) at every point of the first batches, and the five W-path parts
    on sampled heavy-atom pair blocks against the oracle."""
    import torch
    ws = medium_sc[0]
    plan = q.Plan(ws)
    nb = min(plan.info["n_batches"], 40)
    n = plan.tabulate_size(0, nb, 1)
    out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    q.nao_tabulate(plan, 0, nb, 1, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    pt_off, pidx, fn_off, fidx = plan.batches()
    sel = pidx[:pt_off[nb]]
    phi, grad, aphi, agrad = oracle.tabulate(ws, ws.x[sel], ws.y[sel], ws.z[sel], with_abs=True)
    o, worst = 0, 0.0
    for b in range(nb):
        P = pt_off[b + 1] - pt_off[b]
        fns = fidx[fn_off[b]:fn_off[b + 1]]
        blk = got[o:o + 4 * P * len(fns)].reshape(4, P, len(fns))
        o += 4 * P * len(fns)
        rows = slice(pt_off[b], pt_off[b + 1])
        ref = np.concatenate([phi[rows][:, fns][None], np.moveaxis(grad[rows][:, fns, :], 2, 0)], axis=0)
        sref = np.concatenate([aphi[rows][:, fns][None], np.moveaxis(agrad[rows][:, fns, :], 2, 0)], axis=0)
        worst = max(worst, per_point_worst(blk, ref, sref, floor=1e-300))
    print("g-function tabulation: worst |d| / (own scale + 1e-300) %.3g" % worst, flush=True)
    assert worst <= 1e-12, worst
    # W path: sampled pairs of heavy atoms (their small components carry g shells)
    v = torch.from_numpy(ws.v).cuda()
    store = q.new_store(plan)
    q.q4c_integrate_H(plan, v, q.PREC_F64, 0, store)
    torch.cuda.synchronize()
    st = store.cpu().numpy()
    pairs, po = plan.pairs()
    heavy = ws.Z >= 21
    cand = np.nonzero(heavy[pairs[:, 0]] & heavy[pairs[:, 1]])[0]
    rng = np.random.default_rng(7031)
    sel = np.sort(rng.choice(cand, size=min(10, cand.size), replace=False))
    ref, sc = oracle.pair_blocks(ws, pairs[sel], with_abs=True)
    nfn = ws.atom_nfn()
    got = [st[:, po[p]:po[p + 1]].reshape(5, int(nfn[pairs[p, 0]]), int(nfn[pairs[p, 1]])) for p in sel]
    _compare(got, ref, sc)


@pytest.mark.parametrize("component", ["large", "small"])
def test_hs_fullsize_cluster_sampled_pairs(q, component):
    """The 120-atom cluster (2,174,400 points; large component 1,860 functions,
    small component 4,020 with g functions), in every launch shape the
    benchmark chooses from: sampled pair blocks (heavy-heavy, heavy-light,
    light-light, diagonal) against the oracle's whole-grid sums."""
    import torch
    wl = W.with_ket(W.config_cluster(), 7101)
    if component == "small":
        wl = W.small_component(wl, 7102)
    plan = q.Plan(wl)
    plan.set_ket_potential(wl)
    v = torch.from_numpy(wl.v).cuda()
    res = []
    for shape in ((0, 0), (0, 1024), (1, 1024)):
        plan.set_launch(q.KERNEL_HS, *shape)
        hs = q.new_hs(plan)
        q.q4c_integrate_HS(plan, v, 0, hs)
        torch.cuda.synchronize()
        res.append(hs.cpu().numpy())
    assert all(np.array_equal(res[0], r) for r in res[1:])
    pairs, po = plan.pairs()
    heavy = wl.Z >= 21
    a, b = pairs[:, 0], pairs[:, 1]
    rng = np.random.default_rng(7041 if component == "large" else 7042)
    sel = []
    for g in ((a == b) & heavy[a], (a != b) & heavy[a] & heavy[b], (a != b) & (heavy[a] ^ heavy[b]),
              (a != b) & ~heavy[a] & ~heavy[b]):
        idx = np.nonzero(g)[0]
        if idx.size:
            sel.extend(rng.choice(idx, size=min(2, idx.size), replace=False).tolist())
    sel = np.array(sorted(set(sel)))
    print("%s component: %d functions, sampled pairs %s" % (component, wl.n_fn, sel.tolist()), flush=True)
    ref, sc = oracle.pair_blocks_hs(wl, pairs[sel], with_abs=True)
    nfn = wl.atom_nfn()
    got = [res[0][:, po[p]:po[p + 1]].reshape(2, int(nfn[pairs[p, 0]]), int(nfn[pairs[p, 1]])) for p in sel]
    _compare(got, ref, sc)
