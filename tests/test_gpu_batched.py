"""Many independent systems in one plan (q4c_plan_create_batched), launch
shapes (work order, persistent workgroups), the autotuner and HIP-graph
replay.  None of them changes any arithmetic, so every result must be bitwise
equal to the plain per-system calls; the batched plan is also checked against
the oracle on sampled pair blocks.

Workload: 12 molecules of the batched-molecule recipe (sizes drawn from
8..80 atoms, cluster element mix) on 24 x 50 grids per atom."""
import numpy as np
import pytest

import oracle
import workload as W
from helpers import gpu_available

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    if not gpu_available():
        pytest.skip("no GPU")
    import torch
    import paper_2608_00773_amd as q
    wl = W.config_molecules(n_mol=12, nrad=24, nang=50)
    systems = W.split_molecules(wl)
    pb = q.Plan(systems)
    v = torch.from_numpy(np.concatenate([s.v for s in systems])).cuda()
    rng = np.random.default_rng(4101)
    coef = torch.from_numpy(rng.standard_normal((5, pb.info["store_len"]))).cuda()
    return dict(q=q, torch=torch, wl=wl, systems=systems, pb=pb, v=v, coef=coef, off=pb.systems())


def _run(q, torch, plan, v, coef, prec):
    st = q.new_store(plan)
    q.q4c_integrate_H(plan, v, prec, 0, st)
    out = torch.empty(plan.info["n_points"], dtype=torch.float64, device="cuda")
    q.density_on_grid(plan, coef, q.TERM_ALL, 1, out)
    torch.cuda.synchronize()
    return st, out


def test_batched_equals_sequential_bitwise(env):
    q, torch, systems, pb, off = env["q"], env["torch"], env["systems"], env["pb"], env["off"]
    print("batched plan:", pb.info, flush=True)
    for prec in (q.PREC_F64, q.PREC_F32, q.PREC_SPLIT_F32, q.PREC_BF16X3):
        st_b, out_b = _run(q, torch, pb, env["v"], env["coef"], prec)
        for s, ws in enumerate(systems):
            p = q.Plan(ws)
            s0, s1 = int(off["store"][s]), int(off["store"][s + 1])
            g0, g1 = int(off["point"][s]), int(off["point"][s + 1])
            st, out = _run(q, torch, p, env["v"][g0:g1].contiguous(), env["coef"][:, s0:s1].contiguous(), prec)
            assert torch.equal(st_b[:, s0:s1], st), (prec, s)
            assert torch.equal(out_b[g0:g1], out), (prec, s)


def test_batched_matches_oracle(env):
    q, torch, systems, pb, off = env["q"], env["torch"], env["systems"], env["pb"], env["off"]
    st_b, _ = _run(q, torch, pb, env["v"], env["coef"], q.PREC_F64)
    st_b = st_b.cpu().numpy()
    pairs_b, po_b = pb.pairs()
    rng = np.random.default_rng(4102)
    worst = 0.0
    for s in (0, len(systems) - 1):
        ws = systems[s]
        a0, a1 = int(off["pair"][s]), int(off["pair"][s + 1])
        sel = np.sort(rng.choice(np.arange(a0, a1), size=min(4, a1 - a0), replace=False))
        local = pairs_b[sel] - off["atom"][s]
        ref, scale = oracle.pair_blocks(ws, local, with_abs=True)
        nfn = ws.atom_nfn()
        for k, p in enumerate(sel):
            a, b = local[k]
            g = st_b[:, po_b[p]:po_b[p + 1]].reshape(5, nfn[a], nfn[b])
            nz = scale[k] > 0
            assert np.all(g[~nz] == ref[k][~nz])
            worst = max(worst, float(np.max(np.abs(g - ref[k])[nz] / scale[k][nz])))
    assert worst <= 1e-12, worst


def test_launch_shapes_bitwise(env):
    q, torch, pb = env["q"], env["torch"], env["pb"]
    ref = {prec: _run(q, torch, pb, env["v"], env["coef"], prec)
           for prec in (q.PREC_F64, q.PREC_F32, q.PREC_SPLIT_F32, q.PREC_BF16X3)}
    for order in (0, 1):
        for pers in (0, 256, 512, 3000):
            print("launch shape order=%d persistent=%d" % (order, pers), flush=True)
            pb.set_launch(q.KERNEL_CONTRACT, order, pers)
            pb.set_launch(q.KERNEL_DENSITY, order, pers)
            assert pb.get_launch(q.KERNEL_CONTRACT) == (order, pers)
            for prec, (st0, out0) in ref.items():
                st, out = _run(q, torch, pb, env["v"], env["coef"], prec)
                assert torch.equal(st, st0), (order, pers, prec)
                assert torch.equal(out, out0), (order, pers, prec)
    pb.set_launch(q.KERNEL_CONTRACT, 0, 0)
    pb.set_launch(q.KERNEL_DENSITY, 0, 0)


def test_graph_replay_bitwise(env):
    """Captured graphs replayed several times, with eager torch work and
    synchronisations between replays: every replay equals the eager result."""
    q, torch, pb = env["q"], env["torch"], env["pb"]
    pb.set_launch(q.KERNEL_CONTRACT, 0, 512)  # a persistent shape inside the graph too
    st0, out0 = _run(q, torch, pb, env["v"], env["coef"], q.PREC_F64)
    spin0 = q.new_spinor(pb)
    q.q4c_integrate_H(pb, env["v"], q.PREC_F64, q.ASSEMBLE_W, q.new_store(pb), spin0)
    acc0 = st0.clone()
    q.q4c_integrate_H(pb, env["v"], q.PREC_F64, q.ACCUMULATE, acc0)
    torch.cuda.synchronize()
    pb.set_graphs(True)
    st = q.new_store(pb)
    spin = q.new_spinor(pb)
    acc = q.new_store(pb)
    out = torch.empty(pb.info["n_points"], dtype=torch.float64, device="cuda")
    junk = torch.empty(1 << 20, dtype=torch.float64, device="cuda")
    for rep in range(4):
        st.fill_(float("nan"))
        out.fill_(float("nan"))
        spin.fill_(float("nan"))
        q.q4c_integrate_H(pb, env["v"], q.PREC_F64, q.ASSEMBLE_W, st, spin)
        junk.normal_()
        q.density_on_grid(pb, env["coef"], q.TERM_ALL, 1, out)
        acc.copy_(st0)
        q.q4c_integrate_H(pb, env["v"], q.PREC_F64, q.ACCUMULATE, acc)
        torch.cuda.synchronize()
        assert torch.equal(st, st0), rep
        assert torch.equal(spin, spin0), rep
        assert torch.equal(out, out0), rep
        assert torch.equal(acc, acc0), rep
        junk.mul_(2.0).sum().item()
    pb.set_graphs(False)
    pb.set_launch(q.KERNEL_CONTRACT, 0, 0)


def test_autotune_keeps_results(env):
    q, torch, pb = env["q"], env["torch"], env["pb"]
    st0, out0 = _run(q, torch, pb, env["v"], env["coef"], q.PREC_F64)
    tmp_st = q.new_store(pb)
    tmp_out = torch.empty(pb.info["n_points"], dtype=torch.float64, device="cuda")
    table = pb.autotune(env["v"], tmp_st, q.PREC_F64, env["coef"], tmp_out, reps=3)
    print("autotune:", table, flush=True)
    assert len(table) == 12
    for kernel in (q.KERNEL_CONTRACT, q.KERNEL_DENSITY):
        rows = [t for t in table if t[0] == kernel]
        best = min(rows, key=lambda t: t[3])
        best0 = min([t for t in rows if t[1] == 0], key=lambda t: t[3])
        # the fastest shape, or the fastest batch-order shape within 2% of it
        want = best0 if best0[3] <= 1.02 * best[3] else best
        assert pb.get_launch(kernel) == (want[1], want[2])
        assert all(t[3] > 0 for t in rows)
    st, out = _run(q, torch, pb, env["v"], env["coef"], q.PREC_F64)
    assert torch.equal(st, st0)
    assert torch.equal(out, out0)
    pb.set_launch(q.KERNEL_CONTRACT, 0, 0)
    pb.set_launch(q.KERNEL_DENSITY, 0, 0)
