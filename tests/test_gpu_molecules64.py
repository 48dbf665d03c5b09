"""The 64-molecule workload at full size: 64 independent molecules of 8..80
atoms (cluster element mix and recipe, 60 x 302 points per atom, about 5e7
points), all their grid batches in one batched plan with autotuned launch
shapes and HIP-graph replay, against 64 per-molecule plans called one after
another (paper Sec. III A, Eq. 31: batches are independent work units).

  * forward (FP64 with the W spinor blocks, and split FP32) and the adjoint
    of the batched plan equal the sequential plans' results bit for bit
  * sampled pair blocks of the smallest and the largest molecule against the
    oracle, every element within 1e-12 of its own scale A_ij
  * the adjoint at sampled points of those molecules against the oracle,
    every point within 1e-12 of its own scale

About two to three minutes, most of it input generation; every step prints a
progress line.
"""
import numpy as np
import pytest

import oracle
import workload as W
from helpers import gpu_available, per_point_worst, store_to_blocks

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


@pytest.fixture(scope="module")
def env():
    if not gpu_available():
        pytest.skip("no GPU")
    import torch
    import paper_2608_00773_amd as q
    wl = W.config_molecules()
    systems = W.split_molecules(wl)
    print("64 molecules: %d atoms, %d points" % (wl.n_atoms, wl.n_points), flush=True)
    pb = q.Plan(systems)
    print("batched plan:", pb.info, flush=True)
    v = torch.from_numpy(np.concatenate([s.v for s in systems])).cuda()
    rng = np.random.default_rng(4201)
    coef = torch.from_numpy(rng.standard_normal((5, pb.info["store_len"]))).cuda()
    return dict(q=q, torch=torch, wl=wl, systems=systems, pb=pb, v=v, coef=coef, off=pb.systems())


def _batched(env, prec):
    q, torch, pb = env["q"], env["torch"], env["pb"]
    st, spin = q.new_store(pb), q.new_spinor(pb)
    q.q4c_integrate_H(pb, env["v"], prec, q.ASSEMBLE_W, st, spin)
    out = torch.empty(pb.info["n_points"], dtype=torch.float64, device="cuda")
    q.density_on_grid(pb, env["coef"], q.TERM_ALL, 1, out)
    torch.cuda.synchronize()
    return st, spin, out


def test_molecules64_batched_graphs_equal_sequential_bitwise(env):
    q, torch, systems, pb, off = env["q"], env["torch"], env["systems"], env["pb"], env["off"]
    tmp_st = q.new_store(pb)
    tmp_out = torch.empty(pb.info["n_points"], dtype=torch.float64, device="cuda")
    table = pb.autotune(env["v"], tmp_st, q.PREC_F64, env["coef"], tmp_out, reps=2)
    del tmp_st, tmp_out
    print("autotuned: contract %s, density %s" % (pb.get_launch(q.KERNEL_CONTRACT), pb.get_launch(q.KERNEL_DENSITY)),
          flush=True)
    assert len(table) == 12
    pb.set_graphs(True)
    ref = {}
    for prec in (q.PREC_F64, q.PREC_SPLIT_F32, q.PREC_BF16X3):
        _batched(env, prec)  # captures the graphs
        ref[prec] = _batched(env, prec)  # replays them
    pb.set_graphs(False)
    env["ref"] = ref
    for s, ws in enumerate(systems):
        p = q.Plan(ws, staging_bytes=2 << 30)
        s0, s1 = int(off["store"][s]), int(off["store"][s + 1])
        g0, g1 = int(off["point"][s]), int(off["point"][s + 1])
        v = env["v"][g0:g1].contiguous()
        coef = env["coef"][:, s0:s1].contiguous()
        for prec, (st_b, spin_b, out_b) in ref.items():
            st, spin = q.new_store(p), q.new_spinor(p)
            q.q4c_integrate_H(p, v, prec, q.ASSEMBLE_W, st, spin)
            out = torch.empty(p.info["n_points"], dtype=torch.float64, device="cuda")
            q.density_on_grid(p, coef, q.TERM_ALL, 1, out)
            torch.cuda.synchronize()
            assert torch.equal(st_b[:, s0:s1], st), (prec, s)
            assert torch.equal(spin_b[4 * s0:4 * s1], spin), (prec, s)
            assert torch.equal(out_b[g0:g1], out), (prec, s)
        p.close()
        if s % 8 == 7:
            print("molecules 0..%d: batched == sequential bit for bit" % s, flush=True)


def test_molecules64_against_oracle(env):
    q, torch, systems, pb, off = env["q"], env["torch"], env["systems"], env["pb"], env["off"]
    st_b, _, out_b = env["ref"][q.PREC_F64] if "ref" in env else _batched(env, q.PREC_F64)
    st_b, out_b = st_b.cpu().numpy(), out_b.cpu().numpy()
    coef = env["coef"].cpu().numpy()
    pairs_b, po_b = pb.pairs()
    sizes = [s.n_atoms for s in systems]
    rng = np.random.default_rng(4202)
    for s in (int(np.argmin(sizes)), int(np.argmax(sizes))):
        ws = systems[s]
        a0, a1 = int(off["pair"][s]), int(off["pair"][s + 1])
        g0, g1 = int(off["point"][s]), int(off["point"][s + 1])
        sel = np.sort(rng.choice(np.arange(a0, a1), size=min(6, a1 - a0), replace=False))
        local = pairs_b[sel] - off["atom"][s]
        ref, scale = oracle.pair_blocks(ws, local, with_abs=True)
        nfn = ws.atom_nfn()
        worst = 0.0
        for k, p in enumerate(sel):
            a, b = local[k]
            g = st_b[:, po_b[p]:po_b[p + 1]].reshape(5, nfn[a], nfn[b])
            nz = scale[k] > 0
            assert np.all(g[~nz] == ref[k][~nz])
            worst = max(worst, float(np.max(np.abs(g - ref[k])[nz] / scale[k][nz])))
        print("molecule %d (%d atoms): %d pair blocks, worst |d| / A_ij %.3g" % (s, ws.n_atoms, len(sel), worst),
              flush=True)
        assert worst <= 1e-12, (s, worst)
        # the adjoint of this molecule at sampled points, from its own coefficients
        pairs_s = pairs_b[a0:a1] - off["atom"][s]
        blocks = store_to_blocks(coef[:, int(off["store"][s]):int(off["store"][s + 1])], pairs_s,
                                 po_b[a0:a1 + 1] - po_b[a0], nfn)
        idx = np.sort(rng.choice(ws.n_points, size=80, replace=False))
        refd, sc = oracle.density(ws, pairs_s, blocks, idx=idx, weight_mode=1, with_scale=True)
        worst = per_point_worst(out_b[g0:g1][idx], refd, oracle.density_scale(sc, ws.w[idx]))
        print("molecule %d: adjoint at %d points, worst |d| / own scale %.3g" % (s, idx.size, worst), flush=True)
        assert worst <= 1e-12, (s, worst)
