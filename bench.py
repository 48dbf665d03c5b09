#!/usr/bin/env python3
"""Benchmark of Q4C real-space Hamiltonian integration on one MI355X.

Workload: the seeded 120-atom cluster (20% Pb, 30% I, 50% H/C/N in a 20
angstrom cube; 26 NAOs per heavy atom, 5 per light atom, l <= 3; 60 x 302
points per atom = 2,174,400 points; batches of at most 300 points; model
potential plus smooth noise).  Inputs are resident in HBM before timing.

One step = the whole hot path once: q4c_integrate_H (tabulation, weighting,
the five contractions, batch-to-global sums, W spinor assembly) followed by
density_on_grid (the adjoint dL/dv for a seeded upstream gradient).

Prints one JSON line.  `value` is active grid points per second of the step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "H-integration grid points/s & MFMA util: split-FP32 vs FP64 at ≤1e-8 Ha"
PEAK_F64 = 78.6e12    # MI355X dense FP64 MFMA, flop/s
PEAK_F32 = 157.3e12   # MI355X dense FP32 MFMA, flop/s
PEAK_BF16 = 2.5e15    # MI355X dense BF16 MFMA, flop/s
PEAK_HBM = 8.0e12     # MI355X HBM3E, bytes/s
PREC = {"f64": 0, "split": 1, "f32": 2, "bf16x3": 3, "f64valu": 4}

# HBM bytes per launch of the path's kernels on the default cluster workload,
# from two rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE), each scaled by what
# the same counter reads for an elementwise copy of 1 GiB (read x2, write x1):
# the timed launches, and per launch shape the autotuner's trial launches of
# the same runs (persistent sizes 512 and 1024 read the same bytes).  Keyed by
# kernel, the SHA-256 of the kernel sources the counters were taken on
# (q4c_kernels.hip and q4c_device.h), the precision, the workload and the
# launch shape: work order (0: batch order, which keeps a batch's tiles on one
# L2; 1: the cost-sorted queue, which does not) and whether the launch is
# persistent (None for kernels without either).  Any change to those sources
# makes the figure unknown, and it is then reported as null.
_KS = "3988041ce98d2cefbd3169767ac3a161f0c36e4d4c5bb94ed602b3de360c368c"
TRAFFIC = {
    ("k_contract", _KS, "f64", "cluster-120", (0, False)): 21.63e9 + 7.44e9,
    ("k_contract", _KS, "f64", "cluster-120", (0, True)): 23.25e9 + 7.64e9,
    ("k_contract", _KS, "f64", "cluster-120", (1, False)): 42.81e9 + 7.65e9,
    ("k_contract", _KS, "f64", "cluster-120", (1, True)): 39.92e9 + 7.96e9,
    ("k_density_tiles", _KS, "f64", "cluster-120", (0, False)): 19.97e9 + 0.21e9,
    ("k_density_tiles", _KS, "f64", "cluster-120", (0, True)): 21.51e9 + 0.21e9,
    ("k_density_tiles", _KS, "f64", "cluster-120", (1, False)): 70.18e9 + 0.21e9,
    ("k_density_tiles", _KS, "f64", "cluster-120", (1, True)): 67.96e9 + 0.21e9,
    ("k_panel", _KS, "f64", "cluster-120", None): 0.17e9 + 11.49e9,
    ("k_reduce", _KS, "f64", "cluster-120", None): 7.41e9 + 0.03e9,
    ("k_contract", _KS, "bf16x3", "cluster-120", (0, False)): 9.44e9 + 6.95e9,
    ("k_contract", _KS, "bf16x3", "cluster-120", (0, True)): 9.69e9 + 7.15e9,
    ("k_contract", _KS, "bf16x3", "cluster-120", (1, False)): 52.62e9 + 7.84e9,
    ("k_contract", _KS, "bf16x3", "cluster-120", (1, True)): 47.97e9 + 7.79e9,
    ("k_panel", _KS, "bf16x3", "cluster-120", None): 0.16e9 + 9.34e9,
    ("k_reduce", _KS, "bf16x3", "cluster-120", None): 7.41e9 + 0.03e9,
}

# The same for k_contract_hs (q4c_integrate_HS) per component and launch shape,
# keyed by the SHA-256 of q4c_hs_kernels.hip and q4c_device.h.
_HS = "07c101f6ce1cacc7d5df8cc7267adc142c8576d56c73f0659b9e0b7c9665fe60"
HS_TRAFFIC = {
    (_HS, "large", 120, (0, True)): 6.854e9 + 2.994e9,
    (_HS, "small", 120, (0, True)): 7.143e9 + 7.043e9,
}


def source_sha(*names):
    import hashlib
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2608_00773_amd", "csrc", n), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=sorted(PREC), default="f64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes (one workgroup per work item) and eager launches")
    ap.add_argument("--no-graphs", action="store_true",
                    help="autotune but launch eagerly (for per-dispatch counter collection)")
    ap.add_argument("--cpu-sample", type=float, default=0.1,
                    help="fraction of grid points for the oracle timing on all host threads (one thread: a tenth)")
    ap.add_argument("--n-atoms", type=int, default=120)
    ap.add_argument("--mode", choices=["full", "step", "forward", "adjoint", "hs"], default="full",
                    help="step/forward/adjoint: run only the whole step or that one call `steps` times "
                         "(for profiler runs) and print its time; hs: only the H/S leg")
    ap.add_argument("--workload", choices=["cluster", "slab", "pepi", "molecules", "periodic"], default="cluster",
                    help="molecules: 64 independent molecules (8..80 atoms), one batched plan (autotuned launch "
                         "shapes, HIP graph replay) against 64 sequential per-molecule plans; prints its own line")
    ap.add_argument("--contract-order", type=int, choices=[0, 1], default=None,
                    help="after autotuning, keep the contraction's work order fixed (0: batch order, "
                         "1: cost-sorted global queue) with the best persistent size timed for it")
    ap.add_argument("--no-hs", action="store_true",
                    help="skip the H/S leg (the Q4C ket-dependent integrand of both components)")
    ap.add_argument("--hs-component", choices=["both", "large", "small"], default="both",
                    help="--mode hs: run one component only")
    ap.add_argument("--hs-shape", default=None,
                    help="--mode hs: fixed k_contract_hs launch shape 'order,persistent' instead of the best of three")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before the work, run one elementwise copy of this many MiB (read once, written once): "
                         "the reference dispatch for scaling HBM byte counters")
    return ap.parse_args()


def contraction_peak(prec: str) -> float:
    """Peak of the contraction kernel for its operand types: 1 of the 10 P n^2
    algorithmic flops (V) runs on FP64 MFMA in every mode; the other 9 (W parts)
    run on FP64 MFMA (f64), FP32 MFMA (split, f32: one FP32 product per
    product, the hi/lo mode's extra two counted as its own overhead) or BF16
    MFMA with six BF16 products per product (bf16x3)."""
    if prec in ("f64", "f64valu"):
        return PEAK_F64  # the FP64 vector peak equals the FP64 matrix peak on MI355X
    if prec == "bf16x3":
        return 10.0 / (1.0 / PEAK_F64 + 9.0 * 6.0 / PEAK_BF16)
    return 10.0 / (1.0 / PEAK_F64 + 9.0 / PEAK_F32)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, plan, gbar, frac_all: float, frac_one: float, seed: int = 6002):
    """The oracle timed on the host cores for the same step as the GPU line:
    the forward pair blocks (all five parts of every atom pair) plus the
    adjoint (w_g times the density of the seeded upstream gradient gbar,
    weight mode 1) at a seeded sample of the grid points.  The oracle runs
    OpenMP over pairs (forward) and over points (adjoint); each element's
    summation order does not depend on the thread count.  Timed on all host
    threads on a sample of frac_all of the points, and on one thread on a
    sample of frac_one.  Points/s counts active sample points, as the GPU
    figure does."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(seed)
    pairs, po = plan.pairs()
    nfn = wl.atom_nfn()
    g = gbar.cpu().numpy()
    blocks = [g[:, po[p]:po[p + 1]].reshape(5, int(nfn[a]), int(nfn[b])) for p, (a, b) in enumerate(pairs)]
    rc = wl.atom_rcut()
    oracle.build()
    nthreads = oracle.max_threads()

    def run(frac, threads):
        idx = np.sort(rng.choice(wl.n_points, size=max(1, int(frac * wl.n_points)), replace=False))
        sub = wl.subset_points(idx)
        d2 = ((sub.x[:, None] - wl.R[None, :, 0]) ** 2 + (sub.y[:, None] - wl.R[None, :, 1]) ** 2 +
              (sub.z[:, None] - wl.R[None, :, 2]) ** 2)
        n_act = int(np.sum(np.any(d2 < rc[None, :] ** 2, axis=1)))
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        oracle.pair_blocks(sub, pairs)
        t1 = time.perf_counter()
        oracle.density(wl, pairs, blocks, idx=idx, weight_mode=1)
        t2 = time.perf_counter()
        return {"value": n_act / (t2 - t0), "unit": "points/s", "cores": threads, "kind": "oracle",
                "sample": "%d of %d grid points (%d active, seed %d), forward over all %d atom pairs %.1f s + "
                          "adjoint at the same points %.1f s" % (idx.size, wl.n_points, n_act, seed, len(pairs),
                                                                 t1 - t0, t2 - t1),
                "forward_s": t1 - t0, "adjoint_s": t2 - t1}

    res = run(frac_all, nthreads)
    res["single_core"] = run(frac_one, 1)
    oracle.set_threads(nthreads)
    res["nproc"] = os.cpu_count()
    res["cpu_model"] = cpu_model()
    return res


def bench_hs(wl, timed, steps: int, cpu_frac: float, with_cpu: bool, components=("large", "small"),
             shapes=((0, 0), (0, 1024), (1, 1024))):
    """H and S of both components (q4c_integrate_HS: the Q4C integrand of Eq. 19
    in the scalar form of Eq. 29) on the same grid and potential: the large
    component is the workload's basis, the small component its l~ = l +- 1
    partners (seeded radials); seeded ket potentials eps + Z erf(r/0.5)/r.
    Per component: best of three launch shapes, time per call, and the
    k_contract_hs roofline from HIP events (algorithmic 3 P n^2 flops per batch)."""
    import numpy as np
    import torch
    import paper_2608_00773_amd as q
    import workload as W
    dev = torch.device("cuda:0")
    hsha = source_sha("q4c_hs_kernels.hip", "q4c_device.h")
    t0 = time.perf_counter()
    wl_l = W.with_ket(wl, 7101)
    wl_s = W.small_component(wl_l, 7102)
    out = {"workload_gen_s": time.perf_counter() - t0}
    kept = {}
    for name, w in (("large", wl_l), ("small", wl_s)):
        if name not in components:
            continue
        t0 = time.perf_counter()
        plan = q.Plan(w)
        plan.set_ket_potential(w)
        t_plan = time.perf_counter() - t0
        info = plan.info
        v = torch.from_numpy(w.v).to(dev)
        hs = q.new_hs(plan, dev)
        call = lambda: q.q4c_integrate_HS(plan, v, 0, hs)
        tune = []
        for shape in shapes:
            plan.set_launch(q.KERNEL_HS, *shape)
            call()
            tune.append((shape, timed(call, 3)))
        best = min(tune, key=lambda t: t[1])[0]
        plan.set_launch(q.KERNEL_HS, *best)
        plan.set_graphs(True)  # the timed calls replay one captured graph
        call()
        ms = timed(call, steps)
        plan.set_graphs(False)
        plan.profile(True)
        for _ in range(steps):
            call()
        tim = plan.timers()
        plan.profile(False)
        nc = max(tim["contract"][1], 1)
        t_c = tim["contract"][0] / nc * 1e-3
        per_call = tim["contract"][1] / steps
        achieved = info["flops_alg_hs"] / per_call / t_c
        out[name] = {
            "n_fn": info["n_fn"], "max_batch_fn": info["max_batch_fn"], "store_len": info["store_len"],
            "ms": ms, "points_per_s": info["n_active"] / (ms * 1e-3), "plan_s": t_plan,
            "flops_alg": info["flops_alg_hs"],
            "launch": {"order": best[0], "persistent": best[1], "tune_ms": [[list(s_), t] for s_, t in tune]},
            "kernels_ms_per_call": {k: v_[0] / steps for k, v_ in tim.items() if v_[1]},
            "roofline": {"kernel": "k_contract_hs", "bound": "mfma", "achieved": achieved / 1e12,
                         "peak": PEAK_F64 / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_F64,
                         "traffic": HS_TRAFFIC.get((hsha, name, int(wl.n_atoms), (best[0], best[1] > 0))),
                         "avg_launch_ms": t_c * 1e3, "launches_per_call": per_call},
        }
        log("H/S %s component: %d functions, %.3f ms per call, k_contract_hs %.1f%% of FP64 peak" %
            (name, info["n_fn"], ms, 100 * achieved / PEAK_F64))
        kept[name] = (plan, hs)
    if "large" in kept and "small" in kept:
        # scalar -> spinor transformation of both components' H and S (Eq. 33)
        (pl, hsl), (ps, hss) = kept["large"], kept["small"]
        h_sp, s_sp = q.new_spinor(pl, dev), q.new_spinor(pl, dev)
        call = lambda: q.q4c_spinor_transform(pl, ps, hsl, hss, h_sp, s_sp)
        call()
        ms = timed(call, steps)
        Ll, Ls = pl.info["store_len"], ps.info["store_len"]
        # algorithmic bytes: the two parts of both components read once, the two
        # complex spinor blocks (4 elements per scalar element) written once
        nbytes = 16.0 * (Ll + Ls) + 2 * 16.0 * 4 * Ll
        out["spinor_transform"] = {
            "ms": ms, "roofline": {"kernel": "k_spinor_transform", "bound": "hbm", "achieved": nbytes / (ms * 1e-3) / 1e9,
                                   "peak": 8000.0, "unit": "GB/s", "frac": nbytes / (ms * 1e-3) / 8e12,
                                   "bytes_alg": nbytes}}
        log("spinor transform: %.3f ms, %.0f GB/s algorithmic" % (ms, nbytes / (ms * 1e-3) / 1e9))
        # forward density update from a seeded spinor density matrix: the scalar
        # density matrices of both components, then n and grad n of each
        pairs_l, po_l = pl.pairs()
        d_host = np.zeros((4 * Ll, 2))
        for p_, blk in enumerate(W.spinor_density(wl_l, pairs_l, 5101)):
            c_ = np.asarray(blk).reshape(-1)
            d_host[4 * po_l[p_]:4 * po_l[p_ + 1], 0] = c_.real
            d_host[4 * po_l[p_]:4 * po_l[p_ + 1], 1] = c_.imag
        d_sp = torch.from_numpy(d_host).to(dev)
        cl = torch.empty(Ll, dtype=torch.float64, device=dev)
        cs = torch.empty(Ls, dtype=torch.float64, device=dev)
        gl = torch.empty((4, pl.info["n_points"]), dtype=torch.float64, device=dev)
        gs = torch.empty((4, ps.info["n_points"]), dtype=torch.float64, device=dev)

        def upd():
            q.q4c_spinor_density_to_scalar(pl, ps, d_sp, cl, cs)
            q.density_gradient_on_grid(pl, cl, gl)
            q.density_gradient_on_grid(ps, cs, gs)
        upd()
        ms_upd = timed(upd, steps)
        dens = {"ms": ms_upd, "points_per_s": pl.info["n_active"] / (ms_upd * 1e-3)}
        for cname, plan_, c_, g_ in (("large", pl, cl, gl), ("small", ps, cs, gs)):
            plan_.profile(True)
            for _ in range(steps):
                q.density_gradient_on_grid(plan_, c_, g_)
            tim = plan_.timers()
            plan_.profile(False)
            nt = max(tim["density_tiles"][1], 1)
            t_t = tim["density_tiles"][0] / nt * 1e-3
            per = tim["density_tiles"][1] / steps
            # sum_B 2 P n^2: the one symmetric product Y = C phi per batch that
            # n = phi^T C phi and grad n = 2 grad phi^T C phi need (flops_alg
            # counts 10 P n^2)
            f_alg = 0.2 * plan_.info["flops_alg"]
            ach = f_alg / per / t_t
            dens[cname] = {"kernels_ms_per_call": {k: v_[0] / steps for k, v_ in tim.items() if v_[1]},
                           "roofline": {"kernel": "k_grad_gemm", "bound": "mfma", "achieved": ach / 1e12,
                                        "peak": PEAK_F64 / 1e12, "unit": "TFLOP/s", "frac": ach / PEAK_F64,
                                        "avg_launch_ms": t_t * 1e3, "launches_per_call": per,
                                        "flops_alg_per_call": f_alg}}
        out["density_update"] = dens
        log("density update (D -> scalar, n and grad n of both components): %.3f ms" % ms_upd)
    kept.clear()
    if with_cpu:
        import oracle
        rng = np.random.default_rng(6102)
        idx = np.sort(rng.choice(wl.n_points, size=max(1, int(cpu_frac * wl.n_points)), replace=False))
        sub = wl_l.subset_points(idx)
        pairs = W.atom_pairs(wl_l)
        oracle.build()
        t0 = time.perf_counter()
        oracle.pair_blocks_hs(sub, pairs)
        dt = time.perf_counter() - t0
        out["cpu_oracle_large"] = {"value": idx.size / dt, "unit": "input points/s", "cores": oracle.max_threads(),
                                   "kind": "oracle",
                                   "sample": "%d of %d grid points (seed 6102), all %d atom pairs, %.2f s" %
                                             (idx.size, wl.n_points, len(pairs), dt)}
    return out


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def bench_molecules(a):
    """64 independent molecules: one batched plan (all systems' batches in the
    same launches, autotuned launch shapes, each call one HIP graph launch)
    against 64 per-molecule plans called one after another."""
    import numpy as np
    import torch
    import paper_2608_00773_amd as q
    import workload as W

    t0 = time.perf_counter()
    wl = W.config_molecules()
    systems = W.split_molecules(wl)
    log("workload: %d molecules, %d atoms, %d points (%.1f s)" % (len(systems), wl.n_atoms, wl.n_points,
                                                                    time.perf_counter() - t0))
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    pb = q.Plan(systems)
    t_plan_b = time.perf_counter() - t0
    log("batched plan: %s (%.1f s)" % (pb.info, t_plan_b))
    t0 = time.perf_counter()
    seq = [q.Plan(s, staging_bytes=2 << 30) for s in systems]
    t_plan_s = time.perf_counter() - t0
    log("64 sequential plans (%.1f s), scratch %.1f GiB in total" %
        (t_plan_s, sum(p.info["scratch_bytes"] for p in seq) / 2 ** 30))
    off = pb.systems()
    v = torch.from_numpy(np.concatenate([s.v for s in systems])).to(dev)
    rng = np.random.default_rng(5004)
    L = pb.info["store_len"]
    coef = torch.from_numpy(rng.standard_normal((5, L))).to(dev)
    st_b, sp_b = q.new_store(pb, dev), q.new_spinor(pb, dev)
    out_b = torch.empty(pb.info["n_points"], dtype=torch.float64, device=dev)
    st_s, sp_s = q.new_store(pb, dev), q.new_spinor(pb, dev)
    out_s = torch.empty_like(out_b)
    sl = [(int(off["store"][i]), int(off["store"][i + 1]), int(off["point"][i]), int(off["point"][i + 1]))
          for i in range(len(systems))]
    # per-molecule views of one set of buffers (contiguous slices)
    v_s = [v[g0:g1] for (_, _, g0, g1) in sl]
    coef_s = [coef[:, s0:s1].contiguous() for (s0, s1, _, _) in sl]
    st_m = [q.new_store(p, dev) for p in seq]
    sp_m = [sp_s[4 * s0:4 * s1] for (s0, s1, _, _) in sl]
    out_m = [out_s[g0:g1] for (_, _, g0, g1) in sl]

    def timed(fn, k):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    def seq_fwd():
        for i, p in enumerate(seq):
            q.q4c_integrate_H(p, v_s[i], q.PREC_F64, q.ASSEMBLE_W, st_m[i], sp_m[i])

    def seq_adj():
        for i, p in enumerate(seq):
            q.density_on_grid(p, coef_s[i], q.TERM_ALL, 1, out_m[i])

    fwd_b = lambda: q.q4c_integrate_H(pb, v, q.PREC_F64, q.ASSEMBLE_W, st_b, sp_b)
    adj_b = lambda: q.density_on_grid(pb, coef, q.TERM_ALL, 1, out_b)

    k = max(1, a.steps // 4)
    seq_fwd(); seq_adj()
    r = {"seq_forward_ms": timed(seq_fwd, k), "seq_adjoint_ms": timed(seq_adj, k)}
    log("sequential: %s" % r)
    fwd_b(); adj_b()
    r["batched_default_forward_ms"] = timed(fwd_b, k)
    r["batched_default_adjoint_ms"] = timed(adj_b, k)
    log("batched, default launch: %s" % r)
    t0 = time.perf_counter()
    table = pb.autotune(v, st_b, q.PREC_F64, coef, out_b, reps=3)
    t_tune = time.perf_counter() - t0
    log("autotune (%.1f s): %s" % (t_tune, table))
    pb.set_graphs(True)
    fwd_b(); adj_b()
    r["batched_forward_ms"] = timed(fwd_b, k)
    r["batched_adjoint_ms"] = timed(adj_b, k)
    torch.cuda.synchronize()
    same = all(torch.equal(st_b[:, s0:s1], st_m[i]) for i, (s0, s1, _, _) in enumerate(sl))
    same = same and torch.equal(sp_b, sp_s) and torch.equal(out_b, out_s)
    n_act = pb.info["n_active"]
    res = {
        "mode": "molecules",
        "workload": "%d independent molecules of %d..%d atoms (%d atoms, %d NAOs), %d points (%d active), "
                    "60 x 302 points per atom" % (len(systems), min(wl.meta["sizes"]), max(wl.meta["sizes"]),
                                                  wl.n_atoms, pb.info["n_fn"], wl.n_points, n_act),
        "unit": "active points/s",
        "sequential_forward_points_per_s": n_act / (r["seq_forward_ms"] * 1e-3),
        "batched_forward_points_per_s": n_act / (r["batched_forward_ms"] * 1e-3),
        "forward_speedup": r["seq_forward_ms"] / r["batched_forward_ms"],
        "sequential_step_points_per_s": n_act / ((r["seq_forward_ms"] + r["seq_adjoint_ms"]) * 1e-3),
        "batched_step_points_per_s": n_act / ((r["batched_forward_ms"] + r["batched_adjoint_ms"]) * 1e-3),
        "step_speedup": (r["seq_forward_ms"] + r["seq_adjoint_ms"]) / (r["batched_forward_ms"] +
                                                                        r["batched_adjoint_ms"]),
        "ms": r,
        "flops_alg_batched": pb.info["flops_alg"],
        "contract_tflops_alg_batched": pb.info["flops_alg"] / (r["batched_forward_ms"] * 1e-3) / 1e12,
        "batched_launch": {"contract": pb.get_launch(q.KERNEL_CONTRACT), "density": pb.get_launch(q.KERNEL_DENSITY),
                           "graphs": True},
        "autotune_table": table,
        "autotune_s": t_tune,
        "bitwise_equal_to_sequential": bool(same),
        "plan_s": {"batched": t_plan_b, "sequential": t_plan_s},
        "scratch_gib": {"batched": pb.info["scratch_bytes"] / 2 ** 30,
                        "sequential_total": sum(p.info["scratch_bytes"] for p in seq) / 2 ** 30},
        "steps": k,
    }
    print(json.dumps(res), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (requested --gpus %d)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    if a.workload == "molecules":
        bench_molecules(a)
        return
    import numpy as np
    import torch
    import paper_2608_00773_amd as q
    import workload as W

    t0 = time.perf_counter()
    if a.workload == "slab":
        wl = W.config_slab()
    elif a.workload == "pepi":
        wl = W.config_pepi_3383()
    elif a.workload == "periodic":
        wl = W.config_periodic(cells=(2, 2, 2), nrad=60, nang=302)
    else:
        wl = W.config_cluster(n_atoms=a.n_atoms)
    t_gen = time.perf_counter() - t0
    print("[bench] workload %s: %d atoms, %d points (%.1f s)" % (a.workload, wl.n_atoms, wl.n_points, t_gen),
          file=sys.stderr, flush=True)
    if a.mode == "hs":
        def timed_hs(fn, k):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(k):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / k
        if a.calib_copy_mib:
            n = a.calib_copy_mib * (1 << 20) // 8
            src = torch.ones(n, dtype=torch.float64, device="cuda")
            dst = torch.empty_like(src)
            torch.mul(src, 1.0, out=dst)
            torch.cuda.synchronize()
            del src, dst
        comps = ("large", "small") if a.hs_component == "both" else (a.hs_component,)
        kw = {}
        if a.hs_shape:
            kw["shapes"] = (tuple(int(t) for t in a.hs_shape.split(",")),)
        print(json.dumps({"mode": "hs", "hs": bench_hs(wl, timed_hs, a.steps, 0.0, False, comps, **kw)}),
              flush=True)
        return
    t0 = time.perf_counter()
    plan = q.Plan(wl)
    t_plan = time.perf_counter() - t0
    info = plan.info
    L = info["store_len"]
    dev = torch.device("cuda:0")
    v = torch.from_numpy(wl.v).to(dev)
    store = q.new_store(plan, dev)
    spin = q.new_spinor(plan, dev)
    rng = np.random.default_rng(5002)
    gbar = torch.from_numpy(rng.standard_normal((5, L))).to(dev)
    grad = torch.empty(wl.n_points, dtype=torch.float64, device=dev)
    prec = PREC[a.precision]

    def step(p):
        q.q4c_integrate_H(plan, v, p, q.ASSEMBLE_W, store, spin)
        q.density_on_grid(plan, gbar, q.TERM_ALL, 1, grad)

    tune = None
    if not a.no_autotune:
        # launch shapes of both contraction kernels picked on this plan (not timed);
        # every later call is one HIP graph launch
        t0 = time.perf_counter()
        tune = plan.autotune(v, store, prec, gbar, grad, reps=3)
        if a.contract_order is not None:
            rows = [t for t in tune if t[0] == q.KERNEL_CONTRACT and t[1] == a.contract_order]
            best = min(rows, key=lambda t: t[3])
            plan.set_launch(q.KERNEL_CONTRACT, best[1], best[2])
        plan.set_graphs(not a.no_graphs)
        print("[bench] autotune %.1f s: %s" % (time.perf_counter() - t0, tune), file=sys.stderr, flush=True)

    def timed(fn, k):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    def timed_each(fn, k, warm):
        """Milliseconds of each of k calls (HIP events on the current stream) after warm untimed ones."""
        for _ in range(warm):
            fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k)]
        torch.cuda.synchronize()
        for e0, e1 in ev:
            e0.record()
            fn()
            e1.record()
        torch.cuda.synchronize()
        return [e0.elapsed_time(e1) for e0, e1 in ev]

    if a.calib_copy_mib:
        n = a.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    if a.mode != "full":
        if a.mode == "forward":
            call = lambda: q.q4c_integrate_H(plan, v, prec, q.ASSEMBLE_W, store, spin)
        elif a.mode == "adjoint":
            call = lambda: q.density_on_grid(plan, gbar, q.TERM_ALL, 1, grad)
        else:
            call = lambda: step(prec)
        for _ in range(a.warmup):
            call()
        ms = timed(call, a.steps)
        print(json.dumps({"mode": a.mode, "precision": a.precision, "ms": ms, "steps": a.steps,
                          "points_per_s": info["n_active"] / (ms * 1e-3)}), flush=True)
        return

    for _ in range(a.warmup):
        step(prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_step = timed(lambda: step(prec), a.steps)
    wall = time.perf_counter() - t0
    print("[bench] %d steps of %.3f ms" % (a.steps, ms_step), file=sys.stderr, flush=True)

    # per-kernel times of the same step, HIP events on the launch stream
    plan.profile(True)
    for _ in range(a.steps):
        step(prec)
    tim = plan.timers()
    plan.profile(False)
    info = plan.info
    n_act = info["n_active"]
    ksha = source_sha("q4c_kernels.hip", "q4c_device.h")
    c_launch = plan.get_launch(q.KERNEL_CONTRACT)
    d_launch = plan.get_launch(q.KERNEL_DENSITY)
    c_shape = (c_launch[0], c_launch[1] > 0)  # work order, persistent
    d_shape = (d_launch[0], d_launch[1] > 0)
    wkey = "%s-%d" % (a.workload, wl.n_atoms)

    def kernel_roofline(name, timer, bound, work_per_step, peak, unit, shape=None):
        """achieved = algorithmic work of one launch / average launch time of
        the kernel (HIP events around each launch over the timed steps)."""
        n = max(tim[timer][1], 1)
        t = tim[timer][0] / n * 1e-3
        per_step = tim[timer][1] / a.steps
        work = work_per_step / max(per_step, 1e-300)
        scale = 1e12 if unit == "TFLOP/s" else 1e9
        return {"kernel": name, "bound": bound, "achieved": work / t / scale, "peak": peak / scale, "unit": unit,
                "frac": work / t / peak, "traffic": TRAFFIC.get((name, ksha, a.precision, wkey, shape)),
                "alg_per_launch": work, "avg_launch_ms": t * 1e3, "launches_per_step": per_step,
                "ms_per_step": tim[timer][0] / a.steps}

    rl = [
        kernel_roofline("k_contract", "contract", "mfma", info["flops_alg"], contraction_peak(a.precision),
                        "TFLOP/s", c_shape),
        kernel_roofline("k_density_tiles", "density_tiles", "mfma", info["flops_alg"], PEAK_F64, "TFLOP/s",
                        d_shape),
        # tabulation: 32 B (phi and its gradient, FP64) per (point, relevant function) per
        # tabulation of all passes; the adjoint tabulates only passes whose panels are not resident
        kernel_roofline("k_panel", "tabulate", "hbm",
                        32.0 * info["tab_elems"] * tim["tabulate"][1] / a.steps / max(info["n_passes"], 1),
                        PEAK_HBM, "GB/s"),
        # batch-to-global sum: the staged partial blocks read once, the five parts written once
        kernel_roofline("k_reduce", "reduce", "hbm", info["staging_bytes"] + 40.0 * info["store_len"], PEAK_HBM,
                        "GB/s"),
    ]
    dominant = max(rl, key=lambda r: r["ms_per_step"])

    # q4c_integrate_H alone (the metric's t_H): each precision, all five parts
    # and the W spinor, median of 20 calls timed one by one after 3 warm-ups;
    # error of each split mode against the FP64 path
    h_only, outs = {}, {}
    for name, p in PREC.items():
        st = q.new_store(plan, dev)
        call = lambda: q.q4c_integrate_H(plan, v, p, q.ASSEMBLE_W, st, spin)
        ms_list = timed_each(call, 20, 3)
        med = float(np.median(ms_list))
        h_only[name] = {"ms_median": med, "points_per_s": n_act / (med * 1e-3),
                        "gflops_alg": info["flops_alg"] / (med * 1e-3) / 1e9, "ms_min": float(np.min(ms_list))}
        outs[name] = st
    for name in h_only:
        h_only[name]["speedup_vs_f64"] = h_only["f64"]["ms_median"] / h_only[name]["ms_median"]
    err = {n: [float(torch.max(torch.abs(outs[n][k] - outs["f64"][k]))) for k in range(5)] for n in outs}
    ms_adj = float(np.median(timed_each(lambda: q.density_on_grid(plan, gbar, q.TERM_ALL, 1, grad), 20, 3)))
    ms_adj32 = float(np.median(timed_each(
        lambda: q.density_on_grid(plan, gbar, q.TERM_ALL, 1, grad, precision=q.PREC_F32), 20, 3)))

    # nao_tabulate (the ABI call; the same tabulation as the panels) over the
    # first quarter of the batches: FP64 phi and grad phi, 32 B written per
    # (point, relevant function), HIP events around each call
    nb_t = max(1, info["n_batches"] // 4)
    n_t = plan.tabulate_size(0, nb_t, 1)
    tab_out = torch.empty(n_t, dtype=torch.float64, device=dev)
    ms_tab = float(np.median(timed_each(lambda: q.nao_tabulate(plan, 0, nb_t, 1, tab_out), 10, 2)))
    del tab_out
    tab_bytes = 8.0 * n_t
    nao_tab = {"batches": nb_t, "ms_median": ms_tab, "bytes_alg": tab_bytes,
               "roofline": {"kernel": "k_tabulate", "bound": "hbm", "achieved": tab_bytes / (ms_tab * 1e-3) / 1e9,
                            "peak": PEAK_HBM / 1e9, "unit": "GB/s", "frac": tab_bytes / (ms_tab * 1e-3) / PEAK_HBM}}

    res = {
        "metric": METRIC,
        "value": n_act / (ms_step * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "split": "f32-hi/lo+f64", "f32": "f32+f64", "bf16x3": "bf16x3+f64",
                  "f64valu": "f64"}[a.precision],
        "data": "synthetic",
        "config": {
            "workload": "%s, %d atoms, %d NAOs, %d points (%d active), %d batches <= 300 pts" %
                        ({"cluster": "random cluster (Pb/I/H,C,N)", "slab": "perovskite-like slab",
                          "pepi": "(6x6)x2 perovskite-like slab",
                          "periodic": "periodic 2x2x2 CsPbBr3-like supercell (40 atoms) with its images"}[a.workload],
                         wl.n_atoms, info["n_fn"], info["n_points"], n_act, info["n_batches"]),
            "precision": a.precision,
            "step": "q4c_integrate_H (all parts + W spinor) + density_on_grid (adjoint, all terms)",
            "flops_alg_per_H": info["flops_alg"],
        },
        "roofline": {k: dominant[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel",
                                              "avg_launch_ms")},
        "roofline_kernels": rl,
        "h_only": h_only,
        "h_only_points_per_s": h_only[a.precision]["points_per_s"],
        "adjoint_ms_median": ms_adj,
        "adjoint_ms_median_f32": ms_adj32,
        "nao_tabulate": nao_tab,
        "launch": {"contract": plan.get_launch(q.KERNEL_CONTRACT), "density": plan.get_launch(q.KERNEL_DENSITY),
                   "graphs": tune is not None and not a.no_graphs, "autotune_table": tune},
        "kernels_ms_per_step": {k: v_[0] / a.steps for k, v_ in tim.items() if v_[1]},
        "staging_bytes_per_call": info["staging_bytes"],
        "max_abs_diff_vs_f64_Ha": {k: dict(zip(q.PART_NAMES, e)) for k, e in err.items() if k != "f64"},
        "plan_s": t_plan,
        "workload_gen_s": t_gen,
        "wall_timed_s": wall,
    }
    if a.workload == "periodic":
        # Bloch sums of the store at 8 seeded k-points (Sec. II C)
        m = wl.meta
        plan.set_cells(m["n_cell_atoms"], m["cell_atom"], m["shift"])
        cpa, cpo = plan.cell_pairs()
        B = 2 * np.pi * np.linalg.inv(m["lattice"]).T
        kp = np.random.default_rng(8601).uniform(-0.5, 0.5, size=(8, 3)) @ B.T
        bout = torch.empty((kp.shape[0], 5, int(cpo[-1]), 2), dtype=torch.float64, device=dev)
        q.q4c_integrate_H(plan, v, prec, 0, store)
        bl = lambda: q.q4c_bloch_sum(plan, 5, store, kp, bout)
        bl()
        nrep = max(3, a.steps // 4)
        ms_b = timed(bl, nrep)
        # k_bloch_sum alone (HIP events on the launch stream): algorithmic
        # bytes = the 5 store parts read once + the complex output written once
        plan.profile(True)
        for _ in range(nrep):
            bl()
        tim = plan.timers()
        plan.profile(False)
        k_ms = tim["bloch"][0] / max(1, tim["bloch"][1])
        alg_b = 8.0 * 5 * plan.info["store_len"] + 16.0 * kp.shape[0] * 5 * int(cpo[-1])
        res["bloch"] = {"n_k": int(kp.shape[0]), "ms_per_call": ms_b, "cell_atoms": int(m["n_cell_atoms"]),
                        "cell_pairs": int(len(cpa)), "cell_store_len": int(cpo[-1]),
                        "k_bloch_sum_ms": k_ms, "alg_bytes": alg_b,
                        "roofline": {"bound": "hbm", "achieved": alg_b / (k_ms * 1e-3) / 1e9, "peak": 8000.0,
                                     "unit": "GB/s", "frac": alg_b / (k_ms * 1e-3) / 1e9 / 8000.0}}
        log("Bloch sums: %d k-points x 5 parts x %d elements: %.3f ms per call, k_bloch_sum %.3f ms (%.0f GB/s alg.)"
            % (kp.shape[0], int(cpo[-1]), ms_b, k_ms, alg_b / (k_ms * 1e-3) / 1e9))
        # the reverse: one k-space density matrix part at the same k-points
        # (seeded values; the kernel's work does not depend on them) to
        # coefficients on the stored image pairs.  Algorithmic bytes: rho read
        # once + the coefficients written once.
        rho = torch.from_numpy(np.random.default_rng(8602).standard_normal((kp.shape[0], 1, int(cpo[-1]), 2))).to(dev)
        kw = np.full(kp.shape[0], 1.0 / kp.shape[0])
        coef_k = torch.empty((1, plan.info["store_len"]), dtype=torch.float64, device=dev)
        bd = lambda: q.q4c_bloch_density(plan, 1, rho, kp, kw, coef_k)
        bd()
        ms_d = timed(bd, nrep)
        plan.profile(True)
        for _ in range(nrep):
            bd()
        tim = plan.timers()
        plan.profile(False)
        kd_ms = tim["bloch"][0] / max(1, tim["bloch"][1])
        alg_d = 16.0 * kp.shape[0] * int(cpo[-1]) + 8.0 * plan.info["store_len"]
        res["bloch"]["density_matrix"] = {
            "ms_per_call": ms_d, "k_bloch_density_ms": kd_ms, "alg_bytes": alg_d,
            "reads_per_k_bytes": 16.0 * plan.info["store_len"],
            "roofline": {"bound": "hbm", "achieved": alg_d / (kd_ms * 1e-3) / 1e9, "peak": 8000.0, "unit": "GB/s",
                         "frac": alg_d / (kd_ms * 1e-3) / 1e9 / 8000.0}}
        log("Bloch density matrix: %d k-points -> %d stored elements: %.3f ms per call, k_bloch_density %.3f ms"
            % (kp.shape[0], plan.info["store_len"], ms_d, kd_ms))
    if not a.no_hs and a.workload == "cluster":
        res["hs"] = bench_hs(wl, timed, a.steps, 0.2 * a.cpu_sample, not a.no_cpu_baseline)
    if not a.no_cpu_baseline and a.workload == "cluster":
        res["cpu_baseline"] = cpu_baseline(wl, plan, gbar, a.cpu_sample, 0.1 * a.cpu_sample)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
