"""GPU parity of the forward density update from a spinor density matrix:
q4c_spinor_density_to_scalar (the scalar density matrices of both components)
and density_gradient_on_grid (n and grad n), against the oracle.

Bars: the reverse transform per element <= 1e-14 of sum f |G| |D| |G|;
n and grad n at points <= 1e-12 of the largest |value| of that column over the
checked points (FP64 sums of products of the same magnitudes).  End to end on
the GPU: sum_g w_g n_g = Re sum D_mu,nu S+_mu,nu (the density convention
n = Re sum D_mu,nu chi*_mu chi_nu integrated) with S+ from q4c_integrate_HS and
q4c_spinor_transform.  A cloud of one-function atoms takes the gradient
kernels' paths for tiles that span many atoms."""
import numpy as np
import pytest

import oracle
import workload as W
from helpers import gpu_available, per_point_worst, spinor_from_blocks

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_2608_00773_amd as q4c
    return q4c


def _env(q, wl, seed_d):
    import torch
    ws = W.small_component(wl, 7002)
    pl, ps = q.Plan(wl), q.Plan(ws)
    pairs, po = pl.pairs()
    _, pos = ps.pairs()
    D = W.spinor_density(wl, pairs, seed_d)
    d = torch.from_numpy(spinor_from_blocks(D, po)).cuda()
    cl = torch.full((pl.info["store_len"],), float("nan"), dtype=torch.float64, device="cuda")
    cs = torch.full((ps.info["store_len"],), float("nan"), dtype=torch.float64, device="cuda")
    q.q4c_spinor_density_to_scalar(pl, ps, d, cl, cs)
    torch.cuda.synchronize()
    return dict(wl=wl, ws=ws, pl=pl, ps=ps, pairs=pairs, po=po, pos=pos, D=D, d=d, cl=cl, cs=cs)


@pytest.fixture(scope="module")
def small(q):
    return _env(q, W.with_ket(W.config_small(), 7001), 5001)


@pytest.fixture(scope="module")
def medium(q):
    return _env(q, W.with_ket(W.config_cluster(n_atoms=24, nrad=24, nang=50, box_ang=9.0, k=7), 7011), 5007)


@pytest.mark.parametrize("case", ["small", "medium"])
def test_reverse_transform_against_oracle(q, case, request):
    e = request.getfixturevalue(case)
    GL, GS = oracle.spinor_G(e["wl"], e["ws"])
    ref = oracle.spinor_density_to_scalar(e["pairs"], e["D"], GL, GS)
    scale = oracle.spinor_density_to_scalar(e["pairs"], [np.abs(x) for x in e["D"]],
                                            [np.abs(g) for g in GL], [np.abs(g) for g in GS])
    got = (e["cl"].cpu().numpy(), e["cs"].cpu().numpy())
    nfn = (e["wl"].atom_nfn(), e["ws"].atom_nfn())
    offs = (e["po"], e["pos"])
    worst = 0.0
    for p, (a, b) in enumerate(e["pairs"]):
        for c in range(2):
            g = got[c][offs[c][p]:offs[c][p + 1]].reshape(int(nfn[c][a]), int(nfn[c][b]))
            worst = max(worst, float(np.max(np.abs(g - ref[p][c]) / (1e-14 * scale[p][c] + 1e-300))))
    print("%s: worst |d| / bar = %.3g" % (case, worst), flush=True)
    assert worst <= 1.0


def _grad(q, plan, coef, npts):
    import torch
    out = torch.full((4, npts), float("nan"), dtype=torch.float64, device="cuda")
    q.density_gradient_on_grid(plan, coef, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("case", ["small", "medium"])
def test_density_gradient_against_oracle(q, case, request):
    e = request.getfixturevalue(case)
    rng = np.random.default_rng(8301)
    for c, (wl, plan, coef, offs) in enumerate(((e["wl"], e["pl"], e["cl"], e["po"]),
                                                 (e["ws"], e["ps"], e["cs"], e["pos"]))):
        got = _grad(q, plan, coef, wl.n_points)
        idx = np.arange(wl.n_points) if case == "small" else np.sort(rng.choice(wl.n_points, 400, replace=False))
        if case == "small":
            idx = idx[::3]
        nfn = wl.atom_nfn()
        cb = coef.cpu().numpy()
        blocks = [cb[offs[p]:offs[p + 1]].reshape(int(nfn[a]), int(nfn[b])) for p, (a, b) in enumerate(e["pairs"])]
        ref, sref = oracle.density_grad(wl, e["pairs"], blocks, idx=idx, with_scale=True)
        for k in range(4):
            worst = per_point_worst(got[k, idx], ref[:, k], sref[:, k])
            print("%s comp %d col %d: worst |d| / own scale %.3g" % (case, c, k, worst), flush=True)
            assert worst <= 1e-12


def test_density_equals_adjoint_ll_and_repeats(q, small):
    """n from density_gradient_on_grid equals density_on_grid's LL term with the
    same coefficients; repeated calls and every launch shape give the same bits."""
    import torch
    e = small
    plan, wl = e["pl"], e["wl"]
    a = _grad(q, plan, e["cl"], wl.n_points)
    coef5 = torch.zeros((5, plan.info["store_len"]), dtype=torch.float64, device="cuda")
    coef5[0] = e["cl"]
    n = torch.empty(wl.n_points, dtype=torch.float64, device="cuda")
    q.density_on_grid(plan, coef5, q.TERM_LL, 0, n)
    torch.cuda.synchronize()
    n = n.cpu().numpy()
    # both within 1e-12 of each point's own scale of the oracle (the sum of
    # the magnitudes of the terms of n there)
    nfn = wl.atom_nfn()
    cb = e["cl"].cpu().numpy()
    blocks = [cb[e["po"][p]:e["po"][p + 1]].reshape(int(nfn[i]), int(nfn[j])) for p, (i, j) in enumerate(e["pairs"])]
    _, sref = oracle.density_grad(wl, e["pairs"], blocks, idx=np.arange(wl.n_points), with_scale=True)
    assert per_point_worst(a[0], n, 2e-12 * sref[:, 0]) <= 1.0
    assert np.array_equal(a, _grad(q, plan, e["cl"], wl.n_points))
    for shape in ((1, 0), (0, 512), (1, 512)):
        plan.set_launch(q.KERNEL_DENSITY, *shape)
        assert np.array_equal(a, _grad(q, plan, e["cl"], wl.n_points)), shape
    plan.set_launch(q.KERNEL_DENSITY, 0, 0)


@pytest.mark.parametrize("case", ["small", "medium"])
def test_electron_count_end_to_end_on_gpu(q, case, request):
    import torch
    e = request.getfixturevalue(case)
    wl, ws = e["wl"], e["ws"]
    nl = _grad(q, e["pl"], e["cl"], wl.n_points)[0]
    ns = _grad(q, e["ps"], e["cs"], ws.n_points)[0]
    lhs = float(np.sum(wl.w * (nl + ns)))
    hs = []
    for w, plan in ((wl, e["pl"]), (ws, e["ps"])):
        plan.set_ket_potential(w)
        h = q.new_hs(plan)
        q.q4c_integrate_HS(plan, torch.from_numpy(w.v).cuda(), 0, h)
        hs.append(h)
    hp, sp = q.new_spinor(e["pl"]), q.new_spinor(e["pl"])
    q.q4c_spinor_transform(e["pl"], e["ps"], hs[0], hs[1], hp, sp)
    torch.cuda.synchronize()
    s = sp.cpu().numpy()
    s = s[:, 0] + 1j * s[:, 1]
    rhs = 0.0
    for p, (a, b) in enumerate(e["pairs"]):
        blk = s[4 * e["po"][p]:4 * e["po"][p + 1]]
        rhs += (1.0 if a == b else 2.0) * float(np.real(np.sum(e["D"][p].reshape(-1) * blk)))
    print("%s: sum w n = %.15g, Re sum D S+ = %.15g" % (case, lhs, rhs), flush=True)
    assert abs(lhs - rhs) <= 1e-11 * float(np.sum(wl.w * (np.abs(nl) + np.abs(ns))))


def test_density_gradient_single_function_atoms(q):
    """100 atoms with one s function each in an 8 angstrom cube: every function
    is its own slot, so a 64 x 64 tile of a batch's coefficient matrix spans up
    to 64 x 64 slot pairs (beyond the LDS pair-offset table: the global lookup
    path), and batches hold up to 100 functions (several function tiles,
    ragged).  n and grad n at sampled points against the oracle, same bar."""
    import torch
    rng = np.random.default_rng(8311)
    nat = 100
    R = rng.uniform(0.0, 8.0 * W.ANGSTROM, size=(nat, 3))
    shells = [[(0, (0.3, 1.0, 4.0), (0.5, 0.4, 0.3))] for _ in range(nat)]
    wl = W.pin_workload(np.ones(nat, dtype=np.int32), R, shells, nrad=12, ntheta=4, nphi=8, nint=512,
                        name="s-cloud")
    plan = q.Plan(wl)
    _, _, fo, _ = plan.batches()
    assert np.max(np.diff(fo)) > 64
    pairs, po = plan.pairs()
    coef = np.random.default_rng(8312).standard_normal(plan.info["store_len"])
    got = _grad(q, plan, torch.from_numpy(coef).cuda(), wl.n_points)
    idx = np.sort(rng.choice(wl.n_points, 300, replace=False))
    nfn = wl.atom_nfn()
    blocks = [coef[po[p]:po[p + 1]].reshape(int(nfn[a]), int(nfn[b])) for p, (a, b) in enumerate(pairs)]
    ref, sref = oracle.density_grad(wl, pairs, blocks, idx=idx, with_scale=True)
    for k in range(4):
        worst = per_point_worst(got[k, idx], ref[:, k], sref[:, k])
        print("s-cloud col %d: worst |d| / own scale %.3g" % (k, worst), flush=True)
        assert worst <= 1e-12
