"""GPU parity of q4c_spinor_transform (Eq. 33: H+ and S+ in the (kappa, m_j)
spinor basis from the large- and small-component H and S) against the oracle.

* Whole pipeline on the 3-atom case: q4c_integrate_HS of both components,
  then the transform, against the oracle's H/S blocks transformed by the
  oracle; bar 1e-12 of the propagated error scale sum |G| A |G| (+1e-300).
* The transform alone, on the GPU's own H/S (24-atom multi-tile case, all
  pairs; the 120-atom cluster, sampled pairs): against the oracle's transform
  of the same inputs; bar 1e-14 of sum |G| |X| |G|.
* Plans that do not pair are rejected."""
import numpy as np
import pytest

import oracle
import workload as W
from helpers import gpu_available

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def q():
    if not gpu_available():
        pytest.skip("no GPU")
    import paper_2608_00773_amd as q4c
    return q4c


def _hs(q, wl):
    import torch
    plan = q.Plan(wl)
    plan.set_ket_potential(wl)
    hs = q.new_hs(plan)
    q.q4c_integrate_HS(plan, torch.from_numpy(wl.v).cuda(), 0, hs)
    return plan, hs


def _transform(q, pl, ps, hsl, hss):
    import torch
    h = q.new_spinor(pl)
    s = q.new_spinor(pl)
    h.fill_(float("nan"))
    s.fill_(float("nan"))
    q.q4c_spinor_transform(pl, ps, hsl, hss, h, s)
    torch.cuda.synchronize()
    h, s = h.cpu().numpy(), s.cpu().numpy()
    return h[:, 0] + 1j * h[:, 1], s[:, 0] + 1j * s[:, 1]


def _blocks(st, pairs, po, nfn):
    return [st[:, po[p]:po[p + 1]].reshape(2, int(nfn[a]), int(nfn[b])) for p, (a, b) in enumerate(pairs)]


def _spinor_blocks(h, s, pairs, po, nfn):
    out = []
    for p, (a, b) in enumerate(pairs):
        na, nb = 2 * int(nfn[a]), 2 * int(nfn[b])
        sl = slice(4 * po[p], 4 * po[p + 1])
        out.append(np.stack([h[sl].reshape(na, nb), s[sl].reshape(na, nb)]))
    return out


def _check(got, ref, scale, tol, floor=1e-300):
    worst = 0.0
    for g, r, sc in zip(got, ref, scale):
        err = np.abs(g - r)
        worst = max(worst, float(np.max(err / (tol * sc + floor))))
    print("worst |d| / (tol scale + floor) = %.3g" % worst, flush=True)
    assert worst <= 1.0


def test_pipeline_small_against_oracle(q):
    wl = W.with_ket(W.config_small(), 7001)
    ws = W.small_component(wl, 7002)
    pl, hsl = _hs(q, wl)
    ps, hss = _hs(q, ws)
    h, s = _transform(q, pl, ps, hsl, hss)
    pairs, po = pl.pairs()
    GL, GS = oracle.spinor_G(wl, ws)
    refl, scl = oracle.pair_blocks_hs(wl, pairs, with_abs=True)
    refs, scs = oracle.pair_blocks_hs(ws, pairs, with_abs=True)
    ref = oracle.spinor_transform(pairs, refl, refs, GL, GS)
    aGL = [np.abs(g) for g in GL]
    aGS = [np.abs(g) for g in GS]
    scale = [np.abs(x) for x in oracle.spinor_transform(pairs, scl, scs, aGL, aGS)]
    got = _spinor_blocks(h, s, pairs, po, wl.atom_nfn())
    _check(got, ref, scale, 1e-12)


def _transform_only(q, wl, ws, sel=None):
    pl, hsl = _hs(q, wl)
    ps, hss = _hs(q, ws)
    h, s = _transform(q, pl, ps, hsl, hss)
    pairs, po = pl.pairs()
    _, pos = ps.pairs()
    bl = _blocks(hsl.cpu().numpy(), pairs, po, wl.atom_nfn())
    bs = _blocks(hss.cpu().numpy(), pairs, pos, ws.atom_nfn())
    idx = np.arange(len(pairs)) if sel is None else sel
    GL, GS = oracle.spinor_G(wl, ws)
    ref = oracle.spinor_transform(pairs[idx], [bl[i] for i in idx], [bs[i] for i in idx], GL, GS)
    scale = [np.abs(x) for x in oracle.spinor_transform(
        pairs[idx], [np.abs(bl[i]) for i in idx], [np.abs(bs[i]) for i in idx],
        [np.abs(g) for g in GL], [np.abs(g) for g in GS])]
    got = _spinor_blocks(h, s, pairs, po, wl.atom_nfn())
    _check([got[i] for i in idx], ref, scale, 1e-14)
    return pl, ps


def test_transform_only_multitile(q):
    wl = W.with_ket(W.config_cluster(n_atoms=24, nrad=24, nang=50, box_ang=9.0, k=7), 7011)
    ws = W.small_component(wl, 7012)
    _transform_only(q, wl, ws)


def test_transform_only_fullsize_cluster_sampled(q):
    wl = W.with_ket(W.config_cluster(), 7101)
    ws = W.small_component(wl, 7102)
    npair = len(W.atom_pairs(wl))
    sel = np.sort(np.random.default_rng(8101).choice(npair, size=40, replace=False))
    _transform_only(q, wl, ws, sel)


def test_unpaired_plans_rejected(q):
    import torch
    wl = W.with_ket(W.config_small(), 7001)
    ws = W.small_component(wl, 7002)
    pl, hsl = _hs(q, wl)
    ps, hss = _hs(q, ws)
    h, s = q.new_spinor(pl), q.new_spinor(pl)
    # the large plan given as its own small partner: shells do not pair
    with pytest.raises(q.Q4CError) as e:
        q.q4c_spinor_transform(pl, pl, hsl, hsl, h, s)
    assert e.value.status == q.Q4C_EINVAL
    # other atoms: a different system
    wo = W.small_component(W.with_ket(W.config_small(nrad=20, nang=50).translated([0.3, 0.0, 0.0]), 7001), 7002)
    po_, hso = _hs(q, wo)
    with pytest.raises(q.Q4CError) as e:
        q.q4c_spinor_transform(pl, po_, hsl, hso, h, s)
    assert e.value.status == q.Q4C_EINVAL
    # the right partner still works after the rejections
    q.q4c_spinor_transform(pl, ps, hsl, hss, h, s)
    torch.cuda.synchronize()
    assert torch.isfinite(h).all() and torch.isfinite(s).all()
