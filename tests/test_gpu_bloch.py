"""GPU parity of q4c_bloch_sum (Bloch sums of unit-cell integrals, Sec. II C)
for periodic cells whose plans hold the cell's atoms and their images.

* One Pb atom per cubic cell (small basis): the W-path store integrated on
  the GPU and summed at seeded k-points, against the oracle's Bloch sum of the
  oracle's pair blocks; bar 1e-12 of the summed error scales (+1e-300).
* The CsPbBr3-like cell: the Bloch sums of the GPU's own W-path store (5
  parts) and H/S store (2 parts) against the oracle's sum of the same blocks;
  bar 1e-14 of sum |terms|; k -> k + G on the GPU.
* 70 k-points (the k chunking) and 1-, 2- and 5-part sums.
* q4c_bloch_density (k-space density matrices to coefficients on the image
  pairs) against the oracle's (3 and 70 k-points, both cell-atom orders), end
  to end with density_gradient_on_grid against explicit Bloch states, and the
  energy identity with q4c_bloch_sum on the CsPbBr3-like cell."""
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


def _kpoints(wl, n, seed):
    B = 2 * np.pi * np.linalg.inv(wl.meta["lattice"]).T
    return np.random.default_rng(seed).uniform(-0.5, 0.5, size=(n, 3)) @ B.T


def _run(q, wl, n_parts, kp, hs=False):
    import torch
    plan = q.Plan(wl)
    m = wl.meta
    plan.set_cells(m["n_cell_atoms"], m["cell_atom"], m["shift"])
    v = torch.from_numpy(wl.v).cuda()
    if hs:
        plan.set_ket_potential(wl)
        st = q.new_hs(plan)
        q.q4c_integrate_HS(plan, v, 0, st)
    else:
        st = q.new_store(plan)
        q.q4c_integrate_H(plan, v, q.PREC_F64, 0, st)
    cpa, cpo = plan.cell_pairs()
    out = torch.full((kp.shape[0], n_parts, int(cpo[-1]), 2), float("nan"), dtype=torch.float64, device="cuda")
    q.q4c_bloch_sum(plan, n_parts, st, kp, out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return plan, st.cpu().numpy(), cpa, cpo, o[..., 0] + 1j * o[..., 1]


def _cell_blocks(o, cpa, cpo, nc):
    return {(int(a), int(b)): o[:, :, cpo[c]:cpo[c + 1]].reshape(o.shape[0], o.shape[1], nc[a], nc[b])
            for c, (a, b) in enumerate(cpa)}


def _abs_scale(m, pairs, abs_blocks):
    """sum over contributions of |term| per element at k = 0: one part at a
    time, so that no orientation sign enters (with the signs of the
    spin-orbit parts, the two orientations of a pair of distinct images of
    one cell atom cancel on the diagonal of the (a, a) block)."""
    n_parts = abs_blocks[0].shape[0]
    per = [oracle.bloch_sum(m["cell_atom"], m["shift"], pairs, [x[q:q + 1] for x in abs_blocks], np.zeros((1, 3)))
           for q in range(n_parts)]
    return {key: np.concatenate([per[q][key][0].real for q in range(n_parts)], axis=0) for key in per[0]}


def _ncell(wl):
    nfn, ca = wl.atom_nfn(), wl.meta["cell_atom"]
    return [int(nfn[list(ca).index(c)]) for c in range(wl.meta["n_cell_atoms"])]


def test_pb_cell_end_to_end(q):
    wl = W.config_periodic(species=((82, (0.0, 0.0, 0.0)),), a_ang=4.0, recipe="small", nrad=20, nang=50, k=61)
    kp = _kpoints(wl, 4, 8501)
    plan, _, cpa, cpo, o = _run(q, wl, 5, kp)
    pairs, _ = plan.pairs()
    ref_b, sc_b = oracle.pair_blocks(wl, pairs, with_abs=True)
    m = wl.meta
    ref = oracle.bloch_sum(m["cell_atom"], m["shift"], pairs, ref_b, kp)
    sc = _abs_scale(m, pairs, sc_b)
    got = _cell_blocks(o, cpa, cpo, _ncell(wl))
    worst = 0.0
    for key, g in got.items():
        bound = 1e-12 * sc[key][None] + 1e-300
        worst = max(worst, float(np.max(np.abs(g - ref[key]) / bound)))
    print("worst |d| / bar = %.3g" % worst, flush=True)
    assert worst <= 1.0


def test_k_chunks_and_part_counts(q):
    """70 k-points (one full 64-point phase chunk plus a ragged one, ragged
    8-point register passes) and the 1- and 2-part sums of a W store, against
    the oracle's sum of the GPU's own blocks."""
    import torch
    wl = W.config_periodic(species=((82, (0.0, 0.0, 0.0)),), a_ang=4.0, recipe="small", nrad=14, nang=26, k=63)
    kp = _kpoints(wl, 70, 8503)
    plan, st, cpa, cpo, o5 = _run(q, wl, 5, kp)
    pairs, po = plan.pairs()
    nfn = wl.atom_nfn()
    m = wl.meta
    nc = _ncell(wl)
    for n_parts in (5, 2, 1):
        blocks = [st[:n_parts, po[p]:po[p + 1]].reshape(n_parts, int(nfn[a]), int(nfn[b]))
                  for p, (a, b) in enumerate(pairs)]
        if n_parts == 5:
            o = o5
        else:
            out = torch.full((kp.shape[0], n_parts, int(cpo[-1]), 2), float("nan"), dtype=torch.float64, device="cuda")
            q.q4c_bloch_sum(plan, n_parts, torch.from_numpy(st).cuda(), kp, out)
            torch.cuda.synchronize()
            o = out.cpu().numpy()
            o = o[..., 0] + 1j * o[..., 1]
            # the leading parts do not depend on how many parts are summed
            assert np.array_equal(o, o5[:, :n_parts])
        ref = oracle.bloch_sum(m["cell_atom"], m["shift"], pairs, blocks, kp)
        sc = _abs_scale(m, pairs, [np.abs(x) for x in blocks])
        got = _cell_blocks(o, cpa, cpo, nc)
        worst = max(float(np.max(np.abs(g - ref[key]) / (1e-14 * sc[key][None] + 1e-300))) for key, g in got.items())
        print("n_parts %d, %d k-points: worst |d| / bar = %.3g" % (n_parts, kp.shape[0], worst), flush=True)
        assert worst <= 1.0


@pytest.mark.parametrize("hs", [False, True])
def test_perovskite_cell_against_oracle_sum(q, hs):
    wl = W.config_periodic(nrad=24, nang=50)
    if hs:
        wl = W.with_ket(wl, 7201)
    n_parts = 2 if hs else 5
    kp = _kpoints(wl, 3, 8502)
    plan, st, cpa, cpo, o = _run(q, wl, n_parts, kp, hs=hs)
    pairs, po = plan.pairs()
    nfn = wl.atom_nfn()
    blocks = [st[:n_parts, po[p]:po[p + 1]].reshape(n_parts, int(nfn[a]), int(nfn[b]))
              for p, (a, b) in enumerate(pairs)]
    m = wl.meta
    ref = oracle.bloch_sum(m["cell_atom"], m["shift"], pairs, blocks, kp)
    sc = _abs_scale(m, pairs, [np.abs(x) for x in blocks])
    got = _cell_blocks(o, cpa, cpo, _ncell(wl))
    assert set(got) == set(ref)
    worst = 0.0
    for key, g in got.items():
        worst = max(worst, float(np.max(np.abs(g - ref[key]) / (1e-14 * sc[key][None] + 1e-300))))
    print("hs=%s: %d cell pairs, worst |d| / bar = %.3g" % (hs, len(got), worst), flush=True)
    assert worst <= 1.0
    # k -> k + G on the GPU
    import torch
    G = 2 * np.pi * np.linalg.inv(m["lattice"]).T @ np.array([2.0, -1.0, 1.0])
    out = torch.empty((kp.shape[0], n_parts, int(cpo[-1]), 2), dtype=torch.float64, device="cuda")
    q.q4c_bloch_sum(plan, n_parts, torch.from_numpy(st).cuda(), kp + G[None, :], out)
    torch.cuda.synchronize()
    o2 = out.cpu().numpy()
    o2 = o2[..., 0] + 1j * o2[..., 1]
    # per element, against the sum of the magnitudes of its terms: the phases
    # of k + G differ from those of k by the rounding of arguments of a few
    # tens of radians
    got2 = _cell_blocks(o2, cpa, cpo, _ncell(wl))
    worst = max(float(np.max(np.abs(g - got[key]) / (1e-12 * sc[key][None] + 1e-300))) for key, g in got2.items())
    print("k -> k + G: worst |d| / bar = %.3g" % worst, flush=True)
    assert worst <= 1.0


# ---------------------------------------------------------------------------
# q4c_bloch_density: k-space density matrices -> coefficients on the stored
# image pairs (the periodic density matrix of Sec. II C)
# ---------------------------------------------------------------------------

def _pbn_cell():
    return W.config_periodic(species=((82, (0.0, 0.0, 0.0)), (7, (0.5, 0.5, 0.5))), a_ang=4.5, recipe="main",
                             nrad=10, nang=26, k=62)


def _states(wl, n_k, seed, nocc=4):
    m = wl.meta
    rng = np.random.default_rng(seed)
    nc = sum(_ncell(wl))
    C = rng.standard_normal((n_k, nc, nocc)) + 1j * rng.standard_normal((n_k, nc, nocc))
    f = rng.uniform(0.5, 2.0, size=nocc)
    kw = rng.uniform(0.2, 1.0, size=n_k)
    return _kpoints(wl, n_k, seed + 1), kw, C, f


def _rho_dev(q, plan, wl, C, f, n_parts=1):
    """rho(k) = sum_l f_l C*_l C_l^T of the cell's functions in the cell-pair
    layout (n_parts copies, the second scaled by 0.5) as a device tensor, and
    the oracle's {(a, b): blocks}."""
    import torch
    ncell = _ncell(wl)
    off = np.concatenate([[0], np.cumsum(ncell)])
    rho = np.einsum("l,kml,knl->kmn", f, C.conj(), C)
    cpa, cpo = plan.cell_pairs()
    n_k = C.shape[0]
    flat = np.zeros((n_k, n_parts, int(cpo[-1])), dtype=np.complex128)
    blocks = {}
    for c, (a, b) in enumerate(cpa):
        blk = rho[:, off[a]:off[a + 1], off[b]:off[b + 1]]
        stack = np.stack([blk * (1.0 if p == 0 else 0.5) for p in range(n_parts)], axis=1)
        blocks[(int(a), int(b))] = stack
        flat[:, :, cpo[c]:cpo[c + 1]] = stack.reshape(n_k, n_parts, -1)
    dev = torch.from_numpy(np.stack([flat.real, flat.imag], axis=-1).copy()).cuda()
    return dev, blocks


def _density_plan(q, wl):
    plan = q.Plan(wl)
    m = wl.meta
    plan.set_cells(m["n_cell_atoms"], m["cell_atom"], m["shift"])
    return plan


def _coef_scale(m, pairs, blocks, kw, nfn):
    """f sum_k |w_k| |rho| per stored element (the bound of every term)."""
    ab = {key: np.abs(v) for key, v in blocks.items()}
    return oracle.bloch_density(m["cell_atom"], m["shift"], pairs, ab, np.zeros((len(kw), 3)), np.abs(kw), nfn)


@pytest.mark.parametrize("n_k", [3, 70])
def test_density_matrix_against_oracle(q, n_k):
    """GPU coefficients against the oracle's on the Pb + N cell (both
    cell-atom orders among the image pairs); 70 k-points cross the 64-point
    phase chunk.  Bar 1e-14 of f sum_k w_k |rho| per element."""
    import torch
    wl = _pbn_cell()
    plan = _density_plan(q, wl)
    kp, kw, C, f = _states(wl, n_k, 8601)
    rho, blocks = _rho_dev(q, plan, wl, C, f, n_parts=2)
    L = plan.info["store_len"]
    out = torch.full((2, L), float("nan"), dtype=torch.float64, device="cuda")
    q.q4c_bloch_density(plan, 2, rho, kp, kw, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    pairs, po = plan.pairs()
    nfn = wl.atom_nfn()
    m = wl.meta
    ref = oracle.bloch_density(m["cell_atom"], m["shift"], pairs, blocks, kp, kw, nfn)
    sc = _coef_scale(m, pairs, blocks, kw, nfn)
    worst = 0.0
    for p in range(len(pairs)):
        g = got[:, po[p]:po[p + 1]].reshape(ref[p].shape)
        worst = max(worst, float(np.max(np.abs(g - ref[p]) / (1e-14 * sc[p] + 1e-300))))
    print("n_k %d: worst |d| / bar = %.3g" % (n_k, worst), flush=True)
    assert worst <= 1.0
    # one part at a time gives the same first part, bit for bit
    out1 = torch.full((1, L), float("nan"), dtype=torch.float64, device="cuda")
    q.q4c_bloch_density(plan, 1, rho[:, :1].contiguous(), kp, kw, out1)
    torch.cuda.synchronize()
    assert np.array_equal(out1.cpu().numpy()[0], got[0])


def test_density_matrix_no_kpoints_gives_zeros(q):
    import torch
    wl = _pbn_cell()
    plan = _density_plan(q, wl)
    out = torch.full((1, plan.info["store_len"]), float("nan"), dtype=torch.float64, device="cuda")
    q.q4c_bloch_density(plan, 1, None, np.zeros((0, 3)), np.zeros(0), out)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0


def test_periodic_density_end_to_end(q):
    """k-space density matrices -> q4c_bloch_density -> density_gradient_on_grid,
    all on the GPU, against n = sum_k w_k sum_l f_l |psi_lk|^2 and its
    gradient from explicit Bloch states at the grid points inside the cell box."""
    import torch
    wl = _pbn_cell()
    plan = _density_plan(q, wl)
    kp, kw, C, f = _states(wl, 3, 8611)
    rho, _ = _rho_dev(q, plan, wl, C, f)
    L = plan.info["store_len"]
    coef = torch.empty((1, L), dtype=torch.float64, device="cuda")
    q.q4c_bloch_density(plan, 1, rho, kp, kw, coef)
    out = torch.empty((4, wl.n_points), dtype=torch.float64, device="cuda")
    q.density_gradient_on_grid(plan, coef[0], out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().T
    m = wl.meta
    pts = np.stack([wl.x, wl.y, wl.z], axis=1)
    frac = pts @ np.linalg.inv(m["lattice"])
    idx = np.nonzero(np.all((frac >= 0.0) & (frac < 1.0), axis=1))[0]
    phi, grad = oracle.tabulate(wl, wl.x[idx], wl.y[idx], wl.z[idx])
    nfn = wl.atom_nfn()
    ca, sh = m["cell_atom"], m["shift"]
    coff = np.concatenate([[0], np.cumsum(_ncell(wl))])
    ref = np.zeros((idx.size, 4))
    for ik, k in enumerate(kp):
        psi = np.zeros((idx.size, C.shape[2]), dtype=np.complex128)
        dpsi = np.zeros((idx.size, C.shape[2], 3), dtype=np.complex128)
        f0 = 0
        for A in range(wl.n_atoms):
            a, n = int(ca[A]), int(nfn[A])
            ph = np.exp(1j * (k @ sh[A]))
            Cc = C[ik, coff[a]:coff[a] + n, :]
            psi += ph * phi[:, f0:f0 + n] @ Cc
            dpsi += ph * np.einsum("gic,il->glc", grad[:, f0:f0 + n, :], Cc)
            f0 += n
        ref[:, 0] += kw[ik] * np.einsum("l,gl->g", f, np.abs(psi) ** 2)
        ref[:, 1:] += kw[ik] * 2.0 * np.einsum("l,gl,glc->gc", f, psi.conj(), dpsi).real
    sc = np.max(np.abs(ref), axis=0)
    errs = [float(np.max(np.abs(got[idx, c] - ref[:, c])) / sc[c]) for c in range(4)]
    print("%d in-box points: relative errors n, grad n = %s" % (idx.size, ["%.2e" % e for e in errs]), flush=True)
    assert max(errs) <= 1e-11


def test_density_matrix_energy_identity_on_perovskite(q):
    """sum over stored elements of q4c_bloch_density's coefficients times a
    GPU H store equals sum_k w_k sum over all cell function pairs
    rho_mn(k) H_mn(k) with H(k) from q4c_bloch_sum on the same store: the
    two periodic kernels are each other's adjoint (CsPbBr3-like cell)."""
    import torch
    wl = W.with_ket(W.config_periodic(nrad=24, nang=50), 7202)
    plan = _density_plan(q, wl)
    plan.set_ket_potential(wl)
    hs = q.new_hs(plan)
    q.q4c_integrate_HS(plan, torch.from_numpy(wl.v).cuda(), 0, hs)
    kp, kw, C, f = _states(wl, 5, 8621)
    rho, blocks = _rho_dev(q, plan, wl, C, f)
    L = plan.info["store_len"]
    coef = torch.empty((1, L), dtype=torch.float64, device="cuda")
    q.q4c_bloch_density(plan, 1, rho, kp, kw, coef)
    cpa, cpo = plan.cell_pairs()
    hk = torch.empty((kp.shape[0], 1, int(cpo[-1]), 2), dtype=torch.float64, device="cuda")
    q.q4c_bloch_sum(plan, 1, hs, kp, hk)
    torch.cuda.synchronize()
    e_r = float(torch.sum(coef[0] * hs[0]).item())
    hkn = hk.cpu().numpy()
    hkn = hkn[..., 0] + 1j * hkn[..., 1]
    rhon = rho.cpu().numpy()
    rhon = rhon[..., 0] + 1j * rhon[..., 1]
    e_k, scale = 0.0, 0.0
    for c, (a, b) in enumerate(cpa):
        t = np.einsum("k,ke,ke->", kw, rhon[:, 0, cpo[c]:cpo[c + 1]], hkn[:, 0, cpo[c]:cpo[c + 1]])
        e_k += t.real if a == b else 2.0 * t.real
        scale += (1.0 if a == b else 2.0) * float(np.einsum("k,ke,ke->", kw, np.abs(rhon[:, 0, cpo[c]:cpo[c + 1]]),
                                                             np.abs(hkn[:, 0, cpo[c]:cpo[c + 1]])))
    print("energy: image pairs %.12e, k space %.12e, scale %.3e" % (e_r, e_k, scale), flush=True)
    assert abs(e_r - e_k) <= 1e-13 * scale
