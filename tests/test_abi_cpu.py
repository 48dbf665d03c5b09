"""C-ABI checks that need no GPU: every function declared in include/q4c.h is
exported by libq4c.so, argument validation returns the documented status
codes, and the host-side plan (batching, relevance lists, pair layout) is
correct.  No kernel is launched."""
import ctypes
import os
import re

import numpy as np
import pytest

import workload as W
from helpers import ROOT

HEADER = os.path.join(ROOT, "include", "q4c.h")


def _lib():
    import paper_2608_00773_amd as q
    return q, q._load()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char)\s*\*?\s*([A-Za-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_three_calls():
    names = declared_functions()
    for n in ("nao_tabulate", "q4c_integrate_H", "density_on_grid", "q4c_plan_create", "q4c_plan_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    q, lib = _lib()
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert set(declared_functions()) == set(q.EXPORTS)


def test_status_strings():
    q, lib = _lib()
    for s in range(0, -9, -1):
        assert lib.q4c_status_string(s).decode() != "unknown status"


def _host_plan(q, wl, **kw):
    return q.Plan(wl, host_only=True, **kw)


def test_host_only_plan_and_nodev_errors():
    q, lib = _lib()
    wl = W.config_small(nrad=10, nang=26)
    p = _host_plan(q, wl)
    assert p.info["n_atoms"] == 3 and p.info["n_fn"] == 42
    assert p.info["device_bytes"] == 0
    rc = lib.q4c_integrate_H(p.handle, ctypes.c_void_p(1), 0, 7, 0, ctypes.c_void_p(1), None, None, None)
    assert rc == q.Q4C_ENODEV
    rc = lib.density_on_grid(p.handle, ctypes.c_void_p(1), 7, 0, 0, ctypes.c_void_p(1), None)
    assert rc == q.Q4C_ENODEV


def test_store_layout_matches_pairs_and_sizes():
    """q4c_store_layout (Sec. III A: locally indexed dense pair blocks): the
    pair list and offsets equal q4c_plan_pairs, the block shapes are the
    atoms' function counts, the byte sizes follow from store_len."""
    q, lib = _lib()
    wl = W.config_small(nrad=10, nang=26)
    p = _host_plan(q, wl)
    lay = p.store_layout()
    pairs, po = p.pairs()
    nfn = wl.atom_nfn()
    L = p.info["store_len"]
    assert lay["n_pairs"] == len(pairs) and lay["store_len"] == L
    assert np.array_equal(lay["pair_atoms"], pairs) and np.array_equal(lay["pair_off"], po)
    assert np.array_equal(lay["pair_nfn"], np.stack([nfn[pairs[:, 0]], nfn[pairs[:, 1]]], axis=1))
    assert np.array_equal(np.diff(po), lay["pair_nfn"][:, 0] * lay["pair_nfn"][:, 1])
    assert (lay["part_bytes"], lay["store_bytes"], lay["hs_bytes"], lay["spinor_bytes"]) == (8 * L, 40 * L, 16 * L,
                                                                                         64 * L)
    out = q._StoreLayout()
    assert lib.q4c_store_layout(p.handle, ctypes.byref(out), None, None, None) == q.Q4C_OK
    assert out.store_len == L
    assert lib.q4c_store_layout(p.handle, None, None, None, None) == q.Q4C_EINVAL


def test_integrate_part_selection_checks():
    """parts (Q4C_PART_*) must be a nonempty subset; spinor assembly needs its parts."""
    q, lib = _lib()
    p = _host_plan(q, W.config_small(nrad=10, nang=26))
    one = ctypes.c_void_p(1)
    call = lambda parts, flags: lib.q4c_integrate_H(p.handle, one, 0, parts, flags, one, one, one, None)
    assert call(0, 0) == q.Q4C_EINVAL
    assert call(8, 0) == q.Q4C_EINVAL
    assert call(q.PART_V | q.PART_WS, q.ASSEMBLE_W) == q.Q4C_EINVAL
    assert call(q.PART_WS | q.PART_WSO, q.ASSEMBLE_V) == q.Q4C_EINVAL
    for parts in (1, 2, 4, 3, 6, 7):
        assert call(parts, 0) == q.Q4C_ENODEV  # valid: fails only for want of device data
    assert call(7, q.ASSEMBLE_W | q.ASSEMBLE_V) == q.Q4C_ENODEV


def test_nao_tabulate_argument_checks():
    q, lib = _lib()
    wl = W.config_small(nrad=10, nang=26)
    p = _host_plan(q, wl)
    n = p.tabulate_size(0, 2, 1)
    buf = ctypes.c_void_p(1)
    assert lib.nao_tabulate(p.handle, 0, 2, 1, 7, buf, 8 * n, None) == q.Q4C_EINVAL  # unknown dtype
    for dt in (q.DTYPE_F64, q.DTYPE_F32_HILO):
        assert lib.nao_tabulate(p.handle, 0, 2, 1, dt, buf, 8 * n - 1, None) == q.Q4C_ESIZE
        assert lib.nao_tabulate(p.handle, 0, 2, 1, dt, buf, 8 * n, None) == q.Q4C_ENODEV
    assert lib.nao_tabulate(p.handle, 2, 1, 1, 0, buf, 8 * n, None) == q.Q4C_EINVAL


def test_argument_validation():
    q, lib = _lib()
    wl = W.config_small(nrad=10, nang=26)
    p = _host_plan(q, wl)
    # bad precision / flags / terms / weight mode are rejected before any device work
    assert lib.q4c_integrate_H(p.handle, ctypes.c_void_p(1), 7, 7, 0, ctypes.c_void_p(1), None, None, None) == q.Q4C_EINVAL
    assert lib.q4c_integrate_H(p.handle, ctypes.c_void_p(1), 0, 7, 1 << 10, ctypes.c_void_p(1), None, None,
                               None) == q.Q4C_EINVAL
    assert lib.q4c_integrate_H(p.handle, None, 0, 7, 0, ctypes.c_void_p(1), None, None, None) == q.Q4C_EINVAL
    assert lib.q4c_integrate_H(p.handle, ctypes.c_void_p(1), 0, 7, q.ASSEMBLE_W, ctypes.c_void_p(1), None, None,
                               None) == q.Q4C_EINVAL
    assert lib.density_on_grid(p.handle, ctypes.c_void_p(1), 0, 0, 0, ctypes.c_void_p(1), None) == q.Q4C_EINVAL
    assert lib.density_on_grid(p.handle, ctypes.c_void_p(1), 7, 0, 2, ctypes.c_void_p(1), None) == q.Q4C_EINVAL
    assert lib.density_on_grid(p.handle, ctypes.c_void_p(1), 7, q.PREC_SPLIT_F32, 1, ctypes.c_void_p(1), None) == q.Q4C_EINVAL
    assert lib.density_on_grid(p.handle, ctypes.c_void_p(1), 7, 9, 1, ctypes.c_void_p(1), None) == q.Q4C_EINVAL
    for prec in (q.PREC_BF16X3, q.PREC_F64_VALU):  # forward-only precisions
        assert lib.density_on_grid(p.handle, ctypes.c_void_p(1), 7, prec, 1, ctypes.c_void_p(1), None) == q.Q4C_EINVAL
    # every forward precision passes validation and then needs a device
    for prec in (q.PREC_F64, q.PREC_SPLIT_F32, q.PREC_F32, q.PREC_BF16X3, q.PREC_F64_VALU):
        assert lib.q4c_integrate_H(p.handle, ctypes.c_void_p(1), prec, 7, 0, ctypes.c_void_p(1), None, None,
                                   None) == q.Q4C_ENODEV
    assert lib.q4c_integrate_H(p.handle, ctypes.c_void_p(1), 5, 7, 0, ctypes.c_void_p(1), None, None,
                               None) == q.Q4C_EINVAL
    assert lib.q4c_integrate_H(None, ctypes.c_void_p(1), 0, 7, 0, ctypes.c_void_p(1), None, None, None) == q.Q4C_EINVAL
    n = ctypes.c_int64()
    assert lib.q4c_tabulate_size(p.handle, 0, p.info["n_batches"] + 1, 1, ctypes.byref(n)) == q.Q4C_EINVAL
    assert lib.q4c_tabulate_size(p.handle, 0, 1, 2, ctypes.byref(n)) == q.Q4C_EINVAL
    assert lib.nao_tabulate(p.handle, 0, 1, 1, 0, ctypes.c_void_p(1), 0, None) == q.Q4C_ESIZE


def test_unsupported_l_and_malformed_basis():
    q, lib = _lib()
    wl = W.config_small(nrad=10, nang=26)
    bad = W.Workload(**{**wl.__dict__})
    bad.shell_l = wl.shell_l.copy()
    bad.shell_l[0] = 5
    with pytest.raises(q.Q4CError) as e:
        _host_plan(q, bad)
    assert e.value.status == q.Q4C_EUNSUPPORTED
    bad2 = W.Workload(**{**wl.__dict__})
    bad2.atom_shell_off = wl.atom_shell_off.copy()
    bad2.atom_shell_off[1] = wl.atom_shell_off[2] + 1
    with pytest.raises(q.Q4CError) as e:
        _host_plan(q, bad2)
    assert e.value.status == q.Q4C_EINVAL
    bad3 = W.Workload(**{**wl.__dict__})
    bad3.w = wl.w.copy()
    bad3.w[5] = np.nan
    with pytest.raises(q.Q4CError) as e:
        _host_plan(q, bad3)
    assert e.value.status == q.Q4C_EINVAL
    bad4 = W.Workload(**{**wl.__dict__})
    bad4.shell_coef_off = wl.shell_coef_off.copy()
    bad4.shell_coef_off[-1] = wl.coef.size
    with pytest.raises(q.Q4CError) as e:
        _host_plan(q, bad4)
    assert e.value.status == q.Q4C_EINVAL


def test_empty_grid_and_no_active_points():
    q, lib = _lib()
    wl = W.config_small(nrad=10, nang=26)
    empty = wl.subset_points(np.arange(0))
    p = _host_plan(q, empty)
    assert p.info["n_batches"] == 0 and p.info["n_active"] == 0 and p.info["flops_alg"] == 0.0
    assert p.info["n_pairs"] == 6
    far = wl.translated([0.0, 0.0, 0.0])
    far.x = far.x + 1e4
    p2 = _host_plan(q, far)
    assert p2.info["n_active"] == 0 and p2.info["n_batches"] == 0


def test_batching_properties():
    q, lib = _lib()
    wl = W.config_cluster(n_atoms=30, nrad=12, nang=26, box_ang=10.0)
    for pmax in (1, 7, 64, 300):
        p = _host_plan(q, wl, p_max=pmax)
        pt_off, pidx, fn_off, fidx = p.batches()
        sizes = np.diff(pt_off)
        assert sizes.max() <= pmax and sizes.min() >= 1
        if p.info["n_active"] > pmax:
            assert sizes.min() >= pmax // 2  # median bisection
        assert len(np.unique(pidx)) == len(pidx)
        # relevance: atom-level exact set
        rc = wl.atom_rcut()
        aoff = np.concatenate([[0], np.cumsum(wl.atom_nfn())])
        for b in np.random.default_rng(0).choice(p.info["n_batches"], size=min(20, p.info["n_batches"]),
                                                 replace=False):
            pts = pidx[pt_off[b]:pt_off[b + 1]]
            d = np.sqrt(np.sum((np.stack([wl.x[pts], wl.y[pts], wl.z[pts]], 1)[:, None, :] - wl.R[None]) ** 2, -1))
            atoms = np.nonzero(np.any(d < rc[None], axis=0))[0]
            want = np.concatenate([np.arange(aoff[a], aoff[a + 1]) for a in atoms])
            assert np.array_equal(fidx[fn_off[b]:fn_off[b + 1]], want)
        # F_alg = sum_B 10 P_B n_B^2
        assert p.info["flops_alg"] == pytest.approx(float(np.sum(10.0 * sizes * np.diff(fn_off) ** 2)), rel=1e-12)


def test_staging_passes_split_by_budget():
    q, lib = _lib()
    wl = W.config_cluster(n_atoms=30, nrad=12, nang=26, box_ang=10.0)
    p1 = _host_plan(q, wl)
    p2 = _host_plan(q, wl, staging_bytes=1 << 20)
    assert p1.info["n_passes"] == 1
    assert p2.info["n_passes"] > 1
    assert p1.info["n_work"] == p2.info["n_work"]


def _small_molecules(n_mol=5, seed_sizes=(8, 14, 9, 11, 8)):
    return W.config_molecules(n_mol=n_mol, sizes=list(seed_sizes[:n_mol]), nrad=12, nang=26)


def test_batched_plan_reproduces_each_system():
    """q4c_plan_create_batched: each system's batches (point sets, relevant
    functions), pairs and store offsets are exactly those of its own plan,
    shifted by the system offsets."""
    q, lib = _lib()
    wl = _small_molecules()
    systems = W.split_molecules(wl)
    pb = q.Plan(systems, host_only=True)
    assert pb.info["n_systems"] == len(systems)
    off = pb.systems()
    pairs_b, po_b = pb.pairs()
    pt_b, pidx_b, fo_b, fidx_b = pb.batches()
    fn_off = 0
    for s, ws in enumerate(systems):
        p = q.Plan(ws, host_only=True)
        assert off["atom"][s + 1] - off["atom"][s] == ws.n_atoms
        assert off["point"][s + 1] - off["point"][s] == ws.n_points
        pairs, po = p.pairs()
        a0, a1 = off["pair"][s], off["pair"][s + 1]
        assert np.array_equal(pairs_b[a0:a1] - off["atom"][s], pairs)
        assert np.array_equal(po_b[a0:a1 + 1] - po_b[a0], po)
        assert off["store"][s] == po_b[a0]
        pt, pidx, fo, fidx = p.batches()
        b0, b1 = off["batch"][s], off["batch"][s + 1]
        assert b1 - b0 == p.info["n_batches"]
        for b in range(b1 - b0):
            got = pidx_b[pt_b[b0 + b]:pt_b[b0 + b + 1]] - off["point"][s]
            assert np.array_equal(got, pidx[pt[b]:pt[b + 1]])
            gotf = fidx_b[fo_b[b0 + b]:fo_b[b0 + b + 1]] - fn_off
            assert np.array_equal(gotf, fidx[fo[b]:fo[b + 1]])
        fn_off += ws.n_fn
    # the systems' pairs never couple two systems
    mol = wl.molecule
    assert np.all(mol[pairs_b[:, 0]] == mol[pairs_b[:, 1]])


def test_batched_plan_validation():
    q, lib = _lib()
    h = ctypes.c_void_p()
    assert lib.q4c_plan_create_batched(0, None, None, None, ctypes.byref(h)) == q.Q4C_EINVAL
    assert lib.q4c_plan_set_launch(None, 0, 0, 0) == q.Q4C_EINVAL
    wl = _small_molecules(n_mol=2)
    p = q.Plan(W.split_molecules(wl), host_only=True)
    assert lib.q4c_plan_set_launch(p.handle, 0, 0, 0) == q.Q4C_ENODEV
    assert lib.q4c_plan_set_graphs(p.handle, 1) == q.Q4C_ENODEV
    assert lib.q4c_plan_autotune(p.handle, None, 0, None, None, None, 1, None, 0, None, None) == q.Q4C_ENODEV


def test_ket_potential_validation_and_hs_flop_count():
    """q4c_plan_set_ket_potential checks its tables; q4c_integrate_HS needs a
    device plan; flops_alg_hs = sum_B 3 P_B n_B^2 over the plan's batches."""
    import dataclasses
    q, lib = _lib()
    wl = W.with_ket(W.config_small(nrad=10, nang=26), 7001)
    p = _host_plan(q, wl)
    p.set_ket_potential(wl)
    for bad in (dataclasses.replace(wl, shell_u_off=wl.shell_u_off + 2),
                dataclasses.replace(wl, shell_u_off=wl.shell_u_off + wl.u_coef.size)):
        with pytest.raises(q.Q4CError) as e:
            p.set_ket_potential(bad)
        assert e.value.status == q.Q4C_EINVAL
    nan = wl.u_coef.copy()
    nan[5] = np.nan
    with pytest.raises(q.Q4CError) as e:
        p.set_ket_potential(dataclasses.replace(wl, u_coef=nan))
    assert e.value.status == q.Q4C_EINVAL
    assert lib.q4c_plan_set_ket_potential(p.handle, None, 0, None) == q.Q4C_EINVAL
    rc = lib.q4c_integrate_HS(p.handle, ctypes.c_void_p(1), 0, ctypes.c_void_p(1), None)
    assert rc == q.Q4C_ENODEV
    assert lib.q4c_integrate_HS(p.handle, ctypes.c_void_p(1), 1 << 20, ctypes.c_void_p(1), None) == q.Q4C_EINVAL
    pt_off, _, fn_off, _ = p.batches()
    P = np.diff(pt_off).astype(np.float64)
    nf = np.diff(fn_off).astype(np.float64)
    assert p.info["flops_alg_hs"] == pytest.approx(float(np.sum(3.0 * P * nf * nf)), rel=1e-15)
    assert p.info["flops_alg"] == pytest.approx(float(np.sum(10.0 * P * nf * nf)), rel=1e-15)


def test_spinor_transform_needs_device_plans():
    q, lib = _lib()
    wl = W.config_small(nrad=10, nang=26)
    p = _host_plan(q, wl)
    rc = lib.q4c_spinor_transform(p.handle, p.handle, ctypes.c_void_p(1), ctypes.c_void_p(1), ctypes.c_void_p(1),
                                  ctypes.c_void_p(1), None)
    assert rc == q.Q4C_ENODEV
    assert lib.q4c_spinor_transform(None, p.handle, None, None, None, None, None) == q.Q4C_EINVAL


def test_density_update_calls_need_device_plans():
    q, lib = _lib()
    wl = W.config_small(nrad=10, nang=26)
    p = _host_plan(q, wl)
    one = ctypes.c_void_p(1)
    assert lib.q4c_spinor_density_to_scalar(p.handle, p.handle, one, one, one, None) == q.Q4C_ENODEV
    assert lib.density_gradient_on_grid(p.handle, one, one, None) == q.Q4C_ENODEV
    assert lib.density_gradient_on_grid(None, one, one, None) == q.Q4C_EINVAL


def test_periodic_cells_validation_and_layout():
    """q4c_plan_set_cells checks its map; the cell-pair layout is the set of
    (a <= b) reached by a stored pair of images, in ascending order."""
    q, lib = _lib()
    # Pb (26 functions) and N (5): images of the two have different bases
    wl = W.config_periodic(species=((82, (0.0, 0.0, 0.0)), (7, (0.5, 0.5, 0.5))), a_ang=4.5, recipe="main",
                           nrad=10, nang=26, k=62)
    p = _host_plan(q, wl)
    m = wl.meta
    p.set_cells(m["n_cell_atoms"], m["cell_atom"], m["shift"])
    pa, po = p.cell_pairs()
    pairs, _ = p.pairs()
    ca = m["cell_atom"]
    want = sorted({(min(ca[a], ca[b]), max(ca[a], ca[b])) for a, b in pairs})
    assert [tuple(x) for x in pa] == want
    nfn = wl.atom_nfn()
    n_cell = [int(nfn[list(ca).index(c)]) for c in range(m["n_cell_atoms"])]
    assert list(np.diff(po)) == [n_cell[a] * n_cell[b] for a, b in want]
    bad = m["cell_atom"].copy()
    bad[-1] = m["n_cell_atoms"]
    with pytest.raises(q.Q4CError) as e:
        p.set_cells(m["n_cell_atoms"], bad, m["shift"])
    assert e.value.status == q.Q4C_EINVAL
    bad = m["cell_atom"].copy()
    bad[-1] = 1 - bad[-1]  # an image of Pb mapped to N (different basis) or the reverse
    with pytest.raises(q.Q4CError) as e:
        p.set_cells(m["n_cell_atoms"], bad, m["shift"])
    assert e.value.status == q.Q4C_EINVAL
    rc = lib.q4c_bloch_sum(p.handle, 5, ctypes.c_void_p(1), 1, ctypes.c_void_p(1), ctypes.c_void_p(1), None)
    assert rc == q.Q4C_ENODEV
    for n_parts in (0, 3, 4, 6):  # 3 or 4 would split the spin-orbit parts
        rc = lib.q4c_bloch_sum(p.handle, n_parts, ctypes.c_void_p(1), 1, ctypes.c_void_p(1), ctypes.c_void_p(1), None)
        assert rc == q.Q4C_EINVAL, n_parts
    one = ctypes.c_void_p(1)
    for n_parts in (0, 3, 5):  # Hermitian parts only
        rc = lib.q4c_bloch_density(p.handle, n_parts, one, 1, one, one, one, None)
        assert rc == q.Q4C_EINVAL, n_parts
    assert lib.q4c_bloch_density(p.handle, 1, one, 1, one, one, one, None) == q.Q4C_ENODEV
    assert lib.q4c_bloch_density(p.handle, 1, one, -1, one, one, one, None) == q.Q4C_EINVAL
    assert lib.q4c_bloch_density(None, 1, one, 1, one, one, one, None) == q.Q4C_EINVAL


def _one_atom_of_g_shells(wl, n_shells):
    """Atom 0 of wl alone, its basis n_shells copies of its first shell as
    l = 4 (9 functions each), the grid points it owns."""
    import dataclasses
    s0 = int(wl.atom_shell_off[0])
    rep = np.full(n_shells, s0)
    pts = np.nonzero(wl.pt_atom == 0)[0][:64]
    return dataclasses.replace(
        wl, name="one atom, %d g shells" % n_shells, Z=wl.Z[:1].copy(), R=wl.R[:1].copy(),
        atom_shell_off=np.array([0, n_shells], dtype=np.int32), shell_l=np.full(n_shells, 4, dtype=np.int32),
        shell_rcut=wl.shell_rcut[rep].copy(), shell_nint=wl.shell_nint[rep].copy(),
        shell_coef_off=wl.shell_coef_off[rep].copy(), shell_alpha=wl.shell_alpha[rep].copy(),
        shell_gcoef=wl.shell_gcoef[rep].copy(), x=wl.x[pts].copy(), y=wl.y[pts].copy(), z=wl.z[pts].copy(),
        w=wl.w[pts].copy(), pt_atom=np.zeros(pts.size, dtype=np.int32), v=wl.v[pts].copy(),
        molecule=None, shell_u_off=None, u_coef=None, shell_eps=None)


def test_pair_block_limit_of_the_batch_sum():
    """The batch-to-global sum spreads one atom pair's five blocks over
    256-element workgroups along the grid's second dimension (at most 65535),
    so an atom pair block of more than 65535 * 256 / 5 elements is rejected
    when the plan is built: 1,818 functions on one atom build, 1,836 do not."""
    q, lib = _lib()
    wl = W.config_small(nrad=10, nang=26)
    p = _host_plan(q, _one_atom_of_g_shells(wl, 202))
    assert p.info["n_fn"] == 1818 and p.info["store_len"] == 1818 * 1818
    with pytest.raises(q.Q4CError) as e:
        _host_plan(q, _one_atom_of_g_shells(wl, 204))
    assert e.value.status == q.Q4C_EUNSUPPORTED
