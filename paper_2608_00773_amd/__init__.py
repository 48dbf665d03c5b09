"""Python binding of libq4c (Q4C real-space Hamiltonian integration on MI355X).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory and the current stream.  The names
follow the C ABI in include/q4c.h: ``nao_tabulate``, ``q4c_integrate_H``,
``density_on_grid`` (plus plan helpers).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libq4c.so")

Q4C_OK = 0
Q4C_EINVAL, Q4C_ENOMEM, Q4C_EHIP, Q4C_ENOTIMPL, Q4C_EUNSUPPORTED, Q4C_ESIZE, Q4C_ENONFINITE, Q4C_ENODEV = \
    -1, -2, -3, -4, -5, -6, -7, -8
PREC_F64, PREC_SPLIT_F32, PREC_F32, PREC_BF16X3, PREC_F64_VALU = 0, 1, 2, 3, 4
TIMER_NAMES = ("tabulate", "contract", "reduce", "spinor", "bloch", "density_tiles", "density_points", "other")
ACCUMULATE, ASSEMBLE_W, ASSEMBLE_V, CHECK_FINITE = 1, 2, 4, 8
PLAN_HOST_ONLY = 1
TERM_LL, TERM_SS, TERM_SO, TERM_ALL = 1, 2, 4, 7
DTYPE_F64, DTYPE_F32_HILO = 0, 1
PART_V, PART_WS, PART_WSO, PART_ALL = 1, 2, 4, 7
PART_NAMES = ("V", "Ws", "Wso_x", "Wso_y", "Wso_z")


class Q4CError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("q4c status %d (%s): %s" % (status, _status_string(status), msg))
        self.status = status


_lib = None


def _status_string(s):
    try:
        return _load().q4c_status_string(s).decode()
    except Exception:  # pragma: no cover
        return "?"


class _Basis(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("R", ctypes.c_void_p), ("atom_shell_off", ctypes.c_void_p),
                ("n_shells", ctypes.c_int32), ("shell_l", ctypes.c_void_p), ("shell_rcut", ctypes.c_void_p),
                ("shell_nint", ctypes.c_void_p), ("shell_coef_off", ctypes.c_void_p), ("n_coef", ctypes.c_int64),
                ("coef", ctypes.c_void_p)]


class _Grid(ctypes.Structure):
    _fields_ = [("n_points", ctypes.c_int64), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p),
                ("z", ctypes.c_void_p), ("w", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("c_light", ctypes.c_double), ("p_max", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("staging_bytes", ctypes.c_int64)]


class _Info(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("n_fn", ctypes.c_int32), ("n_points", ctypes.c_int64),
                ("n_active", ctypes.c_int64), ("n_batches", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
                ("store_len", ctypes.c_int64), ("fn_entries", ctypes.c_int64), ("max_batch_points", ctypes.c_int64),
                ("max_batch_fn", ctypes.c_int64), ("n_work", ctypes.c_int64), ("n_passes", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("flops_alg", ctypes.c_double), ("n_systems", ctypes.c_int32),
                ("scratch_bytes", ctypes.c_int64), ("flops_alg_hs", ctypes.c_double), ("staging_bytes", ctypes.c_int64),
                ("tab_elems", ctypes.c_int64)]


class _TuneEntry(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("order", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("ms", ctypes.c_double)]


KERNEL_CONTRACT, KERNEL_DENSITY, KERNEL_HS = 0, 1, 2


class _StoreLayout(ctypes.Structure):
    _fields_ = [("n_pairs", ctypes.c_int64), ("store_len", ctypes.c_int64), ("part_bytes", ctypes.c_int64),
                ("store_bytes", ctypes.c_int64), ("hs_bytes", ctypes.c_int64), ("spinor_bytes", ctypes.c_int64)]


EXPORTS = ("q4c_plan_create", "q4c_plan_destroy", "q4c_plan_info", "q4c_plan_pairs", "q4c_plan_batches",
           "q4c_store_layout",
           "q4c_tabulate_size", "nao_tabulate", "q4c_integrate_H", "density_on_grid", "q4c_coef_from_spinor",
           "q4c_plan_sync", "q4c_plan_profile", "q4c_plan_timers", "q4c_status_string",
           "q4c_last_error", "q4c_plan_create_batched", "q4c_plan_systems", "q4c_plan_set_launch",
           "q4c_plan_get_launch", "q4c_plan_autotune", "q4c_plan_set_graphs", "q4c_plan_set_ket_potential",
           "q4c_integrate_HS", "q4c_spinor_transform", "q4c_spinor_density_to_scalar", "density_gradient_on_grid",
           "q4c_plan_set_cells", "q4c_plan_cell_pairs", "q4c_bloch_sum", "q4c_bloch_density",
           "q4c_bloch_sum_noalloc")


def _load():
    """Load libq4c.so.  There is no fallback: a missing library is an error."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libq4c.so not built (run __graft_entry__.build() or "
                              "python paper_2608_00773_amd/build.py): %s" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        lib.q4c_plan_create.argtypes = [ctypes.POINTER(_Basis), ctypes.POINTER(_Grid), ctypes.POINTER(_Opts),
                                        ctypes.POINTER(vp)]
        lib.q4c_plan_destroy.argtypes = [vp]
        lib.q4c_plan_destroy.restype = None
        lib.q4c_plan_info.argtypes = [vp, ctypes.POINTER(_Info)]
        lib.q4c_plan_pairs.argtypes = [vp, vp, vp]
        lib.q4c_plan_batches.argtypes = [vp, vp, vp, vp, vp]
        lib.q4c_tabulate_size.argtypes = [vp, i64, i64, i32, ctypes.POINTER(i64)]
        lib.nao_tabulate.argtypes = [vp, i64, i64, i32, i32, vp, i64, vp]
        lib.q4c_store_layout.argtypes = [vp, ctypes.POINTER(_StoreLayout), vp, vp, vp]
        lib.q4c_integrate_H.argtypes = [vp, vp, i32, u32, u32, vp, vp, vp, vp]
        lib.density_on_grid.argtypes = [vp, vp, u32, i32, i32, vp, vp]
        lib.q4c_coef_from_spinor.argtypes = [vp, vp, vp, vp]
        lib.q4c_plan_sync.argtypes = [vp, vp]
        lib.q4c_plan_profile.argtypes = [vp, ctypes.c_int]
        lib.q4c_plan_timers.argtypes = [vp, vp, vp]
        lib.q4c_plan_create_batched.argtypes = [i32, ctypes.POINTER(_Basis), ctypes.POINTER(_Grid),
                                                ctypes.POINTER(_Opts), ctypes.POINTER(vp)]
        lib.q4c_plan_systems.argtypes = [vp, vp, vp, vp, vp, vp]
        lib.q4c_plan_set_launch.argtypes = [vp, i32, i32, i32]
        lib.q4c_plan_get_launch.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        lib.q4c_plan_autotune.argtypes = [vp, vp, i32, vp, vp, vp, i32, ctypes.POINTER(_TuneEntry), i32,
                                          ctypes.POINTER(i32), vp]
        lib.q4c_plan_set_graphs.argtypes = [vp, ctypes.c_int]
        lib.q4c_plan_set_ket_potential.argtypes = [vp, vp, i64, vp]
        lib.q4c_integrate_HS.argtypes = [vp, vp, u32, vp, vp]
        lib.q4c_spinor_transform.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        lib.q4c_spinor_density_to_scalar.argtypes = [vp, vp, vp, vp, vp, vp]
        lib.density_gradient_on_grid.argtypes = [vp, vp, vp, vp]
        lib.q4c_plan_set_cells.argtypes = [vp, i32, vp, vp]
        lib.q4c_plan_cell_pairs.argtypes = [vp, ctypes.POINTER(i64), vp, vp]
        lib.q4c_bloch_sum.argtypes = [vp, i32, vp, i32, vp, vp, vp]
        lib.q4c_bloch_density.argtypes = [vp, i32, vp, i32, vp, vp, vp, vp]
        lib.q4c_bloch_sum_noalloc.argtypes = [vp, i32, vp, i32, vp, vp, vp]
        lib.q4c_status_string.argtypes = [ctypes.c_int]
        lib.q4c_status_string.restype = ctypes.c_char_p
        lib.q4c_last_error.argtypes = []
        lib.q4c_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("q4c_plan_destroy", "q4c_status_string", "q4c_last_error"):
                getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != Q4C_OK:
        raise Q4CError(rc, _load().q4c_last_error().decode())


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _stream_handle():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, dtype_name="float64", min_numel=0, name="tensor"):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if str(t.dtype) != "torch." + dtype_name:
        raise TypeError("%s must be %s, got %s" % (name, dtype_name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < min_numel:
        raise ValueError("%s has %d elements, needs %d" % (name, t.numel(), min_numel))
    return ctypes.c_void_p(t.data_ptr())


def _descriptors(wl, keep):
    k = dict(
        R=_np(wl.R, np.float64).reshape(-1), aso=_np(wl.atom_shell_off, np.int32), sl=_np(wl.shell_l, np.int32),
        sr=_np(wl.shell_rcut, np.float64), sn=_np(wl.shell_nint, np.int32),
        so=_np(wl.shell_coef_off, np.int64), coef=_np(wl.coef, np.float64), x=_np(wl.x, np.float64),
        y=_np(wl.y, np.float64), z=_np(wl.z, np.float64), w=_np(wl.w, np.float64))
    keep.append(k)
    b = _Basis(int(k["aso"].size - 1), k["R"].ctypes.data, k["aso"].ctypes.data, int(k["sl"].size),
               k["sl"].ctypes.data, k["sr"].ctypes.data, k["sn"].ctypes.data, k["so"].ctypes.data,
               int(k["coef"].size), k["coef"].ctypes.data)
    g = _Grid(int(k["x"].size), k["x"].ctypes.data, k["y"].ctypes.data, k["z"].ctypes.data, k["w"].ctypes.data)
    return b, g


class Plan:
    """An integration plan (q4c_plan_create) for one system and grid, or, given
    a list of systems, one plan over all of them (q4c_plan_create_batched):
    the union is system-major and every call runs all systems at once."""

    def __init__(self, wl, p_max: Optional[int] = None, c_light: Optional[float] = None, host_only: bool = False,
                 staging_bytes: int = 0):
        lib = _load()
        systems = list(wl) if isinstance(wl, (list, tuple)) else [wl]
        first = systems[0]
        keep = []
        coef_cache = {}
        descs = []
        for w in systems:
            # systems sharing one coefficient array pass the same pointer (shared tables)
            key = id(w.coef)
            b, g = _descriptors(w, keep)
            if key in coef_cache:
                b.coef, b.n_coef = coef_cache[key]
            else:
                coef_cache[key] = (b.coef, b.n_coef)
            descs.append((b, g))
        if p_max is None:
            p_max = int(getattr(first, "meta", {}).get("p_max", 300))
        o = _Opts(float(c_light if c_light is not None else getattr(first, "c_light", 0.0)), int(p_max),
                  PLAN_HOST_ONLY if host_only else 0, int(staging_bytes))
        h = ctypes.c_void_p()
        if isinstance(wl, (list, tuple)):
            B = (_Basis * len(descs))(*[d[0] for d in descs])
            G = (_Grid * len(descs))(*[d[1] for d in descs])
            _check(lib.q4c_plan_create_batched(len(descs), B, G, ctypes.byref(o), ctypes.byref(h)))
        else:
            _check(lib.q4c_plan_create(ctypes.byref(descs[0][0]), ctypes.byref(descs[0][1]), ctypes.byref(o),
                                       ctypes.byref(h)))
        self._h = h
        del keep
        self.info = self._info()

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _load().q4c_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _info(self):
        inf = _Info()
        _check(_load().q4c_plan_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in _Info._fields_}

    def pairs(self):
        n = self.info["n_pairs"]
        pa = np.zeros(2 * max(n, 1), dtype=np.int32)
        po = np.zeros(n + 1, dtype=np.int64)
        _check(_load().q4c_plan_pairs(self._h, pa.ctypes.data, po.ctypes.data))
        return pa[:2 * n].reshape(n, 2), po

    def store_layout(self):
        """q4c_store_layout: sizes, pair list, block offsets and block shapes."""
        lay = _StoreLayout()
        n = self.info["n_pairs"]
        pa = np.zeros(2 * max(n, 1), dtype=np.int32)
        po = np.zeros(n + 1, dtype=np.int64)
        nf = np.zeros(2 * max(n, 1), dtype=np.int32)
        _check(_load().q4c_store_layout(self._h, ctypes.byref(lay), pa.ctypes.data, po.ctypes.data, nf.ctypes.data))
        out = {f: getattr(lay, f) for f, _ in _StoreLayout._fields_}
        out.update(pair_atoms=pa[:2 * n].reshape(n, 2), pair_off=po, pair_nfn=nf[:2 * n].reshape(n, 2))
        return out

    def batches(self):
        nb, na, fe = self.info["n_batches"], self.info["n_active"], self.info["fn_entries"]
        pt_off = np.zeros(nb + 1, dtype=np.int64)
        pidx = np.zeros(max(na, 1), dtype=np.int64)
        fn_off = np.zeros(nb + 1, dtype=np.int64)
        fidx = np.zeros(max(fe, 1), dtype=np.int32)
        _check(_load().q4c_plan_batches(self._h, pt_off.ctypes.data, pidx.ctypes.data, fn_off.ctypes.data,
                                        fidx.ctypes.data))
        return pt_off, pidx[:na], fn_off, fidx[:fe]

    def tabulate_size(self, b0: int, b1: int, deriv: int = 1) -> int:
        n = ctypes.c_int64()
        _check(_load().q4c_tabulate_size(self._h, int(b0), int(b1), int(deriv), ctypes.byref(n)))
        return int(n.value)

    def profile(self, enable: bool = True):
        """Bracket every kernel launch of this plan with HIP events (q4c_plan_profile)."""
        _check(_load().q4c_plan_profile(self._h, 1 if enable else 0))

    def timers(self):
        """{kernel kind: (total ms, launches)} since the last call (q4c_plan_timers)."""
        ms = np.zeros(len(TIMER_NAMES))
        n = np.zeros(len(TIMER_NAMES), dtype=np.int64)
        _check(_load().q4c_plan_timers(self._h, ms.ctypes.data, n.ctypes.data))
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(TIMER_NAMES)}

    def sync(self):
        _check(_load().q4c_plan_sync(self._h, _stream_handle()))

    def systems(self):
        """{atom, point, batch, pair, store}: [n_systems + 1] offsets of each system in the union."""
        n = self.info["n_systems"] + 1
        out = {k: np.zeros(n, dtype=np.int64) for k in ("atom", "point", "batch", "pair", "store")}
        _check(_load().q4c_plan_systems(self._h, *[out[k].ctypes.data for k in ("atom", "point", "batch", "pair",
                                                                                 "store")]))
        return out

    def set_ket_potential(self, wl):
        """Ket-potential tables u = eps - V per shell (q4c_plan_set_ket_potential)
        from a workload's shell_u_off / u_coef, or from a list of workloads in
        the system order of a batched plan (their shells concatenated)."""
        systems = list(wl) if isinstance(wl, (list, tuple)) else [wl]
        offs, tabs, base = [], [], 0
        for w in systems:
            if w.u_coef is None or w.shell_u_off is None:
                raise ValueError("workload has no ket-potential tables")
            offs.append(np.asarray(w.shell_u_off, dtype=np.int64) + base)
            tabs.append(np.asarray(w.u_coef, dtype=np.float64))
            base += tabs[-1].size
        off = np.ascontiguousarray(np.concatenate(offs))
        tab = np.ascontiguousarray(np.concatenate(tabs))
        _check(_load().q4c_plan_set_ket_potential(self._h, off.ctypes.data, int(tab.size), tab.ctypes.data))

    def set_cells(self, n_cell_atoms: int, cell_atom, shift):
        """Periodic cell map (q4c_plan_set_cells): cell atom and lattice
        translation (bohr) of every atom of the plan."""
        ca = np.ascontiguousarray(cell_atom, dtype=np.int32)
        sh = np.ascontiguousarray(shift, dtype=np.float64).reshape(-1)
        _check(_load().q4c_plan_set_cells(self._h, int(n_cell_atoms), ca.ctypes.data, sh.ctypes.data))

    def cell_pairs(self):
        """(pair_atoms int32[n, 2], pair_off int64[n + 1]) of the Bloch-sum output."""
        n = ctypes.c_int64()
        _check(_load().q4c_plan_cell_pairs(self._h, ctypes.byref(n), None, None))
        pa = np.zeros((n.value, 2), dtype=np.int32)
        po = np.zeros(n.value + 1, dtype=np.int64)
        _check(_load().q4c_plan_cell_pairs(self._h, ctypes.byref(n), pa.ctypes.data, po.ctypes.data))
        return pa, po

    def set_launch(self, kernel: int, order: int, persistent: int):
        _check(_load().q4c_plan_set_launch(self._h, int(kernel), int(order), int(persistent)))

    def get_launch(self, kernel: int):
        o, p = ctypes.c_int32(), ctypes.c_int32()
        _check(_load().q4c_plan_get_launch(self._h, int(kernel), ctypes.byref(o), ctypes.byref(p)))
        return int(o.value), int(p.value)

    def set_graphs(self, enable: bool = True):
        _check(_load().q4c_plan_set_graphs(self._h, 1 if enable else 0))

    def autotune(self, v, store, precision: int = PREC_F64, coef=None, out=None, reps: int = 3):
        """Time the candidate launch shapes (q4c_plan_autotune), keep the fastest;
        returns [(kernel, order, persistent, ms), ...]."""
        L = self.info["store_len"]
        tab = (_TuneEntry * 32)()
        n = ctypes.c_int32()
        _check(_load().q4c_plan_autotune(
            self._h, _dev_ptr(v, min_numel=self.info["n_points"], name="v"), int(precision),
            _dev_ptr(store, min_numel=5 * L, name="store"),
            _dev_ptr(coef, min_numel=5 * L, name="coef") if coef is not None else None,
            _dev_ptr(out, min_numel=self.info["n_points"], name="out") if out is not None else None,
            int(reps), tab, 32, ctypes.byref(n), _stream_handle()))
        return [(e.kernel, e.order, e.persistent, e.ms) for e in tab[:min(n.value, 32)]]


# ---------------------------------------------------------------------------
# C-ABI calls on torch device tensors
# ---------------------------------------------------------------------------

def nao_tabulate(plan: Plan, b0: int, b1: int, deriv: int, out, dtype: int = DTYPE_F64):
    """phi (and grad phi) of batches [b0, b1) into `out`: a float64 CUDA tensor
    for DTYPE_F64, a float32 one (hi and lo planes) for DTYPE_F32_HILO."""
    need = plan.tabulate_size(b0, b1, deriv)
    dt = "float32" if dtype == DTYPE_F32_HILO else "float64"
    ptr = _dev_ptr(out, dt, name="out")
    _check(_load().nao_tabulate(plan.handle, int(b0), int(b1), int(deriv), int(dtype), ptr,
                                int(out.numel() * out.element_size()), _stream_handle()))
    return need


def q4c_integrate_H(plan: Plan, v, precision: int = PREC_F64, flags: int = 0, store=None, spin_w=None,
                    spin_v=None, parts: int = PART_ALL):
    """Integrate the selected real parts into `store` ([5, store_len] float64;
    unselected parts keep their values)."""
    L = plan.info["store_len"]
    _check(_load().q4c_integrate_H(
        plan.handle, _dev_ptr(v, min_numel=plan.info["n_points"], name="v"), int(precision), int(parts), int(flags),
        _dev_ptr(store, min_numel=5 * L, name="store"),
        _dev_ptr(spin_w, min_numel=8 * L, name="spin_w") if spin_w is not None else None,
        _dev_ptr(spin_v, min_numel=8 * L, name="spin_v") if spin_v is not None else None, _stream_handle()))
    return store


def q4c_integrate_HS(plan: Plan, v, flags: int = 0, hs=None):
    """H and S of the plan's component into `hs` ([2, store_len] float64)."""
    L = plan.info["store_len"]
    _check(_load().q4c_integrate_HS(plan.handle, _dev_ptr(v, min_numel=plan.info["n_points"], name="v"),
                                    int(flags), _dev_ptr(hs, min_numel=2 * L, name="hs"), _stream_handle()))
    return hs


def q4c_spinor_transform(plan_large: Plan, plan_small: Plan, hs_large, hs_small, h_out, s_out):
    """H+ and S+ in the spinor basis into h_out, s_out ([4 store_len, 2] float64
    each, complex as (re, im), store_len of the large plan)."""
    L, Ls = plan_large.info["store_len"], plan_small.info["store_len"]
    _check(_load().q4c_spinor_transform(
        plan_large.handle, plan_small.handle, _dev_ptr(hs_large, min_numel=2 * L, name="hs_large"),
        _dev_ptr(hs_small, min_numel=2 * Ls, name="hs_small"), _dev_ptr(h_out, min_numel=8 * L, name="h_out"),
        _dev_ptr(s_out, min_numel=8 * L, name="s_out"), _stream_handle()))
    return h_out, s_out


def q4c_spinor_density_to_scalar(plan_large: Plan, plan_small: Plan, d_spin, c_large, c_small):
    """Scalar density matrices of both components (one part each) from a spinor
    density matrix d_spin ([4 store_len, 2] float64, store_len of the large plan)."""
    L, Ls = plan_large.info["store_len"], plan_small.info["store_len"]
    _check(_load().q4c_spinor_density_to_scalar(
        plan_large.handle, plan_small.handle, _dev_ptr(d_spin, min_numel=8 * L, name="d_spin"),
        _dev_ptr(c_large, min_numel=L, name="c_large"), _dev_ptr(c_small, min_numel=Ls, name="c_small"),
        _stream_handle()))
    return c_large, c_small


def density_gradient_on_grid(plan: Plan, coef, out):
    """n and grad n ([4, n_points] float64) from one coefficient part ([store_len])."""
    _check(_load().density_gradient_on_grid(plan.handle, _dev_ptr(coef, min_numel=plan.info["store_len"], name="coef"),
                                            _dev_ptr(out, min_numel=4 * plan.info["n_points"], name="out"),
                                            _stream_handle()))
    return out


def q4c_bloch_sum(plan: Plan, n_parts: int, store, k_points, out):
    """Bloch sums of the first n_parts parts of `store` at k_points ([n_k, 3],
    host) into out ([n_k, n_parts, cell_len, 2] float64, complex as re, im)."""
    kp = np.ascontiguousarray(k_points, dtype=np.float64).reshape(-1, 3)
    _, po = plan.cell_pairs()
    _check(_load().q4c_bloch_sum(plan.handle, int(n_parts), _dev_ptr(store, min_numel=n_parts * plan.info["store_len"],
                                                                     name="store"),
                                 int(kp.shape[0]), kp.ctypes.data,
                                 _dev_ptr(out, min_numel=2 * kp.shape[0] * n_parts * int(po[-1]), name="out"),
                                 _stream_handle()))
    return out


def q4c_bloch_sum_noalloc(plan: Plan, n_parts: int, store, k_points_dev, out):
    """q4c_bloch_sum with the k-points on the device (k_points_dev: float64 CUDA
    tensor [n_k, 3]) and the library's fixed scratch: allocates nothing."""
    n_k = int(k_points_dev.numel() // 3)
    _, po = plan.cell_pairs()
    _check(_load().q4c_bloch_sum_noalloc(
        plan.handle, int(n_parts), _dev_ptr(store, min_numel=n_parts * plan.info["store_len"], name="store"), n_k,
        _dev_ptr(k_points_dev, min_numel=3 * n_k, name="k_points_dev"),
        _dev_ptr(out, min_numel=2 * n_k * n_parts * int(po[-1]), name="out"), _stream_handle()))
    return out


def q4c_bloch_density(plan: Plan, n_parts: int, rho, k_points, k_weights, out):
    """Coefficients on the stored image pairs (n_parts x store_len, device)
    from k-space density matrices rho ([n_k, n_parts, cell_len, 2] float64,
    device, the layout of q4c_bloch_sum's output) at k_points ([n_k, 3]) with
    weights k_weights ([n_k]) (host)."""
    kp = np.ascontiguousarray(k_points, dtype=np.float64).reshape(-1, 3)
    kw = np.ascontiguousarray(k_weights, dtype=np.float64).reshape(-1)
    if kw.size != kp.shape[0]:
        raise ValueError("one weight per k-point")
    _, po = plan.cell_pairs()
    nk = int(kp.shape[0])
    rp = _dev_ptr(rho, min_numel=2 * nk * n_parts * int(po[-1]), name="rho") if nk > 0 else None
    _check(_load().q4c_bloch_density(plan.handle, int(n_parts), rp, nk, kp.ctypes.data if nk else None,
                                     kw.ctypes.data if nk else None,
                                     _dev_ptr(out, min_numel=n_parts * plan.info["store_len"], name="out"),
                                     _stream_handle()))
    return out


def density_on_grid(plan: Plan, coef, terms: int = TERM_ALL, weight_mode: int = 0, out=None,
                    precision: int = PREC_F64):
    L = plan.info["store_len"]
    _check(_load().density_on_grid(plan.handle, _dev_ptr(coef, min_numel=5 * L, name="coef"), int(terms),
                                   int(precision), int(weight_mode),
                                   _dev_ptr(out, min_numel=plan.info["n_points"], name="out"), _stream_handle()))
    return out


def q4c_coef_from_spinor(plan: Plan, spin_d, out):
    L = plan.info["store_len"]
    _check(_load().q4c_coef_from_spinor(plan.handle, _dev_ptr(spin_d, min_numel=8 * L, name="spin_d"),
                                        _dev_ptr(out, min_numel=5 * L, name="out"), _stream_handle()))
    return out


# ---------------------------------------------------------------------------
# Convenience: allocation through torch
# ---------------------------------------------------------------------------

def new_store(plan: Plan, device="cuda"):
    import torch
    return torch.empty((5, plan.info["store_len"]), dtype=torch.float64, device=device)


def new_hs(plan: Plan, device="cuda"):
    import torch
    return torch.empty((2, plan.info["store_len"]), dtype=torch.float64, device=device)


def new_spinor(plan: Plan, device="cuda"):
    import torch
    return torch.empty((4 * plan.info["store_len"], 2), dtype=torch.float64, device=device)


def integrate(plan: Plan, v, precision: int = PREC_F64, assemble: bool = False):
    """Allocate outputs and run q4c_integrate_H; returns (store, spin_w or None)."""
    store = new_store(plan, v.device)
    spin_w = new_spinor(plan, v.device) if assemble else None
    q4c_integrate_H(plan, v, precision, ASSEMBLE_W if assemble else 0, store, spin_w)
    return store, spin_w
