"""ORACLE -- test infrastructure, not part of the library.

A plain FP64 CPU statement of Q4C real-space grid integration (paper Sec. III A,
Eq. 29/31), of the paper's ket-dependent H and S integrand for one component
(Sec. II, Eq. 19, symmetrised), of its spinor assembly (Eq. 16a with the Eq. 8b kinetic balance at
V_A -> 0) and of the density / adjoint contraction (Eq. 39, Eq. 4).  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may import it; the
library never does.  Shares no code with the HIP path: the C part
(q4c_oracle.c) is compiled with gcc, and the spinor algebra below is written
out from the Pauli matrices.

Layout convention (shared as a *format* with the library, not as code): the
result for an atom pair (A, B), A <= B, is five nA x nB row-major blocks
(V, Ws, Wso_x, Wso_y, Wso_z), rows = functions of A in shell order and
m = -l..l, columns = functions of B.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "q4c_oracle.c")
_lib = None

SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no GPU toolchain involved)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp", _SRC, "-o", tmp,
                               "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _Basis(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("R", ctypes.POINTER(ctypes.c_double)),
                ("atom_shell_off", ctypes.POINTER(ctypes.c_int32)), ("shell_l", ctypes.POINTER(ctypes.c_int32)),
                ("shell_rcut", ctypes.POINTER(ctypes.c_double)), ("shell_nint", ctypes.POINTER(ctypes.c_int32)),
                ("shell_coef_off", ctypes.POINTER(ctypes.c_int64)), ("coef", ctypes.POINTER(ctypes.c_double))]


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        bp = ctypes.POINTER(_Basis)
        lib.orc_solid_harmonic.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, dp, dp]
        lib.orc_radial.argtypes = [dp, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]
        lib.orc_n_functions.argtypes = [bp]
        lib.orc_tabulate.argtypes = [bp, ctypes.c_int64, dp, dp, dp, dp, dp, dp, dp]
        lib.orc_pair_blocks.argtypes = [bp, ctypes.c_int64, dp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int,
                                        ip, ip, ctypes.c_int, dp, dp]
        lib.orc_pair_blocks_hs.argtypes = [bp, ctypes.POINTER(ctypes.c_int64), dp, ctypes.c_int64, dp, dp, dp, dp,
                                           dp, ctypes.c_int, ip, ip, ctypes.c_int, dp, dp]
        lib.orc_density_grad_points.argtypes = [bp, ctypes.c_int64, dp, dp, dp, ctypes.c_int, ip, ip, dp, dp, dp]
        lib.orc_density_points.argtypes = [bp, ctypes.c_int64, dp, dp, dp, dp, ctypes.c_double, ctypes.c_int,
                                           ip, ip, dp, ctypes.c_int, dp, dp, dp]
        lib.orc_max_threads.argtypes = []
        lib.orc_max_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_set_threads.restype = None
        _lib = lib
    return _lib


def max_threads() -> int:
    """Threads the oracle's parallel loops use (OpenMP over pairs or points;
    each element's summation order does not depend on it)."""
    return int(_load().orc_max_threads())


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class _BasisHandle:
    """Keeps the arrays referenced by the C struct alive."""

    def __init__(self, wl):
        self.R = _c(wl.R, np.float64).reshape(-1)
        self.aso = _c(wl.atom_shell_off, np.int32)
        self.sl = _c(wl.shell_l, np.int32)
        self.sr = _c(wl.shell_rcut, np.float64)
        self.sn = _c(wl.shell_nint, np.int32)
        self.so = _c(wl.shell_coef_off, np.int64)
        self.coef = _c(wl.coef, np.float64)
        self.s = _Basis(int(wl.n_atoms), _dp(self.R), _ip(self.aso), _ip(self.sl), _dp(self.sr), _ip(self.sn),
                        self.so.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(self.coef))

    @property
    def ptr(self):
        return ctypes.byref(self.s)


def solid_harmonic(l: int, m: int, x: float, y: float, z: float):
    """(S, grad S) with S = s^l Y_lm (App. B real harmonics)."""
    lib = _load()
    S = ctypes.c_double()
    g = np.zeros(3)
    lib.orc_solid_harmonic(l, m, x, y, z, ctypes.byref(S), _dp(g))
    return S.value, g


def radial(table: np.ndarray, rcut: float, s: float):
    lib = _load()
    t = _c(table, np.float64).reshape(-1)
    v = ctypes.c_double()
    d = ctypes.c_double()
    lib.orc_radial(_dp(t), int(t.size // 4), float(rcut), float(s), ctypes.byref(v), ctypes.byref(d))
    return v.value, d.value


def tabulate(wl, x, y, z, with_abs: bool = False):
    """phi [npts, nfn] and grad phi [npts, nfn, 3] of every function (brute force).

    with_abs: also the magnitudes of the terms each value is summed from (the
    radial cubic's sum_k |c_k t^k| times the sum of |monomials| of S_lm, and
    the gradient analogues), the error scale of each tabulated value."""
    lib = _load()
    h = _BasisHandle(wl)
    x, y, z = _c(x, np.float64), _c(y, np.float64), _c(z, np.float64)
    nfn = lib.orc_n_functions(h.ptr)
    phi = np.zeros((x.size, nfn))
    grad = np.zeros((x.size, nfn, 3))
    aphi = np.zeros_like(phi) if with_abs else None
    agrad = np.zeros_like(grad) if with_abs else None
    lib.orc_tabulate(h.ptr, x.size, _dp(x), _dp(y), _dp(z), _dp(phi), _dp(grad),
                     _dp(aphi) if with_abs else None, _dp(agrad) if with_abs else None)
    return (phi, grad, aphi, agrad) if with_abs else (phi, grad)


def pair_blocks(wl, pairs: np.ndarray, v: Optional[np.ndarray] = None, screened: bool = True,
                with_abs: bool = False):
    """Five real parts (V, Ws, Wso_x, Wso_y, Wso_z) per requested atom pair.

    Returns a list of float64[5, nA, nB] (and the matching sum-|term| scales if
    with_abs)."""
    lib = _load()
    h = _BasisHandle(wl)
    pairs = _c(pairs, np.int32).reshape(-1, 2)
    pa, pb = _c(pairs[:, 0], np.int32), _c(pairs[:, 1], np.int32)
    nfn = wl.atom_nfn()
    sizes = [5 * int(nfn[a]) * int(nfn[b]) for a, b in pairs]
    out = np.zeros(int(sum(sizes)))
    absout = np.zeros_like(out) if with_abs else None
    vv = _c(wl.v if v is None else v, np.float64)
    x, y, z, w = (_c(t, np.float64) for t in (wl.x, wl.y, wl.z, wl.w))
    lib.orc_pair_blocks(h.ptr, x.size, _dp(x), _dp(y), _dp(z), _dp(w), _dp(vv), float(wl.c_light),
                        int(pairs.shape[0]), _ip(pa), _ip(pb), 1 if screened else 0, _dp(out),
                        _dp(absout) if with_abs else None)
    res, ares, o = [], [], 0
    for (a, b), s in zip(pairs, sizes):
        res.append(out[o:o + s].reshape(5, int(nfn[a]), int(nfn[b])))
        if with_abs:
            ares.append(absout[o:o + s].reshape(5, int(nfn[a]), int(nfn[b])))
        o += s
    return (res, ares) if with_abs else res


def pair_blocks_hs(wl, pairs: np.ndarray, v: Optional[np.ndarray] = None, screened: bool = True,
                   with_abs: bool = False, u_coef: Optional[np.ndarray] = None,
                   shell_u_off: Optional[np.ndarray] = None):
    """H and S of one component per requested atom pair (Eq. 19 in the scalar
    form of Eq. 29, symmetrised): H_ij = sum_g w phi_i phi_j (v + (u_i + u_j)/2),
    S_ij = sum_g w phi_i phi_j, with the per-shell ket potential u = eps - V
    tabulated like the radials (wl.u_coef at wl.shell_u_off, unless given).

    Returns a list of float64[2, nA, nB] (and the error scales if with_abs)."""
    lib = _load()
    h = _BasisHandle(wl)
    uc = _c(wl.u_coef if u_coef is None else u_coef, np.float64)
    uo = _c(wl.shell_u_off if shell_u_off is None else shell_u_off, np.int64)
    pairs = _c(pairs, np.int32).reshape(-1, 2)
    pa, pb = _c(pairs[:, 0], np.int32), _c(pairs[:, 1], np.int32)
    nfn = wl.atom_nfn()
    sizes = [2 * int(nfn[a]) * int(nfn[b]) for a, b in pairs]
    out = np.zeros(int(sum(sizes)))
    absout = np.zeros_like(out) if with_abs else None
    vv = _c(wl.v if v is None else v, np.float64)
    x, y, z, w = (_c(t, np.float64) for t in (wl.x, wl.y, wl.z, wl.w))
    lib.orc_pair_blocks_hs(h.ptr, uo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(uc), x.size, _dp(x),
                           _dp(y), _dp(z), _dp(w), _dp(vv), int(pairs.shape[0]), _ip(pa), _ip(pb),
                           1 if screened else 0, _dp(out), _dp(absout) if with_abs else None)
    res, ares, o = [], [], 0
    for (a, b), s in zip(pairs, sizes):
        res.append(out[o:o + s].reshape(2, int(nfn[a]), int(nfn[b])))
        if with_abs:
            ares.append(absout[o:o + s].reshape(2, int(nfn[a]), int(nfn[b])))
        o += s
    return (res, ares) if with_abs else res


def density(wl, pairs: np.ndarray, coef_blocks: Sequence[np.ndarray], idx: Optional[np.ndarray] = None,
            weight_mode: int = 0, with_parts: bool = False, with_scale: bool = False):
    """Density / adjoint at grid points `idx` (default all) from per-pair
    coefficient blocks float64[5, nA, nB] (V, Ws, x, y, z; each stored element
    counts once).

    with_parts: also the unweighted parts [npts, 3] (nL, nS scalar, nS spin-orbit).
    with_scale: also the per-point error scale of each part [npts, 3]
    (unweighted; see orc_density_points): sum over its terms of |C| times the
    magnitudes of the two function factors.  Returned last."""
    lib = _load()
    h = _BasisHandle(wl)
    pairs = _c(pairs, np.int32).reshape(-1, 2)
    pa, pb = _c(pairs[:, 0], np.int32), _c(pairs[:, 1], np.int32)
    coef = _c(np.concatenate([np.asarray(c, dtype=np.float64).reshape(-1) for c in coef_blocks]), np.float64)
    if idx is None:
        idx = np.arange(wl.n_points)
    x, y, z, w = (_c(t[idx], np.float64) for t in (wl.x, wl.y, wl.z, wl.w))
    out = np.zeros(x.size)
    parts = np.zeros((x.size, 3)) if with_parts else None
    scale = np.zeros((x.size, 3)) if with_scale else None
    lib.orc_density_points(h.ptr, x.size, _dp(x), _dp(y), _dp(z), _dp(w), float(wl.c_light),
                           int(pairs.shape[0]), _ip(pa), _ip(pb), _dp(coef), int(weight_mode), _dp(out),
                           _dp(parts) if with_parts else None, _dp(scale) if with_scale else None)
    res = (out,)
    if with_parts:
        res += (parts,)
    if with_scale:
        res += (scale,)
    return res if len(res) > 1 else out


def density_scale(scale_parts: np.ndarray, w: Optional[np.ndarray] = None, terms: int = 7) -> np.ndarray:
    """Per-point error scale of the selected terms (bit 1 LL, 2 SS scalar, 4 SS
    spin-orbit) from density(..., with_scale=True), times |w_g| when the
    weights are given (the adjoint, weight mode 1)."""
    sel = [k for k in range(3) if terms & (1 << k)]
    sc = np.sum(scale_parts[:, sel], axis=1)
    return sc * np.abs(w) if w is not None else sc


# ---------------------------------------------------------------------------
# Spinor algebra (Eq. 16a with K = sigma.p / 2c; Pauli identity)
# ---------------------------------------------------------------------------

def spinor_W(parts: np.ndarray) -> np.ndarray:
    """W_sp = Ws (x) I2 + i sum_m Wso_m (x) sigma_m for one pair block.

    parts: float64[5, nA, nB].  Returns complex128[2 nA, 2 nB] with rows
    (spin, function) spin-major: [[uu, ud], [du, dd]]."""
    Ws, Wx, Wy, Wz = parts[1], parts[2], parts[3], parts[4]
    nA, nB = Ws.shape
    out = np.zeros((2 * nA, 2 * nB), dtype=np.complex128)
    for s in range(2):
        for t in range(2):
            blk = Ws * (1.0 if s == t else 0.0) + 0j
            for m, Wm in enumerate((Wx, Wy, Wz)):
                blk = blk + 1j * Wm * SIGMA[m][s, t]
            out[s * nA:(s + 1) * nA, t * nB:(t + 1) * nB] = blk
    return out


def spinor_V(parts: np.ndarray) -> np.ndarray:
    """V_sp = V (x) I2, same layout as spinor_W."""
    V = parts[0]
    nA, nB = V.shape
    out = np.zeros((2 * nA, 2 * nB), dtype=np.complex128)
    out[:nA, :nB] = V
    out[nA:, nB:] = V
    return out


def coef_from_spinor_density(pairs: np.ndarray, D_blocks: Sequence[np.ndarray]) -> List[np.ndarray]:
    """Coefficients on the stored elements such that the density / adjoint of
    L = Re Tr(D H), H = V_sp + W_sp, is a sum over stored elements.

    Re tr2(D_ji H_ij) = (V_ij + Ws_ij) d_ij - sum_m Wso_m,ij e^m_ij with
    d_ij = Re tr2 D_ji and e^m_ij = Im tr2(D_ji sigma_m).  Off-diagonal pair
    blocks are stored once for (i,j) and stand for (j,i) too; both terms are
    equal for Hermitian D, so their coefficient is doubled.  D_blocks[p] is the
    (2 nA) x (2 nB) block D_AB; D_ji (j on B, i on A) = conj(D_AB)^T entries."""
    out = []
    for (a, b), D in zip(pairs, D_blocks):
        nA, nB = D.shape[0] // 2, D.shape[1] // 2
        # D_ji as a 2x2 spin matrix for each (i, j): (D_ji)_{s t} = D[(s, j), (t, i)] = conj(D_AB[(t,i),(s,j)])
        Dab = D.reshape(2, nA, 2, nB)  # [t, i, s, j]
        Dji = np.conj(Dab).transpose(1, 3, 2, 0)  # [i, j, s, t]
        d = np.real(Dji[:, :, 0, 0] + Dji[:, :, 1, 1])
        e = [np.imag(np.einsum("ijst,ts->ij", Dji, SIGMA[m])) for m in range(3)]
        f = 1.0 if a == b else 2.0
        out.append(np.stack([f * d, f * d, -f * e[0], -f * e[1], -f * e[2]]))
    return out


def loss_re_tr(pairs: np.ndarray, D_blocks: Sequence[np.ndarray], parts_blocks: Sequence[np.ndarray]) -> float:
    """Re Tr(D H) for the full Hermitian matrices rebuilt from the A <= B blocks."""
    tot = 0.0
    for (a, b), D, P in zip(pairs, D_blocks, parts_blocks):
        H = spinor_V(P) + spinor_W(P)
        # Tr over this block and its mirror: sum_{IJ} D_JI H_IJ, with D_JI = conj(D_IJ) for the stored block
        t = np.sum(np.conj(D) * H)  # = sum_IJ conj(D_IJ) H_IJ = sum_IJ D_JI H_IJ
        tot += np.real(t) * (1.0 if a == b else 2.0)
    return float(tot)


# ---------------------------------------------------------------------------
# Scalar -> spinor transformation (Sec. III A, Eq. 33; Eq. 10, 13, 14; App. A)
# ---------------------------------------------------------------------------
#
# Spinor basis per large shell s (angular momentum l): kappa = -(l+1)
# (j = l + 1/2) with m_j = -j..j, then, for l >= 1, kappa = l (j = l - 1/2);
# 2 (2l+1) spinor functions per shell, m_j ascending.  Half-integers are
# handled as twice their value (j2 = 2j, mj2 = 2 m_j).
#
# The small component of spinor (s, kappa, m_j) is the spin-angular function
# Upsilon_{-kappa, m_j} (l~ = l + 1 for kappa < 0, l - 1 for kappa > 0) on the
# small shell paired with (s, kappa); small shells follow the large shells in
# the order l + 1, then l - 1 (as workload.small_component builds them).
#
# Complex harmonics: the Condon-Shortley ones that the coupling of App. A
# assumes.  App. B's real harmonics already carry (-1)^m, so in their terms
# Y~_l^m = (Y_l,|m| + i Y_l,-|m|)/sqrt2 for m > 0 and (-1)^m (Y_l,|m| -
# i Y_l,-|m|)/sqrt2 for m < 0: Eq. 13 without its extra (-1)^m (applying both
# factors would break (sigma.r) Upsilon_kappa = -Upsilon_-kappa).


def complex_harmonic_coefs(l: int, m: int):
    """Y~_l^m as a combination of App. B real harmonics: [(m', coefficient)]."""
    if m == 0:
        return [(0, 1.0 + 0j)]
    s = 1.0 / math.sqrt(2.0)
    if m > 0:
        return [(m, s + 0j), (-m, 1j * s)]
    sg = -1.0 if (m & 1) else 1.0
    return [(-m, sg * s + 0j), (m, -1j * sg * s)]


def cg_half(l: int, j2: int, mj2: int, spin: int) -> float:
    """C_alpha (spin 0, m_s = +1/2) or C_beta (spin 1, m_s = -1/2) of Eq. 10 for
    j = j2/2, m_j = mj2/2: with a = 2(j - l) = +-1,
    C_alpha = a sqrt(l + a m_j + 1/2) / sqrt(2l + 1),
    C_beta  = sqrt(l - a m_j + 1/2) / sqrt(2l + 1)."""
    a = j2 - 2 * l
    mj = 0.5 * mj2
    if spin == 0:
        return a * math.sqrt(max(l + a * mj + 0.5, 0.0)) / math.sqrt(2 * l + 1)
    return math.sqrt(max(l - a * mj + 0.5, 0.0)) / math.sqrt(2 * l + 1)


def spinor_labels(wl_large):
    """Per atom: list of (large shell, l, kappa, mj2) in spinor order."""
    out = []
    for a in range(wl_large.n_atoms):
        lab = []
        for s in range(wl_large.atom_shell_off[a], wl_large.atom_shell_off[a + 1]):
            l = int(wl_large.shell_l[s])
            for kappa in ((-(l + 1), l) if l >= 1 else (-(l + 1),)):
                j2 = 2 * abs(kappa) - 1
                for mj2 in range(-j2, j2 + 1, 2):
                    lab.append((s, l, kappa, mj2))
        out.append(lab)
    return out


def _shell_fn_offsets(wl, a):
    offs, f = [], 0
    for s in range(wl.atom_shell_off[a], wl.atom_shell_off[a + 1]):
        offs.append(f)
        f += 2 * int(wl.shell_l[s]) + 1
    return offs, f


def spinor_G(wl_large, wl_small):
    """Transformation matrices of Eq. 14 per atom: GL[a] complex[2, nL_a, NS_a]
    and GS[a] complex[2, nS_a, NS_a] (spin, scalar function, spinor function),
    NS_a = 2 nL_a.  G[sigma][t, mu] is the coefficient of scalar function t
    with spin sigma in spinor function mu.  The i of the small component
    (Eq. 12b) is left out: it cancels in every bra-ket of the same component."""
    labels = spinor_labels(wl_large)
    GL, GS = [], []
    for a in range(wl_large.n_atoms):
        offL, nL = _shell_fn_offsets(wl_large, a)
        offS, nS = _shell_fn_offsets(wl_small, a)
        lab = labels[a]
        gl = np.zeros((2, nL, len(lab)), dtype=np.complex128)
        gs = np.zeros((2, nS, len(lab)), dtype=np.complex128)
        s0 = wl_large.atom_shell_off[a]
        # small shell index (atom-local) paired with (large shell, kappa)
        small_of, k = {}, 0
        for s in range(s0, wl_large.atom_shell_off[a + 1]):
            l = int(wl_large.shell_l[s])
            small_of[(s, -(l + 1))] = k
            k += 1
            if l >= 1:
                small_of[(s, l)] = k
                k += 1
        for mu, (s, l, kappa, mj2) in enumerate(lab):
            j2 = 2 * abs(kappa) - 1
            lt = l + 1 if kappa < 0 else l - 1
            ks = small_of[(s, kappa)]
            assert int(wl_small.shell_l[wl_small.atom_shell_off[a] + ks]) == lt
            for spin in (0, 1):
                ml2 = mj2 - (1 if spin == 0 else -1)  # 2 m_l = 2 m_j - 2 m_s
                ml = ml2 // 2
                if abs(ml) <= l:
                    c = cg_half(l, j2, mj2, spin)
                    for mp, z in complex_harmonic_coefs(l, ml):
                        gl[spin, offL[s - s0] + mp + l, mu] += c * z
                if abs(ml) <= lt:
                    c = cg_half(lt, j2, mj2, spin)
                    for mp, z in complex_harmonic_coefs(lt, ml):
                        gs[spin, offS[ks] + mp + lt, mu] += c * z
        GL.append(gl)
        GS.append(gs)
    return GL, GS


def spinor_transform(pairs, blocks_large, blocks_small, GL, GS):
    """H+ and S+ in the spinor basis for each atom pair (Eq. 33, summed over the
    two components and the two spins):
        X+_AB = sum_comp sum_sigma G_A[sigma]^H X^comp_AB G_B[sigma]
    blocks_*: per pair float64[2, n_A, n_B] (H, S) of that component.
    Returns a list of complex128[2, NS_A, NS_B] (H+, S+)."""
    out = []
    for p, (a, b) in enumerate(pairs):
        res = np.zeros((2, GL[a].shape[2], GL[b].shape[2]), dtype=np.complex128)
        for q in range(2):
            for sp in range(2):
                res[q] += GL[a][sp].conj().T @ blocks_large[p][q] @ GL[b][sp]
                res[q] += GS[a][sp].conj().T @ blocks_small[p][q] @ GS[b][sp]
        out.append(res)
    return out


def spinor_density_to_scalar(pairs, D_blocks, GL, GS):
    """The scalar density matrices of both components from a Hermitian spinor
    density matrix given on the pair blocks (the reverse of Eq. 33, as the
    paper's D'_ij = sum_mu,nu D_mu,nu G*_i,mu G_j,nu, summed over spins):
        D'^c_AB = Re sum_sigma conj(G^c_A[sigma]) D_AB G^c_B[sigma]^T
    times 2 on off-diagonal pairs (each stored block stands for its mirror),
    so that a density sums every stored element once.
    Returns a list of (C^L_AB float64[nL_A, nL_B], C^S_AB float64[nS_A, nS_B])."""
    out = []
    for p, (a, b) in enumerate(pairs):
        f = 1.0 if a == b else 2.0
        res = []
        for G in (GL, GS):
            acc = np.zeros((G[a].shape[1], G[b].shape[1]), dtype=np.complex128)
            for sp in range(2):
                acc += G[a][sp].conj() @ D_blocks[p] @ G[b][sp].T
            res.append(f * acc.real)
        out.append(tuple(res))
    return out


def density_grad(wl, pairs, coef_blocks, idx=None, with_scale: bool = False):
    """n and its gradient at grid points `idx` (default all) from one real
    coefficient block per pair (each stored element once): float64[npts, 4]
    with columns n, dn/dx, dn/dy, dn/dz.  with_scale: also the per-point error
    scale of each column (see orc_density_grad_points)."""
    lib = _load()
    h = _BasisHandle(wl)
    pairs = _c(pairs, np.int32).reshape(-1, 2)
    pa, pb = _c(pairs[:, 0], np.int32), _c(pairs[:, 1], np.int32)
    coef = _c(np.concatenate([np.asarray(c, dtype=np.float64).reshape(-1) for c in coef_blocks]), np.float64)
    if idx is None:
        idx = np.arange(wl.n_points)
    x, y, z = (_c(np.asarray(t)[idx], np.float64) for t in (wl.x, wl.y, wl.z))
    out = np.zeros((x.size, 4))
    scale = np.zeros((x.size, 4)) if with_scale else None
    lib.orc_density_grad_points(h.ptr, x.size, _dp(x), _dp(y), _dp(z), int(pairs.shape[0]), _ip(pa), _ip(pb),
                                _dp(coef), _dp(out), _dp(scale) if with_scale else None)
    return (out, scale) if with_scale else out


# ---------------------------------------------------------------------------
# Periodic systems: Bloch sums of unit-cell integrals (Sec. II C, Eq. 26-28)
# ---------------------------------------------------------------------------

def bloch_sum(cell_atom, shift, pairs, blocks, k_points):
    """O_ab(k) = sum over ordered pairs (A', B') of image atoms of the cell
    atoms a, b of exp(i k.(T_B' - T_A')) O_A'B' (the unit-cell integrals of
    the image-extended system summed with the Bloch phases; Eq. 27 with the
    restricted sum of Eq. 28).  blocks: per stored pair (A' <= B') float64
    [n_parts, nA', nB']; the other orientation is O_B'A' = s_q O_A'B'^T with
    s_q = -1 for the spin-orbit parts q >= 2 of a five-part store, +1
    otherwise.  k_points: [n_k, 3] (bohr^-1); shift: [n_atoms, 3] (bohr).
    Returns {(a, b): complex128[n_k, n_parts, n_a, n_b]} for a <= b."""
    k_points = np.asarray(k_points, dtype=np.float64).reshape(-1, 3)
    out = {}
    for p, (A, B) in enumerate(pairs):
        blk = np.asarray(blocks[p])
        npart = blk.shape[0]
        sgn = np.array([(-1.0 if (npart == 5 and q >= 2) else 1.0) for q in range(npart)])
        orients = [(A, B, blk)]
        if A != B:
            orients.append((B, A, sgn[:, None, None] * np.transpose(blk, (0, 2, 1))))
        for (X, Y, M) in orients:
            a, b = int(cell_atom[X]), int(cell_atom[Y])
            if a > b:
                continue
            ph = np.exp(1j * (k_points @ (np.asarray(shift[Y]) - np.asarray(shift[X]))))
            acc = out.setdefault((a, b), np.zeros((k_points.shape[0],) + M.shape, dtype=np.complex128))
            acc += ph[:, None, None, None] * M[None]
    return out


def bloch_density(cell_atom, shift, pairs, rho, k_points, k_weights, nfn):
    """Density-matrix coefficients on the stored image pairs from k-space
    density matrices (Sec. II C, the periodic density matrix and density):
    D_A'B' = sum_k w_k exp(i k.(T_B' - T_A')) rho_ab(k), a, b the cell atoms
    of A', B', with rho_ab(k) = rho_ba(k)^H when a > b (Hermitian rho, e.g.
    sum_l f_l C*_al C_bl).  The density of the extended system is
    n(r) = Re sum over ordered image pairs D phi phi; with the stored pairs
    (A' <= B') standing for both orders the coefficient of a stored element is
    f Re D_A'B' with f = 2 for A' != B' and 1 for A' = B'.
    rho: {(a, b): complex128[n_k, n_parts, n_a, n_b]} for a <= b (the layout
    of bloch_sum's output); nfn: functions per plan atom.
    Returns per stored pair float64 [n_parts, nA', nB']."""
    k_points = np.asarray(k_points, dtype=np.float64).reshape(-1, 3)
    k_weights = np.asarray(k_weights, dtype=np.float64).reshape(-1)
    n_parts = next(iter(rho.values())).shape[1]
    out = []
    for A, B in pairs:
        a, b = int(cell_atom[A]), int(cell_atom[B])
        if a <= b:
            r = rho[(a, b)]                                      # [n_k, n_parts, nA, nB]
        else:
            r = np.conj(np.transpose(rho[(b, a)], (0, 1, 3, 2)))  # rho_ab = rho_ba^H
        ph = k_weights * np.exp(1j * (k_points @ (np.asarray(shift[B]) - np.asarray(shift[A]))))
        D = np.einsum("k,kqij->qij", ph, r)
        f = 1.0 if A == B else 2.0
        blk = f * D.real
        assert blk.shape == (n_parts, int(nfn[A]), int(nfn[B]))
        out.append(blk)
    return out
