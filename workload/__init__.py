"""Seeded synthetic workloads for Q4C grid integration.

This module produces INPUTS only: atoms, NAO radial tables (piecewise-cubic
coefficients of the tapered Gaussian-sum radial part), atom-centred grids with
Becke partition weights, the model potential on the grid, and seeded Hermitian
spinor density matrices.  It contains none of the integration arithmetic and
imports neither the library nor the oracle; both receive these arrays.

Recipes follow the paper's statement of the problem (atoms, radial tables x
real Y_lm, overlapping atom-centred grids with partition weights, potential
on the grid; Sec. III A, Eq. 29) with the synthetic stand-ins described in
the design notes: Gaussian-sum radials instead of DFTATOM solutions,
spherical-Fibonacci angular sets instead of Lebedev/Delley tables, Becke
instead of modified-Stratmann weights.

Units: bohr and hartree throughout.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

ANGSTROM = 1.0 / 0.529177210903  # bohr per angstrom
C_LIGHT = 137.035999084          # speed of light, atomic units

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_gridgen.so")
_lib = None


def build_helper(force: bool = False) -> str:
    """Compile the C input-generation helper (gcc, OpenMP)."""
    src = os.path.join(_HERE, "_gridgen.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", src, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _helper():
    global _lib
    if _lib is None:
        build_helper()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lib.becke_weights.argtypes = [ctypes.c_int, dp, ctypes.c_int64, dp, dp, dp, ip, ctypes.c_double, dp]
        lib.model_potential.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int64, dp, dp, dp,
                                        ctypes.c_double, ctypes.c_double, dp]
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


# ----------------------------------------------------------------------------
# Radial tables
# ----------------------------------------------------------------------------

def taper(s, rcut, width=1.0):
    """C2 smootherstep taper: 1 inside rcut-width, 0 at rcut; and its derivative."""
    u = np.clip((np.asarray(s, dtype=np.float64) - (rcut - width)) / width, 0.0, 1.0)
    t = 1.0 - u ** 3 * (10.0 - 15.0 * u + 6.0 * u * u)
    dt = -30.0 * u * u * (1.0 - u) ** 2 / width
    return t, dt


def gauss_norm(l: int, alpha: Sequence[float], coef: Sequence[float]) -> float:
    """Normalisation N so that phi = N sum_k c_k exp(-a_k s^2) s^l Y_lm has unit norm
    (untapered): int_0^inf s^(2l+2) exp(-p s^2) ds = Gamma(l+3/2) / (2 p^(l+3/2))."""
    tot = 0.0
    for a1, c1 in zip(alpha, coef):
        for a2, c2 in zip(alpha, coef):
            p = a1 + a2
            tot += c1 * c2 * math.gamma(l + 1.5) / (2.0 * p ** (l + 1.5))
    return 1.0 / math.sqrt(tot)


def radial_values(s, alpha, coef, rcut, tapered=True):
    """Tilde-R(s) = taper(s) * sum_k coef_k exp(-alpha_k s^2) and its s-derivative.
    `coef` already includes the normalisation."""
    s = np.asarray(s, dtype=np.float64)
    g = np.zeros_like(s)
    dg = np.zeros_like(s)
    for a, c in zip(alpha, coef):
        e = c * np.exp(-a * s * s)
        g += e
        dg += -2.0 * a * s * e
    if not tapered:
        return g, dg
    t, dt = taper(s, rcut)
    val = g * t
    der = dg * t + g * dt
    inside = s < rcut
    return np.where(inside, val, 0.0), np.where(inside, der, 0.0)


def spline_table(alpha, coef, rcut, nint, tapered=True):
    """Cubic-Hermite coefficients on knots r_j = rcut (j/nint)^2.

    Interval j covers [r_j, r_{j+1}); with t = (s - r_j)/h_j in [0,1) the value
    is c0 + c1 t + c2 t^2 + c3 t^3.  Returns float64[nint, 4]."""
    j = np.arange(nint + 1, dtype=np.float64)
    r = rcut * (j / nint) ** 2
    f, d = radial_values(r, alpha, coef, rcut, tapered)
    f[-1] = 0.0
    d[-1] = 0.0
    h = r[1:] - r[:-1]
    f0, f1 = f[:-1], f[1:]
    d0, d1 = d[:-1] * h, d[1:] * h
    out = np.empty((nint, 4))
    out[:, 0] = f0
    out[:, 1] = d0
    out[:, 2] = 3.0 * (f1 - f0) - 2.0 * d0 - d1
    out[:, 3] = 2.0 * (f0 - f1) + d0 + d1
    return out


# ----------------------------------------------------------------------------
# Grids
# ----------------------------------------------------------------------------

def radial_grid(nr: int, rm: float = 1.0):
    """Gauss-Chebyshev (2nd kind) nodes with Becke's map r = rm (1+x)/(1-x).
    Returns (r, w) with sum_i w_i F(r_i) ~ int_0^inf F(r) r^2 dr."""
    i = np.arange(1, nr + 1, dtype=np.float64)
    ang = i * np.pi / (nr + 1)
    x = np.cos(ang)
    wx = np.pi / (nr + 1) * np.sin(ang) ** 2 / np.sqrt(1.0 - x * x)
    r = rm * (1.0 + x) / (1.0 - x)
    drdx = 2.0 * rm / (1.0 - x) ** 2
    return r, wx * r * r * drdx


def fibonacci_sphere(n: int):
    """Spherical-Fibonacci unit vectors and equal weights 4 pi / n."""
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    phi = k * np.pi * (3.0 - math.sqrt(5.0))
    sxy = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    pts = np.stack([sxy * np.cos(phi), sxy * np.sin(phi), z], axis=1)
    return pts, np.full(n, 4.0 * np.pi / n)


def random_rotation(rng: np.random.Generator):
    """Uniform random rotation matrix from a normalised Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    a, b, c, d = q
    return np.array([
        [a * a + b * b - c * c - d * d, 2 * (b * c - a * d), 2 * (b * d + a * c)],
        [2 * (b * c + a * d), a * a - b * b + c * c - d * d, 2 * (c * d - a * b)],
        [2 * (b * d - a * c), 2 * (c * d + a * b), a * a - b * b - c * c + d * d],
    ])


def product_sphere(ntheta: int, nphi: int):
    """Gauss-Legendre(cos theta) x uniform(phi) product grid: exact for
    spherical harmonics up to degree min(2 ntheta - 1, nphi - 1)."""
    xg, wg = np.polynomial.legendre.leggauss(ntheta)
    ph = (np.arange(nphi) + 0.5) * 2.0 * np.pi / nphi
    ct = np.repeat(xg, nphi)
    st = np.sqrt(1.0 - ct * ct)
    pp = np.tile(ph, ntheta)
    pts = np.stack([st * np.cos(pp), st * np.sin(pp), ct], axis=1)
    w = np.repeat(wg, nphi) * (2.0 * np.pi / nphi)
    return pts, w


# ----------------------------------------------------------------------------
# Workload container
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    Z: np.ndarray            # int32[na]
    R: np.ndarray            # float64[na, 3] bohr
    atom_shell_off: np.ndarray  # int32[na+1]
    shell_l: np.ndarray      # int32[ns]
    shell_rcut: np.ndarray   # float64[ns] bohr
    shell_nint: np.ndarray   # int32[ns]
    shell_coef_off: np.ndarray  # int64[ns] offset (in doubles) into coef
    coef: np.ndarray         # float64[...] 4 per interval, interval-major
    shell_alpha: np.ndarray  # float64[ns, 3] Gaussian exponents (pins)
    shell_gcoef: np.ndarray  # float64[ns, 3] normalised contraction coefficients (pins)
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    w: np.ndarray            # quadrature x partition weight
    pt_atom: np.ndarray      # int32[N] owner centre of each point
    v: np.ndarray            # float64[N] potential, Ha
    c_light: float = C_LIGHT
    molecule: Optional[np.ndarray] = None  # int32[na] molecule id (batched workloads)
    meta: Dict = dataclasses.field(default_factory=dict)
    # ket potential u_s(r) = eps_s - V_s(r) per shell (Q4C H integrand), tables
    # in the radial format on the shell's own knots; None when not set
    shell_u_off: Optional[np.ndarray] = None  # int64[ns] offsets (doubles) into u_coef
    u_coef: Optional[np.ndarray] = None       # float64[...] 4 per interval
    shell_eps: Optional[np.ndarray] = None    # float64[ns] eps_s (recipe record)

    @property
    def n_atoms(self) -> int:
        return int(self.Z.shape[0])

    @property
    def n_points(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_shells(self) -> int:
        return int(self.shell_l.shape[0])

    def atom_nfn(self) -> np.ndarray:
        out = np.zeros(self.n_atoms, dtype=np.int64)
        for a in range(self.n_atoms):
            s0, s1 = self.atom_shell_off[a], self.atom_shell_off[a + 1]
            out[a] = int(np.sum(2 * self.shell_l[s0:s1] + 1))
        return out

    @property
    def n_fn(self) -> int:
        return int(np.sum(2 * self.shell_l + 1))

    def atom_rcut(self) -> np.ndarray:
        out = np.zeros(self.n_atoms)
        for a in range(self.n_atoms):
            s0, s1 = self.atom_shell_off[a], self.atom_shell_off[a + 1]
            out[a] = float(np.max(self.shell_rcut[s0:s1])) if s1 > s0 else 0.0
        return out

    def subset_points(self, idx: np.ndarray) -> "Workload":
        idx = np.asarray(idx)
        return dataclasses.replace(self, x=self.x[idx].copy(), y=self.y[idx].copy(), z=self.z[idx].copy(),
                                   w=self.w[idx].copy(), pt_atom=self.pt_atom[idx].copy(), v=self.v[idx].copy(),
                                   name=self.name + "-sub")

    def with_v(self, v: np.ndarray) -> "Workload":
        return dataclasses.replace(self, v=np.ascontiguousarray(v, dtype=np.float64))

    def translated(self, shift) -> "Workload":
        shift = np.asarray(shift, dtype=np.float64)
        return dataclasses.replace(self, R=self.R + shift[None, :], x=self.x + shift[0], y=self.y + shift[1],
                                   z=self.z + shift[2], name=self.name + "-shifted")


# ----------------------------------------------------------------------------
# Basis sets
# ----------------------------------------------------------------------------

HEAVY_SHELLS = [0, 0, 0, 1, 1, 2, 2, 3]   # 3s2p2d1f = 26 functions
LIGHT_SHELLS = [0, 0, 1]                  # 2s1p = 5 functions
SMALL_SHELLS = [0, 0, 0, 1, 1, 2]         # 3s2p1d = 14 functions


def _species_shells(Z: int, recipe: str) -> List[int]:
    if recipe == "small":
        return SMALL_SHELLS
    return HEAVY_SHELLS if Z >= 21 else LIGHT_SHELLS


def make_basis(Z: np.ndarray, recipe: str, seed: int, rcut: float, nint: int,
               alpha_range=(0.1, 20.0)):
    """Per-species shells of 3-Gaussian radials; atoms of one species share tables."""
    species = sorted(set(int(z) for z in Z))
    tables = {}
    coef_chunks: List[np.ndarray] = []
    off = 0
    for sp in species:
        rng = np.random.default_rng(np.random.PCG64([seed, sp]))
        sh = []
        for l in _species_shells(sp, recipe):
            lo, hi = np.log(alpha_range[0]), np.log(alpha_range[1])
            alpha = np.sort(np.exp(rng.uniform(lo, hi, size=3)))
            c = rng.uniform(0.2, 1.0, size=3)
            c = c * gauss_norm(l, alpha, c)
            tab = spline_table(alpha, c, rcut, nint)
            coef_chunks.append(tab.reshape(-1))
            sh.append((l, alpha, c, off))
            off += tab.size
        tables[sp] = sh
    coef = np.concatenate(coef_chunks) if coef_chunks else np.zeros(0)
    atom_shell_off = [0]
    sl, sr, sn, so, sa, sc = [], [], [], [], [], []
    for z in Z:
        for (l, alpha, c, o) in tables[int(z)]:
            sl.append(l); sr.append(rcut); sn.append(nint); so.append(o); sa.append(alpha); sc.append(c)
        atom_shell_off.append(len(sl))
    return dict(atom_shell_off=np.array(atom_shell_off, dtype=np.int32),
                shell_l=np.array(sl, dtype=np.int32), shell_rcut=np.array(sr, dtype=np.float64),
                shell_nint=np.array(sn, dtype=np.int32), shell_coef_off=np.array(so, dtype=np.int64),
                coef=np.ascontiguousarray(coef), shell_alpha=np.array(sa).reshape(-1, 3),
                shell_gcoef=np.array(sc).reshape(-1, 3))


def custom_basis(Z, shells_per_atom, rcut, nint, tapered=True):
    """Explicit basis for pins: shells_per_atom[a] = list of (l, alpha[3], raw_coef[3]).
    Coefficients are normalised here (untapered norm)."""
    coef_chunks = []
    off = 0
    atom_shell_off = [0]
    sl, sr, sn, so, sa, sc = [], [], [], [], [], []
    for a in range(len(Z)):
        for (l, alpha, c) in shells_per_atom[a]:
            alpha = np.asarray(alpha, dtype=np.float64)
            c = np.asarray(c, dtype=np.float64)
            c = c * gauss_norm(l, alpha, c)
            tab = spline_table(alpha, c, rcut, nint, tapered)
            coef_chunks.append(tab.reshape(-1))
            sl.append(l); sr.append(rcut); sn.append(nint); so.append(off); sa.append(alpha); sc.append(c)
            off += tab.size
        atom_shell_off.append(len(sl))
    return dict(atom_shell_off=np.array(atom_shell_off, dtype=np.int32),
                shell_l=np.array(sl, dtype=np.int32), shell_rcut=np.array(sr, dtype=np.float64),
                shell_nint=np.array(sn, dtype=np.int32), shell_coef_off=np.array(so, dtype=np.int64),
                coef=np.concatenate(coef_chunks), shell_alpha=np.array(sa).reshape(-1, 3),
                shell_gcoef=np.array(sc).reshape(-1, 3))


# ----------------------------------------------------------------------------
# Atom-centred grids
# ----------------------------------------------------------------------------

def atom_grids(R: np.ndarray, Z: np.ndarray, nrad_of, nang_of, seed: int, r_comp: float,
               rm: float = 1.0, chunk_atoms: Optional[int] = None, R_partition: Optional[np.ndarray] = None):
    """Overlapping atom-centred grids (radial shells x rotated Fibonacci sphere)
    with Becke partition weights.  Returns x, y, z, w, owner.  R_partition
    (optional) is the atom list the partition runs over; atoms of R must be its
    first entries (periodic cells: the cell's atoms, then their images)."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    xs, ys, zs, ws, own = [], [], [], [], []
    cache = {}
    for a in range(len(Z)):
        nr, na = nrad_of(int(Z[a])), nang_of(int(Z[a]))
        if (nr, na) not in cache:
            r, wr = radial_grid(nr, rm)
            u, wu = fibonacci_sphere(na)
            cache[(nr, na)] = (r, wr, u, wu)
        r, wr, u, wu = cache[(nr, na)]
        rot = random_rotation(rng)
        uu = u @ rot.T
        p = (r[:, None, None] * uu[None, :, :]).reshape(-1, 3) + R[a][None, :]
        xs.append(p[:, 0]); ys.append(p[:, 1]); zs.append(p[:, 2])
        ws.append((wr[:, None] * wu[None, :]).reshape(-1))
        own.append(np.full(p.shape[0], a, dtype=np.int32))
    x = np.ascontiguousarray(np.concatenate(xs))
    y = np.ascontiguousarray(np.concatenate(ys))
    z = np.ascontiguousarray(np.concatenate(zs))
    wq = np.concatenate(ws)
    owner = np.ascontiguousarray(np.concatenate(own))
    wb = becke(R if R_partition is None else R_partition, x, y, z, owner, r_comp)
    return x, y, z, np.ascontiguousarray(wq * wb), owner


def becke(R, x, y, z, owner, r_comp):
    lib = _helper()
    Rc = np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
    out = np.empty(x.shape[0])
    lib.becke_weights(int(R.shape[0]), _dp(Rc), int(x.shape[0]), _dp(x), _dp(y), _dp(z), _ip(owner),
                      float(r_comp), _dp(out))
    return out


def model_potential(R, Z, x, y, z, a_smear=0.5, r_cut=0.0):
    """v(r) = sum_A -Z_A erf(|r-R_A|/a)/|r-R_A| (a = 0.5 bohr)."""
    lib = _helper()
    Rc = np.ascontiguousarray(R, dtype=np.float64).reshape(-1)
    Zf = np.ascontiguousarray(Z, dtype=np.float64)
    out = np.empty(x.shape[0])
    lib.model_potential(int(R.shape[0]), _dp(Rc), _dp(Zf), int(x.shape[0]), _dp(x), _dp(y), _dp(z),
                        float(a_smear), float(r_cut), _dp(out))
    return out


def smooth_noise(x, y, z, seed: int, amp: float = 1e-2, nwaves: int = 8):
    """amp * (1/8) sum_k cos(k_k . r + phi_k), |k_k| uniform in [0.2, 1] bohr^-1."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    out = np.zeros_like(x)
    for _ in range(nwaves):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        k = d * rng.uniform(0.2, 1.0)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        out += np.cos(k[0] * x + k[1] * y + k[2] * z + ph)
    return amp * out / nwaves


# ----------------------------------------------------------------------------
# Geometries
# ----------------------------------------------------------------------------

def _random_cluster(rng, n, box, min_dist, Zpool):
    pos = []
    tries = 0
    while len(pos) < n:
        p = rng.uniform(0.0, box, size=3)
        tries += 1
        if tries > 200000:
            raise RuntimeError("cannot place atoms")
        if pos and np.min(np.linalg.norm(np.array(pos) - p, axis=1)) < min_dist:
            continue
        pos.append(p)
    return np.array(pos), np.array(Zpool, dtype=np.int32)


def cluster_composition(rng, n):
    n_pb = int(round(0.2 * n))
    n_i = int(round(0.3 * n))
    n_l = n - n_pb - n_i
    light = rng.choice([1, 6, 7], size=n_l)
    Z = np.concatenate([np.full(n_pb, 82), np.full(n_i, 53), light]).astype(np.int32)
    return Z


def perovskite_slab(rng, nx, ny, nlayers, n_target=None, bi_sites=1, vacancies=0, a=6.3,
                    period=16.0, dist=0.2):
    """2D hybrid perovskite-like slab (angstrom): per site one Pb/Bi, two
    bridging and two apical I, and C16 H24 N2 placed at seeded interlayer
    positions with a 1.0 angstrom minimum spacing."""
    sites = [(i, j, k) for k in range(nlayers) for j in range(ny) for i in range(nx)]
    nsite = len(sites)
    perm = rng.permutation(nsite)
    vac = set(perm[:vacancies].tolist())
    bi = set(perm[vacancies:vacancies + bi_sites].tolist())
    inorg_pos, inorg_Z = [], []
    for s, (i, j, k) in enumerate(sites):
        base = np.array([i * a, j * a, k * period])
        if s not in vac:
            inorg_pos.append(base); inorg_Z.append(83 if s in bi else 82)
        for off in ([a / 2, 0, 0], [0, a / 2, 0], [0, 0, a / 2], [0, 0, -a / 2]):
            inorg_pos.append(base + np.array(off)); inorg_Z.append(53)
    inorg_pos = np.array(inorg_pos) + rng.uniform(-dist, dist, size=(len(inorg_pos), 3))
    org_unit = [6] * 16 + [1] * 24 + [7] * 2
    org_pos, org_Z = [], []
    allpos = list(inorg_pos)
    for s, (i, j, k) in enumerate(sites):
        for zc in org_unit:
            for _ in range(100000):
                p = np.array([i * a + rng.uniform(-a / 2, a / 2), j * a + rng.uniform(-a / 2, a / 2),
                              k * period + a / 2 + 1.0 + rng.uniform(0.0, period - a - 2.0)])
                d = np.min(np.linalg.norm(np.array(allpos) - p, axis=1))
                if d >= 1.0:
                    break
            else:
                raise RuntimeError("cannot place organic atom")
            allpos.append(p); org_pos.append(p); org_Z.append(zc)
    org_pos = np.array(org_pos)
    org_Z = np.array(org_Z, dtype=np.int32)
    if n_target is not None:
        n_keep = n_target - len(inorg_Z)
        keep = np.sort(rng.permutation(len(org_Z))[:n_keep])
        org_pos, org_Z = org_pos[keep], org_Z[keep]
    pos = np.concatenate([inorg_pos, org_pos])
    Z = np.concatenate([np.array(inorg_Z, dtype=np.int32), org_Z])
    return pos, Z


# ----------------------------------------------------------------------------
# Named configurations
# ----------------------------------------------------------------------------

def _assemble(name, Z, R, basis, grid, v, molecule=None, meta=None):
    x, y, z, w, owner = grid
    return Workload(name=name, Z=np.ascontiguousarray(Z, dtype=np.int32),
                    R=np.ascontiguousarray(R, dtype=np.float64), x=x, y=y, z=z, w=w, pt_atom=owner,
                    v=np.ascontiguousarray(v), molecule=molecule, meta=meta or {}, **basis)


def config_small(nint: int = 512, nrad: int = 40, nang: int = 110):
    """Pb at the origin and two I at +-2.9 angstrom on x; 3s2p1d per atom (42 NAOs),
    40 x 110 points per atom (13,200), Becke weights, v = sum -Z erf(r/0.5)/r."""
    k = 1
    Z = np.array([82, 53, 53], dtype=np.int32)
    R = np.array([[0.0, 0, 0], [2.9, 0, 0], [-2.9, 0, 0]]) * ANGSTROM
    basis = make_basis(Z, "small", 2000 + k, 6.0 * ANGSTROM, nint)
    grid = atom_grids(R, Z, lambda z: nrad, lambda z: nang, 3000 + k, r_comp=12.0 * ANGSTROM)
    v = model_potential(R, Z, grid[0], grid[1], grid[2])
    return _assemble("pb-i2-42nao", Z, R, basis, grid, v,
                     meta=dict(config="small-3-atom", p_max=128, seeds=dict(basis=2001, grid=3001)))


def config_cluster(n_atoms: int = 120, nint: int = 512, nrad: int = 60, nang: int = 302, k: int = 2,
                   box_ang: float = 20.0, noise: bool = True):
    """Seeded random cluster: 20% Pb, 30% I, 50% {H,C,N} in a 20 angstrom cube,
    1.8 angstrom minimum spacing; heavy 26 NAOs, light 5; 60 x 302 points/atom."""
    rng = np.random.default_rng(np.random.PCG64(1000 + k))
    Z = cluster_composition(rng, n_atoms)
    R, _ = _random_cluster(rng, n_atoms, box_ang, 1.8, Z)
    R = R * ANGSTROM
    basis = make_basis(Z, "main", 2000 + k, 6.0 * ANGSTROM, nint)
    grid = atom_grids(R, Z, lambda z: nrad, lambda z: nang, 3000 + k, r_comp=12.0 * ANGSTROM)
    v = model_potential(R, Z, grid[0], grid[1], grid[2])
    if noise:
        v = v + smooth_noise(grid[0], grid[1], grid[2], 4000 + k)
    return _assemble("cluster-%d" % n_atoms, Z, R, basis, grid, v,
                     meta=dict(config="random-cluster-%d" % n_atoms, p_max=300,
                               seeds=dict(geometry=1000 + k, basis=2000 + k, grid=3000 + k, noise=4000 + k)))


def config_slab(n_target: int = 1000, nx: int = 4, ny: int = 3, nlayers: int = 2, bi_sites: int = 1,
                vacancies: int = 0, light_grid=(50, 146), k: int = 3, nint: int = 512):
    """Perovskite-like slab (2D hybrid perovskite composition), heavy atoms 60 x 302
    points, light atoms per `light_grid`, Becke competing radius 5 angstrom and a
    12 angstrom shifted cut on the model potential (both documented input choices)."""
    rng = np.random.default_rng(np.random.PCG64(1000 + k))
    pos, Z = perovskite_slab(rng, nx, ny, nlayers, n_target=n_target, bi_sites=bi_sites,
                             vacancies=vacancies)
    R = pos * ANGSTROM
    basis = make_basis(Z, "main", 2000 + k, 6.0 * ANGSTROM, nint)
    heavy = lambda z: z >= 21
    grid = atom_grids(R, Z, lambda z: 60 if heavy(z) else light_grid[0],
                      lambda z: 302 if heavy(z) else light_grid[1], 3000 + k, r_comp=5.0 * ANGSTROM)
    v = model_potential(R, Z, grid[0], grid[1], grid[2], r_cut=12.0 * ANGSTROM)
    v = v + smooth_noise(grid[0], grid[1], grid[2], 4000 + k)
    return _assemble("slab-%d" % len(Z), Z, R, basis, grid, v,
                     meta=dict(config="perovskite-slab-%d" % len(Z), p_max=300,
                               seeds=dict(geometry=1000 + k, basis=2000 + k, grid=3000 + k, noise=4000 + k)))


def config_pepi_3383():
    """(6x6)x2 PEPI-shaped slab: 72 sites, one Pb vacancy, two Bi -> 3,383 atoms;
    light atoms on 40 x 86 grids."""
    return config_slab(n_target=None, nx=6, ny=6, nlayers=2, bi_sites=2, vacancies=1, light_grid=(40, 86), k=5)


def config_molecules(n_mol: int = 64, k: int = 4, nint: int = 512, nrad: int = 60, nang: int = 302,
                     sizes: Optional[Sequence[int]] = None):
    """Independent molecules of 8..80 atoms (cluster element mix), each in its own
    cube of side 20 angstrom (N/120)^(1/3), placed on a lattice far enough apart that
    no basis function or partition weight couples two molecules."""
    rng = np.random.default_rng(np.random.PCG64(1000 + k))
    if sizes is None:
        sizes = rng.integers(8, 81, size=n_mol)
    Zs, Rs, mol = [], [], []
    spacing = 20.0 + 2 * 6.0 + 14.0  # angstrom: cube + two cutoffs + Becke competing radius margin
    side = int(math.ceil(len(sizes) ** (1.0 / 3.0)))
    for m, n in enumerate(sizes):
        Zm = cluster_composition(rng, int(n))
        box = 20.0 * (n / 120.0) ** (1.0 / 3.0)
        Rm, _ = _random_cluster(rng, int(n), box, 1.8, Zm)
        cell = np.array([m % side, (m // side) % side, m // (side * side)], dtype=np.float64)
        Rs.append(Rm + cell * spacing)
        Zs.append(Zm)
        mol.append(np.full(int(n), m, dtype=np.int32))
    Z = np.concatenate(Zs)
    R = np.concatenate(Rs) * ANGSTROM
    molecule = np.concatenate(mol)
    basis = make_basis(Z, "main", 2000 + k, 6.0 * ANGSTROM, nint)
    grid = atom_grids(R, Z, lambda z: nrad, lambda z: nang, 3000 + k, r_comp=12.0 * ANGSTROM)
    # potential of each molecule from its own atoms only
    v = np.zeros(grid[0].shape[0])
    owner_mol = molecule[grid[4]]
    for m in range(len(sizes)):
        sel = np.nonzero(owner_mol == m)[0]
        am = np.nonzero(molecule == m)[0]
        v[sel] = model_potential(R[am], Z[am], grid[0][sel], grid[1][sel], grid[2][sel])
    v = v + smooth_noise(grid[0], grid[1], grid[2], 4000 + k)
    return _assemble("molecules-%d" % len(sizes), Z, R, basis, grid, v, molecule=molecule,
                     meta=dict(config="molecules-%d" % len(sizes), p_max=300, sizes=[int(s) for s in sizes],
                               seeds=dict(geometry=1000 + k, basis=2000 + k, grid=3000 + k, noise=4000 + k)))


def split_molecules(wl: Workload) -> List[Workload]:
    """The independent systems of a batched-molecule workload, one Workload each."""
    assert wl.molecule is not None
    out = []
    owner_mol = wl.molecule[wl.pt_atom]
    for m in range(int(wl.molecule.max()) + 1):
        am = np.nonzero(wl.molecule == m)[0]
        pts = np.nonzero(owner_mol == m)[0]
        remap = np.full(wl.n_atoms, -1, dtype=np.int32)
        remap[am] = np.arange(am.shape[0], dtype=np.int32)
        s_lo = wl.atom_shell_off[am[0]]
        s_hi = wl.atom_shell_off[am[-1] + 1]
        out.append(Workload(
            name="%s-m%d" % (wl.name, m), Z=wl.Z[am].copy(), R=wl.R[am].copy(),
            atom_shell_off=(wl.atom_shell_off[am[0]:am[-1] + 2] - s_lo).astype(np.int32),
            shell_l=wl.shell_l[s_lo:s_hi].copy(), shell_rcut=wl.shell_rcut[s_lo:s_hi].copy(),
            shell_nint=wl.shell_nint[s_lo:s_hi].copy(), shell_coef_off=wl.shell_coef_off[s_lo:s_hi].copy(),
            coef=wl.coef, shell_alpha=wl.shell_alpha[s_lo:s_hi].copy(), shell_gcoef=wl.shell_gcoef[s_lo:s_hi].copy(),
            x=wl.x[pts].copy(), y=wl.y[pts].copy(), z=wl.z[pts].copy(), w=wl.w[pts].copy(),
            pt_atom=remap[wl.pt_atom[pts]], v=wl.v[pts].copy(), meta=dict(parent=wl.name, molecule=m)))
    return out


CONFIGS = {
    "small": config_small,
    "cluster": config_cluster,
    "slab": config_slab,
    "molecules": config_molecules,
    "pepi": config_pepi_3383,
}


# ----------------------------------------------------------------------------
# Pair list and seeded spinor density matrices
# ----------------------------------------------------------------------------

def atom_pairs(wl: Workload) -> np.ndarray:
    """Atom pairs (A <= B) whose basis supports can overlap: |R_A - R_B| < rcut_A + rcut_B.
    Sorted by (A, B).  int32[npairs, 2]."""
    rc = wl.atom_rcut()
    out = []
    for a in range(wl.n_atoms):
        d = np.linalg.norm(wl.R[a:] - wl.R[a][None, :], axis=1)
        bs = np.nonzero(d < rc[a] + rc[a:])[0] + a
        for b in bs:
            out.append((a, b))
    return np.array(out, dtype=np.int32).reshape(-1, 2)


def spinor_density(wl: Workload, pairs: np.ndarray, seed: int, scale: float = 0.1, decay_bohr: float = 2.0):
    """Seeded Hermitian spinor density matrix on the given pair blocks.

    Off-diagonal blocks (A < B): D_AB = scale exp(-R_AB / decay) (X + iY);
    diagonal blocks: (X + X^H)/2 with X = G1 + i G2; G ~ N(0,1).  Each block is a
    (2 nA) x (2 nB) complex matrix, rows = (spin, function of A), spin-major.
    The block of pair p uses generator stream (seed, A, B)."""
    nfn = wl.atom_nfn()
    blocks = []
    for (a, b) in pairs:
        rng = np.random.default_rng(np.random.PCG64([seed, int(a), int(b)]))
        na, nb = 2 * nfn[a], 2 * nfn[b]
        X = rng.standard_normal((na, nb)) + 1j * rng.standard_normal((na, nb))
        if a == b:
            blocks.append(0.5 * (X + X.conj().T) * scale)
        else:
            rab = float(np.linalg.norm(wl.R[a] - wl.R[b]))
            blocks.append(scale * math.exp(-rab / decay_bohr) * X)
    return blocks


# ----------------------------------------------------------------------------
# Ket potentials and small-component bases (the paper's Q4C H integrand)
# ----------------------------------------------------------------------------

def hermite_table(fun, rcut: float, nint: int) -> np.ndarray:
    """Cubic-Hermite coefficients of fun (returning value and r-derivative on an
    array of radii) on knots r_j = rcut (j/nint)^2, in the radial-table format
    (float64[nint, 4], t in [0,1) per interval).  Exact for cubics in r."""
    j = np.arange(nint + 1, dtype=np.float64)
    r = rcut * (j / nint) ** 2
    f, d = fun(r)
    h = r[1:] - r[:-1]
    f0, f1 = f[:-1], f[1:]
    d0, d1 = d[:-1] * h, d[1:] * h
    out = np.empty((nint, 4))
    out[:, 0] = f0
    out[:, 1] = d0
    out[:, 2] = 3.0 * (f1 - f0) - 2.0 * d0 - d1
    out[:, 3] = 2.0 * (f0 - f1) + d0 + d1
    return out


def smeared_nucleus(r, Z: float, a_smear: float = 0.5):
    """Z erf(r/a)/r (the negative of the smeared-nucleus model potential of one
    atom) and its r-derivative; finite at r = 0 (series below r = 1e-4 a)."""
    r = np.asarray(r, dtype=np.float64)
    x = r / a_smear
    small = x < 1e-4
    xs = np.where(small, 1.0, x)
    c = 2.0 / math.sqrt(math.pi)
    from scipy.special import erf as _erf
    val = np.where(small, Z * c / a_smear * (1.0 - x * x / 3.0),
                   Z * _erf(xs) / (xs * a_smear))
    der = np.where(small, -Z * c / a_smear * (2.0 * x / 3.0) / a_smear,
                   Z * (c * np.exp(-xs * xs) / xs - _erf(xs) / (xs * xs)) / (a_smear * a_smear))
    return val, der


def _species_key(wl: Workload, a: int, k: int):
    return (int(wl.Z[a]), k)


def ket_tables(wl: Workload, shell_eps: np.ndarray, a_smear: float = 0.5) -> Workload:
    """Attach u_s(r) = eps_s + Z_A erf(r/a)/r to every shell s of atom A: the ket
    potential eps_s - V_s(r) of a free-atom-like shell whose defining potential is
    the smeared-nucleus model potential of its own atom.  Shells with the same
    (Z, eps, rcut, nint) share one table."""
    shell_eps = np.asarray(shell_eps, dtype=np.float64)
    tabs: Dict = {}
    chunks: List[np.ndarray] = []
    offs = np.zeros(wl.n_shells, dtype=np.int64)
    off = 0
    for a in range(wl.n_atoms):
        for s in range(wl.atom_shell_off[a], wl.atom_shell_off[a + 1]):
            key = (int(wl.Z[a]), float(shell_eps[s]), float(wl.shell_rcut[s]), int(wl.shell_nint[s]))
            if key not in tabs:
                eps, Z = key[1], key[0]
                t = hermite_table(lambda r: (lambda v, d: (v + eps, d))(*smeared_nucleus(r, Z, a_smear)),
                                  key[2], key[3])
                tabs[key] = off
                chunks.append(t.reshape(-1))
                off += t.size
            offs[s] = tabs[key]
    return dataclasses.replace(wl, shell_u_off=offs, u_coef=np.ascontiguousarray(np.concatenate(chunks)),
                               shell_eps=shell_eps.copy())


def with_ket(wl: Workload, seed: int, eps_range=(-2.0, -0.05)) -> Workload:
    """Seeded orbital energies eps per (species, shell index), uniform in eps_range
    (Ha), and the matching ket-potential tables."""
    eps = np.zeros(wl.n_shells)
    cache: Dict = {}
    for a in range(wl.n_atoms):
        s0 = wl.atom_shell_off[a]
        for k, s in enumerate(range(s0, wl.atom_shell_off[a + 1])):
            key = _species_key(wl, a, k)
            if key not in cache:
                rng = np.random.default_rng(np.random.PCG64([seed, key[0], k]))
                cache[key] = float(rng.uniform(*eps_range))
            eps[s] = cache[key]
    return ket_tables(wl, eps)


def poly_ket_tables(wl: Workload, eps: Sequence[float], kq: Sequence[float]) -> Workload:
    """u_s(r) = eps_s + kq_s r^2 per shell (a quadratic: the cubic table is exact).
    For closed-form pins."""
    chunks, offs, off = [], np.zeros(wl.n_shells, dtype=np.int64), 0
    for s in range(wl.n_shells):
        e, k = float(eps[s]), float(kq[s])
        t = hermite_table(lambda r: (e + k * r * r, 2.0 * k * r), float(wl.shell_rcut[s]), int(wl.shell_nint[s]))
        offs[s] = off
        chunks.append(t.reshape(-1))
        off += t.size
    return dataclasses.replace(wl, shell_u_off=offs, u_coef=np.ascontiguousarray(np.concatenate(chunks)),
                               shell_eps=np.asarray(eps, dtype=np.float64).copy())


def small_component(wl: Workload, seed: int, alpha_range=(0.3, 30.0)) -> Workload:
    """The small-component scalar basis of a large-component workload (Eq. 12b):
    every large shell l gives small shells l~ = l + 1 (j = l + 1/2) and, for
    l >= 1, l~ = l - 1 (j = l - 1/2).  Radials Q(r)/r are seeded normalised
    3-Gaussian sums per (species, shell) on the parent shell's cutoff and knots;
    each small shell takes its parent's eps, and its ket table is rebuilt from
    its own atom's smeared-nucleus potential.  Same grid, atoms and v."""
    rows = []  # (atom, l~, parent shell)
    for a in range(wl.n_atoms):
        for s in range(wl.atom_shell_off[a], wl.atom_shell_off[a + 1]):
            l = int(wl.shell_l[s])
            rows.append((a, l + 1, s))
            if l >= 1:
                rows.append((a, l - 1, s))
    cache: Dict = {}
    chunks: List[np.ndarray] = []
    off = 0
    aso = np.zeros(wl.n_atoms + 1, dtype=np.int32)
    sl, sr, sn, so, sa, sc, eps = [], [], [], [], [], [], []
    k_of_atom: Dict[int, int] = {}
    for (a, lt, s) in rows:
        k = k_of_atom.get(a, 0)
        k_of_atom[a] = k + 1
        key = (int(wl.Z[a]), k, float(wl.shell_rcut[s]), int(wl.shell_nint[s]))
        if key not in cache:
            rng = np.random.default_rng(np.random.PCG64([seed, key[0], k]))
            lo, hi = np.log(alpha_range[0]), np.log(alpha_range[1])
            alpha = np.sort(np.exp(rng.uniform(lo, hi, size=3)))
            c = rng.uniform(0.2, 1.0, size=3)
            c = c * gauss_norm(lt, alpha, c)
            tab = spline_table(alpha, c, key[2], key[3])
            cache[key] = (off, alpha, c)
            chunks.append(tab.reshape(-1))
            off += tab.size
        o, alpha, c = cache[key]
        sl.append(lt); sr.append(key[2]); sn.append(key[3]); so.append(o); sa.append(alpha); sc.append(c)
        eps.append(float(wl.shell_eps[s]) if wl.shell_eps is not None else 0.0)
        aso[a + 1] = len(sl)
    for a in range(wl.n_atoms):
        aso[a + 1] = max(aso[a + 1], aso[a])
    ws = dataclasses.replace(
        wl, name=wl.name + "-small", atom_shell_off=aso, shell_l=np.array(sl, dtype=np.int32),
        shell_rcut=np.array(sr, dtype=np.float64), shell_nint=np.array(sn, dtype=np.int32),
        shell_coef_off=np.array(so, dtype=np.int64), coef=np.ascontiguousarray(np.concatenate(chunks)),
        shell_alpha=np.array(sa).reshape(-1, 3), shell_gcoef=np.array(sc).reshape(-1, 3),
        shell_u_off=None, u_coef=None, shell_eps=None)
    return ket_tables(ws, np.array(eps))


# ----------------------------------------------------------------------------
# Periodic cells (the paper's solids: Sec. II C, Sec. III A)
# ----------------------------------------------------------------------------

def periodic_noise(lat, x, y, z, seed: int, amp: float = 1e-2, nwaves: int = 8):
    """amp * (1/8) sum_k cos(G_k . r + phi_k) with G_k reciprocal lattice vectors
    2 pi L^-T n, n integer in [-2, 2]^3 (not 0): lattice-periodic noise."""
    rng = np.random.default_rng(np.random.PCG64(seed))
    B = 2.0 * np.pi * np.linalg.inv(np.asarray(lat)).T
    out = np.zeros_like(x)
    for _ in range(nwaves):
        n = np.zeros(3)
        while not np.any(n):
            n = rng.integers(-2, 3, size=3).astype(np.float64)
        G = B @ n
        ph = rng.uniform(0.0, 2.0 * np.pi)
        out += np.cos(G[0] * x + G[1] * y + G[2] * z + ph)
    return amp * out / nwaves


CSPBBR3_CELL = ((55, (0.0, 0.0, 0.0)), (82, (0.5, 0.5, 0.5)), (35, (0.5, 0.5, 0.0)), (35, (0.5, 0.0, 0.5)),
                (35, (0.0, 0.5, 0.5)))  # cubic perovskite ABX3: A corner, B body centre, X face centres


def config_periodic(cells=(1, 1, 1), a_ang: float = 5.87, species=CSPBBR3_CELL, recipe: str = "main",
                    nrad: int = 40, nang: int = 110, k: int = 6, nint: int = 512, rcut_ang: float = 6.0,
                    distort_ang: float = 0.1):
    """A periodic cubic-perovskite cell (CsPbBr3-like: the paper's benchmark
    solid), n1 x n2 x n3 primitive cells with seeded displacements, as a plan
    workload: the cell's atoms first, then every periodic image whose
    functions reach the cell (its distance to the cell box below the cutoff).
    The grid holds the cell atoms' grids only, with Becke weights over all
    atoms (cell and images), so it integrates exactly one cell of a periodic
    integrand; v is the cut-and-shifted smeared-nucleus potential of every atom
    within 12 angstrom plus smooth noise.  meta: n_cell_atoms, cell_atom
    (image -> cell atom), shift (lattice translation of each atom, bohr),
    lattice (rows = lattice vectors, bohr).  The Becke competing radius is 5
    angstrom (as for the slabs)."""
    rng = np.random.default_rng(np.random.PCG64(1000 + k))
    n1, n2, n3 = cells
    a = a_ang * ANGSTROM
    lat = np.diag([n1 * a, n2 * a, n3 * a])
    Zc, Rc = [], []
    for i in range(n1):
        for j in range(n2):
            for l in range(n3):
                for z, f in species:
                    Zc.append(z)
                    Rc.append((np.array([i, j, l], dtype=np.float64) + np.array(f)) * a)
    Zc = np.array(Zc, dtype=np.int32)
    Rc = np.array(Rc) + rng.uniform(-1, 1, size=(len(Zc), 3)) * distort_ang * ANGSTROM
    rcut = rcut_ang * ANGSTROM
    lo, hi = np.zeros(3), np.diag(lat)

    def images(reach):
        out = []
        m = [int(np.ceil(reach / lat[d, d])) + 1 for d in range(3)]
        for t1 in range(-m[0], m[0] + 1):
            for t2 in range(-m[1], m[1] + 1):
                for t3 in range(-m[2], m[2] + 1):
                    if t1 == t2 == t3 == 0:
                        continue
                    T = np.array([t1, t2, t3], dtype=np.float64) @ lat
                    for c in range(len(Zc)):
                        p = Rc[c] + T
                        if np.linalg.norm(p - np.clip(p, lo, hi)) < reach:
                            out.append((c, T))
        return out

    img = images(rcut)
    r_comp = 5.0 * ANGSTROM
    Z = np.concatenate([Zc, np.array([Zc[c] for c, _ in img], dtype=np.int32)]).astype(np.int32)
    R = np.concatenate([Rc, np.array([Rc[c] + T for c, T in img]).reshape(-1, 3)])
    cell_atom = np.concatenate([np.arange(len(Zc)), np.array([c for c, _ in img], dtype=np.int64)]).astype(np.int32)
    shift = np.concatenate([np.zeros((len(Zc), 3)), np.array([T for _, T in img]).reshape(-1, 3)])
    basis = make_basis(Z, recipe, 2000 + k, rcut, nint)
    # partition over every atom a competing radius away from any point where a
    # function of the plan lives (those lie within 2 rcut of the cell)
    pimg = images(2 * rcut + r_comp + 1.0)
    Rw = np.concatenate([R, np.array([Rc[c] + T for c, T in pimg
                                      if not any(c == c2 and np.allclose(T, T2) for c2, T2 in img)]).reshape(-1, 3)])
    grid = atom_grids(Rc, Zc, lambda z: nrad, lambda z: nang, 3000 + k, r_comp=r_comp, R_partition=Rw)
    # potential: every atom within 12 angstrom of such points, cut and shifted at 12 angstrom
    vimg = images(2 * rcut + 12.0 * ANGSTROM + 1.0)
    Rp = np.concatenate([Rc, np.array([Rc[c] + T for c, T in vimg]).reshape(-1, 3)])
    Zp = np.concatenate([Zc, np.array([Zc[c] for c, _ in vimg], dtype=np.int32)])
    v = model_potential(Rp, Zp, grid[0], grid[1], grid[2], r_cut=12.0 * ANGSTROM)
    v = v + periodic_noise(lat, grid[0], grid[1], grid[2], 4000 + k)
    return _assemble("periodic-%dx%dx%d" % tuple(cells), Z, R, basis, grid, v,
                     meta=dict(config="periodic-perovskite-%dx%dx%d" % tuple(cells), p_max=300,
                               n_cell_atoms=len(Zc), cell_atom=cell_atom, shift=shift, lattice=lat,
                               seeds=dict(geometry=1000 + k, basis=2000 + k, grid=3000 + k, noise=4000 + k)))


def pin_workload(Z, R_bohr, shells_per_atom, nrad=300, ntheta=12, nphi=24, rcut=6.0 * ANGSTROM, nint=2048,
                 v=None, rm=1.0, tapered=True, name="pin"):
    """Small workload on product grids (Gauss-Chebyshev radial x Gauss-Legendre
    theta x uniform phi) for closed-form pins.  `v` is a callable v(x, y, z) or
    None for v = 1.  Several atoms get Becke weights over all atoms."""
    Z = np.asarray(Z, dtype=np.int32)
    R = np.asarray(R_bohr, dtype=np.float64).reshape(-1, 3)
    basis = custom_basis(Z, shells_per_atom, rcut, nint, tapered)
    r, wr = radial_grid(nrad, rm)
    u, wu = product_sphere(ntheta, nphi)
    xs, ys, zs, ws, own = [], [], [], [], []
    for a in range(len(Z)):
        p = (r[:, None, None] * u[None, :, :]).reshape(-1, 3) + R[a][None, :]
        xs.append(p[:, 0]); ys.append(p[:, 1]); zs.append(p[:, 2])
        ws.append((wr[:, None] * wu[None, :]).reshape(-1))
        own.append(np.full(p.shape[0], a, dtype=np.int32))
    x, y, z = (np.ascontiguousarray(np.concatenate(t)) for t in (xs, ys, zs))
    owner = np.ascontiguousarray(np.concatenate(own))
    wq = np.concatenate(ws)
    wb = becke(R, x, y, z, owner, 1e9) if len(Z) > 1 else np.ones_like(wq)
    vv = np.ones_like(x) if v is None else np.asarray(v(x, y, z), dtype=np.float64)
    return _assemble(name, Z, R, basis, (x, y, z, np.ascontiguousarray(wq * wb), owner), vv)
