"""Pins for the oracle's Bloch sums of unit-cell integrals (Sec. II C):
O_ab(k) = sum over image pairs of exp(i k.(T_b' - T_a')) O_a'b'.

  * the sum itself against explicit Bloch functions
    psi_k(r) = sum_M exp(i k.T_M) phi(r - T_M) tabulated on the cell's grid and
    integrated by brute force (V, Ws and the spin-orbit parts)
  * k -> k + G invariance (G a reciprocal lattice vector), O(-k) = conj O(k)
  * the cell's diagonal blocks Hermitian (V, Ws) / anti-Hermitian (Wso)
"""
import numpy as np
import pytest

import oracle
import workload as W

C = W.C_LIGHT
CP = 1.0 / (4.0 * C * C)


@pytest.fixture(scope="module")
def cell():
    # one Pb atom per simple cubic cell, the small basis (3s2p1d), a coarse grid
    wl = W.config_periodic(species=((82, (0.0, 0.0, 0.0)),), a_ang=4.0, recipe="small", nrad=20, nang=50, k=61)
    pairs = W.atom_pairs(wl)
    blocks = oracle.pair_blocks(wl, pairs)
    lat = wl.meta["lattice"]
    rng = np.random.default_rng(8401)
    B = 2 * np.pi * np.linalg.inv(lat).T
    kp = (rng.uniform(-0.5, 0.5, size=(3, 3)) @ B.T)
    return wl, pairs, blocks, kp, B


def test_against_explicit_bloch_functions(cell):
    wl, pairs, blocks, kp, _ = cell
    ca, sh = wl.meta["cell_atom"], wl.meta["shift"]
    got = oracle.bloch_sum(ca, sh, pairs, blocks, kp)[(0, 0)]
    phi, grad = oracle.tabulate(wl, wl.x, wl.y, wl.z)  # all functions of all images at the cell's points
    nfn = wl.atom_nfn()
    n0 = int(nfn[0])
    om = wl.w * wl.v
    for ik, k in enumerate(kp):
        psi = np.zeros((wl.n_points, n0), dtype=np.complex128)
        dpsi = np.zeros((wl.n_points, n0, 3), dtype=np.complex128)
        f0 = 0
        for A in range(wl.n_atoms):
            ph = np.exp(1j * (k @ sh[A]))
            psi += ph * phi[:, f0:f0 + n0]
            dpsi += ph * grad[:, f0:f0 + n0, :]
            f0 += int(nfn[A])
        V = np.einsum("g,gi,gj->ij", om, psi.conj(), psi)
        Ws = CP * np.einsum("g,gic,gjc->ij", om, dpsi.conj(), dpsi)
        cr = np.cross(dpsi.conj()[:, :, None, :], dpsi[:, None, :, :])  # [g, i, j, 3]
        Wso = CP * np.einsum("g,gijc->cij", om, cr)
        ref = [V, Ws, Wso[0], Wso[1], Wso[2]]
        for q in range(5):
            sc = np.max(np.abs(ref[q])) + 1e-300
            assert np.max(np.abs(got[ik, q] - ref[q])) <= 1e-11 * sc, (ik, q)


def test_reciprocal_lattice_and_time_reversal(cell):
    wl, pairs, blocks, kp, B = cell
    ca, sh = wl.meta["cell_atom"], wl.meta["shift"]
    G = B @ np.array([1.0, -2.0, 1.0])
    a = oracle.bloch_sum(ca, sh, pairs, blocks, kp)[(0, 0)]
    b = oracle.bloch_sum(ca, sh, pairs, blocks, kp + G[None, :])[(0, 0)]
    c = oracle.bloch_sum(ca, sh, pairs, blocks, -kp)[(0, 0)]
    sc = np.max(np.abs(a))
    assert np.max(np.abs(a - b)) <= 1e-11 * sc
    assert np.max(np.abs(c - a.conj())) <= 1e-13 * sc


def test_diagonal_blocks_hermitian(cell):
    wl, pairs, blocks, kp, _ = cell
    a = oracle.bloch_sum(wl.meta["cell_atom"], wl.meta["shift"], pairs, blocks, kp)[(0, 0)]
    for ik in range(kp.shape[0]):
        for q in range(5):
            M = a[ik, q]
            s = 1.0 if q < 2 else -1.0
            assert np.max(np.abs(M - s * M.conj().T)) <= 1e-13 * np.max(np.abs(M))


# ---------------------------------------------------------------------------
# The reverse direction: k-space density matrices -> coefficients on the
# stored image pairs (the periodic density matrix and density of Sec. II C)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def cell2():
    # Pb (26 functions) and N (5) per cubic cell: cell pairs (0,0), (0,1), (1,1)
    # and stored image pairs of both cell-atom orders
    wl = W.config_periodic(species=((82, (0.0, 0.0, 0.0)), (7, (0.5, 0.5, 0.5))), a_ang=4.5, recipe="main",
                           nrad=10, nang=26, k=62)
    pairs = W.atom_pairs(wl)
    m = wl.meta
    nfn = wl.atom_nfn()
    ca = m["cell_atom"]
    ncell = [int(nfn[list(ca).index(c)]) for c in range(m["n_cell_atoms"])]
    rng = np.random.default_rng(8411)
    B = 2 * np.pi * np.linalg.inv(m["lattice"]).T
    kp = rng.uniform(-0.5, 0.5, size=(3, 3)) @ B.T
    kw = rng.uniform(0.2, 1.0, size=3)
    # occupied states: coefficients C(k) over the cell's functions, occupations f
    nc, nocc = sum(ncell), 4
    C = rng.standard_normal((3, nc, nocc)) + 1j * rng.standard_normal((3, nc, nocc))
    f = rng.uniform(0.5, 2.0, size=nocc)
    return wl, pairs, ncell, kp, kw, C, f


def _rho_blocks(ncell, C, f):
    """rho(k)_mn = sum_l f_l C*_ml C_nl cut into cell-pair blocks a <= b."""
    rho = np.einsum("l,kml,knl->kmn", f, C.conj(), C)
    off = np.concatenate([[0], np.cumsum(ncell)])
    na = len(ncell)
    return {(a, b): rho[:, None, off[a]:off[a + 1], off[b]:off[b + 1]].copy()
            for a in range(na) for b in range(a, na)}


def test_density_matrix_against_explicit_bloch_states(cell2):
    """n(r) = sum_k w_k sum_l f_l |psi_lk(r)|^2 with psi_lk(r) = sum over the
    plan's atoms A' of exp(i k.T_A') sum_i C_{i(a),l}(k) phi_A'i(r), and its
    gradient 2 Re(psi* grad psi), at the grid points inside the cell box
    (where every function reaching the point belongs to the plan), against
    sum over stored pairs of the returned coefficients times phi_i phi_j."""
    wl, pairs, ncell, kp, kw, C, f = cell2
    m = wl.meta
    ca, sh = m["cell_atom"], m["shift"]
    nfn = wl.atom_nfn()
    coef = oracle.bloch_density(ca, sh, pairs, _rho_blocks(ncell, C, f), kp, kw, nfn)
    pts = np.stack([wl.x, wl.y, wl.z], axis=1)
    frac = pts @ np.linalg.inv(m["lattice"])
    idx = np.nonzero(np.all((frac >= 0.0) & (frac < 1.0), axis=1))[0]
    assert idx.size > 200
    got = oracle.density_grad(wl, pairs, [c[0] for c in coef], idx=idx)
    phi, grad = oracle.tabulate(wl, wl.x[idx], wl.y[idx], wl.z[idx])
    coff = np.concatenate([[0], np.cumsum(ncell)])
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
    for c in range(4):
        assert np.max(np.abs(got[:, c] - ref[:, c])) <= 1e-12 * sc[c], c


def test_density_matrix_is_the_adjoint_of_the_bloch_sum(cell2):
    """sum_k w_k sum over all cell function pairs rho_mn(k) O_mn(k) equals
    sum over stored pairs of coefficient * O^uc for real unit-cell blocks O
    (self pairs symmetric): the energy of a periodic density matrix, once in k
    space and once on the image pairs."""
    wl, pairs, ncell, kp, kw, C, f = cell2
    m = wl.meta
    ca, sh = m["cell_atom"], m["shift"]
    nfn = wl.atom_nfn()
    rng = np.random.default_rng(8412)
    O = []
    for A, B in pairs:
        x = rng.standard_normal((1, int(nfn[A]), int(nfn[B])))
        if A == B:
            x = 0.5 * (x + np.transpose(x, (0, 2, 1)))
        O.append(x)
    rho = _rho_blocks(ncell, C, f)
    Ok = oracle.bloch_sum(ca, sh, pairs, O, kp)
    e_k = 0.0
    for (a, b), r in rho.items():
        t = np.einsum("k,kqij,kqij->", kw, r, Ok[(a, b)])
        e_k += t.real if a == b else 2.0 * t.real  # the (b, a) block is the conjugate transpose
    coef = oracle.bloch_density(ca, sh, pairs, rho, kp, kw, nfn)
    e_r = sum(float(np.sum(c * o)) for c, o in zip(coef, O))
    assert abs(e_k - e_r) <= 1e-12 * sum(float(np.sum(np.abs(c * o))) for c, o in zip(coef, O))


def test_density_matrix_gamma_point_is_the_real_sum(cell2):
    """At k = 0 with weight 1 every image pair takes its cell pair's block
    unchanged: coefficient = f Re rho_ab (f = 2 off the self pairs), the
    transposed orientation conjugated."""
    wl, pairs, ncell, kp, kw, C, f = cell2
    m = wl.meta
    ca = m["cell_atom"]
    nfn = wl.atom_nfn()
    rho = _rho_blocks(ncell, C[:1], f)
    coef = oracle.bloch_density(ca, m["shift"], pairs, rho, np.zeros((1, 3)), np.ones(1), nfn)
    for (A, B), c in zip(pairs, coef):
        a, b = int(ca[A]), int(ca[B])
        blk = rho[(a, b)][0, 0].real if a <= b else rho[(b, a)][0, 0].T.real
        assert np.array_equal(c[0], (1.0 if A == B else 2.0) * blk)
