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
