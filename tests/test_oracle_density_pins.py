"""Pins for the oracle's forward density update from a spinor density matrix:
the scalar density matrices of both components (the reverse of Eq. 33, the
paper's D' = sum D G* G) and the density with its gradient on the grid.

  * reverse transform                -> duality with the (pinned) forward transform:
                                        sum_c sum C^c X^c = sum f Re sum D X+ for any X
  * density on the grid, both parts  -> electron count sum_g w_g n_g = Re Tr(D S+)
  * gradient                          -> central differences of n
  * n itself                          -> the (pinned) adjoint/density oracle, LL term
"""
import numpy as np
import pytest

import oracle
import workload as W


@pytest.fixture(scope="module")
def setup():
    wl = W.with_ket(W.config_small(nrad=24, nang=50), 7001)
    ws = W.small_component(wl, 7002)
    pairs = W.atom_pairs(wl)
    GL, GS = oracle.spinor_G(wl, ws)
    D = W.spinor_density(wl, pairs, 5001)  # Hermitian, (2 nA) x (2 nB) per pair
    C = oracle.spinor_density_to_scalar(pairs, D, GL, GS)
    return wl, ws, pairs, GL, GS, D, C


def _f(a, b):
    return 1.0 if a == b else 2.0


def test_reverse_is_dual_to_forward(setup):
    wl, ws, pairs, GL, GS, D, C = setup
    rng = np.random.default_rng(8201)
    nL, nS = wl.atom_nfn(), ws.atom_nfn()
    XL = [rng.standard_normal((2, nL[a], nL[b])) for a, b in pairs]
    XS = [rng.standard_normal((2, nS[a], nS[b])) for a, b in pairs]
    Xp = oracle.spinor_transform(pairs, XL, XS, GL, GS)
    for q in range(2):
        lhs = sum(float(np.sum(C[p][0] * XL[p][q]) + np.sum(C[p][1] * XS[p][q])) for p in range(len(pairs)))
        rhs = sum(_f(a, b) * float(np.real(np.sum(D[p] * Xp[p][q]))) for p, (a, b) in enumerate(pairs))
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(rhs)), (q, lhs, rhs)


def test_scalar_density_matrices_symmetric_on_diagonal_pairs(setup):
    wl, ws, pairs, GL, GS, D, C = setup
    for p, (a, b) in enumerate(pairs):
        if a == b:
            for c in C[p]:
                assert np.max(np.abs(c - c.T)) < 1e-14 * max(1.0, np.max(np.abs(c)))


def test_electron_count_on_the_grid(setup):
    """sum_g w_g (n^L_g + n^S_g) = Re Tr(D S+) with S+ the forward transform of
    the oracle's overlap blocks: the same grid sums taken in two orders."""
    wl, ws, pairs, GL, GS, D, C = setup
    nL = oracle.density_grad(wl, pairs, [c[0] for c in C])[:, 0]
    nS = oracle.density_grad(ws, pairs, [c[1] for c in C])[:, 0]
    lhs = float(np.sum(wl.w * (nL + nS)))
    bl = oracle.pair_blocks_hs(wl, pairs)
    bs = oracle.pair_blocks_hs(ws, pairs)
    Sp = oracle.spinor_transform(pairs, bl, bs, GL, GS)
    rhs = sum(_f(a, b) * float(np.real(np.sum(D[p] * Sp[p][1]))) for p, (a, b) in enumerate(pairs))
    assert abs(lhs - rhs) <= 1e-11 * float(np.sum(wl.w * (np.abs(nL) + np.abs(nS)))), (lhs, rhs)


def test_density_matches_the_adjoint_oracle(setup):
    wl, ws, pairs, GL, GS, D, C = setup
    idx = np.arange(0, wl.n_points, 37)
    got = oracle.density_grad(wl, pairs, [c[0] for c in C], idx=idx)[:, 0]
    blocks = [np.concatenate([c[0][None], np.zeros((4,) + c[0].shape)]) for c in C]
    ref = oracle.density(wl, pairs, blocks, idx=idx, weight_mode=0)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_gradient_central_differences(setup):
    wl, ws, pairs, GL, GS, D, C = setup
    rng = np.random.default_rng(8202)
    for comp, w in ((0, wl), (1, ws)):
        cb = [c[comp] for c in C]
        # points near the atoms, where n varies fastest
        idx = np.sort(rng.choice(w.n_points, size=24, replace=False))
        g = oracle.density_grad(w, pairs, cb, idx=idx)
        h = 1e-4
        for k in range(3):
            dx = np.zeros(3)
            dx[k] = h
            wp = w.subset_points(idx).translated([0, 0, 0])
            xp = (wp.x + dx[0], wp.y + dx[1], wp.z + dx[2])
            xm = (wp.x - dx[0], wp.y - dx[1], wp.z - dx[2])
            npl = oracle.density_grad(W.Workload(**{**w.__dict__, "x": xp[0], "y": xp[1], "z": xp[2]}), pairs, cb,
                                      idx=np.arange(idx.size))[:, 0]
            nmi = oracle.density_grad(W.Workload(**{**w.__dict__, "x": xm[0], "y": xm[1], "z": xm[2]}), pairs, cb,
                                      idx=np.arange(idx.size))[:, 0]
            fd = (npl - nmi) / (2 * h)
            sc = np.max(np.abs(g[:, 1:])) + 1e-300
            assert np.max(np.abs(fd - g[:, 1 + k])) <= 1e-6 * sc, (comp, k)
