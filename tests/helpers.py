"""Shared test helpers: layout conversion and comparison against the oracle.

Nothing here computes the method's arithmetic; it only rearranges arrays
between the library's store layout and the oracle's per-pair blocks."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def store_to_blocks(store: np.ndarray, pairs: np.ndarray, pair_off: np.ndarray, nfn: np.ndarray):
    """[5, store_len] -> list of [5, nA, nB] blocks."""
    out = []
    for p, (a, b) in enumerate(pairs):
        na, nb = int(nfn[a]), int(nfn[b])
        out.append(store[:, pair_off[p]:pair_off[p + 1]].reshape(5, na, nb))
    return out


def blocks_to_store(blocks, pair_off: np.ndarray) -> np.ndarray:
    L = int(pair_off[-1])
    st = np.zeros((5, L))
    for p, blk in enumerate(blocks):
        st[:, pair_off[p]:pair_off[p + 1]] = np.asarray(blk).reshape(5, -1)
    return st


def spinor_to_blocks(spin: np.ndarray, pairs, pair_off, nfn):
    """[4 store_len, 2] float64 (re, im) -> list of complex [2nA, 2nB]."""
    c = spin[:, 0] + 1j * spin[:, 1]
    out = []
    for p, (a, b) in enumerate(pairs):
        na, nb = int(nfn[a]), int(nfn[b])
        out.append(c[4 * pair_off[p]:4 * pair_off[p + 1]].reshape(2 * na, 2 * nb))
    return out


def spinor_from_blocks(blocks, pair_off) -> np.ndarray:
    L = int(pair_off[-1])
    out = np.zeros((4 * L, 2))
    for p, blk in enumerate(blocks):
        c = np.asarray(blk).reshape(-1)
        out[4 * pair_off[p]:4 * pair_off[p + 1], 0] = c.real
        out[4 * pair_off[p]:4 * pair_off[p + 1], 1] = c.imag
    return out


def rel_to_scale(got, ref, scale, floor=0.0):
    """max |got - ref| / (scale + floor) elementwise."""
    return float(np.max(np.abs(got - ref) / (scale + floor))) if np.size(got) else 0.0


def gamma(k: int) -> float:
    """gamma_k = k u / (1 - k u) with the FP32 unit roundoff u = 2^-24."""
    return k * 2.0 ** -24 / (1 - k * 2.0 ** -24)


# The stated bound of the split precisions' W elements: FP32 partial sums over
# 16 points, then FP64.  Per 16 points an element sums at most 48 products
# (16 points x 3) whose two operands (sqrt|w v| times a gradient component,
# formed in FP64) are each rounded to FP32 once: gamma_52 of the magnitudes of
# its terms for Q4C_PREC_F32, which also covers operands rounded three times;
# with hi + lo operands every product is three FP32 products, 144 per 16
# points: gamma_150 for Q4C_PREC_SPLIT_F32.  Values below
# FP32's normal range (2^-126) lose their relative precision; the far tails of
# tight functions reach it, hence an absolute floor, far below any bar.
# Q4C_PREC_BF16X3 (BF16 MFMA, operands split into three BF16 parts): the
# split and the dropped terms cost 3 units of 2^-23 per product, and the
# MFMA's FP32 sums over one 16-point chunk at most 7 + 36 (groups of 8
# products aligned to their largest, then added to the accumulator: 9 MFMAs
# of 4 groups per element), the spin-orbit difference and the FP64 addition
# 2 more: 48 2^-23, and 50 with the magnitudes of the six kept terms in place
# of |a b|.
SPLIT_GAMMA = {1: gamma(150), 2: gamma(52), 3: 50 * 2.0 ** -23}
SPLIT_FLOOR = 1e-25  # Ha


def split_bound_worst(got_blocks, ref_blocks, scale_blocks, precision):
    """Largest |got - ref| / ((gamma + 1e-12) A_ij + floor) over the W parts
    (1..4) of every element, A_ij the oracle's per-element scale."""
    worst = 0.0
    g_ = SPLIT_GAMMA[precision] + 1e-12
    for g, r, s in zip(got_blocks, ref_blocks, scale_blocks):
        g, r, s = g[1:], r[1:], s[1:]
        nz = s > 0
        assert np.all(g[~nz] == r[~nz])
        if np.any(nz):
            worst = max(worst, float(np.max(np.abs(g - r)[nz] / (g_ * s[nz] + SPLIT_FLOOR))))
    return worst


def per_point_worst(got, ref, scale, floor=0.0):
    """max |got - ref| / (scale + floor) over the entries whose scale is
    positive; where the scale is 0 (no term reaches the entry: outside every
    support) the two must agree exactly.  The scale of an entry is the
    oracle's sum of the magnitudes of the terms it is summed from.  floor
    (absolute) covers values in the FP64 subnormal range (below 2.2e-308),
    where each operation may lose up to 2^-1074 absolutely and no relative
    bar can hold: tails of tight Gaussians reach it inside the cutoff."""
    got, ref, scale = (np.asarray(t, dtype=np.float64) for t in (got, ref, scale))
    zero = ~(scale > 0)
    assert np.array_equal(got[zero], ref[zero]), "entries with no terms differ"
    nz = ~zero
    return float(np.max(np.abs(got[nz] - ref[nz]) / (scale[nz] + floor))) if np.any(nz) else 0.0


def spinor_coef_scale(pairs, D_blocks):
    """Per stored element and part, the scale of the spinor -> coefficient
    conversion: f times the sum of the magnitudes of the four spin entries of
    D for (i, j) (every coefficient is a signed sum of at most two of them, so
    one rounding leaves it within 2^-53 of this scale), f = 2 for pairs of two
    atoms, 1 within an atom."""
    out = []
    for (a, b), D in zip(pairs, D_blocks):
        nA, nB = D.shape[0] // 2, D.shape[1] // 2
        m = np.abs(D).reshape(2, nA, 2, nB).sum(axis=(0, 2))
        f = 1.0 if a == b else 2.0
        out.append(np.broadcast_to(f * m, (5, nA, nB)).copy())
    return out
