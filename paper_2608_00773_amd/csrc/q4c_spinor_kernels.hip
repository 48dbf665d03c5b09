// Scalar <-> spinor transformations.  Forward, of H and S (paper Sec. III A, Eq. 33, with
// the transformation matrices of Eq. 14): for every atom pair (A, B),
//   X+_AB = sum over components c (large, small) and spins s of
//           G^c_A[s]^H X^c_AB G^c_B[s],      X = H, S,
// where G^c_A[s] maps the scalar functions of component c on atom A to the
// spinor functions (kappa, m_j) of A.  G is very sparse: a spinor function
// takes at most two scalar functions per component and spin (the two real
// harmonics of one complex harmonic), so each output element is a sum of at
// most 16 products per part, gathered straight from the scalar blocks.
// HBM-bound: the scalar blocks are read and the complex blocks written once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "q4c_internal.h"

namespace q4c {
namespace {

// One thread per output element, over all pairs at once: element g of the
// spinor store belongs to the pair p with 4 pair_off[p] <= g < 4 pair_off[p+1]
// (found once per workgroup block, then a few steps per thread), so the
// writes are contiguous and every workgroup is full.
// Outputs: complex128 (re, im interleaved), 4 store_len (large plan) each,
// block (2 nL_A) x (2 nL_B) row-major at complex offset 4 pair_off[p].
__global__ __launch_bounds__(256) void k_spinor_transform(DevPlan d, const SpinorType *types, const SpinorFn *fns,
                                                          const int32_t *sp_off, const int32_t *nL,
                                                          const int32_t *nS, const int64_t *poffS,
                                                          int64_t lenS, int64_t npairs, const double *hsL,
                                                          const double *hsS, double *h_out, double *s_out) {
  const int64_t lenL = d.store_len, total = 4 * lenL;
  for (int64_t g0 = blockIdx.x * (int64_t)blockDim.x; g0 < total; g0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = g0 + threadIdx.x;
    // pair of the block's first element (the last p with 4 pair_off[p] <= g0):
    // a search on a workgroup-uniform key, then a short scan per thread (a
    // block of 256 elements spans few pairs)
    const int64_t key = g0 >> 2;
    int64_t lo = 0, hi = npairs - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (d.pair_off[mid] <= key)
        lo = mid;
      else
        hi = mid - 1;
    }
    if (g >= total) continue;
    int64_t p = lo;
    while (p + 1 < npairs && 4 * d.pair_off[p + 1] <= g) ++p;
    const int A = d.pair_a[p], B = d.pair_b[p];
    const int NB = sp_off[B + 1] - sp_off[B];
    const int nLB = nL[B], nSB = nS[B];
    const int64_t oL = d.pair_off[p], oS = poffS[p];
    const int e = (int)(g - 4 * oL);
    const int mu = e / NB, nu = e - mu * NB;
    const double *HL = hsL + oL, *SL = hsL + lenL + oL;
    const double *HS = hsS + oS, *SS = hsS + lenS + oS;
    const SpinorFn fa = fns[sp_off[A] + mu], fb = fns[sp_off[B] + nu];
    const SpinorType &ta = types[fa.type], &tb = types[fb.type];
    double hre = 0.0, him = 0.0, sre = 0.0, sim = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const double *Hc = c == 0 ? HL : HS, *Sc = c == 0 ? SL : SS;
      const int ncol = c == 0 ? nLB : nSB;
      const int ra = c == 0 ? fa.offL : fa.offS, rb = c == 0 ? fb.offL : fb.offS;
#pragma unroll
      for (int sp = 0; sp < 2; ++sp) {
        for (int k1 = 0; k1 < ta.n[c][sp]; ++k1) {
          // conj(G_A) entry
          const double are = ta.re[c][sp][k1], aim = -ta.im[c][sp][k1];
          const int64_t row = (int64_t)(ra + ta.m[c][sp][k1]) * ncol;
          for (int k2 = 0; k2 < tb.n[c][sp]; ++k2) {
            const double bre = tb.re[c][sp][k2], bim = tb.im[c][sp][k2];
            const double wre = are * bre - aim * bim, wim = are * bim + aim * bre;
            const int64_t ij = row + rb + tb.m[c][sp][k2];
            const double h = Hc[ij], s = Sc[ij];
            hre += wre * h;
            him += wim * h;
            sre += wre * s;
            sim += wim * s;
          }
        }
      }
    }
    h_out[2 * g] = hre;
    h_out[2 * g + 1] = him;
    s_out[2 * g] = sre;
    s_out[2 * g + 1] = sim;
  }
}

// The reverse: scalar density matrices of one component from a spinor
// density matrix D given on the pair blocks (same layout as the transform's
// output), C_ij = f Re sum_spin sum_mu,nu conj(G_i,mu) D_mu,nu G_j,nu with
// f = 2 on off-diagonal pairs (each stored block stands for its mirror).
// One thread per element of the component's store.
__global__ __launch_bounds__(256) void k_spinor_to_scalar(DevPlan d, const ScalarRel *rel, const int32_t *fofs,
                                                          const int32_t *ncnt, const int64_t *poff, int64_t len,
                                                          int64_t npairs, const int32_t *sp_off, const double *dsp,
                                                          double *c_out) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < len; g += (int64_t)gridDim.x * blockDim.x) {
    // pair of element g in this component's store: the last p with poff[p] <= g
    int64_t lo = 0, hi = npairs - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (poff[mid] <= g)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int64_t p = lo;
    const int A = d.pair_a[p], B = d.pair_b[p];
    const int e = (int)(g - poff[p]);
    const int nBc = ncnt[B];                       // this component's functions on B
    const int NB = sp_off[B + 1] - sp_off[B];      // spinor functions on B
    const int i = e / nBc, j = e - i * nBc;
    const ScalarRel &ri = rel[fofs[A] + i], &rj = rel[fofs[B] + j];
    const double *D = dsp + 8 * d.pair_off[p];  // the pair's complex spinor block (re, im)
    double acc = 0.0;
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
      for (int k1 = 0; k1 < ri.n[sp]; ++k1) {
        const double ar = ri.re[sp][k1], ai = ri.im[sp][k1];
        const int64_t row = (int64_t)ri.mu[sp][k1] * NB;
        for (int k2 = 0; k2 < rj.n[sp]; ++k2) {
          const double br = rj.re[sp][k2], bi = rj.im[sp][k2];
          // conj(a) b = (ar br + ai bi) + i (ar bi - ai br); the real part of that times D
          const double wr = ar * br + ai * bi, wi = ar * bi - ai * br;
          const int64_t o = 2 * (row + rj.mu[sp][k2]);
          acc += wr * D[o] - wi * D[o + 1];
        }
      }
    c_out[g] = (A == B ? 1.0 : 2.0) * acc;
  }
}

}  // namespace

int launch_spinor_transform(const q4c_plan *pl, const double *hs_large, const double *hs_small, double *h_out,
                            double *s_out, hipStream_t s) {
  if (pl->n_pairs == 0) return Q4C_OK;
  {
    TimedLaunch tl_(pl, Q4C_TIMER_SPINOR, s);
    const int64_t total = 4 * pl->store_len;
    const unsigned grid = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_spinor_transform, dim3(grid), dim3(256), 0, s, pl->dp, pl->d_sp_types,
                       pl->d_sp_fns, pl->d_sp_off, pl->d_sp_nL, pl->d_sp_nS, pl->d_sp_poffS, pl->sp_store_len_S,
                       pl->n_pairs, hs_large, hs_small, h_out, s_out);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_spinor_transform");
  return Q4C_OK;
}

}  // namespace q4c

namespace q4c {

int launch_spinor_to_scalar(const q4c_plan *pl, const double *d_spin, double *c_large, double *c_small,
                            hipStream_t s) {
  if (pl->n_pairs == 0) return Q4C_OK;
  {
    TimedLaunch tl_(pl, Q4C_TIMER_SPINOR, s);
    const int64_t lenL = pl->store_len, lenS = pl->sp_store_len_S;
    if (lenL > 0)
      hipLaunchKernelGGL(k_spinor_to_scalar, dim3((unsigned)std::min<int64_t>((lenL + 255) / 256, 65536)), dim3(256),
                         0, s, pl->dp, pl->d_sp_relL, pl->d_sp_fL, pl->d_sp_nL, pl->dp.pair_off, lenL, pl->n_pairs,
                         pl->d_sp_off, d_spin, c_large);
    if (lenS > 0)
      hipLaunchKernelGGL(k_spinor_to_scalar, dim3((unsigned)std::min<int64_t>((lenS + 255) / 256, 65536)), dim3(256),
                         0, s, pl->dp, pl->d_sp_relS, pl->d_sp_fS, pl->d_sp_nS, pl->d_sp_poffS, lenS, pl->n_pairs,
                         pl->d_sp_off, d_spin, c_small);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_spinor_to_scalar");
  return Q4C_OK;
}

}  // namespace q4c
