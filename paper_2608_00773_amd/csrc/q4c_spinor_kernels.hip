// Scalar -> spinor transformation of H and S (paper Sec. III A, Eq. 33, with
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

#include <cstdint>

#include "q4c_internal.h"

namespace q4c {
namespace {

// One workgroup per atom pair; threads stride over the (mu, nu) elements.
// Outputs: complex128 (re, im interleaved), 4 store_len (large plan) each,
// block (2 nL_A) x (2 nL_B) row-major at complex offset 4 pair_off[p].
__global__ __launch_bounds__(256) void k_spinor_transform(DevPlan d, const SpinorType *types, const SpinorFn *fns,
                                                          const int32_t *sp_off, const int32_t *nL,
                                                          const int32_t *nS, const int64_t *poffS,
                                                          int64_t lenS, const double *hsL, const double *hsS,
                                                          double *h_out, double *s_out) {
  const int p = blockIdx.x;
  const int A = d.pair_a[p], B = d.pair_b[p];
  const int NA = sp_off[A + 1] - sp_off[A], NB = sp_off[B + 1] - sp_off[B];
  const int nLB = nL[B], nSB = nS[B];
  const int64_t oL = d.pair_off[p], oS = poffS[p], lenL = d.store_len;
  const double *HL = hsL + oL, *SL = hsL + lenL + oL;
  const double *HS = hsS + oS, *SS = hsS + lenS + oS;
  const int64_t out0 = 4 * oL;  // complex offset of the pair's spinor block
  for (int e = threadIdx.x; e < NA * NB; e += blockDim.x) {
    const int mu = e / NB, nu = e - mu * NB;
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
    const int64_t o = 2 * (out0 + e);
    h_out[o] = hre;
    h_out[o + 1] = him;
    s_out[o] = sre;
    s_out[o + 1] = sim;
  }
}

}  // namespace

int launch_spinor_transform(const q4c_plan *pl, const double *hs_large, const double *hs_small, double *h_out,
                            double *s_out, hipStream_t s) {
  if (pl->n_pairs == 0) return Q4C_OK;
  {
    TimedLaunch tl_(pl, Q4C_TIMER_SPINOR, s);
    hipLaunchKernelGGL(k_spinor_transform, dim3((unsigned)pl->n_pairs), dim3(256), 0, s, pl->dp, pl->d_sp_types,
                       pl->d_sp_fns, pl->d_sp_off, pl->d_sp_nL, pl->d_sp_nS, pl->d_sp_poffS, pl->sp_store_len_S,
                       hs_large, hs_small, h_out, s_out);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_spinor_transform");
  return Q4C_OK;
}

}  // namespace q4c
