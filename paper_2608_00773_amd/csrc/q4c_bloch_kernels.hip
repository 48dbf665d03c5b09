// Bloch sums of unit-cell integrals (paper Sec. II C, Eq. 27 with the
// restricted sum of Eq. 28): for a plan whose atoms are a reference cell's
// atoms and their periodic images (q4c_plan_set_cells), every element of
// every cell pair block (a <= b) at every k-point is
//   O_ab(k)[i][j] = sum over contributions (stored pair, orientation, T)
//                   exp(i k.T) O_pair[i][j]   (or s_q O_pair[j][i] transposed),
// s_q = -1 for the spin-orbit parts (q >= 2) of a five-part store.
//
// Two kernels per chunk of at most KB k-points:
//   k_bloch_phase  exp(i k.T) once per (contribution, k-point), [t][k] layout;
//   k_bloch_sum    one thread per (part, cell element): it reads each of its
//                  stored values once per KC k-points and keeps KC complex
//                  accumulators in registers, so the store is streamed
//                  ceil(n_k / KC) times and no sine or cosine is evaluated
//                  per element.  The contributions of a cell pair are a short
//                  list shared by all of its elements (uniform loads).
// The reverse direction (q4c_bloch_density, the periodic density matrix of
// the same section) reuses k_bloch_phase with k-point weights, per stored
// pair, and k_bloch_density sums one stored element per thread.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "q4c_internal.h"

namespace q4c {
namespace {

constexpr int KC = 8;    // k-points per register pass
constexpr int KB = kBlochKChunk;  // k-points per phase-table chunk

// ph[t][k] = w_k exp(i k.T_t) (w_k = 1 without weights)
__global__ __launch_bounds__(256) void k_bloch_phase(int n_k, int64_t n_ct, const double *kpts, const double *kw,
                                                     const double *ct_T, double *ph) {
  const int64_t total = (int64_t)n_k * n_ct;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = g / n_k;
    const int ik = (int)(g - t * n_k);
    double sn, cs;
    sincos(kpts[3 * ik] * ct_T[3 * t] + kpts[3 * ik + 1] * ct_T[3 * t + 1] + kpts[3 * ik + 2] * ct_T[3 * t + 2], &sn,
           &cs);
    const double w = kw ? kw[ik] : 1.0;
    ph[2 * g] = w * cs;
    ph[2 * g + 1] = w * sn;
  }
}

// ph: [n_ct][n_k] complex phases of this chunk; out: [n_k][n_parts][clen] complex.
__global__ __launch_bounds__(256) void k_bloch_sum(DevPlan d, int n_parts, int64_t ncp, const int64_t *cp_off,
                                                   const int64_t *ct_off, const int32_t *ct_pair,
                                                   const int32_t *ct_flag, int n_k, const double *ph,
                                                   const double *store, double *out) {
  const int64_t clen = cp_off[ncp];
  const int64_t total = (int64_t)n_parts * clen;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = g % clen;
    const int q = (int)(g / clen);
    // cell pair of element e: the last c with cp_off[c] <= e
    int64_t lo = 0, hi = ncp - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (cp_off[mid] <= e)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int64_t c = lo;
    const int64_t le = e - cp_off[c];
    const double sq = (n_parts == 5 && q >= 2) ? -1.0 : 1.0;
    const double *sp = store + (int64_t)q * d.store_len;
    const int64_t t0 = ct_off[c], t1 = ct_off[c + 1];
    for (int k0 = 0; k0 < n_k; k0 += KC) {
      double re[KC], im[KC];
#pragma unroll
      for (int kk = 0; kk < KC; ++kk) re[kk] = im[kk] = 0.0;
      for (int64_t t = t0; t < t1; ++t) {
        const int64_t p = ct_pair[t];
        const int nbp = d.pair_nb[p];  // columns of the stored block
        // target block is n_row x n_col with n_col = nbp (direct) or nap (transposed)
        const bool tr = ct_flag[t] != 0;
        const int ncol = tr ? d.pair_na[p] : nbp;
        const int i = (int)(le / ncol), j = (int)(le - (int64_t)i * ncol);
        const double v = tr ? sq * sp[d.pair_off[p] + (int64_t)j * nbp + i] : sp[d.pair_off[p] + (int64_t)i * nbp + j];
        const double *pt = ph + 2 * (t * n_k + k0);
#pragma unroll
        for (int kk = 0; kk < KC; ++kk)
          if (k0 + kk < n_k) {
            re[kk] += pt[2 * kk] * v;
            im[kk] += pt[2 * kk + 1] * v;
          }
      }
#pragma unroll
      for (int kk = 0; kk < KC; ++kk)
        if (k0 + kk < n_k) {
          const int64_t o = ((int64_t)(k0 + kk) * n_parts + q) * clen + e;
          out[2 * o] = re[kk];
          out[2 * o + 1] = im[kk];
        }
    }
  }
}

// The reverse direction (the periodic density matrix of Sec. II C): one
// thread per (part, stored element (i, j) of image pair p = (A', B')):
//   coef = f Re sum_k w_k exp(i k.(T_B' - T_A')) rho_ab(k)[i][j],
// rho_ab(k)[i][j] = conj(rho_ba(k)[j][i]) when the cell atoms run a > b,
// f = 2 off the self pairs.  ph: [n_pairs][n_k] weighted phases of this
// chunk; rho: this chunk's [n_k][n_parts][clen] complex; acc: add to coef.
__global__ __launch_bounds__(256) void k_bloch_density(DevPlan d, int n_parts, int64_t n_pairs, int64_t ncp,
                                                       const int64_t *cp_off, const int32_t *pc_cp,
                                                       const int32_t *pc_flag, int n_k, const double *ph,
                                                       const double *rho, int acc, double *coef) {
  const int64_t L = d.store_len;
  const int64_t clen = cp_off[ncp];
  const int64_t total = (int64_t)n_parts * L;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(g / L);
    const int64_t e = g - (int64_t)q * L;
    // stored pair of element e: the last p with pair_off[p] <= e
    int64_t lo = 0, hi = n_pairs - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (d.pair_off[mid] <= e)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int64_t p = lo;
    const int64_t le = e - d.pair_off[p];
    const int na = d.pair_na[p], nb = d.pair_nb[p];
    const int i = (int)(le / nb), j = (int)(le - (int64_t)i * nb);
    const bool tr = pc_flag[p] != 0;
    // element of the cell-pair block: (i, j) of (a, b), or (j, i) of (b, a)
    const int64_t ce = cp_off[pc_cp[p]] + (tr ? (int64_t)j * na + i : (int64_t)i * nb + j);
    const double sg = tr ? 1.0 : -1.0;  // Re(e^{i t} r) = c Re r - s Im r; conj(r): c Re r + s Im r
    const double *pp = ph + 2 * p * n_k;
    double s = 0.0;
    for (int k = 0; k < n_k; ++k) {
      const double *r = rho + 2 * (((int64_t)k * n_parts + q) * clen + ce);
      s += pp[2 * k] * r[0] + sg * pp[2 * k + 1] * r[1];
    }
    const double f = d.pair_a[p] == d.pair_b[p] ? 1.0 : 2.0;
    coef[g] = acc ? coef[g] + f * s : f * s;
  }
}

}  // namespace

int launch_bloch_sum(const q4c_plan *p, int n_parts, const double *store, int n_k, const double *kpts_dev,
                     double *phase, double *out, hipStream_t s) {
  const int64_t ncp = (int64_t)p->cp_a.size();
  const int64_t clen = p->cp_off.back();
  const int64_t n_ct = p->n_contrib;
  if ((int64_t)n_k * n_parts * clen == 0) return Q4C_OK;
  for (int k0 = 0; k0 < n_k; k0 += KB) {
    const int nk = std::min(KB, n_k - k0);
    {
      TimedLaunch tl_(p, Q4C_TIMER_OTHER, s);
      const int64_t tot = (int64_t)nk * n_ct;
      const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tot + 255) / 256, 65536));
      hipLaunchKernelGGL(k_bloch_phase, dim3(grid), dim3(256), 0, s, nk, n_ct, kpts_dev + 3 * (int64_t)k0,
                         (const double *)nullptr, p->d_ct_T, phase);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_bloch_phase");
    {
      TimedLaunch tl_(p, Q4C_TIMER_BLOCH, s);
      const int64_t tot = (int64_t)n_parts * clen;
      const unsigned grid = (unsigned)std::min<int64_t>((tot + 255) / 256, 65536);
      hipLaunchKernelGGL(k_bloch_sum, dim3(grid), dim3(256), 0, s, p->dp, n_parts, ncp, p->d_cp_off, p->d_ct_off,
                         p->d_ct_pair, p->d_ct_flag, nk, (const double *)phase, store,
                         out + 2 * (int64_t)k0 * n_parts * clen);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_bloch_sum");
  }
  return Q4C_OK;
}

int launch_bloch_density(const q4c_plan *p, int n_parts, const double *rho, int n_k, const double *kpts_dev,
                         const double *kw_dev, double *phase, double *coef, hipStream_t s) {
  const int64_t ncp = (int64_t)p->cp_a.size();
  const int64_t clen = p->cp_off.back();
  const int64_t L = p->store_len, np_ = p->n_pairs;
  if ((int64_t)n_parts * L == 0) return Q4C_OK;
  // no k-points: one pass with an empty sum writes zeros
  for (int k0 = 0; k0 < std::max(n_k, 1); k0 += KB) {
    const int nk = std::min(KB, n_k - k0);
    if (nk > 0) {
      TimedLaunch tl_(p, Q4C_TIMER_OTHER, s);
      const int64_t tot = (int64_t)nk * np_;
      const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tot + 255) / 256, 65536));
      hipLaunchKernelGGL(k_bloch_phase, dim3(grid), dim3(256), 0, s, nk, np_, kpts_dev + 3 * (int64_t)k0,
                         kw_dev + k0, p->d_pc_T, phase);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_bloch_phase");
    {
      TimedLaunch tl_(p, Q4C_TIMER_BLOCH, s);
      const int64_t tot = (int64_t)n_parts * L;
      const unsigned grid = (unsigned)std::min<int64_t>((tot + 255) / 256, 65536);
      hipLaunchKernelGGL(k_bloch_density, dim3(grid), dim3(256), 0, s, p->dp, n_parts, np_, ncp, p->d_cp_off,
                         p->d_pc_cp, p->d_pc_flag, nk, (const double *)phase,
                         rho + 2 * (int64_t)k0 * n_parts * clen, k0 > 0 ? 1 : 0, coef);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_bloch_density");
  }
  return Q4C_OK;
}

}  // namespace q4c
