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
//   k_bloch_sum    one workgroup per (cell pair, part): the cell pair's
//                  contributions and their phases are staged in LDS, each
//                  thread keeps a few elements x KC k-points of complex sums
//                  in registers, so the store is streamed ceil(n_k / KC)
//                  times and no sine or cosine is evaluated per element.
// The reverse direction (q4c_bloch_density, the periodic density matrix of
// the same section) reuses k_bloch_phase with k-point weights, per stored
// pair, and k_bloch_density runs one workgroup per stored pair.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <optional>

#include "q4c_internal.h"
#include "q4c_device.h"

// Fixed device scratch of q4c_bloch_sum_noalloc (the phase table of one
// k-point chunk), for callers that cannot allocate.  Each device the library
// runs on holds its own copy until the process ends; every call on a device
// shares it.  Host code must not pass this name to a kernel (it is a host
// stand-in there): it uses the device address from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[q4c::kNoAllocScratchDoubles];

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

constexpr int BS_EPT = 2;  // cell elements per thread per pass
constexpr int BS_TB = 64;  // contributions staged in LDS at a time

// One workgroup per (cell pair c, part q): the contributions' store offsets,
// column counts, orientations and phases for KC k-points are staged in LDS
// (BS_TB contributions at a time) and read as broadcasts; each thread holds
// BS_EPT elements x KC k-points of complex sums, so that one staged phase
// serves BS_EPT elements and every stored value is read once per pass.
// ph: [n_ct][n_k] complex phases of this chunk; out: [n_k][n_parts][clen] complex.
__global__ __launch_bounds__(256) void k_bloch_sum(DevPlan d, int n_parts, int64_t ncp, const int64_t *cp_off,
                                                   const int64_t *ct_off, const int32_t *ct_pair,
                                                   const int32_t *ct_flag, int n_k, const double *ph,
                                                   const double *__restrict__ store, double *__restrict__ out) {
  __shared__ int64_t s_off[BS_TB];
  __shared__ int s_nbp[BS_TB], s_tr[BS_TB];
  __shared__ double s_ph[BS_TB][KC][2];
  const int64_t c = blockIdx.x / n_parts;
  const int q = (int)(blockIdx.x - c * n_parts);
  const int64_t clen = cp_off[ncp];
  const int64_t e0 = cp_off[c], blk = cp_off[c + 1] - e0;
  const int64_t t0 = ct_off[c], nt = ct_off[c + 1] - t0;
  const double sq = (n_parts == 5 && q >= 2) ? -1.0 : 1.0;
  const int64_t L = d.store_len;
  // columns of the cell-pair block: those of the stored block (direct) or
  // its rows (transposed), the same for every contribution of the cell pair
  const int64_t p0 = ct_pair[t0];
  const int ncol = ct_flag[t0] ? d.pair_na[p0] : d.pair_nb[p0];
  const int tid = threadIdx.x;
  for (int64_t eb = 0; eb < blk; eb += 256 * BS_EPT) {
    int ei[BS_EPT], ej[BS_EPT];
    bool ev[BS_EPT];
#pragma unroll
    for (int x = 0; x < BS_EPT; ++x) {
      const int64_t le = eb + tid + 256 * x;
      ev[x] = le < blk;
      ei[x] = ev[x] ? (int)(le / ncol) : 0;
      ej[x] = ev[x] ? (int)(le - (int64_t)ei[x] * ncol) : 0;
    }
    for (int k0 = 0; k0 < n_k; k0 += KC) {
      double re[BS_EPT][KC], im[BS_EPT][KC];
#pragma unroll
      for (int x = 0; x < BS_EPT; ++x)
#pragma unroll
        for (int kk = 0; kk < KC; ++kk) re[x][kk] = im[x][kk] = 0.0;
      for (int64_t tb = 0; tb < nt; tb += BS_TB) {
        const int nb = (int)min<int64_t>(BS_TB, nt - tb);
        __syncthreads();  // the previous batch is consumed
        for (int x = tid; x < nb; x += 256) {
          const int64_t pp = ct_pair[t0 + tb + x];
          s_off[x] = (int64_t)q * L + d.pair_off[pp];
          s_nbp[x] = d.pair_nb[pp];
          s_tr[x] = ct_flag[t0 + tb + x];
        }
        for (int x = tid; x < nb * KC; x += 256) {
          const int tt = x / KC, kk = x - tt * KC;
          const bool in = k0 + kk < n_k;
          const double *pt = ph + 2 * ((t0 + tb + tt) * n_k + k0 + kk);
          s_ph[tt][kk][0] = in ? pt[0] : 0.0;
          s_ph[tt][kk][1] = in ? pt[1] : 0.0;
        }
        __syncthreads();  // the batch is visible
        for (int tt = 0; tt < nb; ++tt) {
          const int64_t off = s_off[tt];
          const int nbp = s_nbp[tt];
          const bool tr = s_tr[tt] != 0;
          double v[BS_EPT];
#pragma unroll
          for (int x = 0; x < BS_EPT; ++x) {
            const int64_t a = tr ? off + (int64_t)ej[x] * nbp + ei[x] : off + (int64_t)ei[x] * nbp + ej[x];
            v[x] = ev[x] ? store[a] : 0.0;
            if (tr) v[x] *= sq;
          }
#pragma unroll
          for (int kk = 0; kk < KC; ++kk) {
            const double cs = s_ph[tt][kk][0], sn = s_ph[tt][kk][1];
#pragma unroll
            for (int x = 0; x < BS_EPT; ++x) {
              re[x][kk] += cs * v[x];
              im[x][kk] += sn * v[x];
            }
          }
        }
      }
#pragma unroll
      for (int x = 0; x < BS_EPT; ++x)
        if (ev[x]) {
#pragma unroll
          for (int kk = 0; kk < KC; ++kk)
            if (k0 + kk < n_k) {
              const int64_t o = ((int64_t)(k0 + kk) * n_parts + q) * clen + e0 + eb + tid + 256 * x;
              out[2 * o] = re[x][kk];
              out[2 * o + 1] = im[x][kk];
            }
        }
    }
  }
}

// The reverse direction (the periodic density matrix of Sec. II C): one
// workgroup per stored image pair p = (A', B') (grouped by cell pair, so that
// a cell pair's rho is re-read from one L2), one thread per element (i, j):
//   coef = f Re sum_k w_k exp(i k.(T_B' - T_A')) rho_ab(k)[i][j],
// rho_ab(k)[i][j] = conj(rho_ba(k)[j][i]) when the cell atoms run a > b,
// f = 2 off the self pairs.  ph: [n_pairs][n_k] weighted phases of this
// chunk (uniform per workgroup); rho: this chunk's [n_k][n_parts][clen]
// complex; acc: add to coef.
__global__ __launch_bounds__(256) void k_bloch_density(DevPlan d, int n_parts, int64_t n_pairs, int64_t ncp,
                                                       const int64_t *cp_off, const int32_t *pc_cp,
                                                       const int32_t *pc_flag, const int32_t *pc_order, int n_k,
                                                       const double *__restrict__ ph,
                                                       const double *__restrict__ rho, int acc,
                                                       double *__restrict__ coef) {
  // the image pairs of one cell pair run one after another on one XCD
  const int64_t p = pc_order[xcd_map(blockIdx.x, n_pairs)];
  const int64_t L = d.store_len;
  const int64_t clen = cp_off[ncp];
  const int na = d.pair_na[p], nb = d.pair_nb[p];
  const int64_t blk = (int64_t)na * nb, po = d.pair_off[p];
  const bool tr = pc_flag[p] != 0;
  const int64_t ce0 = cp_off[pc_cp[p]];
  const double sg = tr ? 1.0 : -1.0;  // Re(e^{i t} r) = c Re r - s Im r; conj(r): c Re r + s Im r
  const double f = d.pair_a[p] == d.pair_b[p] ? 1.0 : 2.0;
  const double *pp = ph + 2 * p * n_k;
  for (int q = 0; q < n_parts; ++q)
    for (int64_t e = threadIdx.x; e < blk; e += blockDim.x) {
      const int i = (int)(e / nb), j = (int)(e - (int64_t)i * nb);
      // element of the cell-pair block: (i, j) of (a, b), or (j, i) of (b, a)
      const int64_t ce = ce0 + (tr ? (int64_t)j * na + i : (int64_t)i * nb + j);
      double s = 0.0;
      for (int k = 0; k < n_k; ++k) {
        const double *r = rho + 2 * (((int64_t)k * n_parts + q) * clen + ce);
        s += pp[2 * k] * r[0] + sg * pp[2 * k + 1] * r[1];
      }
      double *o = coef + (int64_t)q * L + po + e;
      *o = acc ? *o + f * s : f * s;
    }
}

}  // namespace

// Phase table, then the sums, for chunks of at most kchunk (<= KB) k-points;
// phase holds 2 kchunk n_contrib doubles.  timed: record the plan's profiling
// events (created on demand) when profiling is on.
static int launch_bloch_sum_chunks(const q4c_plan *p, int n_parts, const double *store, int n_k,
                                   const double *kpts_dev, double *phase, int kchunk, bool timed, double *out,
                                   hipStream_t s) {
  const int64_t ncp = (int64_t)p->cp_a.size();
  const int64_t clen = p->cp_off.back();
  const int64_t n_ct = p->n_contrib;
  if ((int64_t)n_k * n_parts * clen == 0) return Q4C_OK;
  for (int k0 = 0; k0 < n_k; k0 += kchunk) {
    const int nk = std::min(kchunk, n_k - k0);
    {
      std::optional<TimedLaunch> tl_;
      if (timed) tl_.emplace(p, Q4C_TIMER_OTHER, s);
      const int64_t tot = (int64_t)nk * n_ct;
      const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tot + 255) / 256, 65536));
      hipLaunchKernelGGL(k_bloch_phase, dim3(grid), dim3(256), 0, s, nk, n_ct, kpts_dev + 3 * (int64_t)k0,
                         (const double *)nullptr, p->d_ct_T, phase);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_bloch_phase");
    {
      std::optional<TimedLaunch> tl_;
      if (timed) tl_.emplace(p, Q4C_TIMER_BLOCH, s);
      const unsigned grid = (unsigned)(ncp * n_parts);
      hipLaunchKernelGGL(k_bloch_sum, dim3(grid), dim3(256), 0, s, p->dp, n_parts, ncp, p->d_cp_off, p->d_ct_off,
                         p->d_ct_pair, p->d_ct_flag, nk, (const double *)phase, store,
                         out + 2 * (int64_t)k0 * n_parts * clen);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_bloch_sum");
  }
  return Q4C_OK;
}

int launch_bloch_sum(const q4c_plan *p, int n_parts, const double *store, int n_k, const double *kpts_dev,
                     double *phase, double *out, hipStream_t s) {
  return launch_bloch_sum_chunks(p, n_parts, store, n_k, kpts_dev, phase, KB, true, out, s);
}

// Device address of `scratch` per device, looked up once per device (with
// that device current) on its first use.
static std::mutex g_scratch_mu;
static double *g_scratch_dev[kMaxDevices] = {};

int noalloc_scratch(int device, double **ptr) {
  if (device < 0 || device >= kMaxDevices) return fail_status(Q4C_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void *addr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[device] = static_cast<double *>(addr);
  }
  *ptr = g_scratch_dev[device];
  return Q4C_OK;
}

int launch_bloch_sum_noalloc(const q4c_plan *p, int n_parts, const double *store, int n_k, const double *kpts_dev,
                             double *out, hipStream_t s) {
  double *phase = nullptr;
  int rc = noalloc_scratch(p->device, &phase);
  if (rc != Q4C_OK) return rc;
  // the phases of one k-point take 2 n_contrib doubles: as many k-points per
  // chunk as the scratch holds (at most KB)
  const int64_t per_k = 2 * std::max<int64_t>(p->n_contrib, 1);
  if (per_k > kNoAllocScratchDoubles)
    return fail_status(Q4C_ESIZE, "the phases of one k-point exceed the fixed scratch of q4c_bloch_sum_noalloc");
  const int kchunk = (int)std::min<int64_t>(KB, kNoAllocScratchDoubles / per_k);
  // no profiling events here: creating one may allocate
  return launch_bloch_sum_chunks(p, n_parts, store, n_k, kpts_dev, phase, kchunk, false, out, s);
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
      hipLaunchKernelGGL(k_bloch_density, dim3((unsigned)np_), dim3(256), 0, s, p->dp, n_parts, np_, ncp,
                         p->d_cp_off, p->d_pc_cp, p->d_pc_flag, p->d_pc_order, nk, (const double *)phase,
                         rho + 2 * (int64_t)k0 * n_parts * clen, k0 > 0 ? 1 : 0, coef);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_bloch_density");
  }
  return Q4C_OK;
}

}  // namespace q4c
