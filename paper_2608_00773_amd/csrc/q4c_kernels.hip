// HIP kernels of libq4c for CDNA4 (gfx950).
//
//  k_tabulate        nao_tabulate: phi and grad phi of a batch's relevant
//                    functions at its points (Eq. 12a, App. B), as the
//                    panels compute them; FP64 or FP32 hi + lo output.
//  k_om              w_g v_g per active point (the weighting of Eq. 29).
//  k_panel           per (batch, 64-function tile): phi and grad phi at all
//                    batch points into the batch's operand panel (HBM).
//  k_contract<prec>  per (batch, tile ti <= tj) work item: 16-point chunks of
//                    the two tiles' panels are copied into LDS (the column
//                    operand weighted by w v on the way) and the five
//                    weighted products
//                        V  = Phi^T diag(w v) Phi
//                        Gs = sum_a dPhi_a^T diag(w v) dPhi_a
//                        Gm = dPhi_b^T diag(w v) dPhi_c - dPhi_c^T diag(w v) dPhi_b
//                    accumulate on MFMA (Eq. 29 restricted to the batch,
//                    Eq. 31).  The lower atom-block triangle follows from
//                    (anti)symmetry.  Results go to a staging buffer laid
//                    out per (batch, atom pair).
//  k_reduce          deterministic batch-to-global sum: every stored atom
//                    pair adds its staged blocks in batch order (FP64).
//  k_spinor          2x2-spinor assembly of the W and V blocks.
//  k_density_tiles,
//  k_density_points  density_on_grid: the transpose of the steps above
//                    (Eq. 39): each quarter of a work item reads its
//                    coefficients from the store, contracts a_g^T C b_g at its
//                    points on MFMA, and every point sums its partials in a
//                    fixed order.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "q4c_internal.h"
#include "q4c_device.h"

namespace q4c {
namespace {


// ---------------------------------------------------------------------------
// Basis functions
// ---------------------------------------------------------------------------

// Real solid harmonics S_lm = s^l Y_lm (App. B convention, Condon-Shortley
// phase as written there: Y_1,1 = -sqrt(3/4pi) x/s) and their gradients,
// l <= 4, indexed by lm = l^2 + l + m.
__device__ __forceinline__ void solid_harmonic(int lm, double x, double y, double z, double &S, double &gx,
                                               double &gy, double &gz) {
  constexpr double C00 = 0.28209479177387814, C1 = 0.4886025119029199, C2a = 1.0925484305920792,
                   C20 = 0.31539156525252005, C22 = 0.5462742152960396, C33 = 0.5900435899266435,
                   C32b = 2.8906114426405543, C31 = 0.4570457994644657, C30 = 0.3731763325901154,
                   C32a = 1.4453057213202771;
  // l = 4: K_4^0 / 8 and sqrt2 K_4^|m| times the integer factors of the polynomials
  constexpr double C40 = 0.10578554691520431, C41 = 0.6690465435572891, C42 = 0.47308734787878,
                   C43 = 1.7701307697799304, C44 = 0.6258357354491761;
  switch (lm) {
    case 0: S = C00; gx = gy = gz = 0.0; break;
    case 1: S = -C1 * y; gx = 0.0; gy = -C1; gz = 0.0; break;
    case 2: S = C1 * z; gx = 0.0; gy = 0.0; gz = C1; break;
    case 3: S = -C1 * x; gx = -C1; gy = 0.0; gz = 0.0; break;
    case 4: S = C2a * x * y; gx = C2a * y; gy = C2a * x; gz = 0.0; break;
    case 5: S = -C2a * y * z; gx = 0.0; gy = -C2a * z; gz = -C2a * y; break;
    case 6: S = C20 * (2.0 * z * z - x * x - y * y); gx = -2.0 * C20 * x; gy = -2.0 * C20 * y; gz = 4.0 * C20 * z; break;
    case 7: S = -C2a * x * z; gx = -C2a * z; gy = 0.0; gz = -C2a * x; break;
    case 8: S = C22 * (x * x - y * y); gx = 2.0 * C22 * x; gy = -2.0 * C22 * y; gz = 0.0; break;
    case 9: S = -C33 * y * (3.0 * x * x - y * y); gx = -6.0 * C33 * x * y; gy = -3.0 * C33 * (x * x - y * y); gz = 0.0; break;
    case 10: S = C32b * x * y * z; gx = C32b * y * z; gy = C32b * x * z; gz = C32b * x * y; break;
    case 11: {
      double q = 4.0 * z * z - x * x - y * y;
      S = -C31 * y * q; gx = 2.0 * C31 * x * y; gy = -C31 * (q - 2.0 * y * y); gz = -8.0 * C31 * y * z;
    } break;
    case 12: S = C30 * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y); gx = -6.0 * C30 * x * z; gy = -6.0 * C30 * y * z;
      gz = C30 * (6.0 * z * z - 3.0 * x * x - 3.0 * y * y); break;
    case 13: {
      double q = 4.0 * z * z - x * x - y * y;
      S = -C31 * x * q; gx = -C31 * (q - 2.0 * x * x); gy = 2.0 * C31 * x * y; gz = -8.0 * C31 * x * z;
    } break;
    case 14: S = C32a * z * (x * x - y * y); gx = 2.0 * C32a * x * z; gy = -2.0 * C32a * y * z; gz = C32a * (x * x - y * y); break;
    case 15: S = -C33 * x * (x * x - 3.0 * y * y); gx = -3.0 * C33 * (x * x - y * y); gy = 6.0 * C33 * x * y; gz = 0.0; break;
    // l = 4 (the small-component partners of f shells), rho = x^2 + y^2 + z^2
    case 16: S = 4.0 * C44 * (x * x * x * y - x * y * y * y); gx = 4.0 * C44 * (3.0 * x * x * y - y * y * y);
      gy = 4.0 * C44 * (x * x * x - 3.0 * x * y * y); gz = 0.0; break;
    case 17: S = -C43 * z * (3.0 * x * x * y - y * y * y); gx = -6.0 * C43 * x * y * z;
      gy = -3.0 * C43 * z * (x * x - y * y); gz = -C43 * (3.0 * x * x * y - y * y * y); break;
    case 18: {
      const double t = 6.0 * z * z - x * x - y * y;  // 7 z^2 - rho
      S = 2.0 * C42 * x * y * t; gx = 2.0 * C42 * y * (t - 2.0 * x * x); gy = 2.0 * C42 * x * (t - 2.0 * y * y);
      gz = 24.0 * C42 * x * y * z;
    } break;
    case 19: {
      const double q = 4.0 * z * z - 3.0 * x * x - 3.0 * y * y;  // 7 z^2 - 3 rho
      S = -C41 * y * z * q; gx = 6.0 * C41 * x * y * z; gy = -C41 * z * (q - 6.0 * y * y); gz = -C41 * y * (q + 8.0 * z * z);
    } break;
    case 20: {
      const double rho = x * x + y * y + z * z, z2 = z * z;
      S = C40 * (35.0 * z2 * z2 - 30.0 * z2 * rho + 3.0 * rho * rho); gx = C40 * x * (12.0 * rho - 60.0 * z2);
      gy = C40 * y * (12.0 * rho - 60.0 * z2); gz = C40 * z * (80.0 * z2 - 48.0 * rho);
    } break;
    case 21: {
      const double q = 4.0 * z * z - 3.0 * x * x - 3.0 * y * y;
      S = -C41 * x * z * q; gx = -C41 * z * (q - 6.0 * x * x); gy = 6.0 * C41 * x * y * z; gz = -C41 * x * (q + 8.0 * z * z);
    } break;
    case 22: {
      const double t = 6.0 * z * z - x * x - y * y;
      S = C42 * (x * x - y * y) * t; gx = 2.0 * C42 * x * (t - x * x + y * y); gy = -2.0 * C42 * y * (t + x * x - y * y);
      gz = 12.0 * C42 * (x * x - y * y) * z;
    } break;
    case 23: S = -C43 * z * (x * x * x - 3.0 * x * y * y); gx = -3.0 * C43 * z * (x * x - y * y);
      gy = 6.0 * C43 * x * y * z; gz = -C43 * (x * x * x - 3.0 * x * y * y); break;
    default: S = C44 * (x * x * x * x - 6.0 * x * x * y * y + y * y * y * y); gx = 4.0 * C44 * (x * x * x - 3.0 * x * y * y);
      gy = 4.0 * C44 * (y * y * y - 3.0 * x * x * y); gz = 0.0; break;
  }
}

// ---------------------------------------------------------------------------
// Contraction
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Tile tabulation: the metadata of a tile's functions is staged in LDS, so
// the per-(function, point) work touches global memory only for the point
// and the four radial coefficients of its interval.
// ---------------------------------------------------------------------------

struct TileMeta {
  double ax[T], ay[T], az[T];  // centres
  double rc[T];                // cutoffs (0 for padding)
  double k1[T], k2[T];         // nint^2 / rcut, rcut / nint^2
  int64_t coef[T];             // offset of the shell's table
  int64_t uoff[T];             // offset of the shell's ket-potential table (H/S panels)
  int nint[T], lm[T];
  int order[T];                // tile functions sorted by lm
};

// Stage metadata of the tile's functions (threads 0 .. T-1) and an ordering
// by lm, so that lanes working on neighbouring items mostly take the same
// solid-harmonic branch.
__device__ __forceinline__ void load_tile_meta(const DevPlan &d, TileMeta &M, int f0, int n, int r0) {
  const int tid = threadIdx.x;
  if (tid < T) {
    const int lf = r0 + tid;
    if (lf < n) {
      const int fn = d.loc_fn[f0 + lf];
      const int a = d.fn_atom[fn], shlm = d.fn_shlm[fn], sh = shlm >> 5;
      M.ax[tid] = d.R[3 * a];
      M.ay[tid] = d.R[3 * a + 1];
      M.az[tid] = d.R[3 * a + 2];
      M.rc[tid] = d.shell_rcut[sh];
      M.k1[tid] = d.shell_knot[2 * sh];
      M.k2[tid] = d.shell_knot[2 * sh + 1];
      M.coef[tid] = d.shell_coef_off[sh];
      M.uoff[tid] = d.shell_u_off ? d.shell_u_off[sh] : 0;
      M.nint[tid] = d.shell_nint[sh];
      M.lm[tid] = shlm & 31;
    } else {
      M.ax[tid] = M.ay[tid] = M.az[tid] = 0.0;
      M.rc[tid] = 0.0;
      M.k1[tid] = M.k2[tid] = 0.0;
      M.coef[tid] = 0;
      M.uoff[tid] = 0;
      M.nint[tid] = 0;
      M.lm[tid] = 32;  // padding sorts last
    }
  }
  __syncthreads();
  if (tid < T) {
    const int mine = M.lm[tid];
    int rank = 0;
    for (int o = 0; o < T; ++o) rank += (M.lm[o] < mine) || (M.lm[o] == mine && o < tid);
    M.order[rank] = tid;
  }
}

// phi and grad phi of tile function m at point (px, py, pz); see tab_one.
// 1/s comes from a Newton-refined reciprocal square root, and the interval
// index from an approximate square root corrected against the exact knots.
__device__ __forceinline__ void tab_meta(const DevPlan &d, const TileMeta &M, int m, double px, double py,
                                         double pz, double &f, double &fx, double &fy, double &fz) {
  const double dx = px - M.ax[m], dy = py - M.ay[m], dz = pz - M.az[m];
  const double s2 = dx * dx + dy * dy + dz * dz;
  const double rc = M.rc[m];
  if (!(s2 < rc * rc)) {
    f = fx = fy = fz = 0.0;
    return;
  }
  double rinv = 0.0, s = 0.0;
  if (s2 > 0.0) {
    rinv = __builtin_amdgcn_rsq(s2);
    rinv = rinv * (1.5 - 0.5 * s2 * rinv * rinv);
    s = s2 * rinv;
  }
  const int n = M.nint[m];
  const double k1 = M.k1[m], k2 = M.k2[m];
  const double u = s * k1;
  int j = u > 0.0 ? (int)(u * __builtin_amdgcn_rsq(u)) : 0;
  j = j < 0 ? 0 : (j > n - 1 ? n - 1 : j);
  double rj = (double)j * (double)j * k2;
  if (s < rj && j > 0) {
    --j;
    rj = (double)j * (double)j * k2;
  } else if (j < n - 1 && s >= (double)(j + 1) * (double)(j + 1) * k2) {
    ++j;
    rj = (double)j * (double)j * k2;
  }
  const double dd = s - rj;
  const dbl4 c = *reinterpret_cast<const dbl4 *>(d.coef + M.coef[m] + 4 * (int64_t)j);
  const double R = ((c[3] * dd + c[2]) * dd + c[1]) * dd + c[0];
  const double q = ((3.0 * c[3] * dd + 2.0 * c[2]) * dd + c[1]) * rinv;  // Rt'(s) / s
  double S, gx, gy, gz;
  solid_harmonic(M.lm[m], dx, dy, dz, S, gx, gy, gz);
  f = R * S;
  fx = q * dx * S + R * gx;
  fy = q * dy * S + R * gy;
  fz = q * dz * S + R * gz;
}

// phi and psi = u phi / 2 of tile function m at (px, py, pz): the H/S panels.
// u, the shell's ket potential, is a cubic on the radial table's own knots,
// so it is evaluated on the same interval.
__device__ __forceinline__ void tab_meta_hs(const DevPlan &d, const TileMeta &M, int m, double px, double py,
                                            double pz, double &f, double &psi) {
  const double dx = px - M.ax[m], dy = py - M.ay[m], dz = pz - M.az[m];
  const double s2 = dx * dx + dy * dy + dz * dz;
  const double rc = M.rc[m];
  if (!(s2 < rc * rc)) {
    f = psi = 0.0;
    return;
  }
  double s = 0.0;
  if (s2 > 0.0) {
    double rinv = __builtin_amdgcn_rsq(s2);
    rinv = rinv * (1.5 - 0.5 * s2 * rinv * rinv);
    s = s2 * rinv;
  }
  const int n = M.nint[m];
  const double k1 = M.k1[m], k2 = M.k2[m];
  const double u = s * k1;
  int j = u > 0.0 ? (int)(u * __builtin_amdgcn_rsq(u)) : 0;
  j = j < 0 ? 0 : (j > n - 1 ? n - 1 : j);
  double rj = (double)j * (double)j * k2;
  if (s < rj && j > 0) {
    --j;
    rj = (double)j * (double)j * k2;
  } else if (j < n - 1 && s >= (double)(j + 1) * (double)(j + 1) * k2) {
    ++j;
    rj = (double)j * (double)j * k2;
  }
  const double dd = s - rj;
  const dbl4 c = *reinterpret_cast<const dbl4 *>(d.coef + M.coef[m] + 4 * (int64_t)j);
  const dbl4 e = *reinterpret_cast<const dbl4 *>(d.ucoef + M.uoff[m] + 4 * (int64_t)j);
  const double R = ((c[3] * dd + c[2]) * dd + c[1]) * dd + c[0];
  const double U = ((e[3] * dd + e[2]) * dd + e[1]) * dd + e[0];
  double S, gx, gy, gz;
  solid_harmonic(M.lm[m], dx, dy, dz, S, gx, gy, gz);
  f = R * S;
  psi = 0.5 * U * f;
}

// ---------------------------------------------------------------------------
// nao_tabulate: one workgroup per (batch, 64-function tile) of the requested
// batch range, the same tabulation as the panels (tile metadata in LDS,
// functions taken in lm order), staged in LDS per 8 points and written as
// runs of the tile's functions: out is [ncomp][P][n] per batch (FP64), or
// [ncomp][2][P][n] floats with the hi and lo planes (F32_HILO).
// ---------------------------------------------------------------------------

template <bool HILO>
__global__ __launch_bounds__(256) void k_tabulate(DevPlan d, const WorkItem *tiles, int64_t t0, int64_t b0, int deriv,
                                                  void *out) {
  constexpr int CP = 8;
  constexpr int SR = T + 1;
  __shared__ TileMeta M;
  __shared__ double st[4 * CP * SR];
  const WorkItem it = tiles[t0 + blockIdx.x];
  const int b = it.batch;
  const int g0 = d.batch_pt_off[b], P = d.batch_pt_off[b + 1] - g0;
  const int f0 = d.batch_fn_off[b], n = d.batch_fn_off[b + 1] - f0;
  const int r0 = it.ti * T;
  const int nrow = n - r0 < T ? n - r0 : T;
  const int nq = deriv ? 4 : 1;
  const int64_t plane = (int64_t)P * n;
  const int64_t base = (int64_t)nq * (d.tab_off[b] - d.tab_off[b0]);  // values before this batch
  load_tile_meta(d, M, f0, n, r0);
  __syncthreads();
  for (int g8 = 0; g8 < P; g8 += CP) {
    for (int e = threadIdx.x; e < T * CP; e += 256) {
      const int k = e / CP, pt = e % CP;
      const int fl = M.order[k];
      double f = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
      const int g = g8 + pt;
      if (M.nint[fl] > 0 && g < P) tab_meta(d, M, fl, d.px[g0 + g], d.py[g0 + g], d.pz[g0 + g], f, fx, fy, fz);
      st[(0 * CP + pt) * SR + fl] = f;
      st[(1 * CP + pt) * SR + fl] = fx;
      st[(2 * CP + pt) * SR + fl] = fy;
      st[(3 * CP + pt) * SR + fl] = fz;
    }
    __syncthreads();
    // (component, point) rows of the tile's functions: 256 threads = 4 rows x 64 functions
    for (int e = threadIdx.x; e < nq * CP * T; e += 256) {
      const int fl = e % T, row = e / T;
      const int q = row / CP, pt = row % CP;
      const int g = g8 + pt;
      if (fl < nrow && g < P) {
        const double x = st[(q * CP + pt) * SR + fl];
        const int64_t o = (int64_t)g * n + r0 + fl;
        if (HILO) {
          float *of = static_cast<float *>(out) + 2 * (base + q * plane);
          const float hi = (float)x;
          of[o] = hi;
          of[plane + o] = (float)(x - (double)hi);
        } else {
          static_cast<double *>(out)[base + q * plane + o] = x;
        }
      }
    }
    __syncthreads();  // st consumed
  }
}

// ---------------------------------------------------------------------------
// Operand panels.  Batch b's panel holds phi, d/dx, d/dy, d/dz of its
// functions at its points, padded to Pp = pad16(P) points and np = pad16(n)
// functions (zeros in the padding), in a 4-point-interleaved layout:
//     element (q, pt, i) at ((q * Pp/4 + pt/4) * np + i) * 4 + pt % 4.
// A 64-lane MFMA operand slice (16 functions x 4 points) is then one
// contiguous 512-byte run, for the forward (functions as rows) and, in
// 128-byte runs, for the adjoint (points as rows).
// ---------------------------------------------------------------------------

__device__ __forceinline__ int64_t panel_index(int q, int pt, int i, int Pp, int np) {
  return ((int64_t)(q * (Pp >> 2) + (pt >> 2)) * np + i) * 4 + (pt & 3);
}

__global__ void k_zero_u32(unsigned *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// w_g v_g for every active point (batch order); 16 zero entries after the end.
__global__ void k_om(DevPlan d, const double *v, double *om, unsigned long long *chunks) {
  if (blockIdx.x == 0 && threadIdx.x < 128) chunks[threadIdx.x] = 0;
  const int64_t n = d.n_active;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n + 16; g += (int64_t)gridDim.x * blockDim.x)
    om[g] = g < n ? d.pw[g] * v[d.perm[g]] : 0.0;
}

// One (batch, function tile of 64): tabulate the tile's functions at all
// points of the batch into the panel, and record for every point the largest
// |gradient component| over the tile's functions (after the batch's panel, at
// 4 Pp np + ti Pp + point): the split-precision routing bound reads it.  Each group of 16 points is computed
// in lm order (few divergent harmonic branches per wave) into LDS, then
// written out as 16 contiguous 2 KB runs.
constexpr int PLD = T + 1;  // padded LDS row of the panel stage

template <bool HS>
__global__ __launch_bounds__(256) void k_panel(DevPlan d, const WorkItem *tiles, int64_t t0, int64_t nt,
                                               double *panel) {
  constexpr int NQ = HS ? 2 : 4;  // components: phi, psi (H/S) or phi and its gradient
  constexpr int CP = 8;           // points per chunk: a small stage keeps 7 workgroups on a CU
  __shared__ TileMeta M;
  __shared__ double st[NQ * CP * PLD];
  __shared__ double s_gx[4][CP];
  const WorkItem it = tiles[t0 + xcd_map(blockIdx.x, nt)];
  const int b = it.batch;
  const int g0 = d.batch_pt_off[b], P = d.batch_pt_off[b + 1] - g0;
  const int f0 = d.batch_fn_off[b], n = d.batch_fn_off[b + 1] - f0;
  const int Pp = (int)pad16(P), np = (int)pad16(n);
  const int r0 = it.ti * T;
  const int nrow = np - r0 < T ? np - r0 : T;  // panel rows of this tile
  load_tile_meta(d, M, f0, n, r0);
  __syncthreads();
  double *pb = panel + d.panel_off[b];
  for (int g8 = 0; g8 < Pp; g8 += CP) {
    for (int e = threadIdx.x; e < T * CP; e += 256) {
      const int k = e / CP, pt = e % CP;
      const int fl = M.order[k];
      double f = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
      const int g = g8 + pt;
      if (HS) {
        if (M.nint[fl] > 0 && g < P) tab_meta_hs(d, M, fl, d.px[g0 + g], d.py[g0 + g], d.pz[g0 + g], f, fx);
      } else {
        if (M.nint[fl] > 0 && g < P) tab_meta(d, M, fl, d.px[g0 + g], d.py[g0 + g], d.pz[g0 + g], f, fx, fy, fz);
      }
      st[(0 * CP + pt) * PLD + fl] = f;
      st[(1 * CP + pt) * PLD + fl] = fx;
      if (!HS) {
        st[(2 * CP + pt) * PLD + fl] = fy;
        st[(3 * CP + pt) * PLD + fl] = fz;
      }
    }
    __syncthreads();
    if (!HS) {
      // largest |d phi / d x_a| per point over the tile's functions: thread
      // (pt, pair of functions), then the 8 pairs of a wave, then the waves
      const int pt = threadIdx.x % CP, fg = threadIdx.x / CP;
      double m = 0.0;
#pragma unroll
      for (int q = 1; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 2; ++k) m = fmax(m, fabs(st[(q * CP + pt) * PLD + 2 * fg + k]));
      m = fmax(m, __shfl_xor(m, 8));
      m = fmax(m, __shfl_xor(m, 16));
      m = fmax(m, __shfl_xor(m, 32));
      if ((threadIdx.x & 63) < CP) s_gx[threadIdx.x >> 6][pt] = m;
    }
    // (q, point quad) runs: rows r0 .. r0 + nrow - 1, 4 points each, contiguous
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int p4 = 0; p4 < CP / 4; ++p4) {
        const int e = threadIdx.x;  // 256 = 64 rows x 4 points
        const int il = e >> 2, pp = e & 3;
        if (il < nrow)
          pb[((int64_t)(q * (Pp >> 2) + (g8 >> 2) + p4) * np + r0 + il) * 4 + pp] = st[(q * CP + 4 * p4 + pp) * PLD + il];
      }
    __syncthreads();  // s_gx written; st consumed
    if (!HS && threadIdx.x < CP)
      pb[(int64_t)4 * Pp * np + (int64_t)it.ti * Pp + g8 + threadIdx.x] =
          fmax(fmax(s_gx[0][threadIdx.x], s_gx[1][threadIdx.x]), fmax(s_gx[2][threadIdx.x], s_gx[3][threadIdx.x]));
  }
}

// Modes of the forward contraction: FP64; split (hi+lo FP32 operands) and
// single FP32 operands for the W parts (V stays FP64), whose chunks with large
// terms are deferred; MODE_HOT adds the deferred chunks' W parts in FP64.
enum { MODE_F64 = 0, MODE_SPLIT = 1, MODE_F32 = 2, MODE_HOT = 3 };


// Split modes: a chunk's W contribution is bounded by c' 48 A B with A the
// largest |grad phi| of the tile's rows and B the largest |w v grad phi| of
// its columns over the chunk's 16 points (16 points x 3 products per term);
// with FP32 rounding 2^-24 that bounds the FP32 error of the chunk.
constexpr double kU32 = 5.9604644775390625e-08;

// Work item positions 0..nw-1 of a pass map to work items w0 + order[w0 + pos]
// (order != NULL: cost-sorted) or w0 + pos.  tickets == NULL: one workgroup
// per position; otherwise a persistent loop (next_item).
//
// Split modes (MODE_SPLIT, MODE_F32): V accumulates in FP64, the W parts in
// FP32; a 16-point chunk whose W bound exceeds tau skips its W products here
// and sets bit k0/16 of hotmask[w] (P <= 1024); MODE_HOT then runs those chunks'
// W products in FP64 and adds them to the staged elements.
template <int MODE, bool PERSIST>
__global__ __launch_bounds__(NT, 2) void k_contract(DevPlan d, const WorkItem *work, const int32_t *order,
                                                    int64_t w0, int64_t nw, const double *om, const double *panel,
                                                    double *staging, double tau, unsigned long long *chunks,
                                                    unsigned *tickets, uint64_t *hotmask) {
  constexpr bool SPLIT = MODE == MODE_SPLIT || MODE == MODE_F32;
  constexpr bool HOTK = MODE == MODE_HOT;
  __shared__ double sa[32 * DROW], sb[32 * DROW];
  __shared__ double s_om[16];
  __shared__ int64_t s_pos;
  unsigned long long n_hot = 0, n_all = 0;
  int64_t pos = PERSIST ? next_item(tickets, nw, order != nullptr, &s_pos)
                        : (order ? (int64_t)blockIdx.x : xcd_map(blockIdx.x, nw));
  while (!PERSIST || pos < nw) {
  const int64_t wi = w0 + (order ? order[w0 + pos] : pos);
  const WorkItem it = work[wi];
  const uint64_t hmask_in = HOTK ? hotmask[wi] : 0;  // MODE_HOT: chunks to add
  uint64_t hmask = 0;                               // split modes: deferred chunks
  const int b = it.batch;
  const int g0 = d.batch_pt_off[b], P = d.batch_pt_off[b + 1] - g0;
  const int f0 = d.batch_fn_off[b], n = d.batch_fn_off[b + 1] - f0;
  const int sbase = d.batch_slot_off[b];
  const int r0 = it.ti * T, c0 = it.tj * T;
  const bool diag = it.ti == it.tj;
  const int Pp = (int)pad16(P), np = (int)pad16(n);
  const double *pb = panel + d.panel_off[b];
  const int64_t plane = (int64_t)Pp * np;
  const int tid = threadIdx.x;
  // wave index as a scalar: conditions derived from it stay uniform
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  (void)diag;
  const int li16 = lane & 15, lk = lane >> 4;
  int brow[4], bcol[4];
  bool act[4];
  wave_blocks(r0, c0, n, wave, brow, bcol, act);

  dbl4 acc[4][5];
#pragma unroll
  for (int sl = 0; sl < 4; ++sl)
#pragma unroll
    for (int q = 0; q < 5; ++q) acc[sl][q] = dbl4{0.0, 0.0, 0.0, 0.0};
  // FP32 accumulators of the four W parts (split modes)
  flt4 accf[4][4];
  if (SPLIT) {
#pragma unroll
    for (int sl = 0; sl < 4; ++sl)
#pragma unroll
      for (int q = 0; q < 4; ++q) accf[sl][q] = flt4{0.f, 0.f, 0.f, 0.f};
  }

  const double cp = d.cprime;
  // Chunks of 8 points in two LDS buffers, the next chunk's DMA in flight
  // while this one is multiplied (one barrier per chunk); the split modes'
  // FP64 routing is decided per 16 points.  MODE_HOT: 16-point chunks, one
  // buffer, only the deferred ones.
  constexpr int CH = HOTK ? 16 : 8;
  constexpr bool DB = !HOTK;  // double-buffered chunk images
  constexpr int RPQ = CH / 2;              // LDS rows per component
  constexpr int BUFD = 4 * RPQ * DROW;     // doubles per chunk image
  bool hot = true;  // W parts of the current 16 points on FP64 MFMA
  // Double-buffered path: the global loads a chunk needs besides its image
  // (w v at its points; the split modes' bound inputs of its 16 points) are
  // issued one chunk ahead, with the next image's DMA, so that nothing
  // consumed between the barrier and the last MFMA of a chunk waits on
  // loads still in flight.
  double omn[CH / 4];  // w v at points 4 ks + lk of the next chunk
  double ga = 0.0, gb = 0.0, gw = 0.0;  // bound inputs of the next 16 points
  const double *gmx = pb + 4 * plane;  // per-point gradient maxima of the row tiles
  auto load_om = [&](int k) {
#pragma unroll
    for (int ks = 0; ks < CH / 4; ++ks) {
      const int pt = k + 4 * ks + lk;
      omn[ks] = pt < P ? om[g0 + pt] : 0.0;
    }
  };
  auto load_bound = [&](int k) {
    // lanes 0..15: row tile maxima; lanes 16..31: column tile maxima and w v
    ga = gb = gw = 0.0;
    if (lane < 16) {
      ga = gmx[(int64_t)it.ti * Pp + k + lane];
    } else if (lane < 32 && k + lane - 16 < P) {
      gb = gmx[(int64_t)it.tj * Pp + k + lane - 16];
      gw = om[g0 + k + lane - 16];
    }
  };
  if (DB) {
    load_om(0);
    if (SPLIT) load_bound(0);
    dma_chunk<NT, CH>(pb, plane, np, r0, 0, sa);
    dma_chunk<NT, CH>(pb, plane, np, c0, 0, sb);
  }
  for (int k0 = 0; k0 < Pp; k0 += CH) {
    if (HOTK && !((hmask_in >> (k0 >> 4)) & 1)) continue;  // WG-uniform
    const int bo = DB ? ((k0 / CH) & 1) * BUFD : 0;  // this chunk's buffer
    double omv[CH / 4];  // FP64 path: w v at points 4 ks + lk of this chunk
    double va = 0.0, vb = 0.0;  // split modes: bound inputs of this lane
    if (!DB) {
      __syncthreads();  // previous chunk's operands consumed
      if (tid < 16) s_om[tid] = k0 + tid < P ? om[g0 + k0 + tid] : 0.0;
      dma_chunk<NT, CH>(pb, plane, np, r0, k0 >> 2, sa);
      dma_chunk<NT, CH>(pb, plane, np, c0, k0 >> 2, sb);
      __builtin_amdgcn_s_waitcnt(0);  // this thread's LDS DMA loads have landed
      __syncthreads();                // the chunk and s_om are visible
    } else {
      __builtin_amdgcn_s_waitcnt(0);  // this thread's loads of this chunk have landed
      __syncthreads();                // ... everyone's; the previous chunk is consumed
#pragma unroll
      for (int ks = 0; ks < CH / 4; ++ks) omv[ks] = omn[ks];
      if (SPLIT && (k0 & 15) == 0) {
        va = ga;
        vb = gb * fabs(gw);
      }
      if (k0 + CH < Pp) {
        const int nbo = BUFD - bo;
        load_om(k0 + CH);
        if (SPLIT && ((k0 + CH) & 15) == 0) load_bound(k0 + CH);
        dma_chunk<NT, CH>(pb, plane, np, r0, (k0 + CH) >> 2, sa + nbo);
        dma_chunk<NT, CH>(pb, plane, np, c0, (k0 + CH) >> 2, sb + nbo);
      }
    }
    const double *ca = sa + bo, *cb = sb + bo;
    if (SPLIT && (k0 & 15) == 0) {
      // bound of the 16 points k0 .. k0+15: A = largest |gradient component|
      // of the row tile, B = largest |w v gradient component| of the column
      // tile, from the panel's per-point maxima; every wave forms the same
      // values, so the decision is uniform over the workgroup
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        va = fmax(va, __shfl_xor(va, off));
        vb = fmax(vb, __shfl_xor(vb, off));
      }
      // equal in every lane after the reductions; as a scalar the branches stay uniform
      hot = __builtin_amdgcn_readfirstlane(kU32 * cp * 48.0 * va * vb > tau ? 1 : 0) != 0;
      n_hot += hot ? 1 : 0;
      n_all += 1;
      if (hot) hmask |= (uint64_t)1 << (k0 >> 4);
    }
#pragma unroll
    for (int ks = 0; ks < CH / 4; ++ks) {
      // K index lk of step ks is point 4 ks + lk of the chunk; the column
      // operand takes its weight w v there (the weighting of Eq. 29)
      const int rowk = 2 * ks + (lk >> 1), ck = lk & 1;
      const double omk = DB ? omv[ks] : s_om[4 * ks + lk];
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) {
        if (!act[sl]) continue;  // wave-uniform
        double av[4], bv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          av[q] = ca[(q * RPQ + rowk) * DROW + 2 * (brow[sl] + li16) + ck];
          bv[q] = cb[(q * RPQ + rowk) * DROW + 2 * (bcol[sl] + li16) + ck] * omk;
        }
        if (!HOTK) acc[sl][0] = mfma64(av[0], bv[0], acc[sl][0]);
        if (MODE == MODE_F64 || HOTK) {
          acc[sl][1] = mfma64(av[1], bv[1], acc[sl][1]);
          acc[sl][2] = mfma64(av[2], bv[3], acc[sl][2]);
          acc[sl][3] = mfma64(av[3], bv[1], acc[sl][3]);
          acc[sl][4] = mfma64(av[1], bv[2], acc[sl][4]);
          acc[sl][1] = mfma64(av[2], bv[2], acc[sl][1]);
          acc[sl][2] = mfma64(-av[3], bv[2], acc[sl][2]);
          acc[sl][3] = mfma64(-av[1], bv[3], acc[sl][3]);
          acc[sl][4] = mfma64(-av[2], bv[1], acc[sl][4]);
          acc[sl][1] = mfma64(av[3], bv[3], acc[sl][1]);
        } else if (hot) {
          // deferred to MODE_HOT
        } else if (MODE == MODE_F32) {
          float af[4], bf[4];
#pragma unroll
          for (int q = 1; q < 4; ++q) {
            af[q] = (float)av[q];
            bf[q] = (float)bv[q];
          }
          accf[sl][0] = mfma32(af[1], bf[1], accf[sl][0]);
          accf[sl][1] = mfma32(af[2], bf[3], accf[sl][1]);
          accf[sl][2] = mfma32(af[3], bf[1], accf[sl][2]);
          accf[sl][3] = mfma32(af[1], bf[2], accf[sl][3]);
          accf[sl][0] = mfma32(af[2], bf[2], accf[sl][0]);
          accf[sl][1] = mfma32(-af[3], bf[2], accf[sl][1]);
          accf[sl][2] = mfma32(-af[1], bf[3], accf[sl][2]);
          accf[sl][3] = mfma32(-af[2], bf[1], accf[sl][3]);
          accf[sl][0] = mfma32(af[3], bf[3], accf[sl][0]);
        } else if (MODE == MODE_SPLIT) {
          // hi + lo split: x = hi + lo with hi = fl(x), lo = fl(x - hi);
          // x y ~ hi_x hi_y + hi_x lo_y + lo_x hi_y (lo_x lo_y dropped)
          float ah[4], al[4], bh[4], bl[4];
#pragma unroll
          for (int q = 1; q < 4; ++q) {
            ah[q] = (float)av[q];
            al[q] = (float)(av[q] - (double)ah[q]);
            bh[q] = (float)bv[q];
            bl[q] = (float)(bv[q] - (double)bh[q]);
          }
#define SPLIT3(ACC, AI, BI, SG)                                  \
  ACC = mfma32(SG ah[AI], bh[BI], ACC);                          \
  ACC = mfma32(SG ah[AI], bl[BI], ACC);                          \
  ACC = mfma32(SG al[AI], bh[BI], ACC);
          SPLIT3(accf[sl][0], 1, 1, +)
          SPLIT3(accf[sl][0], 2, 2, +)
          SPLIT3(accf[sl][0], 3, 3, +)
          SPLIT3(accf[sl][1], 2, 3, +)
          SPLIT3(accf[sl][1], 3, 2, -)
          SPLIT3(accf[sl][2], 3, 1, +)
          SPLIT3(accf[sl][2], 1, 3, -)
          SPLIT3(accf[sl][3], 1, 2, +)
          SPLIT3(accf[sl][3], 2, 1, -)
#undef SPLIT3
        }
      }
    }
  }
  // write the computed blocks to the staged atom-pair blocks
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    if (!act[sl]) continue;
    const int cb = c0 + bcol[sl];
    const int lj = cb + li16;
    if (lj >= n) continue;
    const SlotInfo sj = slot_of(d, f0, sbase, lj);
    const int rb = r0 + brow[sl];
    const bool upper = rb < cb;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // V and, in FP64 modes, the W parts: FP64 MFMA rows lk + 4 r
      const int li = rb + d_row_f64(lk, r);
      if (li < n && !(HOTK && hmask_in == 0)) {
        const SlotInfo si = slot_of(d, f0, sbase, li);
        double vals[5];
        vals[0] = acc[sl][0][r];
#pragma unroll
        for (int q = 1; q < 5; ++q) vals[q] = cp * acc[sl][q][r];
        if (MODE == MODE_F64)
          stage_store<0, 5>(staging, si, sj, li, lj, upper, vals);
        else if (HOTK)
          stage_add<1, 5>(staging, si, sj, li, lj, upper, vals + 1);
        else
          stage_store<0, 1>(staging, si, sj, li, lj, upper, vals);
      }
      if (SPLIT) {
        // the W parts from the FP32 accumulators: FP32 MFMA rows 4 lk + r
        const int lf = rb + d_row_f32(lk, r);
        if (lf < n) {
          const SlotInfo sf = slot_of(d, f0, sbase, lf);
          double w[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) w[q] = cp * (double)accf[sl][q][r];
          stage_store<1, 5>(staging, sf, sj, lf, lj, upper, w);
        }
      }
    }
  }
  if (SPLIT && threadIdx.x == 0) hotmask[wi] = hmask;
  if (!PERSIST) break;
  pos = next_item(tickets, nw, order != nullptr, &s_pos);
  }
  if (SPLIT && threadIdx.x == 0) {
    const int slot = (int)(blockIdx.x & 63);
    atomicAdd(&chunks[2 * slot], n_hot);
    atomicAdd(&chunks[2 * slot + 1], n_all);
  }
}

// Batch-to-global sum for one pass: reduction entry r adds the staged blocks
// of pair red_pair[r] in batch order, one after another onto the running
// value (zero, or the stored value when a previous pass or ACCUMULATE left
// one).  The sum is a single sequential chain in batch order, so results
// repeat bit for bit and do not depend on how batches are split into passes.
// Loads of four incidences are issued together.
__global__ __launch_bounds__(256) void k_reduce(DevPlan d, int64_t r0, const int32_t *red_pair,
                                                const uint8_t *red_first, const int64_t *red_inc_off,
                                                const int64_t *inc_src, const double *staging, double *store,
                                                int accumulate, int nq) {
  __shared__ int64_t s_src[256];
  const int64_t r = r0 + blockIdx.x;
  const int p = red_pair[r];
  const int blk = d.pair_na[p] * d.pair_nb[p];
  const int64_t k0 = red_inc_off[r], k1 = red_inc_off[r + 1];
  const bool add = accumulate || !red_first[r];
  const int64_t po = d.pair_off[p];
  const int m = nq * blk;  // parts 0 .. nq-1 of the staged blocks (the first nq of five)
  // each thread owns elements e = tid, tid + 256, ... (at most 4 at a time in registers)
  for (int e0 = 0; e0 < m; e0 += 4 * 256) {
    double sum[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = e0 + j * 256 + threadIdx.x;
      sum[j] = 0.0;
      if (e < m && add) {
        const int q = e / blk;
        sum[j] = store[q * d.store_len + po + (e - q * blk)];
      }
    }
    for (int64_t kb = k0; kb < k1; kb += 256) {
      const int nk = (int)(k1 - kb < 256 ? k1 - kb : 256);
      __syncthreads();  // previous offsets consumed
      if (threadIdx.x < nk) s_src[threadIdx.x] = inc_src[kb + threadIdx.x];
      __syncthreads();
      int k = 0;
      for (; k + 8 <= nk; k += 8) {
        double a[4][8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int e = e0 + j * 256 + threadIdx.x;
#pragma unroll
          for (int u = 0; u < 8; ++u) a[j][u] = e < m ? staging[s_src[k + u] + e] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int u = 0; u < 8; ++u) sum[j] += a[j][u];
      }
      for (; k < nk; ++k) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int e = e0 + j * 256 + threadIdx.x;
          if (e < m) sum[j] += staging[s_src[k] + e];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = e0 + j * 256 + threadIdx.x;
      if (e < m) {
        const int q = e / blk;
        store[q * d.store_len + po + (e - q * blk)] = sum[j];
      }
    }
  }
}

// Pairs no batch touches are zero unless accumulating.
__global__ void k_zero_pairs(DevPlan d, const int32_t *pairs, double *store, int nq) {
  const int p = pairs[blockIdx.x];
  const int64_t blk = (int64_t)d.pair_na[p] * d.pair_nb[p];
  for (int64_t e = threadIdx.x; e < nq * blk; e += blockDim.x) {
    const int q = (int)(e / blk);
    store[q * d.store_len + d.pair_off[p] + (e - q * blk)] = 0.0;
  }
}

// W_sp = Ws (x) I2 + i sum_m Wso_m (x) sigma_m and V_sp = V (x) I2, per pair a
// (2 nA) x (2 nB) complex block, spin-major rows and columns.
__global__ void k_spinor(DevPlan d, const double *store, double *spin_w, double *spin_v) {
  const int p = blockIdx.x;
  const int na = d.pair_na[p], nb = d.pair_nb[p];
  const int64_t blk = (int64_t)na * nb;
  const int64_t po = d.pair_off[p];
  const int64_t L = d.store_len;
  const int64_t cb = 8 * po;           // doubles: complex offset 4 po
  const int64_t rs = 2 * (int64_t)nb;  // complex row stride
  for (int64_t e = threadIdx.x; e < blk; e += blockDim.x) {
    const int i = (int)(e / nb), j = (int)(e - (int64_t)i * nb);
    const int64_t uu = 2 * ((int64_t)i * rs + j), ud = 2 * ((int64_t)i * rs + nb + j);
    const int64_t du = 2 * ((int64_t)(na + i) * rs + j), dd = 2 * ((int64_t)(na + i) * rs + nb + j);
    if (spin_w) {
      const double ws = store[L + po + e], wx = store[2 * L + po + e], wy = store[3 * L + po + e],
                   wz = store[4 * L + po + e];
      double *o = spin_w + cb;
      o[uu] = ws; o[uu + 1] = wz;
      o[ud] = wy; o[ud + 1] = wx;
      o[du] = -wy; o[du + 1] = wx;
      o[dd] = ws; o[dd + 1] = -wz;
    }
    if (spin_v) {
      const double vv = store[po + e];
      double *o = spin_v + cb;
      o[uu] = vv; o[uu + 1] = 0.0;
      o[ud] = 0.0; o[ud + 1] = 0.0;
      o[du] = 0.0; o[du + 1] = 0.0;
      o[dd] = vv; o[dd + 1] = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint / density
// ---------------------------------------------------------------------------

// The adjoint runs per quarter of a work item: a 32 x 32 block of the
// batch's coefficient matrix (rows ti*64 + 32 rh .., columns tj*64 + 32 ch ..),
// four waves with one 16 x 16 block each.  Positions 4 w + qd, qd = 2 rh + ch.
constexpr int NTD = 256;
constexpr int QW = 32;              // functions per side of a quarter
// LDS image of one 16-point chunk of 32 functions (layout of dma_chunk): row
// (q, u) every RSQ doubles; 2 mod 16, so 16 lanes reading 16 consecutive
// points of one function hit distinct banks
constexpr int RSQ = 2 * QW + 2;
constexpr int QIMG = 4 * 8 * RSQ;   // doubles per image: 4 components x 8 point pairs

// A quarter has work iff its rows and columns start inside the batch's n
// functions and it is not below the diagonal of a diagonal tile.
__device__ __forceinline__ bool quarter_valid(const WorkItem &it, int qd, int n) {
  const int rh = qd >> 1, ch = qd & 1;
  return it.ti * T + 32 * rh < n && it.tj * T + 32 * ch < n && !(it.ti == it.tj && rh > ch);
}

// partial[g] of quarter qd (P doubles at 4 work_part_off[w] + qd P) = sum over
// its stored elements ij of the selected terms at point g:
//   C^V phi_i phi_j + c' C^Ws grad phi_i . grad phi_j + c' sum_m C^m (grad phi_i x grad phi_j)_m
// (Eq. 39 on the scalar basis).  Per wave, the 16 x 16 coefficient block sits
// in registers as the MFMA's first operand (5 parts x 4 K steps of 4 rows),
// and per 16-point chunk four accumulators collect (C^T Y) grouped by the
// column component Z they are multiplied with afterwards:
//   u_phi = C^V phi,  u_x = C^Ws dx - C^z dy + C^y dz,
//   u_y = C^z dx + C^Ws dy - C^x dz,  u_z = -C^y dx + C^x dy + C^Ws dz
// (rows i, the K index: Y = the row functions' values at the chunk's points),
// then one lane-local drain sum_j u . Z per chunk.  Chunk images arrive by LDS
// DMA, double-buffered: the next chunk's loads are in flight while this one
// is multiplied (one barrier per chunk); two workgroups fit on a CU.
template <bool PERSIST>
__global__ __launch_bounds__(NTD, 2) void k_density_tiles(DevPlan d, uint32_t terms, const WorkItem *work,
                                                          const int32_t *order, int64_t w0, int64_t nw,
                                                          const double *coef, const double *panel,
                                                          double *partial, unsigned *tickets) {
  constexpr int NC = 5;  // coefficient parts
  __shared__ double img[2][2][QIMG];     // [buffer][row image, column image]
  __shared__ double s_red[2][4][16];     // per-wave point sums, alternating chunks
  __shared__ int64_t s_pos;
  // slot data of the quarter's 32 rows and 32 columns (slot -1: beyond n)
  __shared__ int s_rslot[QW], s_rfn[QW], s_cslot[QW], s_cfn[QW], s_cnf[QW];
  // store offset of the pair block of (row slot, column slot) for the slots
  // the quarter spans (-1: lower atom-block triangle or not a stored pair)
  __shared__ int64_t s_poff[QW * QW];
  const int64_t npos = 4 * nw;
  int64_t pos = PERSIST ? next_item(tickets, npos, order != nullptr, &s_pos)
                        : (order ? (int64_t)blockIdx.x : xcd_map(blockIdx.x, npos));
  while (!PERSIST || pos < npos) {
  const int qd = (int)(pos & 3);
  const int64_t wi = w0 + (order ? order[w0 + (pos >> 2)] : (pos >> 2));
  const WorkItem it = work[wi];
  const int b = it.batch;
  const int f0 = d.batch_fn_off[b], n = d.batch_fn_off[b + 1] - f0;
  if (quarter_valid(it, qd, n)) {  // workgroup-uniform
  const int g0 = d.batch_pt_off[b], P = d.batch_pt_off[b + 1] - g0;
  const int sbase = d.batch_slot_off[b];
  const int r0 = it.ti * T + 32 * (qd >> 1), c0 = it.tj * T + 32 * (qd & 1);
  const int Pp = (int)pad16(P), np = (int)pad16(n);
  const double *pb = panel + d.panel_off[b];
  const int64_t plane = (int64_t)Pp * np;
  const int tid = threadIdx.x;
  // wave index as a scalar: conditions derived from it stay uniform
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int rb = wave >> 1, cb = wave & 1;  // this wave's 16 x 16 block in the quarter
  const int l16 = lane & 15, lk = lane >> 4;
  const int rowb = r0 + 16 * rb, colb = c0 + 16 * cb;
  const bool act = block_active(rowb, colb, n);
  const bool upper = rowb < colb;
  const int lj = colb + l16;
  if (tid < 2 * QW) {
    const bool row = tid < QW;
    const int lf = row ? r0 + tid : c0 + tid - QW;
    SlotInfo si{-1, 0, 0, 0};
    if (lf < n) si = slot_of(d, f0, sbase, lf);
    if (row) {
      s_rslot[tid] = si.slot;
      s_rfn[tid] = si.fnoff;
    } else {
      s_cslot[tid - QW] = si.slot;
      s_cfn[tid - QW] = si.fnoff;
      s_cnf[tid - QW] = si.nfn;
    }
  }
  __syncthreads();  // slot tables visible
  // slot ranges of the quarter's rows and columns (slots ascend with the
  // functions; rows and columns beyond n carry slot -1)
  const int rs0 = s_rslot[0], cs0 = s_cslot[0];
  const int rs1 = s_rslot[min(QW, n - r0) - 1], cs1 = s_cslot[min(QW, n - c0) - 1];
  const int nrs = rs1 - rs0 + 1, ncs = cs1 - cs0 + 1;
  {
    const int ns = d.batch_slot_off[b + 1] - sbase;
    const int64_t spb = d.batch_sp_off[b];
    for (int t = tid; t < nrs * ncs; t += NTD) {
      const int si = rs0 + t / ncs, sj = cs0 + t % ncs;
      int64_t po = -1;
      if (si <= sj) {
        // upper-triangle index of (si, sj)
        const int q = d.sp_pair[spb + (int64_t)si * ns - (int64_t)si * (si - 1) / 2 + (sj - si)];
        if (q >= 0) po = d.pair_off[q];
      }
      s_poff[t] = po;
    }
  }
  // the first chunk's images load while the coefficients are read
  dma_chunk<NTD, 16, QW, RSQ>(pb, plane, np, r0, 0, img[0][0]);
  dma_chunk<NTD, 16, QW, RSQ>(pb, plane, np, c0, 0, img[0][1]);
  __syncthreads();  // pair offsets visible
  // coefficient block: rows i = rowb + 4 ks + lk (ks = 0..3), column lj, read
  // from the store: element (li, lj) of the pair block of its two atoms
  // (upper atom-block triangle only), plus the mirrored element (lj, li) when
  // the 16 x 16 block is strictly upper inside one atom block (no work item
  // computes the mirrored block); c' on the W parts, zero for unselected
  // terms.  Every load is issued before any is used.
  double creg[NC][4];
  {
    const int64_t L = d.store_len;
    const int cl = 16 * cb + l16;
    const int cslot = s_cslot[cl], cfn = s_cfn[cl], cnf = s_cnf[cl];
    int64_t ea[4], em[4];
    bool live[4], mir[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int rl = 16 * rb + 4 * ks + lk;
      const int li = r0 + rl;
      const int rslot = s_rslot[rl], rfn = s_rfn[rl];
      const int64_t po = (act && rslot >= 0 && cslot >= 0) ? s_poff[(rslot - rs0) * ncs + (cslot - cs0)] : -1;
      live[ks] = po >= 0;
      mir[ks] = live[ks] && upper && rslot == cslot;
      ea[ks] = live[ks] ? po + (int64_t)(li - rfn) * cnf + (lj - cfn) : 0;
      em[ks] = mir[ks] ? po + (int64_t)(lj - rfn) * cnf + (li - cfn) : 0;
    }
    double cv[NC][4], cm[NC][4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        cv[q][ks] = coef[q * L + ea[ks]];
        cm[q][ks] = coef[q * L + em[ks]];
      }
    const bool on[NC] = {(terms & Q4C_TERM_LL) != 0, (terms & Q4C_TERM_SS) != 0, (terms & Q4C_TERM_SO) != 0,
                         (terms & Q4C_TERM_SO) != 0, (terms & Q4C_TERM_SO) != 0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const double c = (live[ks] ? cv[q][ks] : 0.0) + (mir[ks] ? mirror_sign(q) * cm[q][ks] : 0.0);
        creg[q][ks] = on[q] ? (q == 0 ? c : d.cprime * c) : 0.0;
      }
  }
  double *out = partial + 4 * d.work_part_off[wi] + qd * P;

  for (int k0 = 0; k0 < Pp; k0 += 16) {
    const int bi = (k0 >> 4) & 1;
    __builtin_amdgcn_s_waitcnt(0);  // this thread's loads of this chunk have landed
    __syncthreads();                // ... everyone's; the previous chunk is consumed, its sums visible
    if (k0 > 0 && tid < 16 && k0 - 16 + tid < P)
      out[k0 - 16 + tid] = (s_red[bi ^ 1][0][tid] + s_red[bi ^ 1][1][tid]) +
                           (s_red[bi ^ 1][2][tid] + s_red[bi ^ 1][3][tid]);
    if (k0 + 16 < Pp) {
      dma_chunk<NTD, 16, QW, RSQ>(pb, plane, np, r0, (k0 + 16) >> 2, img[bi ^ 1][0]);
      dma_chunk<NTD, 16, QW, RSQ>(pb, plane, np, c0, (k0 + 16) >> 2, img[bi ^ 1][1]);
    }
    double x = 0.0;
    if (act) {
      const double *ia = img[bi][0], *ib = img[bi][1];
      // column values Z[q][pt = l16][j = 16 cb + lk + 4 r]: register r of the
      // MFMA result of lane (l16, lk) is column lk + 4 r of the block at point l16
      double zt[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) zt[q][r] = ib[(q * 8 + (l16 >> 1)) * RSQ + 2 * (16 * cb + d_row_f64(lk, r)) + (l16 & 1)];
      dbl4 uf = dbl4{0.0, 0.0, 0.0, 0.0}, ux = uf, uy = uf, uz = uf;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        // row values Y[q][pt = l16][i = 16 rb + 4 ks + lk]: the K index is lk
        const int col = 2 * (16 * rb + 4 * ks + lk) + (l16 & 1);
        const double y0 = ia[(0 * 8 + (l16 >> 1)) * RSQ + col], y1 = ia[(1 * 8 + (l16 >> 1)) * RSQ + col];
        const double y2 = ia[(2 * 8 + (l16 >> 1)) * RSQ + col], y3 = ia[(3 * 8 + (l16 >> 1)) * RSQ + col];
        uf = mfma64(creg[0][ks], y0, uf);
        ux = mfma64(creg[1][ks], y1, ux);
        uy = mfma64(creg[4][ks], y1, uy);
        uz = mfma64(creg[3][ks], -y1, uz);
        ux = mfma64(creg[4][ks], -y2, ux);
        uy = mfma64(creg[1][ks], y2, uy);
        uz = mfma64(creg[2][ks], y2, uz);
        ux = mfma64(creg[3][ks], y3, ux);
        uy = mfma64(creg[2][ks], -y3, uy);
        uz = mfma64(creg[1][ks], y3, uz);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) x += (uf[r] * zt[0][r] + ux[r] * zt[1][r]) + (uy[r] * zt[2][r] + uz[r] * zt[3][r]);
      // sum over the block's 16 columns: the 4 registers (above), then the 4 lane rows
      x += __shfl_xor(x, 16);
      x += __shfl_xor(x, 32);
    }
    if (lane < 16) s_red[bi][wave][l16] = x;
  }
  __syncthreads();  // the last chunk's per-wave sums
  {
    const int k0 = Pp - 16, bi = (k0 >> 4) & 1;
    if (tid < 16 && k0 + tid < P)
      out[k0 + tid] = (s_red[bi][0][tid] + s_red[bi][1][tid]) + (s_red[bi][2][tid] + s_red[bi][3][tid]);
  }
  }  // quarter_valid
  if (!PERSIST) break;
  pos = next_item(tickets, npos, order != nullptr, &s_pos);
  }
}

// Point sums: out[perm[g]] = (w_g if weighted) * sum over the batch's work
// items (in order) and their valid quarters (in order).
__global__ void k_density_points(DevPlan d, const WorkItem *work, int64_t b0, const double *partial, int weight_mode,
                                 double *out) {
  const int64_t b = b0 + blockIdx.x;
  const int g0 = d.batch_pt_off[b], P = d.batch_pt_off[b + 1] - g0;
  const int n = d.batch_fn_off[b + 1] - d.batch_fn_off[b];
  const int64_t wa = d.batch_work_off[b], wb = d.batch_work_off[b + 1];
  for (int g = threadIdx.x; g < P; g += blockDim.x) {
    double s = 0.0;
    for (int64_t w = wa; w < wb; ++w) {
      const WorkItem it = work[w];
      const double *pw = partial + 4 * d.work_part_off[w];
#pragma unroll
      for (int qd = 0; qd < 4; ++qd)
        if (quarter_valid(it, qd, n)) s += pw[qd * P + g];
    }
    out[d.perm[g0 + g]] = weight_mode ? d.pw[g0 + g] * s : s;
  }
}

__global__ void k_fill(double *p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Coefficients from spinor blocks D_AB (see q4c_coef_from_spinor).
__global__ void k_coef_from_spinor(DevPlan d, const double *spin, double *coef) {
  const int p = blockIdx.x;
  const int na = d.pair_na[p], nb = d.pair_nb[p];
  const int64_t blk = (int64_t)na * nb;
  const int64_t po = d.pair_off[p];
  const int64_t L = d.store_len;
  const int64_t rs = 2 * (int64_t)nb;
  const double f = d.pair_a[p] == d.pair_b[p] ? 1.0 : 2.0;
  const double *D = spin + 8 * po;
  for (int64_t e = threadIdx.x; e < blk; e += blockDim.x) {
    const int i = (int)(e / nb), j = (int)(e - (int64_t)i * nb);
    const double *uu = D + 2 * ((int64_t)i * rs + j), *ud = D + 2 * ((int64_t)i * rs + nb + j);
    const double *du = D + 2 * ((int64_t)(na + i) * rs + j), *dd = D + 2 * ((int64_t)(na + i) * rs + nb + j);
    const double dsum = f * (uu[0] + dd[0]);
    coef[po + e] = dsum;
    coef[L + po + e] = dsum;
    coef[2 * L + po + e] = f * (ud[1] + du[1]);
    coef[3 * L + po + e] = f * (ud[0] - du[0]);
    coef[4 * L + po + e] = f * (uu[1] - dd[1]);
  }
}

__global__ void k_check_finite(const double *v, int64_t n, int32_t *flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    if (!isfinite(v[i])) flag[0] = 1;
}

}  // namespace

static int check_launch(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, what);
  return Q4C_OK;
}

int launch_tabulate(const q4c_plan *p, int64_t b0, int64_t b1, int deriv, int dtype, void *out, hipStream_t s) {
  const int64_t t0 = p->batch_tile_off[b0], nt = p->batch_tile_off[b1] - t0;
  if (nt <= 0) return Q4C_OK;
  {
    TimedLaunch tl_(p, Q4C_TIMER_TABULATE, s);
    if (dtype == Q4C_DTYPE_F32_HILO)
      hipLaunchKernelGGL(k_tabulate<true>, dim3((unsigned)nt), dim3(256), 0, s, p->dp, p->d_ptile, t0, b0, deriv, out);
    else
      hipLaunchKernelGGL(k_tabulate<false>, dim3((unsigned)nt), dim3(256), 0, s, p->dp, p->d_ptile, t0, b0, deriv, out);
  }
  return check_launch("k_tabulate");
}

int launch_integrate(const q4c_plan *p, const double *v, int precision, uint32_t flags, double *store,
                     double *spin_w, double *spin_v, hipStream_t s) {
  const int accumulate = (flags & Q4C_ACCUMULATE) ? 1 : 0;
  int rc;
  {
    TimedLaunch tl_(p, Q4C_TIMER_OTHER, s);
    const unsigned nb = (unsigned)std::min<int64_t>((p->n_active + 16 + 255) / 256, 65535);
    hipLaunchKernelGGL(k_om, dim3(nb), dim3(256), 0, s, p->dp, v, p->d_om, p->d_chunks);
  }
  if ((rc = check_launch("k_om")) != Q4C_OK) return rc;
  const LaunchCfg cfg = p->cfg_contract;
  const int32_t *order = cfg.order ? p->d_order : nullptr;
  if (cfg.persistent > 0) {
    hipLaunchKernelGGL(k_zero_u32, dim3(8), dim3(256), 0, s, p->d_tickets,
                       (int64_t)p->passes.size() * kTicketsPerLaunch);
    if ((rc = check_launch("k_zero_u32")) != Q4C_OK) return rc;
  }
  for (size_t ip = 0; ip < p->passes.size(); ++ip) {
    const Pass &ps = p->passes[ip];
    const int64_t nw = ps.w1 - ps.w0, nt = ps.t1 - ps.t0, nr = ps.r1 - ps.r0;
    unsigned *tickets = cfg.persistent > 0 ? p->d_tickets + ip * kTicketsPerLaunch : nullptr;
    const unsigned grid = (unsigned)(cfg.persistent > 0 ? std::min<int64_t>(cfg.persistent, nw) : nw);
    double *panel = p->d_staging + ps.staging_len + ps.partial_len;
    if (nt > 0) {
      {
        TimedLaunch tl_(p, Q4C_TIMER_TABULATE, s);
        hipLaunchKernelGGL(k_panel<false>, dim3((unsigned)nt), dim3(256), 0, s, p->dp, p->d_ptile, ps.t0, nt, panel);
      }
      if ((rc = check_launch("k_panel")) != Q4C_OK) return rc;
    }
    if (nw > 0) {
      {
        TimedLaunch tl_(p, Q4C_TIMER_CONTRACT, s);
        if (precision == Q4C_PREC_F64)
          {
          if (tickets)
            hipLaunchKernelGGL((k_contract<MODE_F64, true>), dim3(grid), dim3(NT), 0, s, p->dp, p->d_work, order, ps.w0,
                               nw, p->d_om, panel, p->d_staging, p->split_tau, p->d_chunks, tickets, p->d_hotmask);
          else
            hipLaunchKernelGGL((k_contract<MODE_F64, false>), dim3(grid), dim3(NT), 0, s, p->dp, p->d_work, order, ps.w0,
                               nw, p->d_om, panel, p->d_staging, p->split_tau, p->d_chunks, tickets, p->d_hotmask);
        }
        else if (precision == Q4C_PREC_F32)
          {
          if (tickets)
            hipLaunchKernelGGL((k_contract<MODE_F32, true>), dim3(grid), dim3(NT), 0, s, p->dp, p->d_work, order, ps.w0,
                               nw, p->d_om, panel, p->d_staging, p->split_tau, p->d_chunks, tickets, p->d_hotmask);
          else
            hipLaunchKernelGGL((k_contract<MODE_F32, false>), dim3(grid), dim3(NT), 0, s, p->dp, p->d_work, order, ps.w0,
                               nw, p->d_om, panel, p->d_staging, p->split_tau, p->d_chunks, tickets, p->d_hotmask);
        }
        else
          {
          if (tickets)
            hipLaunchKernelGGL((k_contract<MODE_SPLIT, true>), dim3(grid), dim3(NT), 0, s, p->dp, p->d_work, order, ps.w0,
                               nw, p->d_om, panel, p->d_staging, p->split_tau, p->d_chunks, tickets, p->d_hotmask);
          else
            hipLaunchKernelGGL((k_contract<MODE_SPLIT, false>), dim3(grid), dim3(NT), 0, s, p->dp, p->d_work, order, ps.w0,
                               nw, p->d_om, panel, p->d_staging, p->split_tau, p->d_chunks, tickets, p->d_hotmask);
        }
      }
      if ((rc = check_launch("k_contract")) != Q4C_OK) return rc;
      if (precision != Q4C_PREC_F64) {
        // the deferred chunks' W parts in FP64, one workgroup per work item
        {
          TimedLaunch tl_(p, Q4C_TIMER_CONTRACT, s);
          hipLaunchKernelGGL((k_contract<MODE_HOT, false>), dim3((unsigned)nw), dim3(NT), 0, s, p->dp, p->d_work,
                             nullptr, ps.w0, nw, p->d_om, panel, p->d_staging, p->split_tau, p->d_chunks, nullptr,
                             p->d_hotmask);
        }
        if ((rc = check_launch("k_contract<hot>")) != Q4C_OK) return rc;
      }
    }
    if (nr > 0) {
      {
        TimedLaunch tl_(p, Q4C_TIMER_REDUCE, s);
        hipLaunchKernelGGL(k_reduce, dim3((unsigned)nr), dim3(256), 0, s, p->dp, ps.r0, p->d_red_pair, p->d_red_first,
                           p->d_red_inc_off, p->d_inc_src, p->d_staging, store, accumulate, 5);
      }
      if ((rc = check_launch("k_reduce")) != Q4C_OK) return rc;
    }
  }
  if (!accumulate && !p->untouched_pairs.empty()) {
    {
      TimedLaunch tl_(p, Q4C_TIMER_OTHER, s);
      hipLaunchKernelGGL(k_zero_pairs, dim3((unsigned)p->untouched_pairs.size()), dim3(256), 0, s, p->dp,
                         p->d_untouched, store, 5);
    }
    if ((rc = check_launch("k_zero_pairs")) != Q4C_OK) return rc;
  }
  if ((flags & (Q4C_ASSEMBLE_W | Q4C_ASSEMBLE_V)) && p->n_pairs > 0) {
    {
      TimedLaunch tl_(p, Q4C_TIMER_SPINOR, s);
      hipLaunchKernelGGL(k_spinor, dim3((unsigned)p->n_pairs), dim3(256), 0, s, p->dp, store,
                         (flags & Q4C_ASSEMBLE_W) ? spin_w : nullptr, (flags & Q4C_ASSEMBLE_V) ? spin_v : nullptr);
    }
    if ((rc = check_launch("k_spinor")) != Q4C_OK) return rc;
  }
  return Q4C_OK;
}

int launch_integrate_hs(const q4c_plan *p, const double *v, uint32_t flags, double *hs, hipStream_t s) {
  const int accumulate = (flags & Q4C_ACCUMULATE) ? 1 : 0;
  int rc;
  {
    TimedLaunch tl_(p, Q4C_TIMER_OTHER, s);
    const unsigned nb = (unsigned)std::min<int64_t>((p->n_active + 16 + 255) / 256, 65535);
    hipLaunchKernelGGL(k_om, dim3(nb), dim3(256), 0, s, p->dp, v, p->d_om, p->d_chunks);
  }
  if ((rc = check_launch("k_om")) != Q4C_OK) return rc;
  const LaunchCfg cfg = p->cfg_hs;
  const int32_t *order = cfg.order ? p->d_order : nullptr;
  if (cfg.persistent > 0) {
    hipLaunchKernelGGL(k_zero_u32, dim3(8), dim3(256), 0, s, p->d_tickets,
                       (int64_t)p->passes.size() * kTicketsPerLaunch);
    if ((rc = check_launch("k_zero_u32")) != Q4C_OK) return rc;
  }
  for (size_t ip = 0; ip < p->passes.size(); ++ip) {
    const Pass &ps = p->passes[ip];
    const int64_t nw = ps.w1 - ps.w0, nt = ps.t1 - ps.t0, nr = ps.r1 - ps.r0;
    unsigned *tickets = cfg.persistent > 0 ? p->d_tickets + ip * kTicketsPerLaunch : nullptr;
    const unsigned grid = (unsigned)(cfg.persistent > 0 ? std::min<int64_t>(cfg.persistent, nw) : nw);
    double *panel = p->d_staging + ps.staging_len + ps.partial_len;
    if (nt > 0) {
      {
        TimedLaunch tl_(p, Q4C_TIMER_TABULATE, s);
        hipLaunchKernelGGL(k_panel<true>, dim3((unsigned)nt), dim3(256), 0, s, p->dp, p->d_ptile, ps.t0, nt, panel);
      }
      if ((rc = check_launch("k_panel<hs>")) != Q4C_OK) return rc;
    }
    if (nw > 0) {
      {
        TimedLaunch tl_(p, Q4C_TIMER_CONTRACT, s);
        rc = launch_contract_hs(p, ps.w0, nw, order, panel, tickets, grid, s);
      }
      if (rc != Q4C_OK) return rc;
    }
    if (nr > 0) {
      {
        TimedLaunch tl_(p, Q4C_TIMER_REDUCE, s);
        hipLaunchKernelGGL(k_reduce, dim3((unsigned)nr), dim3(256), 0, s, p->dp, ps.r0, p->d_red_pair, p->d_red_first,
                           p->d_red_inc_off, p->d_inc_src, p->d_staging, hs, accumulate, 2);
      }
      if ((rc = check_launch("k_reduce")) != Q4C_OK) return rc;
    }
  }
  if (!accumulate && !p->untouched_pairs.empty()) {
    {
      TimedLaunch tl_(p, Q4C_TIMER_OTHER, s);
      hipLaunchKernelGGL(k_zero_pairs, dim3((unsigned)p->untouched_pairs.size()), dim3(256), 0, s, p->dp,
                         p->d_untouched, hs, 2);
    }
    if ((rc = check_launch("k_zero_pairs")) != Q4C_OK) return rc;
  }
  return Q4C_OK;
}

int launch_density(const q4c_plan *p, const double *coef, uint32_t terms, int weight_mode, double *out,
                   int64_t resident_pass, hipStream_t s) {
  int rc;
  if (p->n_points > 0) {
    {
      TimedLaunch tl_(p, Q4C_TIMER_OTHER, s);
      const unsigned nb = (unsigned)std::min<int64_t>((p->n_points + 255) / 256, 65535);
      hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, s, out, p->n_points, 0.0);
    }
    if ((rc = check_launch("k_fill")) != Q4C_OK) return rc;
  }
  const LaunchCfg cfg = p->cfg_density;
  const int32_t *order = cfg.order ? p->d_order : nullptr;
  unsigned *tick0 = p->d_tickets + p->passes.size() * kTicketsPerLaunch;
  if (cfg.persistent > 0) {
    hipLaunchKernelGGL(k_zero_u32, dim3(8), dim3(256), 0, s, tick0, (int64_t)p->passes.size() * kTicketsPerLaunch);
    if ((rc = check_launch("k_zero_u32")) != Q4C_OK) return rc;
  }
  // passes from the last one down: the first one may find its panels resident
  // (the forward call ends with its last pass); each point's partials lie in
  // one pass, so the order of the passes does not change any result
  for (size_t ipr = p->passes.size(); ipr-- > 0;) {
    const size_t ip = ipr;
    const Pass &ps = p->passes[ip];
    const int64_t nw = ps.w1 - ps.w0, nbt = ps.b1 - ps.b0;
    const int64_t nt = (int64_t)ip == resident_pass ? 0 : ps.t1 - ps.t0;
    unsigned *tickets = cfg.persistent > 0 ? tick0 + ip * kTicketsPerLaunch : nullptr;
    // four workgroup positions (quarters) per work item
    const unsigned grid = (unsigned)(cfg.persistent > 0 ? std::min<int64_t>(cfg.persistent, 4 * nw) : 4 * nw);
    double *partial = p->d_staging + ps.staging_len;
    double *panel = partial + ps.partial_len;
    if (nt > 0) {
      {
        TimedLaunch tl_(p, Q4C_TIMER_TABULATE, s);
        hipLaunchKernelGGL(k_panel<false>, dim3((unsigned)nt), dim3(256), 0, s, p->dp, p->d_ptile, ps.t0, nt, panel);
      }
      if ((rc = check_launch("k_panel")) != Q4C_OK) return rc;
    }
    if (nw > 0) {
      {
        TimedLaunch tl_(p, Q4C_TIMER_DENSITY_TILES, s);
        if (tickets)
          hipLaunchKernelGGL(k_density_tiles<true>, dim3(grid), dim3(NTD), 0, s, p->dp, terms, p->d_work, order, ps.w0,
                             nw, coef, panel, partial, tickets);
        else
          hipLaunchKernelGGL(k_density_tiles<false>, dim3(grid), dim3(NTD), 0, s, p->dp, terms, p->d_work, order,
                             ps.w0, nw, coef, panel, partial, tickets);
      }
      if ((rc = check_launch("k_density_tiles")) != Q4C_OK) return rc;
    }
    if (nbt > 0) {
      {
        TimedLaunch tl_(p, Q4C_TIMER_DENSITY_POINTS, s);
        hipLaunchKernelGGL(k_density_points, dim3((unsigned)nbt), dim3(256), 0, s, p->dp, p->d_work, ps.b0, partial,
                           weight_mode, out);
      }
      if ((rc = check_launch("k_density_points")) != Q4C_OK) return rc;
    }
  }
  return Q4C_OK;
}

int launch_density_grad(const q4c_plan *p, const double *coef, double *out, hipStream_t s) {
  int rc;
  if (p->n_points > 0) {
    {
      TimedLaunch tl_(p, Q4C_TIMER_OTHER, s);
      const unsigned nb = (unsigned)std::min<int64_t>((4 * p->n_points + 255) / 256, 65535);
      hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, s, out, 4 * p->n_points, 0.0);
    }
    if ((rc = check_launch("k_fill")) != Q4C_OK) return rc;
  }
  for (size_t ip = 0; ip < p->passes.size(); ++ip) {
    const Pass &ps = p->passes[ip];
    const int64_t nt = ps.t1 - ps.t0;
    double *panel = p->d_staging + ps.staging_len + ps.partial_len;
    if (nt > 0) {
      {
        TimedLaunch tl_(p, Q4C_TIMER_TABULATE, s);
        hipLaunchKernelGGL(k_panel<false>, dim3((unsigned)nt), dim3(256), 0, s, p->dp, p->d_ptile, ps.t0, nt, panel);
      }
      if ((rc = check_launch("k_panel")) != Q4C_OK) return rc;
    }
    if ((rc = launch_grad_pass(p, ip, coef, panel, out, s)) != Q4C_OK) return rc;
  }
  return Q4C_OK;
}

int launch_coef_from_spinor(const q4c_plan *p, const double *spin_d, double *coef_out, hipStream_t s) {
  if (p->n_pairs == 0) return Q4C_OK;
  {
    TimedLaunch tl_(p, Q4C_TIMER_OTHER, s);
    hipLaunchKernelGGL(k_coef_from_spinor, dim3((unsigned)p->n_pairs), dim3(256), 0, s, p->dp, spin_d, coef_out);
  }
  return check_launch("k_coef_from_spinor");
}

int launch_check_finite(const q4c_plan *p, const double *v, hipStream_t s, bool *finite) {
  hipError_t e = hipMemsetAsync(p->d_flag, 0, sizeof(int32_t), s);
  if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
  if (p->n_points > 0) {
    unsigned nb = (unsigned)std::min<int64_t>((p->n_points + 255) / 256, 65535);
    hipLaunchKernelGGL(k_check_finite, dim3(nb), dim3(256), 0, s, v, p->n_points, p->d_flag);
    int rc = check_launch("k_check_finite");
    if (rc != Q4C_OK) return rc;
  }
  int32_t h = 0;
  e = hipMemcpyAsync(&h, p->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  *finite = (h == 0);
  return Q4C_OK;
}

}  // namespace q4c
