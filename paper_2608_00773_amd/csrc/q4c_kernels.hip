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
//                    (Eq. 39): each column half of a work item reads its
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
__global__ void k_om(DevPlan d, const double *v, double *om) {
  const int64_t n = d.n_active;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n + 16; g += (int64_t)gridDim.x * blockDim.x)
    om[g] = g < n ? d.pw[g] * v[d.perm[g]] : 0.0;
}

// One (batch, function tile of 64): tabulate the tile's functions at all
// points of the batch into the panel.  Each group of 8 points is computed in
// lm order (few divergent harmonic branches per wave) into LDS, then written
// out as contiguous runs of the tile's functions.  Panel kinds:
//   PK_F64:   phi, d/dx, d/dy, d/dz in FP64 (4 planes of Pp np doubles)
//   PK_HS:    phi and psi = u phi / 2 in FP64 (2 planes)
//   PK_F32:   phi in FP64 (1 plane), then sqrt|w v| times d/dx, d/dy, d/dz
//             (formed in FP64) as FP32 planes (Pp np floats each) after it
//   PK_SPLIT: phi in FP64, then d/dx, d/dy, d/dz as FP32 hi planes fl32(x)
//             and the three lo planes fl32(x - hi)
//   PK_BF16:  phi in FP64 (1 plane), then the BF16 region: for component q
//             and split part t of sqrt|w v| times the gradient (formed in
//             FP64), plane 3 q + t of (Pp / 8) point octets x np functions x
//             8 points (16 bytes per function and octet)
// The FP64 and FP32 planes use the 4-point interleave of panel_index (FP32
// planes counted in floats).
enum { PK_F64 = 0, PK_HS = 1, PK_F32 = 2, PK_SPLIT = 3, PK_BF16 = 4 };

// BF16 (8 significant bits) three-way split of two values a, b at once:
// each is rounded to FP32, and each part is the BF16 nearest (ties to even)
// to what the previous parts leave; the remainders are exact in FP32, so
// |x - x1 - x2 - x3| <= (2^-24 + 2^-24) |x|.  Part k of both values comes
// as one word wk (a in the low half, b in the high half), from one packed
// conversion per part.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}
__device__ __forceinline__ void split3_bf16x2(double a, double b, uint32_t &w1, uint32_t &w2, uint32_t &w3) {
  const float fa = (float)a, fb = (float)b;
  w1 = pack_bf16(fa, fb);
  const float ra = fa - __uint_as_float(w1 << 16), rb = fb - __uint_as_float(w1 & 0xffff0000u);
  w2 = pack_bf16(ra, rb);
  w3 = pack_bf16(ra - __uint_as_float(w2 << 16), rb - __uint_as_float(w2 & 0xffff0000u));
}
constexpr int PLD = T + 1;  // padded LDS row of the panel stage

template <int KIND>
__global__ __launch_bounds__(256) void k_panel(DevPlan d, const WorkItem *tiles, int64_t t0, int64_t nt,
                                               double *panel, const double *om) {
  constexpr bool HS = KIND == PK_HS;
  constexpr int NQ = HS ? 2 : 4;  // components: phi, psi (H/S) or phi and its gradient
  constexpr int CP = 8;           // points per chunk: a small stage keeps 7 workgroups on a CU
  __shared__ TileMeta M;
  __shared__ double st[NQ * CP * PLD];
  __shared__ double s_sw[CP];  // PK_BF16: sqrt|w v| at the chunk's points
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
  float *pf = reinterpret_cast<float *>(pb + (int64_t)Pp * np);  // FP32 planes (PK_F32, PK_SPLIT)
  const int64_t fplane = (int64_t)Pp * np;
  for (int g8 = 0; g8 < Pp; g8 += CP) {
    if ((KIND == PK_BF16 || KIND == PK_F32) && threadIdx.x < CP)  // visible after the stage's barrier
      s_sw[threadIdx.x] = g8 + (int)threadIdx.x < P ? sqrt(fabs(om[g0 + g8 + threadIdx.x])) : 0.0;
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
    // (q, point quad) runs: rows r0 .. r0 + nrow - 1, 4 points each, contiguous
    constexpr int NQW = KIND == PK_BF16 ? 1 : NQ;  // PK_BF16: phi here, the gradient below
#pragma unroll
    for (int q = 0; q < NQW; ++q)
#pragma unroll
      for (int p4 = 0; p4 < CP / 4; ++p4) {
        const int e = threadIdx.x;  // 256 = 64 rows x 4 points
        const int il = e >> 2, pp = e & 3;
        if (il < nrow) {
          const double x = st[(q * CP + 4 * p4 + pp) * PLD + il];
          if (KIND == PK_F64 || KIND == PK_HS || q == 0) {
            pb[((int64_t)(q * (Pp >> 2) + (g8 >> 2) + p4) * np + r0 + il) * 4 + pp] = x;
          } else {
            const int64_t o = ((int64_t)((q - 1) * (Pp >> 2) + (g8 >> 2) + p4) * np + r0 + il) * 4 + pp;
            const float hi = KIND == PK_F32 ? (float)(s_sw[4 * p4 + pp] * x) : (float)x;
            pf[o] = hi;
            if (KIND == PK_SPLIT) pf[3 * fplane + o] = (float)(x - (double)hi);
          }
        }
      }
    if (KIND == PK_BF16) {
      // one task per (component, function): the 8 points of this octet,
      // sqrt|w v| times the gradient split into three BF16 parts, 16 bytes
      // per part
      u32x4 *pbf = reinterpret_cast<u32x4 *>(pb + fplane);
      const int64_t noct = Pp >> 3;
      for (int t = threadIdx.x; t < 3 * T; t += 256) {
        const int il = t % T, q = t / T;
        if (il >= nrow) continue;
        u32x4 w[3];
#pragma unroll
        for (int e = 0; e < CP; e += 2) {
          const double xa = s_sw[e] * st[((q + 1) * CP + e) * PLD + il];
          const double xb = s_sw[e + 1] * st[((q + 1) * CP + e + 1) * PLD + il];
          uint32_t w1, w2, w3;
          split3_bf16x2(xa, xb, w1, w2, w3);
          w[0][e >> 1] = w1;
          w[1][e >> 1] = w2;
          w[2][e >> 1] = w3;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) pbf[((int64_t)(3 * q + k) * noct + (g8 >> 3)) * np + r0 + il] = w[k];
      }
    }
    __syncthreads();  // st consumed
  }
}

// Modes of the FP64 contraction: all five parts, or V alone (phi only: the
// V part of the split precisions, and V-only calls).  V alone does one MFMA
// per row and column value, too little work per chunk to hide the next
// chunk's loads at two workgroups per CU: its 16-point chunks (33 KB of LDS)
// and 110 VGPRs let four share a CU.
enum { MODE_F64 = 0, MODE_V = 1 };

// Work item positions 0..nw-1 of a pass map to work items w0 + order[w0 + pos]
// (order != NULL: cost-sorted) or w0 + pos.  tickets == NULL: one workgroup
// per position; otherwise a persistent loop (next_item).
template <int MODE, bool PERSIST>
__global__ __launch_bounds__(NT, MODE == MODE_V ? 4 : 2) void k_contract(
    DevPlan d, const WorkItem *work, const int32_t *order, int64_t w0, int64_t nw, const double *om,
    const double *panel, double *staging, unsigned *tickets) {
  constexpr bool VONLY = MODE == MODE_V;
  constexpr int NQ = VONLY ? 1 : 4;        // panel components multiplied
  constexpr int NP = VONLY ? 1 : 5;        // parts accumulated
  // Chunks of CH points in two LDS buffers, the next chunk's DMA in flight
  // while this one is multiplied (one barrier per chunk)
  constexpr int CH = VONLY ? 16 : 8;
  constexpr int RPQ = CH / 2;              // LDS rows per component
  constexpr int BUFD = NQ * RPQ * DROW;    // doubles per chunk image
  __shared__ double sa[2 * BUFD], sb[2 * BUFD];
  __shared__ int64_t s_pos;
  // slot data of the tile's 64 rows and 64 columns for the epilogue, loaded
  // when the work item starts (slot -1: beyond n)
  __shared__ int s_fslot[2 * T], s_ffn[2 * T], s_fnf[2 * T];
  __shared__ int64_t s_frow[2 * T];
  int64_t pos = PERSIST ? next_item(tickets, nw, order != nullptr, &s_pos)
                        : (order ? (int64_t)blockIdx.x : xcd_map(blockIdx.x, nw));
  while (!PERSIST || pos < nw) {
  const int64_t wi = w0 + (order ? order[w0 + pos] : pos);
  const WorkItem it = work[wi];
  const int b = it.batch;
  const int g0 = d.batch_pt_off[b], P = d.batch_pt_off[b + 1] - g0;
  const int f0 = d.batch_fn_off[b], n = d.batch_fn_off[b + 1] - f0;
  const int r0 = it.ti * T, c0 = it.tj * T;
  const int Pp = (int)pad16(P), np = (int)pad16(n);
  const double *pb = panel + d.panel_off[b];
  const int64_t plane = (int64_t)Pp * np;
  const int tid = threadIdx.x;
  // wave index as a scalar: conditions derived from it stay uniform
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li16 = lane & 15, lk = lane >> 4;
  int brow[4], bcol[4];
  bool act[4];
  wave_blocks(r0, c0, n, wave, brow, bcol, act);

  dbl4 acc[4][NP];
#pragma unroll
  for (int sl = 0; sl < 4; ++sl)
#pragma unroll
    for (int q = 0; q < NP; ++q) acc[sl][q] = dbl4{0.0, 0.0, 0.0, 0.0};

  const double cp = d.cprime;
  // K steps go in pairs over 8 points: K index lk of the first step of the
  // pair is point 2 lk of the 8, of the second point 2 lk + 1 (one 16-byte
  // LDS read per operand gives a lane both).  w v at the points this lane's
  // K index visits in the next chunk, loaded a chunk ahead with the next
  // image's DMA, so that nothing consumed between the barrier and the last
  // MFMA of a chunk waits on loads in flight
  double omn[CH / 4];
  auto load_om = [&](int k) {
#pragma unroll
    for (int ks = 0; ks < CH / 4; ++ks) {
      const int pt = k + 8 * (ks >> 1) + 2 * lk + (ks & 1);
      omn[ks] = pt < P ? om[g0 + pt] : 0.0;
    }
  };
  load_om(0);
  dma_chunk<NT, CH, T, DROW, NQ>(pb, plane, np, r0, 0, sa);
  dma_chunk<NT, CH, T, DROW, NQ>(pb, plane, np, c0, 0, sb);
  if (!VONLY && tid < 2 * T) {  // visible from the first chunk's barrier on
    const int lf = tid < T ? r0 + tid : c0 + tid - T;
    int64_t v = 0, ro = 0;
    if (lf < n) {
      v = d.loc_info[f0 + lf];
      ro = d.loc_rowoff[f0 + lf];
    }
    s_fslot[tid] = lf < n ? (int)(v & 0xFFFFF) : -1;
    s_ffn[tid] = (int)((v >> 20) & 0xFFFFF);
    s_fnf[tid] = (int)(v >> 40);
    s_frow[tid] = ro;
  }
  for (int k0 = 0; k0 < Pp; k0 += CH) {
    const int bo = ((k0 / CH) & 1) * BUFD;  // this chunk's buffer
    __builtin_amdgcn_s_waitcnt(0);  // this thread's loads of this chunk have landed
    __syncthreads();                // ... everyone's; the previous chunk is consumed
    double omv[CH / 4];
#pragma unroll
    for (int ks = 0; ks < CH / 4; ++ks) omv[ks] = omn[ks];
    if (k0 + CH < Pp) {
      const int nbo = BUFD - bo;
      load_om(k0 + CH);
      dma_chunk<NT, CH, T, DROW, NQ>(pb, plane, np, r0, (k0 + CH) >> 2, sa + nbo);
      dma_chunk<NT, CH, T, DROW, NQ>(pb, plane, np, c0, (k0 + CH) >> 2, sb + nbo);
    }
    const double *ca = sa + bo, *cb = sb + bo;
#pragma unroll
    for (int kp = 0; kp < CH / 8; ++kp) {
      // image row 4 kp + lk holds points 8 kp + 2 lk and 8 kp + 2 lk + 1 of
      // the chunk; the column operand takes its weight w v there (the
      // weighting of Eq. 29)
      const int row = 4 * kp + lk;
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) {
        if (!act[sl]) continue;  // wave-uniform
        dbl2 ap[NQ], bp[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          ap[q] = *reinterpret_cast<const dbl2 *>(&ca[(q * RPQ + row) * DROW + 2 * (brow[sl] + li16)]);
          bp[q] = *reinterpret_cast<const dbl2 *>(&cb[(q * RPQ + row) * DROW + 2 * (bcol[sl] + li16)]);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
        const double omk = omv[2 * kp + h];
        double av[NQ], bv[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          av[q] = ap[q][h];
          bv[q] = bp[q][h] * omk;
        }
        acc[sl][0] = mfma64(av[0], bv[0], acc[sl][0]);
        if (!VONLY) {
          acc[sl][1] = mfma64(av[1], bv[1], acc[sl][1]);
          acc[sl][2] = mfma64(av[2], bv[3], acc[sl][2]);
          acc[sl][3] = mfma64(av[3], bv[1], acc[sl][3]);
          acc[sl][4] = mfma64(av[1], bv[2], acc[sl][4]);
          acc[sl][1] = mfma64(av[2], bv[2], acc[sl][1]);
          acc[sl][2] = mfma64(-av[3], bv[2], acc[sl][2]);
          acc[sl][3] = mfma64(-av[1], bv[3], acc[sl][3]);
          acc[sl][4] = mfma64(-av[2], bv[1], acc[sl][4]);
          acc[sl][1] = mfma64(av[3], bv[3], acc[sl][1]);
        }
        }
      }
    }
  }
  // write the computed blocks to the staged atom-pair blocks
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    if (!act[sl]) continue;
    const int cbk = c0 + bcol[sl];
    const int lj = cbk + li16;
    if (lj >= n) continue;
    const int cj = T + bcol[sl] + li16;
    // V alone keeps the two dependent lookups here: with the tables it
    // compiled to 256 VGPRs instead of 148 and ran 45% slower
    const SlotInfo sj = VONLY ? slot_of(d, f0, d.batch_slot_off[b], lj)
                              : SlotInfo{s_fslot[cj], s_ffn[cj], s_fnf[cj], s_frow[cj]};
    const int rb = r0 + brow[sl];
    const bool upper = rb < cbk;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // FP64 MFMA rows lk + 4 r
      const int li = rb + d_row_f64(lk, r);
      if (li < n) {
        const int ri = li - r0;
        const SlotInfo si = VONLY ? slot_of(d, f0, d.batch_slot_off[b], li)
                                  : SlotInfo{s_fslot[ri], s_ffn[ri], s_fnf[ri], s_frow[ri]};
        double vals[5];
        vals[0] = acc[sl][0][r];
#pragma unroll
        for (int q = 1; q < NP; ++q) vals[q] = cp * acc[sl][q][r];
        stage_store<0, NP>(staging, si, sj, li, lj, upper, vals);
      }
    }
  }
  if (!PERSIST) break;
  pos = next_item(tickets, nw, order != nullptr, &s_pos);
  }
}

// The plain FP64 baseline (precision F64_VALU): the five parts of a work
// item on the vector ALU, no matrix cores.  Same work items, FP64 panels,
// chunk DMA and staging as k_contract<MODE_F64>; each thread owns a 4 x 4
// patch of the 64 x 64 tile (rows 4 (t / 16), columns 4 (t % 16)) and adds
// every point's ten products to its 80 FP64 sums with fused multiply-adds,
// point after point.  Patches in blocks no work item computes (below the
// diagonal, beyond n) skip the arithmetic.
__global__ __launch_bounds__(NT, 1) void k_contract_valu(DevPlan d, const WorkItem *work, const int32_t *order,
                                                         int64_t w0, int64_t nw, const double *om,
                                                         const double *panel, double *staging, unsigned *tickets) {
  (void)tickets;
  constexpr int NQ = 4, CH = 8, RPQ = CH / 2;
  constexpr int BUFD = NQ * RPQ * DROW;  // doubles per chunk image
  __shared__ double sa[2 * BUFD], sb[2 * BUFD];
  __shared__ double s_om[2][CH];
  // slot data of the tile's 64 rows and 64 columns for the epilogue, loaded
  // when the work item starts (slot -1: beyond n)
  __shared__ int s_fslot[2 * T], s_ffn[2 * T], s_fnf[2 * T];
  __shared__ int64_t s_frow[2 * T];
  const int64_t pos = order ? (int64_t)blockIdx.x : xcd_map(blockIdx.x, nw);
  const int64_t wi = w0 + (order ? order[w0 + pos] : pos);
  const WorkItem it = work[wi];
  const int b = it.batch;
  const int g0 = d.batch_pt_off[b], P = d.batch_pt_off[b + 1] - g0;
  const int f0 = d.batch_fn_off[b], n = d.batch_fn_off[b + 1] - f0;
  const int r0 = it.ti * T, c0 = it.tj * T;
  const int Pp = (int)pad16(P), np = (int)pad16(n);
  const double *pb = panel + d.panel_off[b];
  const int64_t plane = (int64_t)Pp * np;
  const int tid = threadIdx.x;
  const int pr = 4 * (tid >> 4), pc = 4 * (tid & 15);  // the thread's patch (tile-local)
  const int rb = pr & ~15, cb = pc & ~15;
  const bool live = block_active(r0 + rb, c0 + cb, n);
  double acc[5][4][4];
#pragma unroll
  for (int q = 0; q < 5; ++q)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[q][a][c] = 0.0;
  double omr = tid < CH ? om[g0 + tid] : 0.0;  // om holds 16 zeros past its end
  dma_chunk<NT, CH, T, DROW, NQ>(pb, plane, np, r0, 0, sa);
  dma_chunk<NT, CH, T, DROW, NQ>(pb, plane, np, c0, 0, sb);
  if (tid < 2 * T) {  // visible from the first chunk's barrier on
    const int lf = tid < T ? r0 + tid : c0 + tid - T;
    int64_t v = 0, ro = 0;
    if (lf < n) {
      v = d.loc_info[f0 + lf];
      ro = d.loc_rowoff[f0 + lf];
    }
    s_fslot[tid] = lf < n ? (int)(v & 0xFFFFF) : -1;
    s_ffn[tid] = (int)((v >> 20) & 0xFFFFF);
    s_fnf[tid] = (int)(v >> 40);
    s_frow[tid] = ro;
  }
  __builtin_amdgcn_s_waitcnt(0);
  if (tid < CH) s_om[0][tid] = omr;
  for (int k0 = 0; k0 < Pp; k0 += CH) {
    const int bi = (k0 / CH) & 1;
    __syncthreads();  // this chunk visible; the previous one consumed
    if (k0 + CH < Pp) {
      omr = tid < CH ? om[g0 + k0 + CH + tid] : 0.0;
      dma_chunk<NT, CH, T, DROW, NQ>(pb, plane, np, r0, (k0 + CH) >> 2, sa + (bi ^ 1) * BUFD);
      dma_chunk<NT, CH, T, DROW, NQ>(pb, plane, np, c0, (k0 + CH) >> 2, sb + (bi ^ 1) * BUFD);
    }
    if (live) {
      const double *ca = sa + bi * BUFD, *cbp = sb + bi * BUFD;
      for (int u = 0; u < RPQ; ++u) {  // point pairs of the chunk
        // component q of functions pr + a (rows) and pc + c (columns) at
        // points 2u, 2u + 1 (16 bytes each)
        dbl2 av[NQ][4], bv[NQ][4];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            av[q][a] = *reinterpret_cast<const dbl2 *>(&ca[(q * RPQ + u) * DROW + 2 * (pr + a)]);
            bv[q][a] = *reinterpret_cast<const dbl2 *>(&cbp[(q * RPQ + u) * DROW + 2 * (pc + a)]);
          }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const double w = s_om[bi][2 * u + h];
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const double x0 = av[0][a][h], x1 = av[1][a][h], x2 = av[2][a][h], x3 = av[3][a][h];
              const double y0 = w * bv[0][c][h], y1 = w * bv[1][c][h], y2 = w * bv[2][c][h], y3 = w * bv[3][c][h];
              acc[0][a][c] = fma(x0, y0, acc[0][a][c]);
              acc[1][a][c] = fma(x1, y1, fma(x2, y2, fma(x3, y3, acc[1][a][c])));
              acc[2][a][c] = fma(x2, y3, fma(-x3, y2, acc[2][a][c]));
              acc[3][a][c] = fma(x3, y1, fma(-x1, y3, acc[3][a][c]));
              acc[4][a][c] = fma(x1, y2, fma(-x2, y1, acc[4][a][c]));
            }
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);  // the next chunk's images and w v have landed
    if (k0 + CH < Pp && tid < CH) s_om[bi ^ 1][tid] = omr;
  }
  if (!live) return;
  const double cp = d.cprime;
  const bool upper = r0 + rb < c0 + cb;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int lj = c0 + pc + c;
    if (lj >= n) continue;
    const int cj = lj - c0 + T;
    const SlotInfo sj{s_fslot[cj], s_ffn[cj], s_fnf[cj], s_frow[cj]};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int li = r0 + pr + a;
      if (li >= n) continue;
      const int ri = li - r0;
      const SlotInfo si{s_fslot[ri], s_ffn[ri], s_fnf[ri], s_frow[ri]};
      double vals[5];
      vals[0] = acc[0][a][c];
#pragma unroll
      for (int q = 1; q < 5; ++q) vals[q] = cp * acc[q][a][c];
      stage_store<0, 5>(staging, si, sj, li, lj, upper, vals);
    }
  }
}

// The four W parts on FP32 MFMA (precisions F32 and SPLIT_F32), from the FP32
// gradient planes of a PK_F32 / PK_SPLIT panel; V runs beside it on FP64
// (k_contract<MODE_V>).  Same work items, wave blocks and staging as
// k_contract.  F32: both operands are sqrt|w v| times the gradient (formed in
// FP64, rounded to FP32 once in the panel), the row operand with the sign of
// w v.  Per 16 points, every element's FP32 partial sum (of at most 48
// products: 16 points x 3) is converted to FP64 and added to an FP64 running
// sum, then restarted from zero, so FP32 rounding never accumulates beyond
// one 16-point chunk: with unit roundoff u = 2^-24 each element's error is at
// most gamma_52 = 52 u / (1 - 52 u) times the sum over all points of the
// magnitudes of its terms (two operands rounded to FP32, 48 products and
// additions), plus FP64 rounding and the loss of relative precision of values
// below FP32's normal range (the far tails of tight functions).  SPLIT: each
// operand x enters as hi = fl32(x) and lo = fl32(x - hi) (the column operand
// w v x formed in FP64 and split again), and every product as
// hi hi + hi lo + lo hi (three FP32 MFMAs): the operands' rounding drops to
// about 2^-48, and a 16-point partial sum holds up to 144 products
// (gamma_150).
template <bool SPLIT, bool PERSIST>
__global__ __launch_bounds__(NT, 2) void k_contract_w(DevPlan d, const WorkItem *work, const int32_t *order,
                                                      int64_t w0, int64_t nw, const double *om,
                                                      const double *panel, double *staging, unsigned *tickets) {
  // Chunks of CH points; an image row is one point quad of 64 functions
  // (1 KB of floats, in the panel's own order: element (pt, f) of the quad at
  // 4 f + pt % 4), rows (component q, quad) for q = 0..2 (d/dx, d/dy, d/dz),
  // then, for SPLIT, the same rows of the lo planes.
  constexpr int CH = SPLIT ? 8 : 16;
  constexpr int NQR = CH / 4;                  // quads per chunk
  constexpr int NPL = SPLIT ? 6 : 3;           // FP32 planes read
  constexpr int ROWF = 4 * T;                  // floats per image row
  constexpr int BUFF = NPL * NQR * ROWF;       // floats per chunk image
  constexpr int FLUSH = 16;                    // points per FP32 partial sum
  __shared__ __attribute__((aligned(16))) float fa[2 * BUFF], fb[2 * BUFF];
  __shared__ int64_t s_pos;
  // slot data of the tile's 64 rows and 64 columns for the epilogue, loaded
  // when the work item starts (slot -1: beyond n)
  __shared__ int s_fslot[2 * T], s_ffn[2 * T], s_fnf[2 * T];
  __shared__ int64_t s_frow[2 * T];
  int64_t pos = PERSIST ? next_item(tickets, nw, order != nullptr, &s_pos)
                        : (order ? (int64_t)blockIdx.x : xcd_map(blockIdx.x, nw));
  while (!PERSIST || pos < nw) {
  const int64_t wi = w0 + (order ? order[w0 + pos] : pos);
  const WorkItem it = work[wi];
  const int b = it.batch;
  const int g0 = d.batch_pt_off[b], P = d.batch_pt_off[b + 1] - g0;
  const int f0 = d.batch_fn_off[b], n = d.batch_fn_off[b + 1] - f0;
  const int r0 = it.ti * T, c0 = it.tj * T;
  const int Pp = (int)pad16(P), np = (int)pad16(n);
  const int64_t fplane = (int64_t)Pp * np;
  const float *pf = reinterpret_cast<const float *>(panel + d.panel_off[b] + fplane);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li16 = lane & 15, lk = lane >> 4;
  int brow[4], bcol[4];
  bool act[4];
  wave_blocks(r0, c0, n, wave, brow, bcol, act);

  flt4 accf[4][4];   // FP32 partial sums of the current 16 points
  dbl4 accw[4][4];   // FP64 running sums
#pragma unroll
  for (int sl = 0; sl < 4; ++sl)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      accf[sl][q] = flt4{0.f, 0.f, 0.f, 0.f};
      accw[sl][q] = dbl4{0.0, 0.0, 0.0, 0.0};
    }
  // LDS DMA of one chunk of 64 functions from row0 (a tile): image row r =
  // (plane pl, quad qd) is the 1 KB run of plane pl (hi d/dx, d/dy, d/dz,
  // then the lo planes) at point quad quad0 + qd, 16 bytes (4 points of one
  // function) per lane.  Functions at or beyond np are not loaded (their
  // blocks are never multiplied).
  auto dma = [&](int row0, int quad0, float *dst) {
    const bool ok = row0 + lane < np;
#pragma unroll
    for (int k = 0; k < NPL * NQR / 4; ++k) {
      const int r = wave + 4 * k;
      const int pl = r / NQR, qd = r % NQR;
      if (ok)
        __builtin_amdgcn_global_load_lds(
            (const void *)(pf + (int64_t)pl * fplane + ((int64_t)(quad0 + qd) * np + row0 + lane) * 4),
            (lds_void *)(dst + r * ROWF), 16, 0, 0);
    }
  };
  // w v at the points this lane's K index visits in the next chunk: points
  // 4 ks + lk (SPLIT), or the four points of quad lk (otherwise)
  double omn[CH / 4];
  auto load_om = [&](int k) {
#pragma unroll
    for (int ks = 0; ks < CH / 4; ++ks) {
      const int pt = SPLIT ? k + 4 * ks + lk : k + 4 * lk + ks;
      omn[ks] = pt < P ? om[g0 + pt] : 0.0;
    }
  };
  load_om(0);
  dma(r0, 0, fa);
  dma(c0, 0, fb);
  if (tid < 2 * T) {  // visible from the first chunk's barrier on
    const int lf = tid < T ? r0 + tid : c0 + tid - T;
    int64_t v = 0, ro = 0;
    if (lf < n) {
      v = d.loc_info[f0 + lf];
      ro = d.loc_rowoff[f0 + lf];
    }
    s_fslot[tid] = lf < n ? (int)(v & 0xFFFFF) : -1;
    s_ffn[tid] = (int)((v >> 20) & 0xFFFFF);
    s_fnf[tid] = (int)(v >> 40);
    s_frow[tid] = ro;
  }
  for (int k0 = 0; k0 < Pp; k0 += CH) {
    const int bo = ((k0 / CH) & 1) * BUFF;
    __builtin_amdgcn_s_waitcnt(0);  // this thread's loads of this chunk have landed
    __syncthreads();                // ... everyone's; the previous chunk is consumed
    double omv[CH / 4];
#pragma unroll
    for (int ks = 0; ks < CH / 4; ++ks) omv[ks] = omn[ks];
    if (k0 + CH < Pp) {
      load_om(k0 + CH);
      dma(r0, (k0 + CH) >> 2, fa + BUFF - bo);
      dma(c0, (k0 + CH) >> 2, fb + BUFF - bo);
    }
    const float *ca = fa + bo, *cb = fb + bo;
    if constexpr (!SPLIT) {
      // The panel holds sqrt|w v| times the gradient, so each product is
      // w v times two gradient components once the row operand takes the
      // sign of w v.  MFMA m of the chunk sums over points 4 lk + m (K index
      // lk): one 16-byte LDS read per operand gives a lane all four.
      uint32_t sgn[4];
#pragma unroll
      for (int m = 0; m < 4; ++m)
        sgn[m] = (uint32_t)((uint64_t)__double_as_longlong(omv[m]) >> 32) & 0x80000000u;
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) {
        if (!act[sl]) continue;  // wave-uniform
        flt4 a4[3], b4[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          a4[q] = *reinterpret_cast<const flt4 *>(&ca[(q * NQR + lk) * ROWF + 4 * (brow[sl] + li16)]);
          b4[q] = *reinterpret_cast<const flt4 *>(&cb[(q * NQR + lk) * ROWF + 4 * (bcol[sl] + li16)]);
#pragma unroll
          for (int m = 0; m < 4; ++m) a4[q][m] = __uint_as_float(__float_as_uint(a4[q][m]) ^ sgn[m]);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          // parts: Ws = dx dx + dy dy + dz dz; Wso_x = dy dz - dz dy;
          // Wso_y = dz dx - dx dz; Wso_z = dx dy - dy dx (row x column)
          accf[sl][0] = mfma32(a4[0][m], b4[0][m], accf[sl][0]);
          accf[sl][1] = mfma32(a4[1][m], b4[2][m], accf[sl][1]);
          accf[sl][2] = mfma32(a4[2][m], b4[0][m], accf[sl][2]);
          accf[sl][3] = mfma32(a4[0][m], b4[1][m], accf[sl][3]);
          accf[sl][0] = mfma32(a4[1][m], b4[1][m], accf[sl][0]);
          accf[sl][1] = mfma32(-a4[2][m], b4[1][m], accf[sl][1]);
          accf[sl][2] = mfma32(-a4[0][m], b4[2][m], accf[sl][2]);
          accf[sl][3] = mfma32(-a4[1][m], b4[0][m], accf[sl][3]);
          accf[sl][0] = mfma32(a4[2][m], b4[2][m], accf[sl][0]);
        }
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < CH / 4; ++ks) {
        const double omk = omv[ks];
#pragma unroll
        for (int sl = 0; sl < 4; ++sl) {
          if (!act[sl]) continue;  // wave-uniform
          // A[i][k] = component q of row function brow + i at point 4 ks + k
          // (hi and lo); B[k][j] = w v times component q of column function
          // bcol + j there, formed in FP64 from hi + lo and split again
          float ah[3], bh[3], al[3], bl[3];
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            ah[q] = ca[(q * NQR + ks) * ROWF + 4 * (brow[sl] + li16) + lk];
            const float bx = cb[(q * NQR + ks) * ROWF + 4 * (bcol[sl] + li16) + lk];
            al[q] = ca[((3 + q) * NQR + ks) * ROWF + 4 * (brow[sl] + li16) + lk];
            const float bxl = cb[((3 + q) * NQR + ks) * ROWF + 4 * (bcol[sl] + li16) + lk];
            const double x = omk * ((double)bx + (double)bxl);
            bh[q] = (float)x;
            bl[q] = (float)(x - (double)bh[q]);
          }
          // the same products, each as hi hi + hi lo + lo hi
#define W32(ACC, AI, BI, SG)              \
  ACC = mfma32(SG ah[AI], bh[BI], ACC);   \
  ACC = mfma32(SG ah[AI], bl[BI], ACC);   \
  ACC = mfma32(SG al[AI], bh[BI], ACC);
          W32(accf[sl][0], 0, 0, +)
          W32(accf[sl][1], 1, 2, +)
          W32(accf[sl][2], 2, 0, +)
          W32(accf[sl][3], 0, 1, +)
          W32(accf[sl][0], 1, 1, +)
          W32(accf[sl][1], 2, 1, -)
          W32(accf[sl][2], 0, 2, -)
          W32(accf[sl][3], 1, 0, -)
          W32(accf[sl][0], 2, 2, +)
#undef W32
        }
      }
    }
    if (((k0 + CH) % FLUSH) == 0 || k0 + CH >= Pp) {
      // the 16-point FP32 partial sums join the FP64 running sums
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) {
        if (!act[sl]) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
          for (int r = 0; r < 4; ++r) accw[sl][q][r] += (double)accf[sl][q][r];
          accf[sl][q] = flt4{0.f, 0.f, 0.f, 0.f};
        }
      }
    }
  }
  const double cp = d.cprime;
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    if (!act[sl]) continue;
    const int cbk = c0 + bcol[sl];
    const int lj = cbk + li16;
    if (lj >= n) continue;
    const int cj = T + bcol[sl] + li16;
    const SlotInfo sj{s_fslot[cj], s_ffn[cj], s_fnf[cj], s_frow[cj]};
    const int rb = r0 + brow[sl];
    const bool upper = rb < cbk;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // FP32 MFMA rows 4 lk + r
      const int lf = rb + d_row_f32(lk, r);
      if (lf < n) {
        const int ri = lf - r0;
        const SlotInfo sf{s_fslot[ri], s_ffn[ri], s_fnf[ri], s_frow[ri]};
        double w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = cp * accw[sl][q][r];
        stage_store<1, 5>(staging, sf, sj, lf, lj, upper, w);
      }
    }
  }
  if (!PERSIST) break;
  pos = next_item(tickets, nw, order != nullptr, &s_pos);
  }
}

// BF16X3 precision: V on FP64 MFMA and the four W parts on BF16 MFMA with
// three-way split operands (PK_BF16 panels), in one kernel.  One workgroup
// per column half (32 columns) of a work item's 64 x 64 tile; wave w takes
// the 16-row block w against the half's two 16-column blocks, so each A
// operand it reads serves both.  Per 16-point chunk the four images (FP64 phi
// and the BF16 parts of sqrt|w v| times the gradient, of rows and of
// columns) arrive by LDS DMA, double-buffered, with w v of the chunk's
// points.  The row operand takes the sign of w v (its BF16 sign bits
// flipped), so each product is w v times the two gradient components.
// W products: a b ~ a1 b1 + a2 b1 + a1 b2 + a1 b3 + a2 b2 + a3 b1 (the terms
// of order 2^-16 and above), three MFMAs of K = 32 per component pair: the
// K index runs over two slots of the chunk's 16 points, slot 0 (lanes with
// lk < 2) holding one part and slot 1 another ([a1|a2] x [b1|b1],
// [a1|a1] x [b2|b3], [a2|a3] x [b2|b1]).  Dropped terms and split remainders
// are below 3 2^-23 |a b|.  The spin-orbit parts keep their positive and
// negative products in separate FP32 sums (no operand is negated).  Each
// chunk's FP32 sums start from zero and are added into FP64 running sums
// (the spin-orbit pair as their FP32 difference).
template <bool PERSIST>
__global__ __launch_bounds__(NT, 2) void k_contract_b3(DevPlan d, const WorkItem *work, const int32_t *order,
                                                       int64_t w0, int64_t nw, const double *om,
                                                       const double *panel, double *staging, unsigned *tickets) {
  constexpr int CH = 16;            // points per chunk
  constexpr int RBF = 18 * 64;      // 16-byte items of the row BF16 image: 18 rows (plane, octet) x 64 functions
  constexpr int CBF = 18 * 32;      // ... of the column image (32 functions)
  constexpr int RD = 8 * DROW;      // doubles of the row phi image: 8 point pairs x 64 functions x 2
  constexpr int CDW = 2 * 32;       // doubles per row of the column phi image
  constexpr int CD = 8 * CDW;
  // chunk images (double-buffered), reused after the last chunk to stage the
  // half tile's results for coalesced writes
  constexpr int IMG_BYTES = 2 * 16 * (RBF + CBF) + 2 * 8 * (RD + CD);
  __shared__ __attribute__((aligned(16))) unsigned char smem[IMG_BYTES];
  u32x4(*sr)[RBF] = reinterpret_cast<u32x4(*)[RBF]>(smem);
  u32x4(*sc)[CBF] = reinterpret_cast<u32x4(*)[CBF]>(smem + 2 * 16 * RBF);
  double(*dr)[RD] = reinterpret_cast<double(*)[RD]>(smem + 2 * 16 * (RBF + CBF));
  double(*dc)[CD] = reinterpret_cast<double(*)[CD]>(smem + 2 * 16 * (RBF + CBF) + 2 * 8 * RD);
  __shared__ double som[2][CH];
  __shared__ int64_t s_pos;
  // slot data of the tile's 64 rows and the half's 32 columns (slot -1: beyond n)
  __shared__ int s_rslot[T], s_rfn[T], s_rnf[T], s_cslot[T / 2], s_cfn[T / 2], s_cnf[T / 2];
  __shared__ int64_t s_rrow[T];
  const int64_t npos = 2 * nw;
  int64_t pos = PERSIST ? next_item(tickets, npos, order != nullptr, &s_pos)
                        : (order ? (int64_t)blockIdx.x : xcd_map(blockIdx.x, npos));
  while (!PERSIST || pos < npos) {
  const int half = (int)(pos & 1);
  const int64_t wi = w0 + (order ? order[w0 + (pos >> 1)] : (pos >> 1));
  const WorkItem it = work[wi];
  const int b = it.batch;
  const int f0 = d.batch_fn_off[b], n = d.batch_fn_off[b + 1] - f0;
  if (it.tj * T + 32 * half < n) {  // workgroup-uniform: the half has columns
  const int g0 = d.batch_pt_off[b], P = d.batch_pt_off[b + 1] - g0;
  const int r0 = it.ti * T, c0 = it.tj * T + 32 * half;
  const int Pp = (int)pad16(P), np = (int)pad16(n);
  const double *pb = panel + d.panel_off[b];
  const int64_t fplane = (int64_t)Pp * np, noct = Pp >> 3;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, lk = lane >> 4;
  const int rb = 16 * wave;  // this wave's row block (tile-local)
  bool act[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) act[c] = block_active(r0 + rb, c0 + 16 * c, n);

  // the chunk of 16 points from k0 into buffer bf, by buffer loads straight
  // into LDS: the batch's panel is one buffer, each lane's offset is fixed for
  // the work item and the chunk and image row go into the scalar offset.
  // Lanes whose function lies at or beyond np load nothing.
  const __amdgpu_buffer_rsrc_t prs =
      __builtin_amdgcn_make_buffer_rsrc((void *)pb, (short)0, (int)(26 * fplane), 0x00020000);
  // lanes whose function lies at or beyond np take an offset past the
  // buffer's range: the load is issued by every lane and reads nothing there
  const bool okr = r0 + lane < np, okc = c0 + (lane & 31) < np;
  constexpr uint32_t OOB = 0x80000000u;
  const uint32_t vrow = okr ? lane * 16u : OOB;
  const uint32_t vcol = okc ? (lane & 31) * 16u + (lane >> 5) * (uint32_t)np * 16u : OOB;
  const uint32_t vprow = okr ? lane * 32u : OOB, vpcol = okc ? (lane & 31) * 32u + (lane >> 5) * 16u : OOB;
  auto dma = [&](int k0, int bf) {
    const int og = k0 >> 3;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
      const int k = wave + 4 * i;  // wave-uniform
      if (k < 18) {  // row image row (plane k / 2, octet k % 2), 64 functions
        const uint32_t so = 8u * (uint32_t)fplane + (uint32_t)((((k >> 1) * noct + og + (k & 1)) * np + r0) * 16);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(prs, (lds_void *)(&sr[bf][k * 64]), 16, vrow, so, 0, 0);
      } else if (k < 27) {  // column image rows (plane, octet 0) and (plane, octet 1), 32 functions each
        const int pl = k - 18;
        const uint32_t so = 8u * (uint32_t)fplane + (uint32_t)(((pl * noct + og) * np + c0) * 16);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(prs, (lds_void *)(&sc[bf][pl * 64]), 16, vcol, so, 0, 0);
      }
    }
    // FP64 phi: image row u = point pair u of the chunk (16 bytes per function)
#pragma unroll
    for (int h = 0; h < 2; ++h) {  // rows: two point pairs per wave
      const int u = wave + 4 * h;
      const uint32_t so = (uint32_t)(((((k0 >> 2) + (u >> 1)) * np + r0) * 4 + 2 * (u & 1)) * 8);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(prs, (lds_void *)(&dr[bf][u * DROW]), 16, vprow, so, 0, 0);
    }
    {  // columns: point pairs 2 w and 2 w + 1 (one quad) per wave
      const uint32_t so = (uint32_t)(((((k0 >> 2) + wave) * np + c0) * 4) * 8);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(prs, (lds_void *)(&dc[bf][2 * wave * CDW]), 16, vpcol, so, 0, 0);
    }
  };

  dbl4 accw[2][4];   // FP64 running sums of Ws, Wso_x, Wso_y, Wso_z
  dbl4 accv[2];      // V
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int q = 0; q < 4; ++q) accw[c][q] = dbl4{0.0, 0.0, 0.0, 0.0};
    accv[c] = dbl4{0.0, 0.0, 0.0, 0.0};
  }
  double omr = tid < CH ? om[g0 + tid] : 0.0;  // om holds 16 zeros past its end
  dma(0, 0);
  if (tid < T + T / 2) {
    const bool row = tid < T;
    const int lf = row ? r0 + tid : c0 + tid - T;
    SlotInfo si{-1, 0, 0, 0};
    if (lf < n) {
      const int64_t v = d.loc_info[f0 + lf];
      si = SlotInfo{(int)(v & 0xFFFFF), (int)((v >> 20) & 0xFFFFF), (int)(v >> 40), row ? d.loc_rowoff[f0 + lf] : 0};
    }
    if (row) {
      s_rslot[tid] = si.slot;
      s_rfn[tid] = si.fnoff;
      s_rnf[tid] = si.nfn;
      s_rrow[tid] = si.row_off;
    } else {
      s_cslot[tid - T] = si.slot;
      s_cfn[tid - T] = si.fnoff;
      s_cnf[tid - T] = si.nfn;
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  if (tid < CH) som[0][tid] = omr;
  const int slot = lk >> 1, oc = lk & 1;
  // split parts of the A and B operands of MFMA s for this lane's slot
  const int ta0 = slot ? 1 : 0, ta2 = slot ? 2 : 1;  // A: s = 0 [1|2], s = 1 [1|1], s = 2 [2|3]
  const int tb1 = slot ? 2 : 1, tb2 = slot ? 0 : 1;  // B: s = 0 [1|1], s = 1 [2|3], s = 2 [2|1]
  for (int k0 = 0; k0 < Pp; k0 += CH) {
    const int bi = (k0 / CH) & 1;
    __syncthreads();  // this chunk's images and w v visible; the previous chunk is consumed
    if (k0 + CH < Pp) {
      omr = tid < CH ? om[g0 + k0 + CH + tid] : 0.0;
      dma(k0 + CH, bi ^ 1);
    }
    // the chunk's products for the active column blocks (a compile-time set:
    // both, or one on diagonal and edge tiles), as straight-line code
    auto chunk = [&](auto a0c, auto a1c) {
      constexpr bool ACT[2] = {decltype(a0c)::value, decltype(a1c)::value};
      // V: four K steps of 4 points on FP64 MFMA, in pairs over 8 points as
      // in the FP64 path (the same order)
#pragma unroll
      for (int kp = 0; kp < 2; ++kp) {
        const int row = 4 * kp + lk;
        const dbl2 ap = *reinterpret_cast<const dbl2 *>(&dr[bi][row * DROW + 2 * (rb + l16)]);
        dbl2 bp[2];
#pragma unroll
        for (int c = 0; c < 2; ++c)
          if (ACT[c]) bp[c] = *reinterpret_cast<const dbl2 *>(&dc[bi][row * CDW + 2 * (16 * c + l16)]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const double omk = som[bi][8 * kp + 2 * lk + h];
#pragma unroll
          for (int c = 0; c < 2; ++c)
            if (ACT[c]) accv[c] = mfma64(ap[h], bp[c][h] * omk, accv[c]);
        }
      }
      // W: this chunk's FP32 sums, Ws then (+, -) of Wso_x, Wso_y, Wso_z
      flt4 accf[2][7];
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int q = 0; q < 7; ++q) accf[c][q] = flt4{0.f, 0.f, 0.f, 0.f};
      // the sign of w v at this lane's 8 points (octet oc), on the BF16 sign
      // bits of the row operand
      u32x4 sgn;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const uint64_t ua = (uint64_t)__double_as_longlong(som[bi][8 * oc + 2 * m]);
        const uint64_t ub = (uint64_t)__double_as_longlong(som[bi][8 * oc + 2 * m + 1]);
        sgn[m] = ((uint32_t)(ua >> 48) & 0x8000u) | ((uint32_t)(ub >> 32) & 0x80000000u);
      }
      // A operands of the row block, all components and split pairs
      u32x4 fa[3][3];
#pragma unroll
      for (int qa = 0; qa < 3; ++qa) {
        const int base = rb + l16;
        fa[qa][0] = sr[bi][((3 * qa + ta0) * 2 + oc) * 64 + base] ^ sgn;
        fa[qa][1] = sr[bi][((3 * qa + 0) * 2 + oc) * 64 + base] ^ sgn;
        fa[qa][2] = sr[bi][((3 * qa + ta2) * 2 + oc) * 64 + base] ^ sgn;
      }
#pragma unroll
      for (int qb = 0; qb < 3; ++qb) {
        u32x4 gb[2][3];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          if (!ACT[c]) continue;
          const int base = 16 * c + l16;
          gb[c][0] = sc[bi][((3 * qb + 0) * 2 + oc) * 32 + base];
          gb[c][1] = sc[bi][((3 * qb + tb1) * 2 + oc) * 32 + base];
          gb[c][2] = sc[bi][((3 * qb + tb2) * 2 + oc) * 32 + base];
        }
        // FP32 sum of (row component qa, column component qb): Ws on the
        // diagonal; y z -> 1, z y -> 2, z x -> 3, x z -> 4, x y -> 5, y x -> 6
#pragma unroll
        for (int sp = 0; sp < 3; ++sp)
#pragma unroll
          for (int qa = 0; qa < 3; ++qa) {
            constexpr int MAP[3][3] = {{0, 5, 4}, {6, 0, 1}, {3, 2, 0}};
            const int t = MAP[qa][qb];
#pragma unroll
            for (int c = 0; c < 2; ++c)
              if (ACT[c]) accf[c][t] = mfma_bf16(fa[qa][sp], gb[c][sp], accf[c][t]);
          }
      }
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        if (!ACT[c]) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          accw[c][0][r] += (double)accf[c][0][r];
#pragma unroll
          for (int m = 0; m < 3; ++m) accw[c][1 + m][r] += (double)(accf[c][1 + 2 * m][r] - accf[c][2 + 2 * m][r]);
        }
      }
    };
    if (act[0] && act[1])
      chunk(std::true_type{}, std::true_type{});
    else if (act[0])
      chunk(std::true_type{}, std::false_type{});
    else if (act[1])
      chunk(std::false_type{}, std::true_type{});
    __builtin_amdgcn_s_waitcnt(0);  // the next chunk's images and w v have landed
    if (k0 + CH < Pp && tid < CH) som[bi ^ 1][tid] = omr;
  }
  // the half tile's results go through LDS (parts 0..2, then 3..4; rows of
  // 33 doubles), then every thread writes whole runs of staged rows: element
  // (i, j) of the half by thread (i 32 + j) mod 256, the mirrored element of a
  // strictly upper block of one atom as well
  const double cp = d.cprime;
  double *E = reinterpret_cast<double *>(smem);
  constexpr int ES = 33;
#pragma unroll
  for (int round = 0; round < 2; ++round) {
    const int q0 = round ? 3 : 0, nq = round ? 2 : 3;
    __syncthreads();  // the images (or the previous round) are consumed
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (!act[c]) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = 16 * c + l16;
        if (round == 0) E[(0 * T + rb + d_row_f64(lk, r)) * ES + j] = accv[c][r];
#pragma unroll
        for (int q = 1; q < 5; ++q)
          if (q >= q0 && q < q0 + nq) E[((q - q0) * T + rb + d_row_f32(lk, r)) * ES + j] = cp * accw[c][q - 1][r];
      }
    }
    __syncthreads();
    for (int e = tid; e < T * (T / 2); e += NT) {
      const int i = e >> 5, j = e & 31;
      const int li = r0 + i, lj = c0 + j;
      if (!block_active(r0 + (i & ~15), c0 + (j & ~15), n) || li >= n || lj >= n) continue;
      const int si = s_rslot[i], sj = s_cslot[j];
      if (si > sj) continue;  // lower atom-block triangle: not stored
      const int nfi = s_rnf[i], nfj = s_cnf[j], fi = s_rfn[i], fj = s_cfn[j];
      const int64_t blk = s_rrow[i] + 5 * (int64_t)nfi * (fj - fi);
      const int64_t pq = (int64_t)nfi * nfj;
      const int64_t el = (int64_t)(li - fi) * nfj + (lj - fj);
      const bool mirror = si == sj && r0 + (i & ~15) < c0 + (j & ~15);
      const int64_t em = (int64_t)(lj - fi) * nfj + (li - fj);
      for (int qq = 0; qq < nq; ++qq) {
        const double x = E[(qq * T + i) * ES + j];
        staging[blk + (q0 + qq) * pq + el] = x;
        if (mirror) staging[blk + (q0 + qq) * pq + em] = mirror_sign(q0 + qq) * x;
      }
    }
  }
  }  // the half has columns
  if (!PERSIST) break;
  pos = next_item(tickets, npos, order != nullptr, &s_pos);
  }
}

// Batch-to-global sum for one pass: reduction entry r adds the staged blocks
// of pair red_pair[r] in batch order, one after another onto the running
// value (zero, or the stored value when a previous pass or ACCUMULATE left
// one).  The sum is a single sequential chain in batch order, so results
// repeat bit for bit and do not depend on how batches are split into passes.
// Workgroup (x, y) takes elements y NTR .. y NTR + NTR - 1 of entry x, one per
// thread (gridDim.y covers the largest entry), so the heavy atom pairs are
// spread over many workgroups instead of setting the kernel's tail; the
// loads of eight incidences are issued together.
constexpr int NTR = 256;  // threads of a k_reduce workgroup
__global__ __launch_bounds__(NTR) void k_reduce(DevPlan d, int64_t r0, const int32_t *red_pair,
                                                const uint8_t *red_first, const int64_t *red_inc_off,
                                                const int64_t *inc_src, const double *staging, double *store,
                                                int accumulate, int nq, unsigned part_mask) {
  __shared__ int64_t s_src[NTR];
  const int64_t r = r0 + blockIdx.x;
  const int p = red_pair[r];
  const int blk = d.pair_na[p] * d.pair_nb[p];
  const int m = nq * blk;  // parts 0 .. nq-1 of the staged blocks (the first nq of five)
  if ((int)blockIdx.y * NTR >= m) return;  // workgroup-uniform: past this entry's elements
  const int64_t k0 = red_inc_off[r], k1 = red_inc_off[r + 1];
  const bool add = accumulate || !red_first[r];
  const int64_t po = d.pair_off[p];
  const int e = blockIdx.y * NTR + threadIdx.x;
  const int q = e / blk;
  const bool own = e < m && ((part_mask >> q) & 1);
  double sum = own && add ? store[q * d.store_len + po + (e - q * blk)] : 0.0;
  for (int64_t kb = k0; kb < k1; kb += NTR) {
    const int nk = (int)(k1 - kb < NTR ? k1 - kb : NTR);
    __syncthreads();  // previous offsets consumed
    if (threadIdx.x < nk) s_src[threadIdx.x] = inc_src[kb + threadIdx.x];
    __syncthreads();
    int k = 0;
    for (; k + 8 <= nk; k += 8) {
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = e < m ? staging[s_src[k + u] + e] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) sum += a[u];
    }
    for (; k < nk; ++k)
      if (e < m) sum += staging[s_src[k] + e];
  }
  if (own) store[q * d.store_len + po + (e - q * blk)] = sum;
}

// Pairs no batch touches are zero unless accumulating (selected parts).
__global__ void k_zero_pairs(DevPlan d, const int32_t *pairs, double *store, int nq, unsigned part_mask) {
  const int p = pairs[blockIdx.x];
  const int64_t blk = (int64_t)d.pair_na[p] * d.pair_nb[p];
  for (int64_t e = threadIdx.x; e < nq * blk; e += blockDim.x) {
    const int q = (int)(e / blk);
    if ((part_mask >> q) & 1) store[q * d.store_len + d.pair_off[p] + (e - q * blk)] = 0.0;
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

// The adjoint runs per column half of a work item: the tile's 64 rows and 32
// of its columns (half h: columns tj*64 + 32 h ..), four waves, each with 32
// rows and 16 columns.  Positions 2 w + h.
constexpr int NTD = 256;
// LDS image of one 16-point chunk of the 64 row functions (layout of
// dma_chunk): row (q, u) every RSA doubles; 2 mod 16, so 16 lanes reading 16
// consecutive points of one function hit distinct banks
constexpr int RSA = 2 * T + 2;
constexpr int AIMG = 4 * 8 * RSA;   // doubles per image: 4 components x 8 point pairs

// A column half has work iff its columns start inside the batch's n functions.
__device__ __forceinline__ bool half_valid(const WorkItem &it, int h, int n) { return it.tj * T + 32 * h < n; }

// The row values of K steps KS and KS + 1 of one lane, four components
// each: component q of step k at LDS byte address a + 64 RSA q + 64 k.  Read
// in one asm block that also waits for them, by hand: the compiler cannot
// tell these reads from the next chunk's LDS DMA into the other image buffer
// and would otherwise wait for that DMA before the first read.
template <int KS>
__device__ __forceinline__ void read_rows2(uint32_t a, double (&y)[2][4]) {
  constexpr int QS = 64 * RSA, K = 64 * KS;
  asm volatile(
      "ds_read_b64 %0, %8 offset:%9\n"
      "ds_read_b64 %1, %8 offset:%10\n"
      "ds_read_b64 %2, %8 offset:%11\n"
      "ds_read_b64 %3, %8 offset:%12\n"
      "ds_read_b64 %4, %8 offset:%13\n"
      "ds_read_b64 %5, %8 offset:%14\n"
      "ds_read_b64 %6, %8 offset:%15\n"
      "ds_read_b64 %7, %8 offset:%16\n"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(y[0][0]), "=&v"(y[0][1]), "=&v"(y[0][2]), "=&v"(y[0][3]), "=&v"(y[1][0]), "=&v"(y[1][1]),
        "=&v"(y[1][2]), "=&v"(y[1][3])
      : "v"(a), "i"(K), "i"(K + QS), "i"(K + 2 * QS), "i"(K + 3 * QS), "i"(K + 64), "i"(K + 64 + QS),
        "i"(K + 64 + 2 * QS), "i"(K + 64 + 3 * QS)
      : "memory");
}

// Slot data and pair offsets of one adjoint position (column half of a work
// item) in LDS: the tile's 64 rows and the half's 32 columns (slot -1:
// beyond n), the store offset of the pair block of (row slot, column slot)
// for the slots the half spans (-1: lower atom-block triangle or not a stored
// pair) when they are at most ADJ_POFF pairs (atoms of 5 or more functions:
// at most 14 x 8; otherwise each lane looks its pairs up in the plan), and
// the slot ranges.
constexpr int ADJ_POFF = 256;
struct AdjTab {
  int rslot[T], rfn[T], cslot[T / 2], cfn[T / 2], cnf[T / 2];
  int64_t poff[ADJ_POFF];
  int rs0, cs0, ncs, lds_table;
};

// store offset of the pair block of slots (si, sj) of a batch, -1 if none
__device__ __forceinline__ int64_t adj_pair_offset(const DevPlan &d, const AdjPos &D, int si, int sj) {
  if (si > sj) return -1;
  return d.sp_poff[D.spb + (int64_t)si * D.ns - (int64_t)si * (si - 1) / 2 + (sj - si)];
}

// Fills a position's AdjTab (every thread of the workgroup calls it): two
// dependent rounds of loads, each ended by a barrier: the slot data (threads
// 0 .. 95, one packed load each), then the pair offsets of the slot ranges
// (one load per thread).
__device__ __forceinline__ void adj_fill(const DevPlan &d, const AdjPos &D, AdjTab &tb) {
  const int tid = threadIdx.x;
  const int r0 = D.ti * T, c0 = D.tj * T + 32 * D.half;
  if (tid < T + T / 2) {
    const bool row = tid < T;
    const int lf = row ? r0 + tid : c0 + tid - T;
    int64_t v = 0;
    if (lf < D.n) v = d.loc_info[D.f0 + lf];
    const int slot = lf < D.n ? (int)(v & 0xFFFFF) : -1;
    const int fnoff = (int)((v >> 20) & 0xFFFFF), nfn = (int)(v >> 40);
    if (row) {
      tb.rslot[tid] = slot;
      tb.rfn[tid] = fnoff;
    } else {
      tb.cslot[tid - T] = slot;
      tb.cfn[tid - T] = fnoff;
      tb.cnf[tid - T] = nfn;
    }
  }
  __syncthreads();  // slot data visible
  // slot ranges of the tile's rows and the half's columns (slots ascend with
  // the functions; rows and columns beyond n carry slot -1)
  const int rs0 = tb.rslot[0], cs0 = tb.cslot[0];
  const int rs1 = tb.rslot[min(T, D.n - r0) - 1], cs1 = tb.cslot[min(T / 2, D.n - c0) - 1];
  const int nrs = rs1 - rs0 + 1, ncs = cs1 - cs0 + 1;
  const bool in_lds = nrs * ncs <= ADJ_POFF;  // workgroup-uniform
  if (in_lds && tid < nrs * ncs) tb.poff[tid] = adj_pair_offset(d, D, rs0 + tid / ncs, cs0 + tid % ncs);
  if (tid == 0) {
    tb.rs0 = rs0;
    tb.cs0 = cs0;
    tb.ncs = ncs;
    tb.lds_table = in_lds;
  }
  __syncthreads();  // pair offsets visible
}

// partial[g] of a position (P doubles at its pass-relative part offset) = sum
// over its stored elements ij of the selected terms at point g:
//   C^V phi_i phi_j + c' C^Ws grad phi_i . grad phi_j + c' sum_m C^m (grad phi_i x grad phi_j)_m
// (Eq. 39 on the scalar basis).  A position is one column half of a work
// item (the tile's 64 rows, 32 columns), four waves of 32 rows and 16 columns
// each.  Per wave, the 32 x 16 coefficient block sits in registers as the
// MFMA's second operand (5 parts x 8 K steps of 4 rows), and per 16-point
// chunk four accumulators collect (Y^T C) grouped by the column component Z
// they are multiplied with afterwards:
//   u_phi = C^V phi,  u_x = C^Ws dx - C^z dy + C^y dz,
//   u_y = C^z dx + C^Ws dy - C^x dz,  u_z = -C^y dx + C^x dy + C^Ws dz
// (rows i, the K index: Y = the row functions' values at the chunk's points),
// then one drain sum_j u . Z per chunk.  The row image arrives by LDS DMA,
// double-buffered (the next chunk's loads in flight while this one is
// multiplied, one barrier per chunk); each lane's 16 column values Z come from
// the panel straight into registers, two chunks ahead.  Two workgroups fit on a
// CU.  A persistent workgroup draws its next position after the last chunk of
// a position (drawn when a position starts, the tickets ran one position
// ahead of need and the launch read twice the bytes, at the same speed).
// F32W (density_on_grid in FP32): the nine W-term products per K step run on
// FP32 MFMA with the coefficients and row values rounded to FP32; each
// chunk's FP32 sums over the wave's 32 rows (at most 96 products per column
// and point) are drained into the FP64 point sum, so the FP32 error of a
// point is at most gamma_98 (u = 2^-24) times the magnitudes of its W terms.
// The V term stays FP64.
template <bool F32W, bool PERSIST>
__global__ __launch_bounds__(NTD, 2) void k_density_tiles(DevPlan d, const AdjPos *apos, int64_t npos, int global_queue,
                                                          const double *cf, const double *panel, double *partial,
                                                          unsigned *tickets) {
  constexpr int NC = 5;  // coefficient parts
  __shared__ double img[2][AIMG];        // row images, alternating chunks
  __shared__ double s_red[2][4][16];     // per-wave point sums, alternating chunks
  __shared__ int64_t s_pos, s_next[2];
  __shared__ AdjTab tb;                  // the position's slot and pair tables
  const bool gq = global_queue != 0;
  int64_t pos = PERSIST ? next_item(tickets, npos, gq, &s_pos) : (gq ? (int64_t)blockIdx.x : xcd_map(blockIdx.x, npos));
  if (pos >= npos) return;  // workgroup-uniform
  AdjPos D = adj_uniform(apos[pos]);
  const int tid = threadIdx.x;
  // wave index as a scalar: conditions derived from it stay uniform
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int js = wave & 1, ih = wave >> 1;  // column block, row half
  const int l16 = lane & 15, lk = lane >> 4;
  // column values of a chunk.  FP64 (TR): the MFMA takes the row values as
  // its first operand (lane l16 supplying point 4 (l16 % 4) + l16 / 4) and
  // the coefficients as its second, so result register r of lane (l16, lk)
  // is point 4 lk + r at column colb + l16: each lane's four points of a
  // component are one 32-byte quad of the panel, two 16-byte loads.  F32W:
  // coefficients first, register r is column lk + 4 r (FP64 MFMA) or
  // 4 lk + r (FP32 MFMA) at point l16.
  constexpr bool TR = !F32W;
  const int ptA = TR ? 4 * (l16 & 3) + (l16 >> 2) : l16;  // the point this lane supplies to the row operand
  int par = 0;
  for (;;) {
  const int n = D.n, P = D.P;
  const int r0 = D.ti * T, c0 = D.tj * T + 32 * D.half;
  const int Pp = (int)pad16(P), np = (int)pad16(n);
  const double *pb = panel + D.panel_off;
  const int64_t plane = (int64_t)Pp * np;
  const int colb = c0 + 16 * js;
  const int lj = colb + l16;
  // row origin of this wave's two 16-row blocks.  Column half 0 of a diagonal
  // tile has 3 active blocks, (0,0), (0,1) and (1,1) in 16-blocks: block (1,1)
  // moves from wave (ih 0, js 1) to the otherwise idle wave (ih 1, js 1), so
  // no wave of that half carries two.
  const bool dg0 = D.ti == D.tj && D.half == 0;
  const int iloc = (dg0 && ih == 1 && js == 1) ? 16 : 32 * ih;
  bool act[2], upper[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int rb = r0 + iloc + 16 * h;
    act[h] = block_active(rb, colb, n) && !(dg0 && ih == 0 && js == 1 && h == 1);
    upper[h] = rb < colb;
  }
  const bool any = act[0] || act[1];
  // The row image of a chunk comes by buffer loads straight into LDS: image
  // row r = (component r / 8, point pair r % 8) holds 16 bytes per function;
  // the lane offset is fixed, the chunk and image row go into the scalar offset.
  // Lanes whose function lies at or beyond np, and column loads of a wave
  // without active blocks, take an offset past the end of the buffer: the
  // load is still issued (so every wave issues the same loads per chunk) but
  // reads nothing and returns zero.
  const __amdgpu_buffer_rsrc_t prs =
      __builtin_amdgcn_make_buffer_rsrc((void *)pb, (short)0, (int)(32 * plane), 0x00020000);
  constexpr uint32_t OOB = 0x80000000u;
  const uint32_t vrow = r0 + lane < np ? lane * 32u : OOB;
  auto dma_rows = [&](int ks0, double *dst) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int r = wave + 4 * k, q = r >> 3, u = r & 7;
      const uint32_t so = (uint32_t)((q * plane + ((int64_t)(ks0 + (u >> 1)) * np + r0) * 4 + 2 * (u & 1)) * 8);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(prs, (lds_void *)(dst + r * RSA), 16, vrow, so, 0, 0);
    }
  };
  // column values of two chunks in flight: zb[c & 1] holds chunk c's, loaded
  // at the end of chunk c - 2.  Each wave issues the same ZLOADS buffer loads
  // for every chunk, unconditionally (past the last chunk the last one is read
  // again), so that at each chunk's barrier "this chunk's image and column
  // values have landed" is "at most ZLOADS loads outstanding": only the next
  // chunk's column loads, issued after the image DMA, remain in flight.
  double zb[2][4][4];
  const uint32_t zoob = any ? 0u : OOB;  // or-ed into the offsets: no branch around the loads
  auto load_z = [&](int k, auto zc) {
    constexpr int ZB = decltype(zc)::value;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t qo = (uint32_t)(q * plane * 8);
      if (TR) {
        const uint32_t zo = (uint32_t)(((int64_t)((k >> 2) + lk) * np + colb + l16) * 32) | zoob;
        const dbl2 z01 = __builtin_bit_cast(dbl2, __builtin_amdgcn_raw_buffer_load_b128(prs, zo, qo, 0));
        const dbl2 z23 = __builtin_bit_cast(dbl2, __builtin_amdgcn_raw_buffer_load_b128(prs, zo + 16, qo, 0));
        zb[ZB][q][0] = z01[0];
        zb[ZB][q][1] = z01[1];
        zb[ZB][q][2] = z23[0];
        zb[ZB][q][3] = z23[1];
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int jr = (F32W && q > 0) ? d_row_f32(lk, r) : d_row_f64(lk, r);
          const uint32_t zo = (uint32_t)((((int64_t)((k + l16) >> 2) * np + colb + jr) * 4 + (l16 & 3)) * 8) | zoob;
          zb[ZB][q][r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(prs, zo, qo, 0));
        }
      }
    }
  };
  // column loads per chunk: one buffer load instruction each
  constexpr int ZLOADS = TR ? 8 : 16;
  // the first chunk's loads go out before anything else of the position
  dma_rows(0, img[0]);
  load_z(0, std::integral_constant<int, 0>{});
  load_z(min(16, Pp - 16), std::integral_constant<int, 1>{});
  adj_fill(d, D, tb);
  // coefficient slice: rows i = r0 + iloc + 4 ks + lk (ks = 0..7), column lj:
  // element (li, lj) of the folded coefficients (k_coef_fold) in the pair
  // block of its two atoms (upper atom-block triangle only); lanes without a
  // stored element read the zeros past the end of each part
  double creg[NC][8];
  {
    const int64_t Lf = d.store_len + 16;
    const int cl = 16 * js + l16;
    const int cslot = tb.cslot[cl], cfn = tb.cfn[cl], cnf = tb.cnf[cl];
    const int rs0 = tb.rs0, cs0 = tb.cs0, ncs = tb.ncs;
    const bool lds_table = tb.lds_table != 0;
#pragma unroll
    for (int ks = 0; ks < 8; ++ks) {
      const int rl = iloc + 4 * ks + lk;
      const int li = r0 + rl;
      const int rslot = tb.rslot[rl], rfn = tb.rfn[rl];
      int64_t po = -1;
      if (act[ks >> 2] && rslot >= 0 && cslot >= 0)
        po = lds_table ? tb.poff[(rslot - rs0) * ncs + (cslot - cs0)] : adj_pair_offset(d, D, rslot, cslot);
      const int64_t ea = po >= 0 ? po + (int64_t)(li - rfn) * cnf + (lj - cfn) : d.store_len;
#pragma unroll
      for (int q = 0; q < NC; ++q) creg[q][ks] = cf[q * Lf + ea];
    }
  }
  // F32W: the W coefficients as FP32 MFMA operands
  float cw[4][8];
  if (F32W) {
#pragma unroll
    for (int ks = 0; ks < 8; ++ks)
#pragma unroll
      for (int q = 0; q < 4; ++q) cw[q][ks] = (float)creg[q + 1][ks];
  }
  double *out = partial + D.part;
  // the coefficients (and the first chunks' loads) have landed before the
  // chunks begin, so that no wait for them falls inside a chunk
  __builtin_amdgcn_s_waitcnt(0);


  auto chunk = [&](int k0, auto zc) {
    constexpr int bi = decltype(zc)::value;  // chunk parity: image buffer and column-value set
    // this wave's image and column loads of this chunk have landed (only the
    // next chunk's column loads may be outstanding) ... and everyone's; the
    // previous chunk is consumed, its sums visible
    barrier_vm<ZLOADS>();
    if (k0 > 0 && tid < 16 && k0 - 16 + tid < P)
      out[k0 - 16 + tid] = (s_red[bi ^ 1][0][tid] + s_red[bi ^ 1][1][tid]) +
                           (s_red[bi ^ 1][2][tid] + s_red[bi ^ 1][3][tid]);
    dma_rows(min(k0 + 16, Pp - 16) >> 2, img[bi ^ 1]);
    // this chunk's column values landed before the barrier above; the empty
    // asm makes them its own result, so the compiler, which cannot follow the
    // loads across the barrier, places no wait for them inside the chunk
#pragma unroll
    for (int q = 0; q < 4; ++q)
      asm volatile("" : "+v"(zb[bi][q][0]), "+v"(zb[bi][q][1]), "+v"(zb[bi][q][2]), "+v"(zb[bi][q][3]));
    const double (&zt)[4][4] = zb[bi];
    double x = 0.0;
    if (any && F32W) {
      // this lane's row values of K step 0, component 0 (point ptA, row iloc + lk)
      const uint32_t ybase = lds_addr(img[bi]) + 8u * (uint32_t)((ptA >> 1) * RSA + 2 * (iloc + lk) + (ptA & 1));
      dbl4 uf = dbl4{0.0, 0.0, 0.0, 0.0};
      flt4 vx = flt4{0.f, 0.f, 0.f, 0.f}, vy = vx, vz = vx;
      auto ksteps = [&](auto k0c, auto k1c) {
        constexpr int K0 = decltype(k0c)::value, K1 = decltype(k1c)::value;
        static_for<K0, K1, 2>([&](auto kpc) {
        constexpr int KP = decltype(kpc)::value;
        double yy[2][4];
        read_rows2<KP>(ybase, yy);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int ks = KP + h;
          const double y0 = yy[h][0];
          const float y1 = (float)yy[h][1];
          const float y2 = (float)yy[h][2];
          const float y3 = (float)yy[h][3];
          uf = mfma64(creg[0][ks], y0, uf);
          vx = mfma32(cw[0][ks], y1, vx);
          vy = mfma32(cw[3][ks], y1, vy);
          vz = mfma32(cw[2][ks], -y1, vz);
          vx = mfma32(cw[3][ks], -y2, vx);
          vy = mfma32(cw[0][ks], y2, vy);
          vz = mfma32(cw[1][ks], y2, vz);
          vx = mfma32(cw[2][ks], y3, vx);
          vy = mfma32(cw[1][ks], -y3, vy);
          vz = mfma32(cw[0][ks], y3, vz);
        }
        });
      };
      if (act[0] && act[1])
        ksteps(std::integral_constant<int, 0>{}, std::integral_constant<int, 8>{});
      else if (act[0])
        ksteps(std::integral_constant<int, 0>{}, std::integral_constant<int, 4>{});
      else
        ksteps(std::integral_constant<int, 4>{}, std::integral_constant<int, 8>{});
#pragma unroll
      for (int r = 0; r < 4; ++r)
        x += (uf[r] * zt[0][r] + (double)vx[r] * zt[1][r]) + ((double)vy[r] * zt[2][r] + (double)vz[r] * zt[3][r]);
      x += __shfl_xor(x, 16);
      x += __shfl_xor(x, 32);
    } else if (any) {
      // this lane's row values of K step 0, component 0 (point ptA, row iloc + lk)
      const uint32_t ybase = lds_addr(img[bi]) + 8u * (uint32_t)((ptA >> 1) * RSA + 2 * (iloc + lk) + (ptA & 1));
      dbl4 uf = dbl4{0.0, 0.0, 0.0, 0.0}, ux = uf, uy = uf, uz = uf;
      // the K steps of active 16-row blocks, as straight-line code
      auto ksteps = [&](auto k0c, auto k1c) {
        constexpr int K0 = decltype(k0c)::value, K1 = decltype(k1c)::value;
        static_for<K0, K1, 2>([&](auto kpc) {
        constexpr int KP = decltype(kpc)::value;
        double yy[2][4];
        read_rows2<KP>(ybase, yy);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          // row values Y[q][pt = ptA][i = iloc + 4 ks + lk]: the K index is lk;
          // row values first, so the result is points x columns
          const int ks = KP + h;
          const double y0 = yy[h][0], y1 = yy[h][1], y2 = yy[h][2], y3 = yy[h][3];
          uf = mfma64(y0, creg[0][ks], uf);
          ux = mfma64(y1, creg[1][ks], ux);
          uy = mfma64(y1, creg[4][ks], uy);
          uz = mfma64(-y1, creg[3][ks], uz);
          ux = mfma64(-y2, creg[4][ks], ux);
          uy = mfma64(y2, creg[1][ks], uy);
          uz = mfma64(y2, creg[2][ks], uz);
          ux = mfma64(y3, creg[3][ks], ux);
          uy = mfma64(-y3, creg[2][ks], uy);
          uz = mfma64(y3, creg[1][ks], uz);
        }
        });
      };
      if (act[0] && act[1])
        ksteps(std::integral_constant<int, 0>{}, std::integral_constant<int, 8>{});
      else if (act[0])
        ksteps(std::integral_constant<int, 0>{}, std::integral_constant<int, 4>{});
      else
        ksteps(std::integral_constant<int, 4>{}, std::integral_constant<int, 8>{});
      // per point (register r: point 4 lk + r), the sum over the 16 columns
      // (lanes l16 of the row): halve the points per lane twice (xor 8, 4),
      // then finish the sum (xor 2, 1); lane l16 ends with point 4 lk + r*,
      // r* = 2 (l16 >> 3 & 1) + (l16 >> 2 & 1)
      double xr[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) xr[r] = (uf[r] * zt[0][r] + ux[r] * zt[1][r]) + (uy[r] * zt[2][r] + uz[r] * zt[3][r]);
      const bool h8 = (l16 & 8) != 0, h4 = (l16 & 4) != 0;
      double s0 = h8 ? xr[2] : xr[0], s1 = h8 ? xr[3] : xr[1];
      s0 += dpp_f64<DPP_ROW_MIRROR>(h8 ? xr[0] : xr[2]);
      s1 += dpp_f64<DPP_ROW_MIRROR>(h8 ? xr[1] : xr[3]);
      x = h4 ? s1 : s0;
      x += dpp_f64<DPP_ROW_HALF_MIRROR>(h4 ? s0 : s1);
      x += dpp_f64<DPP_QUAD_XOR2>(x);
      x += dpp_f64<DPP_QUAD_XOR1>(x);
    }
    if (TR) {
      if ((l16 & 3) == 0) s_red[bi][wave][4 * lk + 2 * ((l16 >> 3) & 1) + ((l16 >> 2) & 1)] = x;
    } else {
      if (lane < 16) s_red[bi][wave][l16] = x;
    }
    load_z(min(k0 + 32, Pp - 16), zc);
  };
  // pairs of chunks (even, odd) as straight-line code, then an odd last one
  int k0 = 0;
  for (; k0 + 32 <= Pp; k0 += 32) {
    chunk(k0, std::integral_constant<int, 0>{});
    chunk(k0 + 16, std::integral_constant<int, 1>{});
  }
  if (k0 < Pp) chunk(k0, std::integral_constant<int, 0>{});
  __syncthreads();  // the last chunk's per-wave sums
  {
    const int k0 = Pp - 16, bi = (k0 >> 4) & 1;
    if (tid < 16 && k0 + tid < P)
      out[k0 + tid] = (s_red[bi][0][tid] + s_red[bi][1][tid]) + (s_red[bi][2][tid] + s_red[bi][3][tid]);
  }
  if (!PERSIST) return;
  // the next position, drawn once this one is done; two slots in turn:
  // thread 0 may write the next slot before every thread has read this one
  if (tid == 0) s_next[par] = ticket_pos(tickets, npos, gq, draw_ticket(tickets, gq));
  __syncthreads();
  pos = uniform_i64(s_next[par]);
  par ^= 1;
  if (pos >= npos) return;
  D = adj_uniform(apos[pos]);
  }
}

// The adjoint's coefficients, folded once per call.  Eq. 39 sums every stored
// element ij of the selected terms; the adjoint's work items cover the upper
// 16 x 16 blocks of each batch, so in the diagonal block of one atom element
// (i, j), i < j, takes C_q(i, j) + s_q C_q(j, i) (s_q = +1 for V and Ws, -1
// for the spin-orbit parts, whose terms change sign under i <-> j), (i, i)
// keeps C_q(i, i) and i > j is zero: every term is then carried once.  Blocks
// of two atoms are copied.  c' multiplies the W parts, unselected terms are
// zero, and each part ends in 16 zeros (row stride store_len + 16), the
// element of lanes without a stored one.  One workgroup per pair.
__global__ void k_coef_fold(DevPlan d, const double *coef, uint32_t terms, double *cf) {
  const int64_t L = d.store_len, Lf = L + 16;
  const int64_t q = blockIdx.x;
  const bool on[5] = {(terms & Q4C_TERM_LL) != 0, (terms & Q4C_TERM_SS) != 0, (terms & Q4C_TERM_SO) != 0,
                      (terms & Q4C_TERM_SO) != 0, (terms & Q4C_TERM_SO) != 0};
  if (q == 0 && threadIdx.x < 16)
    for (int p = 0; p < 5; ++p) cf[p * Lf + L + threadIdx.x] = 0.0;
  const int64_t po = d.pair_off[q];
  const int na = d.pair_na[q], nb = d.pair_nb[q];
  const bool diag = d.pair_a[q] == d.pair_b[q];
  for (int t = threadIdx.x; t < na * nb; t += blockDim.x) {
    const int i = t / nb, j = t - i * nb;
#pragma unroll
    for (int p = 0; p < 5; ++p) {
      double c = coef[p * L + po + t];
      if (diag) {
        if (i < j)
          c += mirror_sign(p) * coef[p * L + po + (int64_t)j * nb + i];
        else if (i > j)
          c = 0.0;
      }
      cf[p * Lf + po + t] = on[p] ? (p > 0 ? c * d.cprime : c) : 0.0;
    }
  }
}

// Point sums: out[perm[g]] = (w_g if weighted) * sum over the batch's work
// items (in order) and their valid column halves (in order).
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
      const double *pw = partial + 2 * d.work_part_off[w];
      s += pw[g];
      if (half_valid(it, 1, n)) s += pw[P + g];
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

// Launch one contraction kernel over work positions [w0, w0 + nw) of a pass,
// persistent (tickets) or one workgroup per position.
template <typename K>
static void launch_work(K kernel_p, K kernel_1, unsigned grid, bool persistent, hipStream_t s, const DevPlan &dp,
                        const WorkItem *work, const int32_t *order, int64_t w0, int64_t nw, const double *om,
                        const double *panel, double *staging, unsigned *tickets) {
  if (persistent)
    hipLaunchKernelGGL(kernel_p, dim3(grid), dim3(NT), 0, s, dp, work, order, w0, nw, om, panel, staging, tickets);
  else
    hipLaunchKernelGGL(kernel_1, dim3(grid), dim3(NT), 0, s, dp, work, order, w0, nw, om, panel, staging, tickets);
}

int launch_integrate(const q4c_plan *p, const double *v, int precision, uint32_t parts, uint32_t flags,
                     double *store, double *spin_w, double *spin_v, hipStream_t s) {
  const int accumulate = (flags & Q4C_ACCUMULATE) ? 1 : 0;
  const bool wantV = parts & Q4C_PART_V, wantW = parts & (Q4C_PART_WS | Q4C_PART_WSO);
  // store parts written: 0 V, 1 Ws, 2..4 Wso
  const unsigned pmask = (wantV ? 1u : 0u) | ((parts & Q4C_PART_WS) ? 2u : 0u) | ((parts & Q4C_PART_WSO) ? 28u : 0u);
  // FP64 with W parts: one kernel for all five (PK_F64 panels); otherwise V
  // on FP64 from phi alone and the W parts on FP32 (PK_F32 / PK_SPLIT panels)
  // BF16X3 with W parts: one kernel for all five (PK_BF16 panels)
  const bool full64 = (precision == Q4C_PREC_F64 || precision == Q4C_PREC_F64_VALU) && wantW;
  const bool fused_b3 = precision == Q4C_PREC_BF16X3 && wantW;
  const int kind = (full64 || precision == Q4C_PREC_F64_VALU) ? PK_F64
                   : fused_b3 ? PK_BF16
                              : (precision == Q4C_PREC_SPLIT_F32 && wantW ? PK_SPLIT : PK_F32);
  int rc;
  {
    TimedLaunch tl_(p, Q4C_TIMER_OTHER, s);
    const unsigned nb = (unsigned)std::min<int64_t>((p->n_active + 16 + 255) / 256, 65535);
    hipLaunchKernelGGL(k_om, dim3(nb), dim3(256), 0, s, p->dp, v, p->d_om);
  }
  if ((rc = check_launch("k_om")) != Q4C_OK) return rc;
  const LaunchCfg cfg = p->cfg_contract;
  const int32_t *order = cfg.order ? p->d_order : nullptr;
  const int64_t np_ = (int64_t)p->passes.size();
  if (cfg.persistent > 0) {
    // ticket queues: [V or all-parts kernel][W kernel] x passes
    hipLaunchKernelGGL(k_zero_u32, dim3(8), dim3(256), 0, s, p->d_tickets, 2 * np_ * kTicketsPerLaunch);
    if ((rc = check_launch("k_zero_u32")) != Q4C_OK) return rc;
  }
  for (size_t ip = 0; ip < p->passes.size(); ++ip) {
    const Pass &ps = p->passes[ip];
    const int64_t nw = ps.w1 - ps.w0, nt = ps.t1 - ps.t0, nr = ps.r1 - ps.r0;
    const bool pers = cfg.persistent > 0;
    unsigned *tick_a = pers ? p->d_tickets + ip * kTicketsPerLaunch : nullptr;
    unsigned *tick_w = pers ? p->d_tickets + (np_ + ip) * kTicketsPerLaunch : nullptr;
    const unsigned grid = (unsigned)(pers ? std::min<int64_t>(cfg.persistent, nw) : nw);
    double *panel = p->d_staging + ps.staging_len + ps.partial_len;
    if (nt > 0) {
      {
        TimedLaunch tl_(p, Q4C_TIMER_TABULATE, s);
        if (kind == PK_F64)
          hipLaunchKernelGGL(k_panel<PK_F64>, dim3((unsigned)nt), dim3(256), 0, s, p->dp, p->d_ptile, ps.t0, nt, panel,
                           (const double *)nullptr);
        else if (kind == PK_BF16)
          hipLaunchKernelGGL(k_panel<PK_BF16>, dim3((unsigned)nt), dim3(256), 0, s, p->dp, p->d_ptile, ps.t0, nt,
                             panel, (const double *)p->d_om);
        else if (kind == PK_SPLIT)
          hipLaunchKernelGGL(k_panel<PK_SPLIT>, dim3((unsigned)nt), dim3(256), 0, s, p->dp, p->d_ptile, ps.t0, nt,
                             panel, (const double *)nullptr);
        else
          hipLaunchKernelGGL(k_panel<PK_F32>, dim3((unsigned)nt), dim3(256), 0, s, p->dp, p->d_ptile, ps.t0, nt, panel,
                             (const double *)p->d_om);
      }
      if ((rc = check_launch("k_panel")) != Q4C_OK) return rc;
    }
    if (nw > 0) {
      TimedLaunch tl_(p, Q4C_TIMER_CONTRACT, s);
      if (precision == Q4C_PREC_F64_VALU) {
        // the plain FP64 baseline: one workgroup per work item, every part
        hipLaunchKernelGGL(k_contract_valu, dim3((unsigned)nw), dim3(NT), 0, s, p->dp, p->d_work, order, ps.w0, nw,
                           p->d_om, panel, p->d_staging, (unsigned *)nullptr);
      } else if (full64) {
        launch_work(k_contract<MODE_F64, true>, k_contract<MODE_F64, false>, grid, pers, s, p->dp, p->d_work, order,
                    ps.w0, nw, p->d_om, panel, p->d_staging, tick_a);
      } else if (fused_b3) {
        // one workgroup per column half of each work item
        const unsigned grid2 = (unsigned)(pers ? std::min<int64_t>(cfg.persistent, 2 * nw) : 2 * nw);
        launch_work(k_contract_b3<true>, k_contract_b3<false>, grid2, pers, s, p->dp, p->d_work, order, ps.w0, nw,
                    p->d_om, panel, p->d_staging, tick_a);
      } else {
        if (wantV) {
          // four V-only workgroups fit on a CU, twice the other contraction
          // kernels' two: twice the persistent workgroups
          const unsigned grid_v = (unsigned)(pers ? std::min<int64_t>(2 * (int64_t)cfg.persistent, nw) : nw);
          launch_work(k_contract<MODE_V, true>, k_contract<MODE_V, false>, grid_v, pers, s, p->dp, p->d_work, order,
                      ps.w0, nw, p->d_om, panel, p->d_staging, tick_a);
        }
        if (wantW && precision == Q4C_PREC_SPLIT_F32)
          launch_work(k_contract_w<true, true>, k_contract_w<true, false>, grid, pers, s, p->dp, p->d_work, order,
                      ps.w0, nw, p->d_om, panel, p->d_staging, tick_w);
        else if (wantW)
          launch_work(k_contract_w<false, true>, k_contract_w<false, false>, grid, pers, s, p->dp, p->d_work, order,
                      ps.w0, nw, p->d_om, panel, p->d_staging, tick_w);
      }
    }
    if (nw > 0 && (rc = check_launch("k_contract")) != Q4C_OK) return rc;
    if (nr > 0) {
      {
        TimedLaunch tl_(p, Q4C_TIMER_REDUCE, s);
        hipLaunchKernelGGL(k_reduce, dim3((unsigned)nr, (unsigned)((5 * p->max_pair_block + NTR - 1) / NTR)), dim3(NTR),
                           0, s, p->dp, ps.r0, p->d_red_pair, p->d_red_first, p->d_red_inc_off, p->d_inc_src,
                           p->d_staging, store, accumulate, 5, pmask);
      }
      if ((rc = check_launch("k_reduce")) != Q4C_OK) return rc;
    }
  }
  if (!accumulate && !p->untouched_pairs.empty()) {
    {
      TimedLaunch tl_(p, Q4C_TIMER_OTHER, s);
      hipLaunchKernelGGL(k_zero_pairs, dim3((unsigned)p->untouched_pairs.size()), dim3(256), 0, s, p->dp,
                         p->d_untouched, store, 5, pmask);
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
    hipLaunchKernelGGL(k_om, dim3(nb), dim3(256), 0, s, p->dp, v, p->d_om);
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
        hipLaunchKernelGGL(k_panel<PK_HS>, dim3((unsigned)nt), dim3(256), 0, s, p->dp, p->d_ptile, ps.t0, nt, panel,
                           (const double *)nullptr);
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
        hipLaunchKernelGGL(k_reduce, dim3((unsigned)nr, (unsigned)((2 * p->max_pair_block + NTR - 1) / NTR)), dim3(NTR),
                           0, s, p->dp, ps.r0, p->d_red_pair, p->d_red_first, p->d_red_inc_off, p->d_inc_src,
                           p->d_staging, hs, accumulate, 2, 3u);
      }
      if ((rc = check_launch("k_reduce")) != Q4C_OK) return rc;
    }
  }
  if (!accumulate && !p->untouched_pairs.empty()) {
    {
      TimedLaunch tl_(p, Q4C_TIMER_OTHER, s);
      hipLaunchKernelGGL(k_zero_pairs, dim3((unsigned)p->untouched_pairs.size()), dim3(256), 0, s, p->dp,
                         p->d_untouched, hs, 2, 3u);
    }
    if ((rc = check_launch("k_zero_pairs")) != Q4C_OK) return rc;
  }
  return Q4C_OK;
}

int launch_density(const q4c_plan *p, const double *coef, uint32_t terms, int precision, int weight_mode,
                   double *out, int64_t resident_pass, hipStream_t s) {
  int rc;
  if (p->n_points > 0) {
    {
      TimedLaunch tl_(p, Q4C_TIMER_OTHER, s);
      const unsigned nb = (unsigned)std::min<int64_t>((p->n_points + 255) / 256, 65535);
      hipLaunchKernelGGL(k_fill, dim3(nb), dim3(256), 0, s, out, p->n_points, 0.0);
    }
    if ((rc = check_launch("k_fill")) != Q4C_OK) return rc;
  }
  if (p->n_pairs > 0) {
    {
      TimedLaunch tl_(p, Q4C_TIMER_OTHER, s);
      hipLaunchKernelGGL(k_coef_fold, dim3((unsigned)p->n_pairs), dim3(256), 0, s, p->dp, coef, terms,
                         p->d_coef_fold);
    }
    if ((rc = check_launch("k_coef_fold")) != Q4C_OK) return rc;
  }
  const LaunchCfg cfg = p->cfg_density;
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
    const int64_t nw = ps.ap1 - ps.ap0, nbt = ps.b1 - ps.b0;
    const AdjPos *apos = (cfg.order ? p->d_adjpos_cost : p->d_adjpos) + ps.ap0;
    const int64_t nt = (int64_t)ip == resident_pass ? 0 : ps.t1 - ps.t0;
    unsigned *tickets = cfg.persistent > 0 ? tick0 + ip * kTicketsPerLaunch : nullptr;
    // one workgroup position per column half of a work item
    const unsigned grid = (unsigned)(cfg.persistent > 0 ? std::min<int64_t>(cfg.persistent, nw) : nw);
    double *partial = p->d_staging + ps.staging_len;
    double *panel = partial + ps.partial_len;
    if (nt > 0) {
      {
        TimedLaunch tl_(p, Q4C_TIMER_TABULATE, s);
        hipLaunchKernelGGL(k_panel<PK_F64>, dim3((unsigned)nt), dim3(256), 0, s, p->dp, p->d_ptile, ps.t0, nt, panel,
                           (const double *)nullptr);
      }
      if ((rc = check_launch("k_panel")) != Q4C_OK) return rc;
    }
    if (nw > 0) {
      {
        TimedLaunch tl_(p, Q4C_TIMER_DENSITY_TILES, s);
        if (precision == Q4C_PREC_F32) {
          if (tickets)
            hipLaunchKernelGGL((k_density_tiles<true, true>), dim3(grid), dim3(NTD), 0, s, p->dp, apos, nw,
                               cfg.order, p->d_coef_fold, panel, partial, tickets);
          else
            hipLaunchKernelGGL((k_density_tiles<true, false>), dim3(grid), dim3(NTD), 0, s, p->dp, apos, nw,
                               cfg.order, p->d_coef_fold, panel, partial, tickets);
        } else {
          if (tickets)
            hipLaunchKernelGGL((k_density_tiles<false, true>), dim3(grid), dim3(NTD), 0, s, p->dp, apos, nw,
                               cfg.order, p->d_coef_fold, panel, partial, tickets);
          else
            hipLaunchKernelGGL((k_density_tiles<false, false>), dim3(grid), dim3(NTD), 0, s, p->dp, apos, nw,
                               cfg.order, p->d_coef_fold, panel, partial, tickets);
        }
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
        hipLaunchKernelGGL(k_panel<PK_F64>, dim3((unsigned)nt), dim3(256), 0, s, p->dp, p->d_ptile, ps.t0, nt, panel,
                           (const double *)nullptr);
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
