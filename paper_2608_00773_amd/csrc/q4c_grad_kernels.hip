// The kernels of density_gradient_on_grid: the density and its gradient from
// one real coefficient part C on the stored pairs (a scalar density matrix of
// one component: the forward density update of Eq. 39 with the gradient a
// GGA needs).  Per batch with functions phi_1..phi_n at its points,
//   n = sum over stored elements C_ij phi_i phi_j = phi^T M phi,
//   grad n = 2 grad phi^T M phi,
// with M the symmetric n x n matrix of the batch (half of each stored
// off-diagonal element on both sides, the symmetric part of a self pair's
// block).  So per batch one product Y = M Phi (2 P n^2 flops, on FP64 MFMA)
// and lane-local dot products of Y with phi and grad phi.
//   k_grad_cdense  M of every batch of a pass, dense (np x np, zero padding);
//   k_grad_gemm    one workgroup per (batch, 64-point tile, 64-function tile
//                  i): Y_i(pt) = sum_j phi_j(pt) M_ji over 16-function K
//                  chunks (phi slice and M slice by LDS DMA, double
//                  buffered), then n and grad n partials over its functions;
//   k_grad_points  the partials of a point over the function tiles, in order.
// (Gathering the M slices from the store inside the product instead of
// materialising M was slower: two dependent memory round trips per 16
// functions do not hide behind 16 MFMAs.)
// The panel tabulation and the launches around these are in q4c_kernels.hip.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "q4c_internal.h"
#include "q4c_device.h"

namespace q4c {
namespace {

constexpr int GT = 64;    // points and functions per output tile
constexpr int GK = 16;    // functions per K chunk
constexpr int GS = 1024;  // doubles per slice image (64 x 16)


// packed slot data of a batch function: slot, the slot's first function and
// its function count
__device__ __forceinline__ int fslot(int64_t v) { return (int)(v & 0xFFFFF); }
__device__ __forceinline__ int ffirst(int64_t v) { return (int)((v >> 20) & 0xFFFFF); }
__device__ __forceinline__ int fcount(int64_t v) { return (int)(v >> 40); }

constexpr int CD_T = 64;       // M tile edge
constexpr int CD_PO = 256;     // entries of the (row slot, column slot) pair-offset table of a tile in LDS

// One upper-triangle tile (rt <= ct) of M of one batch: M_rc for the tile's
// rows r and columns c, and by symmetry the mirrored tile M_cr.  Slots
// (relevant atoms) ascend with the batch's functions and with the atom
// index, so slot lo < hi is the stored pair (atom(lo), atom(hi)) with rows =
// lo's functions; above the diagonal (r < c) the row slot never exceeds the
// column slot and the store is read in its own orientation, coalesced along
// c (a self pair also takes its transposed element).  The tile goes through
// LDS so that both it and its mirror are written along rows.
__global__ __launch_bounds__(256) void k_grad_cdense(DevPlan d, const int32_t *items, int64_t it0,
                                                     const int64_t *cd_off, const int64_t *fninfo,
                                                     const double *coef, double *cd) {
  __shared__ double s_t[CD_T][CD_T + 1];
  __shared__ int64_t s_ri[CD_T], s_ci[CD_T];
  __shared__ int64_t s_po[CD_PO];
  const int64_t it = it0 + blockIdx.x;
  const int b = items[3 * it], rt = items[3 * it + 1], ct = items[3 * it + 2];
  const int f0 = d.batch_fn_off[b], n = d.batch_fn_off[b + 1] - f0, np = (int)pad16(n);
  const int sbase = d.batch_slot_off[b], ns = d.batch_slot_off[b + 1] - sbase;
  const int64_t spb = d.batch_sp_off[b];
  double *M = cd + cd_off[b];
  const int r0 = CD_T * rt, c0 = CD_T * ct;  // both below n (tiles start below np - 15)
  const int nr = min(CD_T, np - r0), nc = min(CD_T, np - c0);
  auto stored_po = [&](int rs, int cs) -> int64_t {
    const int lo = min(rs, cs), hi = max(rs, cs);
    const int q = d.sp_pair[spb + (int64_t)lo * ns - (int64_t)lo * (lo - 1) / 2 + (hi - lo)];
    return q >= 0 ? d.pair_off[q] : (int64_t)-1;
  };
  if (threadIdx.x < CD_T) s_ri[threadIdx.x] = fninfo[f0 + min(r0 + (int)threadIdx.x, n - 1)];
  else if (threadIdx.x < 2 * CD_T) s_ci[threadIdx.x - CD_T] = fninfo[f0 + min(c0 + (int)threadIdx.x - CD_T, n - 1)];
  __syncthreads();  // slot data visible
  const int rs0 = fslot(s_ri[0]), rs1 = fslot(s_ri[min(CD_T, n - r0) - 1]);
  const int cs0 = fslot(s_ci[0]), cs1 = fslot(s_ci[min(CD_T, n - c0) - 1]);
  const int nrs = rs1 - rs0 + 1, ncs = cs1 - cs0 + 1;
  const bool po_lds = nrs * ncs <= CD_PO;  // workgroup-uniform
  if (po_lds)
    for (int t = threadIdx.x; t < nrs * ncs; t += blockDim.x) s_po[t] = stored_po(rs0 + t / ncs, cs0 + t % ncs);
  __syncthreads();  // pair offsets visible
  // the tile's elements with r <= c (all of them off the diagonal), four per
  // thread at a time, loads unconditional (element 0 of the store stands in
  // for an absent one) and in flight together
  for (int x0 = threadIdx.x; x0 < CD_T * CD_T; x0 += 4 * blockDim.x) {
    int64_t a1[4], a2[4];
    bool live[4], self[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int x = x0 + u * blockDim.x;
      const int rl = x / CD_T, cl = x % CD_T;
      const int r = r0 + rl, c = c0 + cl;
      const bool in = r < n && c < n && r <= c;
      const int64_t ri = s_ri[rl], ci = s_ci[cl];
      const int rs = fslot(ri), cs = fslot(ci);
      const int64_t po = !in ? -1 : (po_lds ? s_po[(rs - rs0) * ncs + cs - cs0] : stored_po(rs, cs));
      const int ir = r - ffirst(ri), ic = c - ffirst(ci), cn = fcount(ci);
      live[u] = po >= 0;
      self[u] = rs == cs;
      a1[u] = live[u] ? po + (int64_t)ir * cn + ic : 0;                // rs <= cs here
      a2[u] = live[u] && self[u] ? po + (int64_t)ic * cn + ir : 0;     // the self pair's transposed element
    }
    double c1[4], c2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      c1[u] = coef[a1[u]];
      c2[u] = coef[a2[u]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int x = x0 + u * blockDim.x;
      s_t[x / CD_T][x % CD_T] = live[u] ? 0.5 * (c1[u] + (self[u] ? c2[u] : 0.0)) : 0.0;
    }
  }
  __syncthreads();  // the tile is in LDS
  // the tile (r <= c part; on the diagonal tile the rest from its mirror) and,
  // off the diagonal, its mirror, both along rows
  for (int x = threadIdx.x; x < nr * nc; x += blockDim.x) {
    const int rl = x / nc, cl = x % nc;
    const double v = (rt == ct && rl > cl) ? s_t[cl][rl] : s_t[rl][cl];
    M[(int64_t)(r0 + rl) * np + c0 + cl] = v;
  }
  if (rt != ct)
    for (int x = threadIdx.x; x < nr * nc; x += blockDim.x) {
      const int cl = x / nr, rl = x % nr;
      M[(int64_t)(c0 + cl) * np + r0 + rl] = s_t[rl][cl];
    }
}

// LDS DMA of K chunk j0: the phi slice (panel component 0, 16 groups of 4
// points from pt0, functions j0..j0+15; image [group][function][point % 4],
// the panel's own order) and the M slice (rows j0..j0+15, columns
// i0..i0+63; image [row][column]).  Four wave-wide loads per wave, two rows
// of 512 bytes each.  Groups past the batch's points and columns past np
// load valid entries instead: they only feed tile rows and columns the
// epilogue skips.
__device__ __forceinline__ void gemm_dma(const double *pb, int np, int Pp, int pt0, int j0, const double *M, int i0,
                                         double *sA, double *sB) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int half = lane >> 5, piece = lane & 31;
#pragma unroll
  for (int k = wave; k < 8; k += 4) {
    const int g = min((pt0 >> 2) + 2 * k + half, (Pp >> 2) - 1);
    __builtin_amdgcn_global_load_lds(
        (const void *)(pb + ((int64_t)g * np + j0 + (piece >> 1)) * 4 + 2 * (piece & 1)),
        (lds_void *)(sA + k * 128), 16, 0, 0);
    const int col = min(i0 + 2 * piece, np - 2);
    __builtin_amdgcn_global_load_lds((const void *)(M + (int64_t)(j0 + 2 * k + half) * np + col),
                                     (lds_void *)(sB + k * 128), 16, 0, 0);
  }
}

// The 16 MFMA operands of one K chunk of a wave, A[mb][ks] at pa + 2048 mb +
// 128 ks and B[nb][ks] at pb + 2048 ks + 128 nb (bytes), read in one asm
// block that also waits for them.  Issued by hand so that the compiler, which
// cannot tell these reads from the LDS DMA still in flight into the other
// buffers, does not wait for that DMA first.
__device__ __forceinline__ void read_operands(uint32_t pa, uint32_t pb, double (&a)[2][4], double (&b)[2][4]) {
  asm volatile(
      "ds_read_b64 %0, %16\n"
      "ds_read_b64 %1, %16 offset:128\n"
      "ds_read_b64 %2, %16 offset:256\n"
      "ds_read_b64 %3, %16 offset:384\n"
      "ds_read_b64 %4, %16 offset:2048\n"
      "ds_read_b64 %5, %16 offset:2176\n"
      "ds_read_b64 %6, %16 offset:2304\n"
      "ds_read_b64 %7, %16 offset:2432\n"
      "ds_read_b64 %8, %17\n"
      "ds_read_b64 %9, %17 offset:2048\n"
      "ds_read_b64 %10, %17 offset:4096\n"
      "ds_read_b64 %11, %17 offset:6144\n"
      "ds_read_b64 %12, %17 offset:128\n"
      "ds_read_b64 %13, %17 offset:2176\n"
      "ds_read_b64 %14, %17 offset:4224\n"
      "ds_read_b64 %15, %17 offset:6272\n"
      "s_waitcnt lgkmcnt(0)"
      : "=&v"(a[0][0]), "=&v"(a[0][1]), "=&v"(a[0][2]), "=&v"(a[0][3]), "=&v"(a[1][0]), "=&v"(a[1][1]),
        "=&v"(a[1][2]), "=&v"(a[1][3]), "=&v"(b[0][0]), "=&v"(b[0][1]), "=&v"(b[0][2]), "=&v"(b[0][3]),
        "=&v"(b[1][0]), "=&v"(b[1][1]), "=&v"(b[1][2]), "=&v"(b[1][3])
      : "v"(pa), "v"(pb)
      : "memory");
}

// One output tile: 4 waves, wave w owns points 32 (w & 1) .. +31 and functions
// 32 (w >> 1) .. +31 of the tile as 2 x 2 blocks of 16 x 16 (FP64 MFMA
// 16x16x4: A = phi [point][j], B = M [j][i]).  Three buffers: while chunk kc
// is multiplied, chunk kc + 1 may still be in flight and chunk kc + 2 is
// issued.  Per K chunk each wave reads its 16 operands into registers, issues
// the DMA of chunk kc + 2, then its 16 MFMAs.  Epilogue: per
// (point, function) of the wave the products with phi, 2 d_x phi, 2 d_y phi,
// 2 d_z phi, summed over the wave's functions (lane shuffles) and over the two
// waves of a point range (LDS), written as 4 x 64 partials of the tile.
__global__ __launch_bounds__(256, 2) void k_grad_gemm(DevPlan d, const int32_t *items, int64_t it0, int64_t nit,
                                                      const int64_t *cd_off, const int64_t *part_off,
                                                      const double *cd, const double *panel, double *part) {
  __shared__ double sA[3][GS], sB[3][GS];
  __shared__ double s_red[2][GT][4];
  const int64_t it = it0 + xcd_map(blockIdx.x, nit);
  const int b = items[3 * it], tp = items[3 * it + 1], ti = items[3 * it + 2];
  const int g0 = d.batch_pt_off[b], P = d.batch_pt_off[b + 1] - g0;
  const int n = d.batch_fn_off[b + 1] - d.batch_fn_off[b];
  const int Pp = (int)pad16(P), np = (int)pad16(n);
  const int pt0 = GT * tp, i0 = GT * ti;
  const double *pb = panel + d.panel_off[b];
  const int64_t plane = (int64_t)Pp * np;
  const double *M = cd + cd_off[b];
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int l16 = lane & 15, lk = lane >> 4;
  const int mq = wave & 1, nq = wave >> 1;
  dbl4 acc[2][2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = dbl4{0.0, 0.0, 0.0, 0.0};
  const int nk = np / GK;
  // this lane's operand addresses within a buffer (A: point block 0, K step 0;
  // B: function block 0, K step 0), bytes
  const uint32_t oa = 8u * (uint32_t)((8 * mq + (l16 >> 2)) * 64 + 4 * lk + (l16 & 3));
  const uint32_t ob = 8u * (uint32_t)(lk * GT + 32 * nq + l16);
  gemm_dma(pb, np, Pp, pt0, 0, M, i0, sA[0], sB[0]);
  if (nk > 1) gemm_dma(pb, np, Pp, pt0, GK, M, i0, sA[1], sB[1]);
  for (int kc = 0; kc < nk; ++kc) {
    const int buf = kc % 3;
    // chunk kc has landed everywhere (chunk kc + 1, four loads per wave, may
    // still be in flight); every wave has read chunk kc - 1
    if (kc + 1 < nk)
      barrier_vm<4>();
    else
      barrier_vm<0>();
    double a[2][4], bb[2][4];
    read_operands(lds_addr(sA[buf]) + oa, lds_addr(sB[buf]) + ob, a, bb);
    if (kc + 2 < nk) gemm_dma(pb, np, Pp, pt0, GK * (kc + 2), M, i0, sA[(kc + 2) % 3], sB[(kc + 2) % 3]);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = mfma64(a[mb][ks], bb[nb][ks], acc[mb][nb]);
  }
  // epilogue: lane (l16, lk) register r of block (mb, nb) holds Y at point
  // 32 mq + 16 mb + lk + 4 r of the tile and function 32 nq + 16 nb + l16
  double o[2][4][4];  // [mb][r][n, d_x n, d_y n, d_z n]
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int pg = pt0 + 32 * mq + 16 * mb + d_row_f64(lk, r);
#pragma unroll
      for (int c = 0; c < 4; ++c) o[mb][r][c] = 0.0;
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const int fi = i0 + 32 * nq + 16 * nb + l16;
        if (pg < P && fi < n) {
          const double y = acc[mb][nb][r];
          const double *e = pb + ((int64_t)(pg >> 2) * np + fi) * 4 + (pg & 3);
          o[mb][r][0] += y * e[0];
          o[mb][r][1] += 2.0 * y * e[plane];
          o[mb][r][2] += 2.0 * y * e[2 * plane];
          o[mb][r][3] += 2.0 * y * e[3 * plane];
        }
      }
    }
  // over the 16 functions of a block (the lanes l16 of a lane row)
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        double v = o[mb][r][c];
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        o[mb][r][c] = v;
      }
  if (l16 == 0) {
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) s_red[nq][32 * mq + 16 * mb + d_row_f64(lk, r)][c] = o[mb][r][c];
  }
  barrier_vm<63>();  // the waves' sums are visible
  {
    const int pt = tid >> 2, c = tid & 3;
    if (pt0 + pt < Pp)
      part[part_off[b] + ((int64_t)ti * 4 + c) * Pp + pt0 + pt] = s_red[0][pt][c] + s_red[1][pt][c];
  }
}

// The partials of a point summed over the batch's function tiles in tile
// order: out is [4][n_points] (n, d_x n, d_y n, d_z n) in user point order.
__global__ void k_grad_points(DevPlan d, int64_t b0, const int64_t *part_off, const double *part, double *out) {
  const int64_t b = b0 + blockIdx.x;
  const int g0 = d.batch_pt_off[b], P = d.batch_pt_off[b + 1] - g0;
  const int n = d.batch_fn_off[b + 1] - d.batch_fn_off[b];
  const int Pp = (int)pad16(P), nti = ((int)pad16(n) + GT - 1) / GT;
  const double *pp = part + part_off[b];
  for (int e = threadIdx.x; e < 4 * P; e += blockDim.x) {
    const int c = e / P, g = e - c * P;
    double s = 0.0;
    for (int t = 0; t < nti; ++t) s += pp[((int64_t)t * 4 + c) * Pp + g];
    out[(int64_t)c * d.n_points + d.perm[g0 + g]] = s;
  }
}

}  // namespace

int launch_grad_pass(const q4c_plan *p, size_t ip, const double *coef, const double *panel, double *out,
                     hipStream_t s) {
  const Pass &ps = p->passes[ip];
  const int64_t c0 = p->gr_cd_item_off[ip], nc = p->gr_cd_item_off[ip + 1] - c0;
  const int64_t w0 = p->gr_item_off[ip], nw = p->gr_item_off[ip + 1] - w0;
  if (nc > 0) {
    {
      TimedLaunch tl_(p, Q4C_TIMER_OTHER, s);
      hipLaunchKernelGGL(k_grad_cdense, dim3((unsigned)nc), dim3(256), 0, s, p->dp, p->d_gr_cditems, c0,
                         p->d_gr_cd_off, p->d_gr_fninfo, coef, p->d_gr_cd);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_grad_cdense");
  }
  if (nw > 0) {
    {
      TimedLaunch tl_(p, Q4C_TIMER_DENSITY_TILES, s);
      hipLaunchKernelGGL(k_grad_gemm, dim3((unsigned)nw), dim3(256), 0, s, p->dp, p->d_gr_items, w0, nw,
                         p->d_gr_cd_off, p->d_gr_part_off, (const double *)p->d_gr_cd, panel, p->d_gr_part);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_grad_gemm");
  }
  const int64_t nbt = ps.b1 - ps.b0;
  if (nbt > 0) {
    {
      TimedLaunch tl_(p, Q4C_TIMER_DENSITY_POINTS, s);
      hipLaunchKernelGGL(k_grad_points, dim3((unsigned)nbt), dim3(256), 0, s, p->dp, ps.b0, p->d_gr_part_off,
                         (const double *)p->d_gr_part, out);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "k_grad_points");
  }
  return Q4C_OK;
}

}  // namespace q4c
