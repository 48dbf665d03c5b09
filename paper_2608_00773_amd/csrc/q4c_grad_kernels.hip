// The tile kernel of density_gradient_on_grid: the density and its gradient
// from one real coefficient part C on the stored pairs (a scalar density
// matrix of one component, the forward density update of Eq. 39 with the
// gradient a GGA needs).  The panel tabulation, the per-point sums and the
// launches around it are in q4c_kernels.hip.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "q4c_internal.h"
#include "q4c_device.h"

namespace q4c {
namespace {

constexpr int NTG = 256;     // 4 waves = 2 column slices x 2 row halves of a column half
constexpr int RSA = 2 * T + 2;   // LDS row stride of the 64 row functions (2 mod 16: 16 points hit distinct banks)
constexpr int RSB = T + 2;       // ... of the 32 column functions

// LDS DMA of components [Q0, Q1) of one 16-point chunk of W functions from
// row0 into dst (the image layout of dma_chunk, from component Q0: element
// (q, pt, f) at ((q - Q0) * 8 + pt / 2) * RS + 2 f + pt % 2).  Every wave issues the same number of
// load instructions whatever np is, so that a partial vmcnt wait counts the
// same loads in every wave: lanes below W whose function lies at or beyond np
// load function np - 1 instead (into padding entries that lie only in 16 x 16
// blocks that are never multiplied); lanes from W on are masked off.
template <int W, int RS, int Q0, int Q1>
__device__ __forceinline__ void dma_comps(const double *pb, int64_t plane, int np, int row0, int ks0, double *dst) {
  constexpr int RPQ = 8;  // point pairs per component
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int f = min(row0 + lane, np - 1);
#pragma unroll
  for (int k = 0; k < (Q1 - Q0) * RPQ / (NTG / 64); ++k) {
    const int r = Q0 * RPQ + wave + k * (NTG / 64);
    const int q = r / RPQ, u = r % RPQ;
    if (W == 64 || lane < W)
      __builtin_amdgcn_global_load_lds((const void *)(pb + q * plane + ((int64_t)(ks0 + (u >> 1)) * np + f) * 4 + 2 * (u & 1)),
                                       (lds_void *)(dst + (r - Q0 * RPQ) * RS), 16, 0, 0);
  }
}

// Workgroup barrier after this wave's LDS operations have completed and at
// most VM of its vector-memory operations remain outstanding (s_waitcnt
// vmcnt(VM) lgkmcnt(0); VM = 63 waits for none).  The LDS DMA loads count in
// vmcnt.  __syncthreads would
// also fence global memory, i.e. wait for every outstanding load; the memory
// clobber keeps the compiler from moving memory accesses across the barrier.
template <int VM>
__device__ __forceinline__ void barrier_vm() {
  static_assert(VM >= 0 && VM < 64, "vmcnt field");
  __builtin_amdgcn_s_waitcnt((VM & 15) | ((VM >> 4) << 14) | (0x7 << 4));
  asm volatile("s_barrier" ::: "memory");
}

// One half of a work item (positions 2 w + half): for the tile's 64 rows i
// and the half's 32 columns j with effective coefficients K (the stored
// coefficient, plus its mirror inside one atom block's strictly upper 16 x 16
// blocks), per point
//   n     = sum_ij K_ij phi_i phi_j      = sum_j u_j phi_j,
//   d_a n = sum_ij K_ij d_a(phi_i phi_j) = sum_j u_j d_a phi_j + sum_i v_i d_a phi_i,
// with u = K^T phi_rows and v = K phi_cols: two MFMA products per 16-point
// chunk (8 + 8 FP64 MFMAs per wave, four independent chains issued together
// and consumed once), the rest lane-local.  Each wave holds its 32 x 16 slice
// of K twice in registers: as the first operand of K^T phi (lane = column) and
// of K phi (lane = row).  Four partials per point and column half, written in
// the layout the per-point sum reads.
template <bool PERSIST>
__global__ __launch_bounds__(NTG, 2) void k_grad_tiles(DevPlan d, const WorkItem *work, const int32_t *order,
                                                       int64_t w0, int64_t nw, const double *coef,
                                                       const double *panel, double *partial, unsigned *tickets) {
  // chunk images: phi (the MFMA operands; two buffers, the next chunk's
  // arrives while this one is multiplied) and the three gradient components
  __shared__ double sa0[2][8 * RSA], sa1[24 * RSA], sb0[2][8 * RSB], sb1[24 * RSB];
  __shared__ double s_red[2][4][4][16];  // per-wave point sums of n, d_x n, d_y n, d_z n, alternating chunks
  __shared__ int64_t s_pos;
  __shared__ int s_rslot[T], s_rfn[T], s_cslot[T / 2], s_cfn[T / 2], s_cnf[T / 2];
  // stored pair of (row slot, column slot) for the slots the tile spans (-1:
  // lower atom-block triangle or not a stored pair)
  __shared__ int s_pq[T * T / 2];
  const int64_t npos = 2 * nw;
  int64_t pos = PERSIST ? next_item(tickets, npos, order != nullptr, &s_pos)
                        : (order ? (int64_t)blockIdx.x : xcd_map(blockIdx.x, npos));
  while (!PERSIST || pos < npos) {
  const int half = (int)(pos & 1);
  const int64_t wi = w0 + (order ? order[w0 + (pos >> 1)] : (pos >> 1));
  const WorkItem it = work[wi];
  const int b = it.batch;
  const int g0 = d.batch_pt_off[b], P = d.batch_pt_off[b + 1] - g0;
  const int f0 = d.batch_fn_off[b], n = d.batch_fn_off[b + 1] - f0;
  const int sbase = d.batch_slot_off[b];
  const int r0 = it.ti * T, c0 = it.tj * T + 32 * half;
  const int Pp = (int)pad16(P), np = (int)pad16(n);
  const double *pb = panel + d.panel_off[b];
  const int64_t plane = (int64_t)Pp * np;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int js = wave & 1, ih = wave >> 1;  // column slice, row half
  const int l16 = lane & 15, lk = lane >> 4;
  const int cb = c0 + 16 * js;  // column block of this wave
  // row origin of this wave's two row blocks.  Column half 0 of a diagonal
  // tile has 3 active blocks, (0,0), (0,1) and (1,1) in 16-blocks: block (1,1)
  // moves from wave (ih 0, js 1) to the otherwise idle wave (ih 1, js 1).
  const bool dg0 = it.ti == it.tj && half == 0;
  const int iloc = (dg0 && ih == 1 && js == 1) ? 16 : 32 * ih;
  bool act[2], upper[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int rb = r0 + iloc + 16 * h;
    act[h] = block_active(rb, cb, n) && !(dg0 && ih == 0 && js == 1 && h == 1);
    upper[h] = rb < cb;
  }
  if (tid < T + T / 2) {
    const bool row = tid < T;
    const int lf = row ? r0 + tid : c0 + tid - T;
    SlotInfo si{-1, 0, 0, 0};
    if (lf < n) si = slot_of(d, f0, sbase, lf);
    if (row) {
      s_rslot[tid] = si.slot;
      s_rfn[tid] = si.fnoff;
    } else {
      s_cslot[tid - T] = si.slot;
      s_cfn[tid - T] = si.fnoff;
      s_cnf[tid - T] = si.nfn;
    }
  }
  __syncthreads();  // slot tables visible
  const int rs0 = s_rslot[0], cs0 = s_cslot[0];
  int rs1 = rs0, cs1 = cs0;
  if (rs0 >= 0) rs1 = s_rslot[min(T, n - r0) - 1];
  if (cs0 >= 0) cs1 = s_cslot[min(T / 2, n - c0) - 1];
  const int nrs = rs0 >= 0 ? rs1 - rs0 + 1 : 0, ncs = cs0 >= 0 ? cs1 - cs0 + 1 : 0;
  {
    const int ns = d.batch_slot_off[b + 1] - sbase;
    const int64_t spb = d.batch_sp_off[b];
    for (int t = tid; t < nrs * ncs; t += NTG) {
      const int si = rs0 + t / ncs, sj = cs0 + t % ncs;
      s_pq[t] = si <= sj ? d.sp_pair[spb + (int64_t)si * ns - (int64_t)si * (si - 1) / 2 + (sj - si)] : -1;
    }
  }
  __syncthreads();  // pair offsets visible
  // K at tile row rl (0..63) and half column cl (0..31) of row block h: the
  // stored element of the two atoms' pair block (upper atom-block triangle),
  // plus the mirrored element when the 16 x 16 block is strictly upper inside
  // one atom block (no work item computes the mirrored block); 0 off the
  // active blocks.
  // Both loads are unconditional (element 0 of the store, always present,
  // stands in for an absent element) and selected afterwards, so that the
  // loads of all 16 elements of a thread are in flight together.
  auto kval = [&](int rl, int cl, int h) -> double {
    const int rslot = s_rslot[rl], cslot = s_cslot[cl];
    const int pq = (act[h] && rslot >= 0 && cslot >= 0) ? s_pq[(rslot - rs0) * ncs + (cslot - cs0)] : -1;
    const bool live = pq >= 0;
    const int64_t po = d.pair_off[live ? pq : 0];
    const bool mir = live && upper[h] && rslot == cslot;
    const int li = r0 + rl, lj = c0 + cl;
    const int rfn = s_rfn[rl], cfn = s_cfn[cl], cnf = s_cnf[cl];
    const double c = coef[live ? po + (int64_t)(li - rfn) * cnf + (lj - cfn) : 0];
    const double cm = coef[mir ? po + (int64_t)(lj - rfn) * cnf + (li - cfn) : 0];
    return (live ? c : 0.0) + (mir ? cm : 0.0);
  };
  // kt: first operand of u = K^T phi_rows, lane (l16 = column, lk) step ks:
  //     K[iloc + 4 ks + lk][16 js + l16];
  // kr: first operand of v = K phi_cols, lane (l16 = row, lk) row block h,
  //     step s: K[iloc + 16 h + l16][16 js + 4 s + lk].
  double kt[8], kr[2][4];
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) kt[ks] = kval(iloc + 4 * ks + lk, 16 * js + l16, ks >> 2);
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) kr[h][s4] = kval(iloc + 16 * h + l16, 16 * js + 4 * s4 + lk, h);
  // materialise the slices here: left to itself the compiler sinks the
  // selects into the chunk loop, where the wait for their loads (unknown
  // count across the back edge) would also wait for the chunk's DMA
#pragma unroll
  for (int ks = 0; ks < 8; ++ks) asm volatile("" : "+v"(kt[ks]));
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) asm volatile("" : "+v"(kr[h][s4]));
  double *out = partial + 8 * d.work_part_off[wi] + half * 4 * P;
  const int jloc = 16 * js;

  // Per chunk: phi of this chunk is in LDS buffer pbuf (its DMA was issued
  // during the previous chunk); phi goes to registers, then this chunk's
  // gradient components and the next chunk's phi are issued together and land
  // while the MFMAs run; one wait, then the lane-local products.
  dma_comps<T, RSA, 0, 1>(pb, plane, np, r0, 0, sa0[0]);
  dma_comps<T / 2, RSB, 0, 1>(pb, plane, np, c0, 0, sb0[0]);
  for (int k0 = 0; k0 < Pp; k0 += 16) {
    const int rb2 = (k0 >> 4) & 1, pbuf = rb2;
    // this chunk's phi has landed everywhere; the previous chunk's images are
    // consumed and its per-wave sums visible
    barrier_vm<0>();
    if (k0 > 0 && tid < 64 && k0 - 16 + (tid & 15) < P) {
      const int o = tid >> 4, t = tid & 15;
      out[o * P + k0 - 16 + t] = (s_red[rb2 ^ 1][0][o][t] + s_red[rb2 ^ 1][1][o][t]) +
                                 (s_red[rb2 ^ 1][2][o][t] + s_red[rb2 ^ 1][3][o][t]);
    }
    auto issue_loads = [&]() {
      dma_comps<T, RSA, 1, 4>(pb, plane, np, r0, k0 >> 2, sa1);
      dma_comps<T / 2, RSB, 1, 4>(pb, plane, np, c0, k0 >> 2, sb1);
      if (k0 + 16 < Pp) {  // the next chunk's phi, into the other buffer (last read in the previous chunk)
        dma_comps<T, RSA, 0, 1>(pb, plane, np, r0, (k0 + 16) >> 2, sa0[pbuf ^ 1]);
        dma_comps<T / 2, RSB, 0, 1>(pb, plane, np, c0, (k0 + 16) >> 2, sb0[pbuf ^ 1]);
      }
    };
    // image element (component q, point pt of the chunk, function f)
    auto A0 = [&](int f) { return sa0[pbuf][(l16 >> 1) * RSA + 2 * f + (l16 & 1)]; };
    auto A1 = [&](int a, int f) { return sa1[((a - 1) * 8 + (l16 >> 1)) * RSA + 2 * f + (l16 & 1)]; };
    auto B0 = [&](int f) { return sb0[pbuf][(l16 >> 1) * RSB + 2 * f + (l16 & 1)]; };
    auto B1 = [&](int a, int f) { return sb1[((a - 1) * 8 + (l16 >> 1)) * RSB + 2 * f + (l16 & 1)]; };
    double xg[4][4];
#pragma unroll
    for (int o = 0; o < 4; ++o)
#pragma unroll
      for (int r = 0; r < 4; ++r) xg[o][r] = 0.0;
    // Both products over the K steps of the active row blocks [H0, H1), as
    // straight-line code: all MFMAs issued before any result is read.
    auto chunk = [&](auto h0c, auto h1c) {
      constexpr int H0 = decltype(h0c)::value, H1 = decltype(h1c)::value;
      double ya[8], yb[4];
#pragma unroll
      for (int ks = 4 * H0; ks < 4 * H1; ++ks) ya[ks] = A0(iloc + 4 * ks + lk);  // phi_i, B[k = i][n = pt]
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) yb[s4] = B0(jloc + 4 * s4 + lk);          // phi_j, B[k = j][n = pt]
      // the reads of phi stay ahead of the DMA (no LDS read waits for a DMA
      // in flight)
      __builtin_amdgcn_sched_barrier(0);
      issue_loads();
      dbl4 u0 = dbl4{0.0, 0.0, 0.0, 0.0}, u1 = u0, v[2] = {u0, u0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        if (H1 - H0 == 2) {
          u0 = mfma64(kt[2 * s4], ya[2 * s4], u0);
          u1 = mfma64(kt[2 * s4 + 1], ya[2 * s4 + 1], u1);
        } else if ((s4 & 1) == 0) {
          u0 = mfma64(kt[4 * H0 + s4], ya[4 * H0 + s4], u0);
          u1 = mfma64(kt[4 * H0 + s4 + 1], ya[4 * H0 + s4 + 1], u1);
        }
#pragma unroll
        for (int h = H0; h < H1; ++h) v[h] = mfma64(kr[h][s4], yb[s4], v[h]);
      }
      __builtin_amdgcn_sched_barrier(0);  // every MFMA issued before the wait for the loads
      barrier_vm<0>();                    // every wave's gradient images (and next phi) have landed
      // column values at (pt = l16, j = jloc + lk + 4 r): phi, d_x, d_y, d_z
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = jloc + d_row_f64(lk, r);
        const double u = u0[r] + u1[r];
        xg[0][r] += u * B0(j);
#pragma unroll
        for (int a = 1; a < 4; ++a) xg[a][r] += u * B1(a, j);
      }
      // row values at (pt = l16, i = iloc + 16 h + lk + 4 r): d_x, d_y, d_z
#pragma unroll
      for (int h = H0; h < H1; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = iloc + 16 * h + d_row_f64(lk, r);
#pragma unroll
          for (int a = 1; a < 4; ++a) xg[a][r] += v[h][r] * A1(a, i);
        }
    };
    if (act[0] && act[1])
      chunk(std::integral_constant<int, 0>{}, std::integral_constant<int, 2>{});
    else if (act[0])
      chunk(std::integral_constant<int, 0>{}, std::integral_constant<int, 1>{});
    else if (act[1])
      chunk(std::integral_constant<int, 1>{}, std::integral_constant<int, 2>{});
    else {
      // no active block: the same loads and barriers as the others
      issue_loads();
      barrier_vm<0>();
    }
    // sum over the wave's 16 columns (and 32 rows): the 4 registers, then the 4 lane rows
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      double sx = (xg[o][0] + xg[o][1]) + (xg[o][2] + xg[o][3]);
      sx += __shfl_xor(sx, 16);
      sx += __shfl_xor(sx, 32);
      if (lane < 16) s_red[rb2][wave][o][l16] = sx;
    }
  }
  barrier_vm<63>();  // the last chunk's per-wave sums
  {
    const int k0 = Pp - 16, rb2 = (k0 >> 4) & 1;
    if (tid < 64 && k0 + (tid & 15) < P) {
      const int o = tid >> 4, t = tid & 15;
      out[o * P + k0 + t] = (s_red[rb2][0][o][t] + s_red[rb2][1][o][t]) + (s_red[rb2][2][o][t] + s_red[rb2][3][o][t]);
    }
  }
  if (!PERSIST) break;
  pos = next_item(tickets, npos, order != nullptr, &s_pos);
  }
}

}  // namespace

int launch_grad_tiles(const q4c_plan *p, int64_t w0, int64_t nw, const int32_t *order, const double *coef,
                      const double *panel, double *gpart, unsigned *tickets, unsigned grid, hipStream_t s) {
  if (tickets)
    hipLaunchKernelGGL(k_grad_tiles<true>, dim3(grid), dim3(NTG), 0, s, p->dp, p->d_work, order, w0, nw, coef, panel,
                       gpart, tickets);
  else
    hipLaunchKernelGGL(k_grad_tiles<false>, dim3(grid), dim3(NTG), 0, s, p->dp, p->d_work, order, w0, nw, coef, panel,
                       gpart, tickets);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_grad_tiles");
  return Q4C_OK;
}

}  // namespace q4c
