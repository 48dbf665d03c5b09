// Device helpers shared by the contraction kernels (q4c_kernels.hip,
// q4c_hs_kernels.hip): MFMA wrappers and lane layouts, work-item mapping and
// persistent queues, wave block slots, staging addresses, LDS DMA of panel
// chunks.  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>
#include <type_traits>

#include "q4c_internal.h"

namespace q4c {
namespace {

typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

constexpr int T = kTile;
constexpr int NT = 256;     // threads per contraction workgroup (4 waves)

// Work items -> workgroups: the hardware hands workgroup id x to XCD x % 8;
// map it so that every XCD runs one contiguous range of work items (the
// tiles of a batch share that XCD's L2).
__device__ __forceinline__ int64_t xcd_map(int64_t bid, int64_t n) {
  const int64_t nx = 8, x = bid % nx, k = bid / nx, q = n / nx, r = n % nx;
  return x * q + (x < r ? x : r) + k;
}

// Persistent launches: workgroups loop over work items drawn from ticket
// counters (zeroed before the launch).  Without an order map the items are
// split into 8 contiguous ranges, one queue per XCD (workgroup x runs on XCD
// x % 8, so a batch's tiles stay on one L2); a workgroup whose queue is empty
// takes items from the next XCD's queue.  With an order map (items sorted by
// cost, largest first) there is one global queue.  Every counter only grows,
// so every workgroup leaves the loop once all queues are drained.
__device__ __forceinline__ int64_t next_item(unsigned *tickets, int64_t nw, bool global_queue, int64_t *s_pos) {
  __syncthreads();  // every thread has read the previous position
  if (threadIdx.x == 0) {
    int64_t pos = nw;
    if (global_queue) {
      const int64_t t = atomicAdd(&tickets[0], 1u);
      if (t < nw) pos = t;
    } else {
      const int x0 = (int)(blockIdx.x & 7);
      for (int k = 0; k < 8 && pos == nw; ++k) {
        const int x = (x0 + k) & 7;
        const int64_t lo = nw * x / 8, hi = nw * (x + 1) / 8;
        if (hi <= lo) continue;
        if ((int64_t)__hip_atomic_load(&tickets[x * kTicketStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
            hi - lo)
          continue;
        const int64_t t = atomicAdd(&tickets[x * kTicketStride], 1u);
        if (lo + t < hi) pos = lo + t;
      }
    }
    *s_pos = pos;
  }
  __syncthreads();
  return *s_pos;
}

// The same queues in two steps, for a workgroup that passes the position on
// through LDS slots of its own: draw_ticket (one thread) adds to its XCD's
// queue (or the global one), ticket_pos turns the ticket into a position and,
// once the own queue is drained, takes one from the other XCDs' queues as
// next_item does.  A drained queue's counter may grow past its range; it is
// never read as a position.
__device__ __forceinline__ unsigned draw_ticket(unsigned *tickets, bool global_queue) {
  return atomicAdd(&tickets[global_queue ? 0 : (int)(blockIdx.x & 7) * kTicketStride], 1u);
}

__device__ __forceinline__ int64_t ticket_pos(unsigned *tickets, int64_t nw, bool global_queue, unsigned tk) {
  if (global_queue) return (int64_t)tk < nw ? (int64_t)tk : nw;
  const int x0 = (int)(blockIdx.x & 7);
  {
    const int64_t lo = nw * x0 / 8, hi = nw * (x0 + 1) / 8;
    if (lo + (int64_t)tk < hi) return lo + (int64_t)tk;
  }
  for (int k = 1; k < 8; ++k) {
    const int x = (x0 + k) & 7;
    const int64_t lo = nw * x / 8, hi = nw * (x + 1) / 8;
    if (hi <= lo) continue;
    if ((int64_t)__hip_atomic_load(&tickets[x * kTicketStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= hi - lo)
      continue;
    const int64_t t = atomicAdd(&tickets[x * kTicketStride], 1u);
    if (lo + t < hi) return lo + t;
  }
  return nw;
}

// lane exchange within rows of 16 lanes by DPP (no LDS traffic): lane i reads
// lane 15 - i (row mirror), 8 (i / 8) + 7 - i % 8 (half-row mirror), i ^ 2 or
// i ^ 1 (quad permutes); a double moves as its two 32-bit halves
constexpr int DPP_QUAD_XOR1 = 0xB1, DPP_QUAD_XOR2 = 0x4E, DPP_ROW_MIRROR = 0x140, DPP_ROW_HALF_MIRROR = 0x141;
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ dbl4 mfma64(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ flt4 mfma32(float a, float b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// BF16 MFMA 16x16x32 with FP32 accumulation; each operand is 8 BF16 values
// (16 bytes) per lane: lane l holds A[l % 16][8 (l / 16) + e] and
// B[8 (l / 16) + e][l % 16], e = 0..7 (element e in bits 16 (e % 2) of word
// e / 2); register r of D is D[4 (l / 16) + r][l % 16].
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ flt4 mfma_bf16(u32x4 a, u32x4 b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

// Staging address of element (li, lj) of a batch (local function indices) for
// part q, given the slot data of li (row) and lj (column).
struct SlotInfo {
  int slot, fnoff, nfn;
  int64_t row_off;
};

__device__ __forceinline__ SlotInfo slot_of(const DevPlan &d, int fbase, int sbase, int lf) {
  SlotInfo s;
  s.slot = d.loc_slot[fbase + lf];
  s.fnoff = d.slot_fnoff[sbase + s.slot];
  s.nfn = d.slot_nfn[sbase + s.slot];
  s.row_off = d.slot_row_off[sbase + s.slot];
  return s;
}

// A value every lane holds alike, as a scalar (wave-uniform) one.
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xFFFFFFFF));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ AdjPos adj_uniform(const AdjPos &a) {
  int w[16];
  __builtin_memcpy(w, &a, sizeof(w));
#pragma unroll
  for (int i = 0; i < 16; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  AdjPos r;
  __builtin_memcpy(&r, w, sizeof(w));
  return r;
}

// Slot, the slot's first local function and its function count of
// batch-local function lf, from the packed table (one load).
struct SlotFn {
  int slot, fnoff, nfn;
};
__device__ __forceinline__ SlotFn slot_fn(const DevPlan &d, int fbase, int lf) {
  const int64_t v = d.loc_info[fbase + lf];
  return SlotFn{(int)(v & 0xFFFFF), (int)((v >> 20) & 0xFFFFF), (int)(v >> 40)};
}

// The five parts: 0 V, 1 Ws, 2 Wso_x, 3 Wso_y, 4 Wso_z.  Mirror sign under
// (i, j) -> (j, i): + for V, Ws; - for the spin-orbit parts.
__device__ __forceinline__ double mirror_sign(int q) { return q >= 2 ? -1.0 : 1.0; }

// Which 16 x 16 blocks of a batch's local n x n matrix are computed: blocks
// (rb, cb) with rb <= cb (block starts), both inside n.  A strictly upper
// block (rb < cb) also stands for its mirror block (cb, rb), which no work
// item computes.
__device__ __forceinline__ bool block_active(int rb, int cb, int n) { return rb < n && cb < n && rb <= cb; }

// The active 16 x 16 blocks of tile (r0, c0) (inside n, on or above the
// diagonal), listed 2 x 2 square by square; wave w of four takes list entries
// [w nb / 4, (w+1) nb / 4): at most one block more than another wave, and a
// full tile gives every wave one 2 x 2 square.  Slot s of the wave holds block
// (brow[s], bcol[s]) (tile-local offsets) when act[s]; the active slots are
// 0 .. count-1, inactive ones point at block (0, 0).
__device__ __forceinline__ void wave_blocks(int r0, int c0, int n, int wave, int (&brow)[4], int (&bcol)[4],
                                            bool (&act)[4]) {
  int nb = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int R = 2 * (k >> 3) + ((k >> 1) & 1), C = 2 * ((k >> 2) & 1) + (k & 1);
    nb += block_active(r0 + 16 * R, c0 + 16 * C, n) ? 1 : 0;
  }
  const int kb0 = wave * nb / 4, kb1 = (wave + 1) * nb / 4;
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    brow[sl] = 0;
    bcol[sl] = 0;
    act[sl] = false;
  }
  int cnt = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int R = 2 * (k >> 3) + ((k >> 1) & 1), C = 2 * ((k >> 2) & 1) + (k & 1);
    if (block_active(r0 + 16 * R, c0 + 16 * C, n)) {
#pragma unroll
      for (int sl = 0; sl < 4; ++sl)
        if (cnt == kb0 + sl && cnt < kb1) {
          brow[sl] = 16 * R;
          bcol[sl] = 16 * C;
          act[sl] = true;
        }
      ++cnt;
    }
  }
}

// Write one accumulated element (li, lj) of a computed block to the staged
// (batch, atom pair) block; `upper` = the element's block is strictly upper.
template <int Q0, int Q1>
__device__ __forceinline__ void stage_store(double *staging, const SlotInfo &si, const SlotInfo &sj, int li, int lj,
                                            bool upper, const double *v) {
  if (si.slot > sj.slot) return;  // lower atom-block triangle: not stored
  const int64_t blk = si.row_off + 5 * (int64_t)si.nfn * (sj.fnoff - si.fnoff);
  const int64_t pq = (int64_t)si.nfn * sj.nfn;
  const int64_t e = (int64_t)(li - si.fnoff) * sj.nfn + (lj - sj.fnoff);
#pragma unroll
  for (int q = Q0; q < Q1; ++q) staging[blk + q * pq + e] = v[q - Q0];
  if (upper && si.slot == sj.slot) {
    // the mirrored element (lj, li) of the same atom block lies in a block
    // that is never computed
    const int64_t em = (int64_t)(lj - si.fnoff) * sj.nfn + (li - sj.fnoff);
#pragma unroll
    for (int q = Q0; q < Q1; ++q) staging[blk + q * pq + em] = mirror_sign(q) * v[q - Q0];
  }
}

// As stage_store, adding to the staged element (and its mirror) instead.
template <int Q0, int Q1>
__device__ __forceinline__ void stage_add(double *staging, const SlotInfo &si, const SlotInfo &sj, int li, int lj,
                                          bool upper, const double *v) {
  if (si.slot > sj.slot) return;
  const int64_t blk = si.row_off + 5 * (int64_t)si.nfn * (sj.fnoff - si.fnoff);
  const int64_t pq = (int64_t)si.nfn * sj.nfn;
  const int64_t e = (int64_t)(li - si.fnoff) * sj.nfn + (lj - sj.fnoff);
#pragma unroll
  for (int q = Q0; q < Q1; ++q) staging[blk + q * pq + e] += v[q - Q0];
  if (upper && si.slot == sj.slot) {
    const int64_t em = (int64_t)(lj - si.fnoff) * sj.nfn + (li - sj.fnoff);
#pragma unroll
    for (int q = Q0; q < Q1; ++q) staging[blk + q * pq + em] += mirror_sign(q) * v[q - Q0];
  }
}

// MFMA 16x16x4 lane layouts (lane l, l16 = l % 16, lk = l / 16):
//   A[i][k]: lane i + 16 k;  B[k][j]: lane j + 16 k;
//   D (f64_16x16x4): register r of lane l holds D[lk + 4 r][l16];
//   D (f32_16x16x4): register r of lane l holds D[4 lk + r][l16].
__device__ __forceinline__ int d_row_f64(int lk, int r) { return lk + 4 * r; }
__device__ __forceinline__ int d_row_f32(int lk, int r) { return 4 * lk + r; }


// LDS image of one 16-point chunk of a 64-function tile, in the panel's own
// order: row (q, u) holds component q at points 2u and 2u+1 of the chunk,
// the two points of function f as consecutive doubles, so element (q, pt, f)
// sits at (q*8 + pt/2)*DROW + 2f + pt%2.  Each row is one 1 KB run of the
// panel (64 functions x 16 bytes) and is filled by one wave-wide LDS DMA
// load: no registers are involved, and all loads of a chunk are in flight at
// once.
constexpr int DROW = 2 * T;  // doubles per LDS row
typedef __attribute__((address_space(3))) void lds_void;

// Workgroup barrier after this wave's LDS operations have completed and at
// most VM of its vector-memory operations remain outstanding (s_waitcnt
// vmcnt(VM) lgkmcnt(0)).  The LDS DMA loads count in vmcnt.  __syncthreads
// would also fence global memory; the memory clobber keeps the compiler from
// moving memory accesses across the barrier.
template <int VM>
__device__ __forceinline__ void barrier_vm() {
  static_assert(VM >= 0 && VM < 64, "vmcnt field");
  __builtin_amdgcn_s_waitcnt((VM & 15) | ((VM >> 4) << 14) | (0x7 << 4));
  asm volatile("s_barrier" ::: "memory");
}

// LDS byte address of a __shared__ array element
__device__ __forceinline__ uint32_t lds_addr(const double *p) {
  return (uint32_t)(uintptr_t)(const lds_void *)(const void *)p;
}

// Calls f(std::integral_constant<int, K>) for K = K0, K0 + S, ... < K1, as
// straight-line code with K a constant expression in f.
template <int K0, int S, class F, int... I>
__device__ __forceinline__ void static_for_seq(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, K0 + S * I>{}), ...);
}
template <int K0, int K1, int S = 1, class F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_seq<K0, S>(f, std::make_integer_sequence<int, (K1 - K0 + S - 1) / S>{});
}

// Issue the LDS DMA loads of one chunk of CH points (panel K steps ks0 ..
// ks0 + CH/4 - 1) of functions row0 .. row0+T-1 into dst (4 * CH/2 rows of
// DROW doubles, spread over the waves; element (q, pt, f) of the chunk at
// (q * CH/2 + pt/2) * DROW + 2f + pt%2).  Functions at
// or beyond np are not loaded: their LDS entries are stale and lie in 16x16
// blocks that are never multiplied (rows n .. np-1 are zero in the panel).
// W < 64 loads only the first W functions (lanes W.. idle); RS is the row
// stride in doubles (at least 2 W, a multiple of 2).  The caller waits for
// the loads (vmcnt) and synchronises the workgroup.
template <int NTH, int CH = 16, int W = T, int RS = DROW, int NQ = 4>
__device__ __forceinline__ void dma_chunk(const double *pb, int64_t plane, int np, int row0, int ks0, double *dst) {
  constexpr int RPQ = CH / 2;  // rows (point pairs) per component; NQ components
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool ok = lane < W && row0 + lane < np;
#pragma unroll
  for (int k = 0; k < NQ * RPQ / (NTH / 64); ++k) {
    const int r = wave + k * (NTH / 64);
    const int q = r / RPQ, u = r % RPQ;
    if (ok)
      __builtin_amdgcn_global_load_lds(
          (const void *)(pb + q * plane + ((int64_t)(ks0 + (u >> 1)) * np + row0 + lane) * 4 + 2 * (u & 1)),
          (lds_void *)(dst + r * RS), 16, 0, 0);
  }
}

}  // namespace
}  // namespace q4c
