// The contraction of q4c_integrate_HS: H and S of one component, the Q4C
// integrand of Eq. 19 in the scalar form of Eq. 29, symmetrised.  The panel
// tabulation, batch sums and launches around it are in q4c_kernels.hip.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "q4c_internal.h"
#include "q4c_device.h"

namespace q4c {
namespace {

// H and S of one component (the Q4C integrand of Eq. 19 in the scalar form
// of Eq. 29, symmetrised), from panels of phi and psi = u phi / 2:
//   H = Phi^T diag(w) (v Phi + Psi) + Psi^T diag(w) Phi,   S = Phi^T diag(w) Phi
// i.e. per 16 x 16 block and K step of 4 points three FP64 MFMAs: the row
// operands phi_i, psi_i against the column operands w v phi_j + w psi_j and
// w phi_j (shared by the psi_i phi_j part of H and by S).  Same tiles, wave
// slots and staging as the forward contraction; chunks of 16 points in two
// LDS buffers (two components), the next chunk's DMA and weights in flight
// while this one is multiplied.
template <bool PERSIST>
__global__ __launch_bounds__(NT, 2) void k_contract_hs(DevPlan d, const WorkItem *work, const int32_t *order,
                                                       int64_t w0, int64_t nw, const double *om,
                                                       const double *panel, double *staging, unsigned *tickets) {
  constexpr int CH = 16, RPQ = CH / 2, NQ = 2;
  constexpr int BUFD = NQ * RPQ * DROW;  // doubles per chunk image
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
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li16 = lane & 15, lk = lane >> 4;
  int brow[4], bcol[4];
  bool act[4];
  wave_blocks(r0, c0, n, wave, brow, bcol, act);
  dbl4 acc[4][3];  // H (v phi + psi part), S, H (psi phi part)
#pragma unroll
  for (int sl = 0; sl < 4; ++sl)
#pragma unroll
    for (int q = 0; q < 3; ++q) acc[sl][q] = dbl4{0.0, 0.0, 0.0, 0.0};
  // K steps in pairs over 8 points (K index lk: point 2 lk of the 8, then
  // 2 lk + 1), one 16-byte LDS read per operand for both; weights at the
  // points this lane's K index visits in the next chunk: w v and w
  double omn[CH / 4], wn[CH / 4];
  auto load_w = [&](int k) {
#pragma unroll
    for (int ks = 0; ks < CH / 4; ++ks) {
      const int pt = k + 8 * (ks >> 1) + 2 * lk + (ks & 1);
      omn[ks] = pt < P ? om[g0 + pt] : 0.0;
      wn[ks] = pt < P ? d.pw[g0 + pt] : 0.0;
    }
  };
  load_w(0);
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
  for (int k0 = 0; k0 < Pp; k0 += CH) {
    const int bo = ((k0 / CH) & 1) * BUFD;
    double omv[CH / 4], wv[CH / 4];
    __builtin_amdgcn_s_waitcnt(0);  // this thread's loads of this chunk have landed
    __syncthreads();                // ... everyone's; the previous chunk is consumed
#pragma unroll
    for (int ks = 0; ks < CH / 4; ++ks) {
      omv[ks] = omn[ks];
      wv[ks] = wn[ks];
    }
    if (k0 + CH < Pp) {
      const int nbo = BUFD - bo;
      load_w(k0 + CH);
      dma_chunk<NT, CH, T, DROW, NQ>(pb, plane, np, r0, (k0 + CH) >> 2, sa + nbo);
      dma_chunk<NT, CH, T, DROW, NQ>(pb, plane, np, c0, (k0 + CH) >> 2, sb + nbo);
    }
    const double *ca = sa + bo, *cb = sb + bo;
#pragma unroll
    for (int kp = 0; kp < CH / 8; ++kp) {
      const int row = 4 * kp + lk;  // image row: points 8 kp + 2 lk, + 1
#pragma unroll
      for (int sl = 0; sl < 4; ++sl) {
        if (!act[sl]) continue;  // wave-uniform
        const dbl2 fi2 = *reinterpret_cast<const dbl2 *>(&ca[row * DROW + 2 * (brow[sl] + li16)]);
        const dbl2 pi2 = *reinterpret_cast<const dbl2 *>(&ca[(RPQ + row) * DROW + 2 * (brow[sl] + li16)]);
        const dbl2 fj2 = *reinterpret_cast<const dbl2 *>(&cb[row * DROW + 2 * (bcol[sl] + li16)]);
        const dbl2 pj2 = *reinterpret_cast<const dbl2 *>(&cb[(RPQ + row) * DROW + 2 * (bcol[sl] + li16)]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int ks = 2 * kp + h;
          const double bw = wv[ks] * fj2[h];                    // w phi_j
          const double bh = omv[ks] * fj2[h] + wv[ks] * pj2[h];  // w v phi_j + w psi_j
          acc[sl][0] = mfma64(fi2[h], bh, acc[sl][0]);
          acc[sl][1] = mfma64(fi2[h], bw, acc[sl][1]);
          acc[sl][2] = mfma64(pi2[h], bw, acc[sl][2]);
        }
      }
    }
  }
  // write the computed blocks (H, S) to the staged atom-pair blocks
#pragma unroll
  for (int sl = 0; sl < 4; ++sl) {
    if (!act[sl]) continue;
    const int cb = c0 + bcol[sl];
    const int lj = cb + li16;
    if (lj >= n) continue;
    const int cj = T + bcol[sl] + li16;
    const SlotInfo sj{s_fslot[cj], s_ffn[cj], s_fnf[cj], s_frow[cj]};
    const int rb = r0 + brow[sl];
    const bool upper = rb < cb;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int li = rb + d_row_f64(lk, r);
      if (li < n) {
        const int ri = li - r0;
        const SlotInfo si{s_fslot[ri], s_ffn[ri], s_fnf[ri], s_frow[ri]};
        double vals[2];
        vals[0] = acc[sl][0][r] + acc[sl][2][r];
        vals[1] = acc[sl][1][r];
        stage_store<0, 2>(staging, si, sj, li, lj, upper, vals);
      }
    }
  }
  if (!PERSIST) break;
  pos = next_item(tickets, nw, order != nullptr, &s_pos);
  }
}

}  // namespace

int launch_contract_hs(const q4c_plan *p, int64_t w0, int64_t nw, const int32_t *order, const double *panel,
                       unsigned *tickets, unsigned grid, hipStream_t s) {
  if (tickets)
    hipLaunchKernelGGL(k_contract_hs<true>, dim3(grid), dim3(NT), 0, s, p->dp, p->d_work, order, w0, nw, p->d_om,
                       panel, p->d_staging, tickets);
  else
    hipLaunchKernelGGL(k_contract_hs<false>, dim3(grid), dim3(NT), 0, s, p->dp, p->d_work, order, w0, nw, p->d_om,
                       panel, p->d_staging, tickets);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_contract_hs");
  return Q4C_OK;
}

}  // namespace q4c
