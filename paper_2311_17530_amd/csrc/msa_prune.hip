// msa_prune.hip -- exact tile pruning (pruned mode, 3 <= k <= 6).
//
// Section 6 of the paper proposes computing only the partitions where an
// optimal alignment can lie.  This file makes that selection exact with the
// pairwise bound of Carrillo and Lipman: the sum-of-pairs score of any
// alignment through cell v is at most
//     B(v) = sum_{i<j} F_ij[v_i][v_j] + G_ij[v_i][v_j]
// (F: optimal pairwise score of the prefixes, G: of the suffixes), so a tile
// whose bound sum_{i<j} max_{tile}(F_ij + G_ij) is below a lower bound L of
// the optimum holds no cell of any optimal alignment and is skipped.
//
// Launch sequence of one pruned fill (all on one stream, no host round trip):
//   pair_table_kernel     F and G of every pair (one wave per table)
//   pair_blockmax_kernel  per pair and tile pair: max of F + G; U and L1
//   select / scan / compact (pass 1)   keep flags, kept-tile queue
//   fill_kernel (pass 1)  kept tiles only
//   prune_check_kernel    end score s >= L1: exact, done; else L2 = s
//   select / scan / compact / fill (pass 2)   run only after a miss
// A pass whose end score reaches its threshold is exact: the score of a
// kept-only path never exceeds the optimum, and a threshold at or below the
// optimum keeps every cell of every optimal alignment (whose values, and the
// lowest-mask choices between them, are then those of the full tensor).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msa_internal.h"

namespace msa {

namespace {

enum { ST_OK = 0 };

constexpr int kRB = 16;           // rows per lane in one band (band = 1024 rows)
// largest number of tiles along a dimension (T >= 3 for k <= 6)
constexpr int kMaxTilesPerDim = 1 + (kPruneMaxLen - 1 + 2) / 3;

// ---------------------------------------------------------------------------
// Pairwise tables.  Workgroup 2p + d computes table d of pair p = (i, j):
//   d = 0: F[a][b] = best score of s_i[:a] against s_j[:b]
//   d = 1: G[a][b] = best score of s_i[a:] against s_j[b:], computed as the
//          prefix table of the reversed sequences and stored mirrored.
// Both are column-major: (a, b) at b * (n_i + 1) + a.  Standard
// Needleman-Wunsch recurrence (the k = 2 case of Eq. 1 with the Section 5.2
// scores): F[a][b] = max(F[a-1][b] + g, F[a][b-1] + g, F[a-1][b-1] + sub).
//
// One wave per table, rows in bands of 64 * RB: lane l holds rows
// base + l*RB .. base + l*RB + RB - 1 and handles column b = s - l at step s
// (an anti-diagonal pipeline).  The value above a lane's first row arrives
// from the lane below by a one-lane wave shift (DPP), together with the
// column's residue; lane 0 reads the band's upper boundary (the previous
// band's last row) from the table, 64 columns per load.  The substitution
// matrix sits in LDS, so the step loop issues no global load but those
// 64-column refills (on gfx9 a wait for a load also waits for every earlier
// store, and each step stores its cells).
// ---------------------------------------------------------------------------

// Lane l receives lane l - 1's value, lane 0 receives `first` (DPP wave_shr:1).
__device__ __forceinline__ int shift_up1(int v, int first) {
  return __builtin_amdgcn_update_dpp(first, v, 0x138, 0xF, 0xF, false);
}

__global__ __launch_bounds__(64) void pair_table_kernel(PruneDev pd, const Ctrl *ctrl) {
  const int p = blockIdx.x >> 1;
  const int dir = blockIdx.x & 1;
  if (p >= pd.npairs) return;
  const int i = pd.pi[p], j = pd.pj[p];
  const int ni = pd.n[i], nj = pd.n[j];
  const int rows = ni + 1, cols = nj + 1;
  const int alpha = ctrl->alpha;
  const int gap = ctrl->gap;
  const uint8_t *si = pd.seqs + pd.seq_off[i];
  const uint8_t *sj = pd.seqs + pd.seq_off[j];
  int32_t *tab = pd.tabs + pd.tab_off[p] + (dir ? (int64_t)rows * cols : 0);
  // element (a, b) of this direction's recurrence
  auto at = [&](int a, int b) -> int64_t {
    return dir ? (int64_t)(nj - b) * rows + (ni - a) : (int64_t)b * rows + a;
  };
  __shared__ int8_t sub[255 * 255];
  const int lane = threadIdx.x;
  for (int x = lane; x < alpha * alpha; x += 64) sub[x] = pd.sub[x];
  __syncthreads();

  const int RB = min(kRB, (rows + 63) / 64);
  for (int base = 0; base < rows; base += 64 * RB) {
    const int a0 = base + lane * RB;
    int x[kRB];
    int32_t cur[kRB];
#pragma unroll
    for (int r = 0; r < kRB; ++r) {
      const int a = a0 + r;
      const bool in = r < RB && a >= 1 && a < rows;
      // codes >= alpha are reported by the fill; clamped here to stay in the matrix
      x[r] = (in ? min((int)(dir ? si[ni - a] : si[a - 1]), alpha - 1) : 0) * alpha;
      cur[r] = 0;
    }
    int32_t bot = 0;    // this lane's last row at the previous step
    int32_t diag0 = 0;  // the value above the first row, previous column
    int yv = 0;         // residue of this lane's column
    // lane 0's columns c0 .. c0 + 63: residue codes and the band's upper
    // boundary, loaded one chunk ahead so that only the refill waits
    auto load_y = [&](int c0) -> int {
      const int bb = c0 + lane;
      return (bb >= 1 && bb < cols) ? (int)(dir ? sj[nj - bb] : sj[bb - 1]) : 0;
    };
    auto load_b = [&](int c0) -> int32_t {
      const int bb = c0 + lane;
      return (bb < cols && base > 0) ? tab[at(base - 1, bb < cols ? bb : 0)] : 0;
    };
    int ynext = load_y(0), bnext = load_b(0);
    for (int c0 = 0; c0 < cols + 63; c0 += 64) {
     // chunks of 64 steps: the step loop itself issues no load
     const int ychunk = ynext;
     const int32_t bchunk = bnext;
     ynext = load_y(c0 + 64);
     bnext = load_b(c0 + 64);
     const int send = min(c0 + 64, cols + 63);
     for (int s = c0; s < send; ++s) {
      const int b = s - lane;
      const int32_t above = shift_up1(bot, 0);
      const int yin = shift_up1(yv, 0);
      // codes >= alpha are reported by the fill; clamped here to stay in the matrix
      const int y0 = min(__builtin_amdgcn_readlane(ychunk, s & 63), alpha - 1);
      const int32_t b0 = __builtin_amdgcn_readlane(bchunk, s & 63);
      yv = lane == 0 ? y0 : yin;
      int32_t up = lane == 0 ? b0 : above;  // (a0 - 1, b)
      if (b >= 0 && b < cols) {
        int32_t dg = diag0;                 // (a0 - 1, b - 1)
        diag0 = up;
        // this lane's cells of column b: ascending rows (prefix table) or
        // descending (mirrored suffix table)
        int32_t *colp = tab + at(a0, b);
        const int rstep = dir ? -1 : 1;
        int sc[kRB];
#pragma unroll
        for (int r = 0; r < kRB; ++r) sc[r] = (int)sub[x[r] + yv];
#pragma unroll
        for (int r = 0; r < kRB; ++r) {
          const int a = a0 + r;
          if (r < RB && a < rows) {
            int32_t v;
            if (a == 0) {
              v = b * gap;
            } else if (b == 0) {
              v = a * gap;
            } else {
              v = max(max(up, cur[r]) + gap, dg + sc[r]);
            }
            dg = cur[r];  // (a, b - 1): the diagonal of (a + 1, b)
            cur[r] = v;
            up = v;
            bot = v;
            colp[r * rstep] = v;
          }
        }
      }
     }
    }
    // the band's last row is read back by the next band
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
  }
}

// ---------------------------------------------------------------------------
// Block maxima: workgroup (c_j, p) takes the columns of tile c_j along j and
// every row, and writes bm[p][c_i][c_j] = max over the tile pair of F + G.
// Workgroup (0, 0) also sets U = sum_p F_p[n_i][n_j] and the first threshold
// L1 = U - ceil(|U| / 16) - C(k,2) * max(|gap|, max |sub|).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pair_blockmax_kernel(PruneDev pd, Ctrl *ctrl) {
  const int p = blockIdx.y;
  const int cj = blockIdx.x;
  const int tid = threadIdx.x;
  if (p == 0 && cj == 0 && tid == 0) {
    int64_t U = 0;
    for (int q = 0; q < pd.npairs; ++q) {
      const int rq = pd.n[pd.pi[q]] + 1;
      U += pd.tabs[pd.tab_off[q] + (int64_t)pd.n[pd.pj[q]] * rq + (rq - 1)];
    }
    const int64_t L1 = U - ((U < 0 ? -U : U) + 15) / 16 - ctrl->prune_c;
    ctrl->prune_U = U;
    ctrl->prune_L = L1;
    ctrl->prune_passes = 1;
    ctrl->redo = 0;
  }
  const int i = pd.pi[p], j = pd.pj[p];
  if (cj >= pd.P[j]) return;
  const int T = pd.T;
  const int rows = pd.n[i] + 1;
  const int cols = pd.n[j] + 1;
  const int b_lo = cj == 0 ? 0 : (cj - 1) * T + 1;
  const int b_hi = cj == 0 ? 0 : min(cj * T, cols - 1);
  const int Pi = pd.P[i];
  __shared__ int32_t bmx[kMaxTilesPerDim];
  for (int c = tid; c < Pi; c += 256) bmx[c] = INT32_MIN;
  __syncthreads();
  const int32_t *F = pd.tabs + pd.tab_off[p];
  const int32_t *G = F + (int64_t)rows * cols;
  for (int a = tid; a < rows; a += 256) {
    int32_t m = INT32_MIN;
    for (int b = b_lo; b <= b_hi; ++b) {
      const int64_t e = (int64_t)b * rows + a;
      m = max(m, F[e] + G[e]);
    }
    const int ci = a == 0 ? 0 : (a - 1) / T + 1;
    atomicMax(&bmx[ci], m);
  }
  __syncthreads();
  for (int c = tid; c < Pi; c += 256) pd.bm[pd.bm_off[p] + (int64_t)c * pd.P[j] + cj] = bmx[c];
}

// Exclusive prefix sum of `v` over the workgroup (kSelBlock threads); the
// total is returned in *total.
__device__ int block_scan(int v, int *total) {
  __shared__ int wsum[kSelBlock / 64];
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  int incl = v;
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(incl, d, 64);
    if (lane >= d) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int before = 0, all = 0;
  for (int x = 0; x < kSelBlock / 64; ++x) {
    before += x < w ? wsum[x] : 0;
    all += wsum[x];
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

// Pass `pass` selection: keep flag of every tile at the current threshold and
// kept tiles per block of the wave-order queue.  Pass 2 runs only after a miss.
__global__ __launch_bounds__(kSelBlock) void prune_select_kernel(PruneDev pd, const Ctrl *ctrl,
                                                                 int pass) {
  if (pass == 2 && ctrl->redo == 0) return;
  const int64_t L = ctrl->prune_L;
  const int64_t q = (int64_t)blockIdx.x * kSelBlock + threadIdx.x;
  int kp = 0;
  if (q < pd.ntiles) {
    const int tile = pd.order[q];
    int c[kPruneMaxK];
#pragma unroll
    for (int i = 0; i < kPruneMaxK; ++i)
      c[i] = i < pd.k ? (tile / pd.tstride[i]) % pd.P[i] : 0;
    int64_t tb = 0;
    for (int p = 0; p < pd.npairs; ++p) {
      int ci = 0, cj = 0;
#pragma unroll
      for (int i = 0; i < kPruneMaxK; ++i) {
        ci = i == pd.pi[p] ? c[i] : ci;
        cj = i == pd.pj[p] ? c[i] : cj;
      }
      tb += pd.bm[pd.bm_off[p] + (int64_t)ci * pd.P[pd.pj[p]] + cj];
    }
    kp = tb >= L ? 1 : 0;
    pd.keep[tile] = (uint8_t)kp;
  }
  int total;
  block_scan(kp, &total);
  if (threadIdx.x == 0) pd.bcnt[blockIdx.x] = total;
}

// Exclusive offsets of the blocks' kept counts (one workgroup); the total is
// the queue length of the pass.
__global__ __launch_bounds__(kSelBlock) void prune_scan_kernel(PruneDev pd, Ctrl *ctrl,
                                                               int pass) {
  if (pass == 2 && ctrl->redo == 0) return;
  int carry = 0;
  for (int base = 0; base < pd.nblocks; base += kSelBlock) {
    const int x = base + (int)threadIdx.x;
    const int v = x < pd.nblocks ? pd.bcnt[x] : 0;
    int total;
    const int ex = block_scan(v, &total);
    if (x < pd.nblocks) pd.bcnt[x] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) {
    ctrl->nqueue = carry;
    ctrl->prune_kept = carry;
  }
}

// Kept tiles in wave order: korder[offset of the block + rank in the block].
__global__ __launch_bounds__(kSelBlock) void prune_compact_kernel(PruneDev pd, const Ctrl *ctrl,
                                                                  int pass) {
  if (pass == 2 && ctrl->redo == 0) return;
  const int64_t q = (int64_t)blockIdx.x * kSelBlock + threadIdx.x;
  const int tile = q < pd.ntiles ? pd.order[q] : 0;
  const int kp = q < pd.ntiles ? (int)pd.keep[tile] : 0;
  int total;
  const int rank = block_scan(kp, &total);
  if (kp) pd.korder[pd.bcnt[blockIdx.x] + rank] = tile;
}

// After pass 1: an end score at or above the threshold is exact.  Otherwise
// pass 2 runs with L2 = s when s is the score of a real path (at least the
// closed-form lower bound of every score; a path through pruned cells only
// carries a value far below it), else with no pruning.
__global__ __launch_bounds__(64) void prune_check_kernel(PruneDev pd, Ctrl *ctrl) {
  if (threadIdx.x != 0) return;
  const int64_t s = *pd.score;
  if (ctrl->status != ST_OK || s >= ctrl->prune_L) {
    ctrl->redo = 0;
    return;
  }
  ctrl->redo = 1;
  ctrl->prune_L = s >= ctrl->lo ? s : INT64_MIN;
  ctrl->prune_passes = 2;
  ctrl->head = 0;
  ctrl->epoch = ctrl->epoch + 1;
}

}  // namespace

int launch_prune_bounds(const PruneDev &pd, Ctrl *ctrl, hipStream_t s) {
  launch_begin();
  hipLaunchKernelGGL(pair_table_kernel, dim3(2 * pd.npairs), dim3(64), 0, s, pd, ctrl);
  int pmax = 1;
  for (int q = 0; q < pd.npairs; ++q) pmax = max(pmax, pd.P[pd.pj[q]]);
  hipLaunchKernelGGL(pair_blockmax_kernel, dim3(pmax, pd.npairs), dim3(256), 0, s, pd, ctrl);
  return launch_end();
}

int launch_prune_select(const PruneDev &pd, Ctrl *ctrl, int pass, hipStream_t s) {
  launch_begin();
  hipLaunchKernelGGL(prune_select_kernel, dim3(pd.nblocks), dim3(kSelBlock), 0, s, pd, ctrl,
                     pass);
  hipLaunchKernelGGL(prune_scan_kernel, dim3(1), dim3(kSelBlock), 0, s, pd, ctrl, pass);
  hipLaunchKernelGGL(prune_compact_kernel, dim3(pd.nblocks), dim3(kSelBlock), 0, s, pd, ctrl,
                     pass);
  return launch_end();
}

int launch_prune_check(const PruneDev &pd, Ctrl *ctrl, hipStream_t s) {
  launch_begin();
  hipLaunchKernelGGL(prune_check_kernel, dim3(1), dim3(64), 0, s, pd, ctrl);
  return launch_end();
}

}  // namespace msa
