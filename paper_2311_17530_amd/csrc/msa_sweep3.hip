// msa_sweep3.hip -- streaming fill of the three-sequence tensor.
//
// The cells of one computation wave (Section 3: cells, or partitions, at
// equal distance from the origin are independent) are the hyperplane
// v0 + v1 + v2 = h.  This kernel sweeps those hyperplanes in a pipeline
// instead of tile by tile:
//
//   - Lines.  A line is the run of cells (v0, v1, 0..n2) along dimension 2.
//     A workgroup owns kSwRows x 64 lines: rows v0 = B0*kSwRows + kSwRPW*w
//     + u, u = 0 .. kSwRPW - 1 (wave w's rows, top to bottom) and columns
//     v1 = B1*64 + j (lane j), and sweeps them over the whole length in
//     steps: at block step s, lane j of wave w computes cell t = s - j - w of
//     each of its lines, top row first.  Every neighbour v - b of that cell
//     was computed by the same lane (in this step for a row's neighbours in
//     the row above it in the same wave), the lane to its left (v1 - 1) or
//     the wave above (v0 - 1) one to three steps earlier, so a step needs no
//     wait beyond one barrier.  Several rows per wave divide the workgroups
//     along dimension 0, and with them the hand-offs between workgroups on
//     the sweep's critical path, at the cost of longer steps.
//   - Exchange inside a wave: lane j - 1's previous output arrives by a DPP
//     wave shift (wave_shr:1); outputs of two steps back are kept in
//     registers.  Between waves: each wave writes its last row's outputs to
//     an LDS ring of 4 steps, read by the wave below one or two steps later.
//     Entry 0 of a ring row is the value of the row's lane -1 (the workgroup
//     to the left), so every lane reads its neighbours at fixed offsets; the
//     other rows' lane -1 values have an array of their own (h0).
//   - Exchange between workgroups: the outputs of the last row go to region
//     X0 and those of lane 63 of every row to region X1, each value tagged
//     with the launch's epoch in its low 3 bits (keys keep those bits clear);
//     the compute waves store them as they compute them.  A loader wave
//     (wave kSwNW) does every global load of the exchange: it loads the
//     neighbours' values kSwPf steps ahead, checks their tags (reloading
//     while any is stale) and writes them to LDS one step before they are
//     read.  Compute waves issue no global load, and no wave waits on their
//     stores (exchange values, and direction bytes every 16 steps).
//   - Workgroups take tickets in order of their block diagonal B0 + B1; a
//     workgroup only waits for workgroups with smaller tickets, which are
//     already running, so the grid cannot deadlock.
//
// Per cell (Section 2, Eq. 1 for three sequences; Section 4 per-cell steps):
// seven candidates key(v - b) + column(b), the column score being the sum of
// the pair scores of the residues the mask b takes plus gap * 2 for a one- or
// two-residue column, all pre-shifted by 3 bits with the tie bits 7 - b in
// the low bits, so one signed maximum gives the score and, among equal
// scores, the lowest mask.  Direction bytes are stored in the same
// tile-major blocks (edge 16) as the tile kernel's, so the traceback, the
// decision export and the other modes read them unchanged: each lane keeps
// the bytes of its current and previous 16-cell run in LDS, and every 16
// steps the whole wave stores the runs completed since.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msa_internal.h"
#include "msa_plan.h"

namespace msa {

namespace {

constexpr int kSwRing = 4;        // LDS rings (outputs, halo rows): 4 steps
constexpr int kSwPf = 2;          // loader prefetch distance (steps)
constexpr int kSwUnroll = 16;     // steps per unrolled group (direction flush)
constexpr int kSwRow = 65;        // ring row: the lane-(-1) entry + 64 lanes
constexpr int kSwSeqPad = 128;    // LDS bytes around the third sequence
constexpr int kSwThreads = (kSwNW + 1) * 64;
constexpr int kSwT = 16;          // tile edge of the direction blocks (k = 3)
constexpr int kSwDbs = kSwT * kSwT * kSwT;
constexpr int64_t kSwWaitTicks = 200000000;  // 2 s of waiting (WaitClock ticks)

static_assert(kSwDbs == 4096, "direction blocks of edge 16");
static_assert(kSwRPW >= 2 && kSwRows < 64, "loader lanes 1 .. kSwRows");
static_assert(tile_edge_for_k(3) == kSwT, "same blocks as the tile kernel");
static_assert(kSwUnroll % kSwRing == 0 && kSwUnroll % kSwPf == 0, "ring slots fixed per group");

struct Sweep3Dev {
  int32_t n0, n1, n2;
  int32_t nb0, nb1;           // workgroups along dimensions 0 and 1
  const uint8_t *s0, *s1, *s2;
  const int8_t *sub;
  int32_t *x0;                // X0[b][d][v1], b < nb0 - 1, d = v1 + v2
  int64_t x0_plane;
  int32_t *x1;                // X1[b][e][v0], b < nb1 - 1, e = v2 + w (w: the row's wave)
  int64_t x1_plane;
  uint8_t *dir;               // tile-major direction blocks
  int32_t ts0, ts1;           // tile strides of dimensions 0 and 1 (dimension 2: 1)
  int64_t *score_out;
  int64_t *trace;             // debug builds: 8 words per workgroup ticket
  int32_t egf;                // end-gap-free mode
  int64_t *best;              // end-gap-free: max of (score << 32 | row-major
                              // cell index) over the far faces
};

struct SwSmem {
  int32_t ring[kSwRing][kSwNW][kSwRow];    // wave w's last row at step s: slot s % 4
  int32_t in0[kSwRing][kSwRow];            // the row above the workgroup (wave -1)
  int32_t h0[kSwRing][kSwNW][kSwRPW - 1];  // lane -1 of wave w's rows above its last
  int32_t junk[64];                        // loader lanes without a halo value write here
  int32_t sub8[kSwSubMax * kSwSubMax];     // substitution matrix << 3
  alignas(16) uint8_t stage[kSwRows][64][32];  // per row and lane: two 16-cell runs
  uint8_t s2[kSwSeqPad + kSwSeqMax + kSwSeqPad];
  int32_t ticket;
};

// LDS writes of this wave complete, then every wave of the workgroup meets.
// Global stores stay in flight: no wave waits on them.
__device__ __forceinline__ void sw_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ int32_t sw_load(const int32_t *p) {
  return __hip_atomic_load(const_cast<int32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void sw_store(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The loader wave.  During step s it writes step s + 1's halo to LDS:
//   - the row above: in0[s % 4] entry i = cell (B0*kSwRows - 1, B1*64 - 1 + i,
//     s + 2 - i) = X0[B0-1][B1*64 + s + 1][B1*64 - 1 + i] (element 0 of lane
//     i; entry 64 is element 1 of lane 0);
//   - lane -1 of row r = kSwRPW*w + u (wave w's row u): cell
//     (B0*kSwRows + r, B1*64 - 1, s + 2 - w) = X1[B1-1][s + 2][B0*kSwRows + r]
//     (element 1 of lane 1 + r), to h0[(s + 1) % 4][w][u] (u < kSwRPW - 1) or
//     ring[(s + 1) % 4][w][0] (the wave's last row);
// and issues the loads of step s + kSwPf.  A cell outside the tensor, or
// without a workgroup before this one, reads -infinity.  Every lane issues
// both loads every step (an address clamped into its element's window of
// cells, or a dummy word), so the wait for a step's values counts exactly the
// younger loads.
struct SwLoader {
  // Element x of step s is the word at wbase[x] + (s - llo[x]) * linc[x], a
  // cell for s - llo[x] in [0, span].  acc[x] = (s - llo[x]) * linc[x] for
  // the next step to issue (steps are issued in order, one per call); an
  // element with no cell has linc 0 and acc -1.
  const int32_t *wbase[2];
  int32_t acc[2], linc[2], ohi[2], lag[2];  // ohi = span * linc, lag = kSwPf * linc
  int32_t dst1[kSwRing];  // LDS word index (in the ring array) of element 1, per slot s % 4

  // (set-up code is force-inlined as well: a call would need the kernel's
  // by-value descriptor in memory, a copy to scratch)
  __device__ __forceinline__ void set(int x, const int32_t *base, int llo, int inc, int span,
                                      int s_first) {
    wbase[x] = base;
    linc[x] = inc;
    acc[x] = (s_first - llo) * inc;
    ohi[x] = span * inc;
    lag[x] = kSwPf * inc;
  }

  __device__ __forceinline__ SwLoader(const Sweep3Dev &sd, SwSmem &sm, int B0, int B1,
                                      int lane, const int32_t *dummy, int s_first) {
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      wbase[x] = dummy;
      acc[x] = -1;
      linc[x] = 0;
      ohi[x] = 0;
      lag[x] = 0;
    }
    // element 0: in0 entry lane, cells for s in [lane - 2, n2 + lane - 2]
    {
      const int v1 = B1 * kSwLanes - 1 + lane;
      if (B0 > 0 && v1 >= 0 && v1 <= sd.n1)
        set(0, sd.x0 + (int64_t)(B0 - 1) * sd.x0_plane +
                   (int64_t)(B1 * kSwLanes + lane - 1) * (sd.n1 + 1) + v1,
            lane - 2, sd.n1 + 1, sd.n2, s_first);
    }
    // element 1: in0 entry 64 (lane 0) or lane -1 of row lane - 1
    const int32_t *const rbase = &sm.ring[0][0][0];
#pragma unroll
    for (int k = 0; k < kSwRing; ++k) dst1[k] = (int32_t)(&sm.junk[lane] - rbase);
    if (lane == 0) {
      const int v1 = B1 * kSwLanes + 63;
#pragma unroll
      for (int k = 0; k < kSwRing; ++k) dst1[k] = (int32_t)(&sm.in0[k][64] - rbase);
      if (B0 > 0 && v1 <= sd.n1)
        set(1, sd.x0 + (int64_t)(B0 - 1) * sd.x0_plane +
                   (int64_t)(B1 * kSwLanes + 63) * (sd.n1 + 1) + v1,
            62, sd.n1 + 1, sd.n2, s_first);
    } else if (lane <= kSwRows) {
      const int r = lane - 1;
      const int w = r / kSwRPW;
      const int v0 = B0 * kSwRows + r;
#pragma unroll
      for (int k = 0; k < kSwRing; ++k)
        dst1[k] = (int32_t)((r % kSwRPW < kSwRPW - 1
                                 ? &sm.h0[(k + 1) & (kSwRing - 1)][w][r % kSwRPW]
                                 : &sm.ring[(k + 1) & (kSwRing - 1)][w][0]) -
                            rbase);
      // X1 is indexed by e = t + w, so one step's values of all rows are
      // adjacent words (the left workgroup stores them in one step too)
      if (B1 > 0 && v0 <= sd.n0)
        set(1, sd.x1 + (int64_t)(B1 - 1) * sd.x1_plane + (int64_t)w * (sd.n0 + 1) + v0, w - 2,
            sd.n0 + 1, sd.n2, s_first);
    }
  }

  // the word of element x at window offset a, clamped into the window
  __device__ __forceinline__ const int32_t *addr(int x, int32_t a) const {
    return wbase[x] + (uint32_t)min(max(a, 0), ohi[x]);
  }

  __device__ __forceinline__ void issue(int32_t (&v)[2]) {
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      v[x] = sw_load(addr(x, acc[x]));
      acc[x] += linc[x];
    }
  }

  // some value of a step (window offsets a) is a cell's and not yet this
  // launch's
  __device__ __forceinline__ bool stale(const int32_t (&a)[2], const int32_t (&v)[2],
                                        int tag) const {
    int st = 0;
#pragma unroll
    for (int x = 0; x < 2; ++x)
      st |= (int)((unsigned)a[x] <= (unsigned)ohi[x]) & (int)((v[x] & 7) != tag);
    return __builtin_amdgcn_ballot_w64(st != 0) != 0;
  }

  // Slow path: reloads the values (into registers of its own) until every
  // one carries this launch's tag or the watchdog fires (WaitClock: pauses of
  // the queue do not count as waiting).
  __device__ __forceinline__ void respin(const int32_t (&a)[2], int32_t (&v)[2], int tag,
                                         Ctrl *ctrl) const {
    int32_t u[2];
    WaitClock wc;
    for (int it = 0;; ++it) {
      __builtin_amdgcn_s_sleep(1);
#pragma unroll
      for (int x = 0; x < 2; ++x) u[x] = sw_load(addr(x, a[x]));
      if (!stale(a, u, tag)) break;
      if ((it & 15) == 15) {
        const int st = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&ctrl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (st == -4) break;  // another workgroup timed out: stop waiting
        if (wc.tick() > kSwWaitTicks) {
          atomicCAS(&ctrl->status, 0, -4);
          break;
        }
      }
    }
    wc.report(ctrl);
    v[0] = u[0];
    v[1] = u[1];
  }

  // The values of step s, issued `back` steps before the next one to issue
  // (reloaded while any carries another launch's tag), to LDS.  The first
  // check is straight-line code, so its wait counts only the younger loads.
  __device__ __forceinline__ void finish(int s, int back, int32_t (&v)[2], int tag, SwSmem &sm,
                                         int lane, Ctrl *ctrl, int &nspin) const {
    int32_t a[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) a[x] = acc[x] - (back == kSwPf ? lag[x] : back * linc[x]);
    if (stale(a, v, tag)) {
      respin(a, v, tag, ctrl);
      ++nspin;
    }
    const bool r0 = (unsigned)a[0] <= (unsigned)ohi[0];
    const bool r1 = (unsigned)a[1] <= (unsigned)ohi[1];
    sm.in0[s & (kSwRing - 1)][lane] = r0 ? (v[0] & ~7) : kNegKey;
    (&sm.ring[0][0][0])[dst1[s & (kSwRing - 1)]] = r1 ? (v[1] & ~7) : kNegKey;
  }
};

// One compute wave: rows v0 = B0*kSwRows + kSwRPW*w + u, u = 0 .. kSwRPW - 1
// (top to bottom), lane j: column v1 = B1*64 + j.  kX0: the workgroup's last
// row has a workgroup below it (this wave stores X0 from its last row); kX1:
// the workgroup has one to its right (lane 63 stores X1); kOrigin: wave 0 of
// workgroup (0, 0), whose top row's lane 0 holds the origin.  kEgf:
// end-gap-free mode (Section 2's reading of free end gaps): every cell with
// some v_i = 0 scores 0 with no decision, and the best far-face cell is
// reported.
template <bool kX0, bool kX1, bool kOrigin, bool kEgf>
__device__ __forceinline__ void sweep_row(const Sweep3Dev &sd, SwSmem &sm, int B0, int B1, int w,
                                          int j, const bool (&ok)[kSwRPW],
                                          const int (&r0)[kSwRPW], int r1, int gap, int tag,
                                          int total, bool cw, int sc, int uc, int jc) {
  constexpr int R = kSwRPW;
  const int v0top = B0 * kSwRows + R * w;
  const int v1 = B1 * kSwLanes + j;
  const int g16 = gap * 16;  // (gap * 2 column pairs) << 3
  const int32_t K1 = g16 + 6, K2 = g16 + 5, K4 = g16 + 3, K5 = g16 + 2, K6 = g16 + 1;
  const int n2 = sd.n2;
  const int c1 = v1 == 0 ? 0 : (v1 - 1) / kSwT + 1, q1 = v1 == 0 ? 0 : (v1 - 1) % kSwT;
  int32_t p01[R], C3[R];
  const int32_t *sub0[R];
  uint8_t *dline[R];
  uint8_t *stage[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int v0 = v0top + u;
    p01[u] = sm.sub8[r0[u] * kSwSubMax + r1];
    C3[u] = p01[u] + g16 + 4;
    sub0[u] = sm.sub8 + r0[u] * kSwSubMax;
    // direction bytes: tile (c0, c1, c2), line q0 * 16 + q1, byte q2
    const int c0 = v0 == 0 ? 0 : (v0 - 1) / kSwT + 1, q0 = v0 == 0 ? 0 : (v0 - 1) % kSwT;
    dline[u] =
        sd.dir + ((int64_t)c0 * sd.ts0 + (int64_t)c1 * sd.ts1) * kSwDbs + (q0 * kSwT + q1) * kSwT;
    stage[u] = &sm.stage[R * w + u][j][0];
  }
  // rows of the wave above: the loader's in0 for wave 0, else the ring
  const int32_t *const prow = (w == 0 ? &sm.in0[0][0] : &sm.ring[0][w - 1][0]) + j;
  const int pstride = w == 0 ? kSwRow : kSwNW * kSwRow;
  const int32_t *const sub_r1 = sm.sub8 + r1 * kSwSubMax;
  const int jw = j + w;
  // exchange stores: cell (v0, v1, t) of the last row at X0[B0][v1 + t][v1]
  // (v1 + t = B1*64 + s - w); lane 63's cells at X1[B1][t + w][v0] = X1[B1][s - 63][v0]
  int32_t *const x0b = sd.x0 + (int64_t)B0 * sd.x0_plane +
                       (int64_t)(B1 * kSwLanes - w) * (sd.n1 + 1) + v1;
  const int64_t x0inc = sd.n1 + 1;
  int32_t *const x1t = sd.x1 + (int64_t)B1 * sd.x1_plane - (int64_t)63 * (sd.n0 + 1) + v0top;
  const int64_t x1inc = sd.n0 + 1;
  const bool lane63 = j == 63;
  // end-gap-free: boundary cells (some v_i = 0), far lanes (v0 = n0 or
  // v1 = n1; every lane's cell t = n2 is far too), and the row-major index of
  // each row's cell t = 0 (below 2^32, checked by the plan's set-up).  The
  // wave's cells t = 0 fall in steps w .. w + 63 and its cells t = n2 in
  // steps n2 + w .. n2 + w + 63; outside those windows only waves holding a
  // boundary or far lane test their cells (wave-uniform branches).
  bool ebz[R], efar[R];
  bool anyfar = false;
  uint32_t elin[R];
  int32_t eout[R];
  int et[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int v0 = v0top + u;
    ebz[u] = v0 == 0 || v1 == 0;
    efar[u] = v0 == sd.n0 || v1 == sd.n1;
    anyfar = anyfar || efar[u];
    elin[u] = ((uint32_t)v0 * (uint32_t)(sd.n1 + 1) + (uint32_t)v1) * (uint32_t)(sd.n2 + 1);
    // the row's best far cell so far: its key (score << 3) and t; among equal
    // scores the later t, whose row-major index is larger
    eout[u] = INT32_MIN;
    et[u] = 0;
  }
  const bool wbz = __builtin_amdgcn_ballot_w64(ebz[0]) != 0;  // (ebz[u > 0] implies ebz[0])
  const bool wfar = __builtin_amdgcn_ballot_w64(anyfar) != 0;

  // per row: own previous output, lane -1's value, and (v0, v1 - 1, t - 1);
  // the top row also keeps its other neighbours of one step back
  int32_t outp[R], hl[R], l6[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    outp[u] = kNegKey;
    l6[u] = kNegKey;
    hl[u] = u < R - 1 ? sm.h0[kSwRing - 1][w][u] : sm.ring[kSwRing - 1][w][0];
  }
  int32_t b5 = kNegKey, b7 = kNegKey;
  // pair scores of the third residue one step ahead (they do not depend on
  // the scores), and its code two steps ahead; s2_j[s] is the residue of t
  const uint8_t *s2_j = sm.s2 + kSwSeqPad - 1 - jw;
  int32_t p02n[R];
#pragma unroll
  for (int u = 0; u < R; ++u) p02n[u] = sub0[u][s2_j[0]];
  int32_t p12n = sub_r1[s2_j[0]];
  int r2n = s2_j[1];
  for (int s0 = 0; s0 < total; s0 += kSwUnroll) {
#pragma unroll
    for (int i = 0; i < kSwUnroll; ++i) {
      const int s = s0 + i;
      const int t = s - jw;
      const bool in_t = (unsigned)t <= (unsigned)n2;
      int32_t p02[R];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        p02[u] = p02n[u];
        p02n[u] = sub0[u][r2n];
      }
      const int32_t p12 = p12n;
      p12n = sub_r1[r2n];
      r2n = s2_j[s + 2];
      // the top row's neighbours in the row above: (v0-1, v1, t), (v0-1, v1-1, t)
      const int32_t b1 = prow[((i - 1) & (kSwRing - 1)) * pstride + 1];
      const int32_t b3 = prow[((i - 2) & (kSwRing - 1)) * pstride];
      int32_t hnext[R];
#pragma unroll
      for (int u = 0; u < R; ++u)
        hnext[u] = u < R - 1 ? sm.h0[i & (kSwRing - 1)][w][u] : sm.ring[i & (kSwRing - 1)][w][0];
      // (v0, v1-1, t) per row: lane j-1's previous output; lane 0 takes lane -1's
      int32_t l2[R];
#pragma unroll
      for (int u = 0; u < R; ++u)
        l2[u] = __builtin_amdgcn_update_dpp(hl[u], outp[u], 0x138, 0xF, 0xF, false);
      int32_t best[R], out[R];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        // neighbours in the row above: (v0-1, v1, t), (v0-1, v1-1, t),
        // (v0-1, v1, t-1), (v0-1, v1-1, t-1); below the top row they are the
        // row above's values of this step, from registers
        const int32_t a1 = u == 0 ? b1 : out[u - 1];
        const int32_t a3 = u == 0 ? b3 : l2[u - 1];
        const int32_t a5 = u == 0 ? b5 : outp[u - 1];
        const int32_t a7 = u == 0 ? b7 : l6[u - 1];
        const int32_t c2 = l2[u] + K2;
        const int32_t c3 = a3 + C3[u];
        const int32_t c4 = outp[u] + K4;
        const int32_t c5 = a5 + p02[u] + K5;
        const int32_t c6 = l6[u] + p12 + K6;
        const int32_t c7 = a7 + p01[u] + (p02[u] + p12);
        // c1 waits for the row above's output (below the top row): take it last
        int32_t bst = max(max(max(max(c4, c2), c3), max(max(c5, c6), c7)), a1 + K1);
        // the origin takes key 7: score 0, and the byte decodes to mask 0
        // (end-gap-free: every cell with some v_i = 0)
        if constexpr (kEgf) {
          if (wbz || (unsigned)(s - w) < 64u) bst = (ebz[u] || t == 0) ? 7 : bst;
        } else if constexpr (kOrigin) {
          if (u == 0) bst = (j == 0 && t == 0) ? 7 : bst;
        }
        best[u] = bst;
        // Plain mode: a cell outside the tensor (t < 0, t > n2, v0 > n0,
        // v1 > n1) may keep what its neighbours give it, since no cell inside
        // reads it (a cell's neighbours have no larger coordinate), and cells
        // t < 0 see only -infinity from the halo and stay far below any score.
        // (Exchange stores and direction runs test validity themselves.)
        // End-gap-free mode keeps -infinity there: that form measured faster.
        if constexpr (kEgf)
          out[u] = (ok[u] && in_t) ? (bst & ~7) : kNegKey;
        else
          out[u] = bst & ~7;
      }
      if constexpr (kEgf) {
        if (wfar || (unsigned)(s - w - n2) < 64u) {
#pragma unroll
          for (int u = 0; u < R; ++u) {
            const bool take = ok[u] && in_t && (efar[u] ? out[u] >= eout[u] : t == n2);
            eout[u] = take ? out[u] : eout[u];
            et[u] = take ? t : et[u];
          }
        }
      }
      sm.ring[i & (kSwRing - 1)][w][j + 1] = out[R - 1];
      // direction bytes of cell t at (t - 1) mod 32 (see the flush below)
#pragma unroll
      for (int u = 0; u < R; ++u) stage[u][(t - 1) & 31] = (uint8_t)best[u];
      if constexpr (kX0) {
        if (ok[R - 1] && in_t) sw_store(x0b + (int64_t)s * x0inc, out[R - 1] | tag);
      }
      if constexpr (kX1) {
        if (lane63) {
#pragma unroll
          for (int u = 0; u < R; ++u)
            if (ok[u] && in_t) sw_store(x1t + (int64_t)s * x1inc + u, out[u] | tag);
        }
      }
      // the score: the corner cell (n0, n1, n2) (wave-uniform test)
      if (cw && s == sc) {
        int32_t o = out[0];
#pragma unroll
        for (int u = 1; u < R; ++u) o = uc == u ? out[u] : o;
        if (j == jc) *sd.score_out = (int64_t)(o >> 3);
      }
      b5 = b1;
      b7 = b3;
#pragma unroll
      for (int u = 0; u < R; ++u) {
        l6[u] = l2[u];
        outp[u] = out[u];
        hl[u] = hnext[u];
      }
      sw_barrier();
    }
    // ---- direction runs completed in the last 16 steps ----
    // Run c (cells 16c - 15 .. 16c) sits at half (c - 1) & 1 of the lane's
    // 32 bytes, cell 0 at byte 31.  The flush after cell t = tf runs once per
    // 16 cells, so a run is stored before any later cell reaches its half;
    // cells past n2 only touch the tail of the last run (bytes of no cell)
    // or halves that are never stored again.
    const int tf = s0 + kSwUnroll - 1 - jw;
    const int c = tf >> 4;                         // run c: cells 16c - 15 .. 16c
    const int cl = (n2 >> 4) + 1;                  // the last, partial run
#pragma unroll
    for (int u = 0; u < R; ++u) {
      if (ok[u]) {
        if (tf >= 0 && tf < 16) dline[u][0] = stage[u][31];  // cell t = 0 (its own block)
        if (c >= 1 && 16 * c <= n2)
          *reinterpret_cast<uint4 *>(dline[u] + (int64_t)c * kSwDbs) =
              *reinterpret_cast<const uint4 *>(stage[u] + ((c - 1) & 1) * 16);
        if ((n2 & 15) != 0 && tf >= n2 && tf - 15 <= n2)
          *reinterpret_cast<uint4 *>(dline[u] + (int64_t)cl * kSwDbs) =
              *reinterpret_cast<const uint4 *>(stage[u] + ((cl - 1) & 1) * 16);
      }
    }
  }
  if constexpr (kEgf) {
    // the lane's far-face key (score << 32 | row-major index), the wave's
    // best, then one atomic per wave
    int64_t ekey = INT64_MIN;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int64_t k = eout[u] == INT32_MIN
                            ? INT64_MIN
                            : ((int64_t)(eout[u] >> 3) << 32) | (int64_t)(elin[u] + (uint32_t)et[u]);
      ekey = k > ekey ? k : ekey;
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t o = __shfl_xor(ekey, d, 64);
      ekey = o > ekey ? o : ekey;
    }
    if (j == 0 && ekey != INT64_MIN) atomicMax((long long *)sd.best, (long long)ekey);
  }
}

// The wave's variant: exchange stores (x0, x1) and the origin.
template <bool kEgf>
__device__ __forceinline__ void sweep_rows(const Sweep3Dev &sd, SwSmem &sm, int B0, int B1,
                                           int w, int j, const bool (&ok)[kSwRPW],
                                           const int (&r0)[kSwRPW], int r1, int gap, int tag,
                                           int total, bool x0, bool x1, bool cw, int sc, int uc,
                                           int jc) {
#define MSA_SW_ARGS sd, sm, B0, B1, w, j, ok, r0, r1, gap, tag, total, cw, sc, uc, jc
  if (B0 == 0 && B1 == 0 && w == 0) {
    if (x1)
      sweep_row<false, true, true, kEgf>(MSA_SW_ARGS);
    else
      sweep_row<false, false, true, kEgf>(MSA_SW_ARGS);
  } else if (x0 && x1)
    sweep_row<true, true, false, kEgf>(MSA_SW_ARGS);
  else if (x0)
    sweep_row<true, false, false, kEgf>(MSA_SW_ARGS);
  else if (x1)
    sweep_row<false, true, false, kEgf>(MSA_SW_ARGS);
  else
    sweep_row<false, false, false, kEgf>(MSA_SW_ARGS);
#undef MSA_SW_ARGS
}

}  // namespace

__global__ __launch_bounds__(kSwThreads) void sweep3_kernel(Sweep3Dev sd, Ctrl *ctrl) {
  __shared__ SwSmem sm;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid) >> 6;
  const int j = tid & 63;
  const int alpha = ctrl->alpha;
  const int gap = ctrl->gap;
  const int epoch = __hip_atomic_load(&ctrl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int tag = (epoch - 1) % 7 + 1;

  // ---- ticket: workgroups in order of their block diagonal B0 + B1 ----
  if (tid == 0) sm.ticket = atomicAdd(&ctrl->head, 1);
  // ---- tables: matrix << 3, third sequence with zero padding ----
  bool bad = false;
  for (int e = tid; e < alpha * alpha; e += kSwThreads)
    sm.sub8[(e / alpha) * kSwSubMax + e % alpha] = (int32_t)sd.sub[e] * 8;
  for (int x = tid; x < kSwSeqPad + sd.n2 + kSwSeqPad; x += kSwThreads) {
    const int q = x - kSwSeqPad;
    int r = (q >= 0 && q < sd.n2) ? (int)sd.s2[q] : 0;
    bad = bad || r >= alpha;
    sm.s2[x] = (uint8_t)(r >= alpha ? 0 : r);
  }
  // the rings before step 0 hold cells t < 0: -infinity
  for (int e = tid; e < kSwRing * kSwNW * kSwRow; e += kSwThreads)
    (&sm.ring[0][0][0])[e] = kNegKey;
  for (int e = tid; e < kSwRing * kSwNW * (kSwRPW - 1); e += kSwThreads)
    (&sm.h0[0][0][0])[e] = kNegKey;
  sw_barrier();
  const int ticket = __builtin_amdgcn_readfirstlane(sm.ticket);
  // A ticket past the grid means the counter was not reset since the last
  // fill (a fill must be followed by its traceback): nothing to do.
  if (ticket >= sd.nb0 * sd.nb1) return;
  int T = ticket;
  int B0 = 0, B1 = 0;
  for (int a = 0; a <= sd.nb0 + sd.nb1 - 2; ++a) {  // diagonals B0 + B1 = a
    const int lo = a - (sd.nb1 - 1) > 0 ? a - (sd.nb1 - 1) : 0;
    const int hi = a < sd.nb0 - 1 ? a : sd.nb0 - 1;
    const int cnt = hi - lo + 1;
    if (T < cnt) {
      B0 = lo + T;
      B1 = a - B0;
      break;
    }
    T -= cnt;
  }
  // Steps until the block's last cell inside the tensor: lane j of wave w
  // computes t = n2 at step n2 + j + w.  A ragged block (the last along
  // dimension 0 or 1) stops after its last valid lane and wave instead of
  // sweeping the skew of lanes and waves that hold no cell; such a block has
  // no workgroup after it along that dimension, so no one waits for the
  // exchange values it skips.  (Every wave and the loader take the same count.)
  const int jmax = min(kSwLanes - 1, sd.n1 - B1 * kSwLanes);
  const int wmax = min(kSwNW - 1, (sd.n0 - B0 * kSwRows) / kSwRPW);
  const int nsteps = sd.n2 + 1 + jmax + wmax;
  const int total = (nsteps + kSwUnroll - 1) / kSwUnroll * kSwUnroll;

  if (wave == kSwNW) {
    // ---------------- loader wave ----------------
    if (bad) atomicCAS(&ctrl->status, 0, -1);
    SwLoader ld(sd, sm, B0, B1, j, reinterpret_cast<const int32_t *>(ctrl), -2);
#ifdef MSA_TRACE
    const int64_t t0 = (int64_t)wall_clock64();
#endif
    int nspin = 0;
    {
      // the halo of steps -1 (rows -2 / -1's lane -1) and 0, then steps 1 ..
      // kSwPf in flight
      int32_t a[2], b[2];
      ld.issue(a);
      ld.issue(b);
      ld.finish(-2, 2, a, tag, sm, j, ctrl, nspin);
      ld.finish(-1, 1, b, tag, sm, j, ctrl, nspin);
    }
    int32_t q[kSwPf][2];
#pragma unroll
    for (int i = 0; i < kSwPf; ++i) ld.issue(q[i]);
    sw_barrier();
#ifdef MSA_TRACE
    const int64_t t1 = (int64_t)wall_clock64();
#endif
    for (int s0 = 0; s0 < total; s0 += kSwUnroll) {
#pragma unroll
      for (int i = 0; i < kSwUnroll; ++i) {
        const int s = s0 + i;
        // during step s: step s + 1's halo (loaded kSwPf steps ago)
        ld.finish(s, kSwPf, q[i % kSwPf], tag, sm, j, ctrl, nspin);
        sw_barrier();
        ld.issue(q[i % kSwPf]);  // step s + kSwPf
      }
    }
#ifdef MSA_TRACE
    if (sd.trace && j == 0) {
      int64_t *tr = sd.trace + (int64_t)ticket * 8;
      tr[0] = B0;
      tr[1] = B1;
      tr[2] = t0;
      tr[3] = t1;
      tr[4] = (int64_t)wall_clock64();
      tr[5] = nspin;
      tr[6] = total;
    }
#endif
    return;
  }

  // ---------------- compute waves ----------------
  const int w = wave;
  const int v0top = B0 * kSwRows + kSwRPW * w;
  const int v1 = B1 * kSwLanes + j;
  const bool col_ok = v1 <= sd.n1;
  bool ok[kSwRPW];
  int r0[kSwRPW];
#pragma unroll
  for (int u = 0; u < kSwRPW; ++u) {
    const int v0 = v0top + u;
    const bool row = v0 <= sd.n0;
    ok[u] = row && col_ok;
    int r = (row && v0 >= 1) ? (int)sd.s0[v0 - 1] : 0;
    bad = bad || r >= alpha;
    r0[u] = __builtin_amdgcn_readfirstlane(r >= alpha ? 0 : r);
  }
  int r1 = (v0top <= sd.n0 && col_ok && v1 >= 1) ? (int)sd.s1[v1 - 1] : 0;
  bad = bad || r1 >= alpha;
  if (bad) atomicCAS(&ctrl->status, 0, -1);
  r1 = r1 >= alpha ? 0 : r1;
  const bool x0 = w == kSwNW - 1 && B0 < sd.nb0 - 1 && v0top + kSwRPW - 1 <= sd.n0;
  const bool x1 = B1 < sd.nb1 - 1 && v0top <= sd.n0;
  // the score: the corner cell's t = n2 is row uc of wave wc, lane jc, at
  // step sc of workgroup (n0 / kSwRows, n1 / 64)
  const int rc = sd.n0 % kSwRows;
  const bool cw = B0 == sd.n0 / kSwRows && B1 == sd.n1 / kSwLanes && w == rc / kSwRPW;
  const int jc = sd.n1 % kSwLanes;
  const int sc = sd.n2 + jc + w;
  const int uc = rc % kSwRPW;
  sw_barrier();  // the loader's halo of steps -1 and 0 is in LDS
  if (sd.egf)
    sweep_rows<true>(sd, sm, B0, B1, w, j, ok, r0, r1, gap, tag, total, x0, x1, cw, sc, uc, jc);
  else
    sweep_rows<false>(sd, sm, B0, B1, w, j, ok, r0, r1, gap, tag, total, x0, x1, cw, sc, uc, jc);
}

int launch_sweep3(const Plan &p, char *ws, const JobDev &jd, Ctrl *ctrl, int32_t flags,
                  hipStream_t s) {
  Sweep3Dev sd;
  sd.n0 = p.n[0];
  sd.n1 = p.n[1];
  sd.n2 = p.n[2];
  sd.nb0 = p.sw_nb0;
  sd.nb1 = p.sw_nb1;
  sd.s0 = jd.seqs;
  sd.s1 = jd.seqs + p.n[0];
  sd.s2 = jd.seqs + p.n[0] + p.n[1];
  sd.sub = jd.sub;
  sd.x0 = reinterpret_cast<int32_t *>(ws + p.off_x0);
  sd.x0_plane = p.x0_plane;
  sd.x1 = reinterpret_cast<int32_t *>(ws + p.off_x1);
  sd.x1_plane = p.x1_plane;
  sd.dir = jd.dir;
  sd.ts0 = p.tstride[0];
  sd.ts1 = p.tstride[1];
  sd.score_out = jd.score_out;
  sd.trace = jd.trace;
  sd.egf = (flags & kEndGapsFree) != 0;
  sd.best = &ctrl->best;
  // One workgroup per CU: a second one would share the SIMDs and stretch the
  // steps of both, and every step sits on the sweep's critical path.  The
  // launch asks for unused LDS beyond half of a CU's.
  int dev = 0, lds_cu = 0, lds_wg = 0;
  size_t pad = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) ==
          hipSuccess &&
      hipDeviceGetAttribute(&lds_wg, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess) {
    const size_t want = (size_t)lds_cu / 2 + 1024;
    if (want > sizeof(SwSmem) && want <= (size_t)lds_wg) pad = want - sizeof(SwSmem);
  }
  const int grid = p.sw_nb0 * p.sw_nb1;
  launch_begin();
  hipLaunchKernelGGL(sweep3_kernel, dim3(grid), dim3(kSwThreads), pad, s, sd, ctrl);
  return launch_end();
}

}  // namespace msa
