// msa_kernels.hip -- gfx950 kernels for the k-dimensional alignment DP.
//
// fill       : persistent tile-dataflow kernel.  Workgroups pop tiles from a
//              queue ordered by computation wave (Section 3: partitions at
//              equal distance from the origin are independent), wait for the
//              k face-predecessor tiles, import the halo from HBM face
//              planes, sweep the tile's local hyperplanes in LDS, export the
//              tile's upper faces and its direction block, then publish a
//              completion flag.
// traceback  : one wave walks the direction blocks from the far corner to the
//              origin (Section 2), then expands the masks into gapped rows.
// export     : decision tensor in row-major order (verification only).
//
// Per cell (Section 2 / Eq. 1 generalised; Section 4 per-cell steps): the
// pair scores of the column, the 2^k - 1 lower neighbours, one candidate per
// neighbour, the maximum.  Candidates are packed keys
//     key = (score << k) | (2^k - 1 - b)
// so one signed integer max yields the best score and, among equal scores,
// the lowest neighbour mask b.  Stored scores keep the low k bits clear.
#include <hip/hip_runtime.h>
#include <stdlib.h>

#include "msa_internal.h"

namespace msa {

enum { ST_OK = 0, ST_EINVAL = -1, ST_EDEVICE = -4 };

constexpr int kSubLds = 32;  // substitution matrices up to 32x32 live in LDS

// 16-byte vector moved as one value (plain loads and stores, no memcpy)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// LDS word strides of the tile with halo, dimension k-1 last (stride 1).  Each
// stride exceeds T times the sum of the strides after it, so every cell of the
// (T+1)^k box has its own word.  Within that freedom they are chosen to spread
// one sweep step's accesses over the LDS banks for the lanes' lines
// (LineOrder): consecutive lines for k <= 3, coordinate-sum order for k = 4;
// k = 5 keeps the strides chosen for consecutive lines.
template <int K> struct Strides;
template <> struct Strides<2> { static constexpr int v[2] = {34, 1}; };
template <> struct Strides<3> { static constexpr int v[3] = {305, 18, 1}; };
template <> struct Strides<4> { static constexpr int v[4] = {743, 82, 9, 1}; };
template <> struct Strides<5> { static constexpr int v[5] = {709, 145, 26, 5, 1}; };
template <> struct Strides<6> { static constexpr int v[6] = {1024, 256, 64, 16, 4, 1}; };
template <> struct Strides<7> { static constexpr int v[7] = {733, 244, 81, 27, 9, 3, 1}; };
template <> struct Strides<8> { static constexpr int v[8] = {2197, 733, 244, 81, 27, 9, 3, 1}; };

template <int K>
struct Cfg {
  static constexpr int T = tile_edge_for_k(K);
  static constexpr int E = T + 1;           // LDS edge including the halo
  static constexpr int KL = K - 1;          // sweep dimension: one lane per line along it
  static constexpr int L = ipow(T, K - 1);  // lines of a full tile
  static constexpr int NC = ipow(T, K);     // cells of a full tile
  static constexpr int NP = K * (K - 1) / 2;
  static constexpr int M = (1 << K) - 1;
  static constexpr int ML = (1 << (K - 1)) - 1;  // neighbour masks over dimensions 0..k-2
  static constexpr int DBS = (NC + 15) / 16 * 16;
  // Direction bytes of a line accumulate in registers (T/4 words per lane) and
  // are stored straight to the tile's block when T is a multiple of 4;
  // otherwise they are staged in LDS.
  static constexpr bool REGDIR = T % 4 == 0;
  // Neighbours one step back along the line are the values the lane read (or
  // wrote) in the previous step: carried in registers for k <= 5.
  static constexpr bool CARRY = K <= 5;
  static constexpr int sstride(int i) { return Strides<K>::v[i]; }
  static constexpr int ns() {
    int s = 0;
    for (int i = 0; i < K; ++i) s += sstride(i);
    return T * s + 1;
  }
  static constexpr int NS = ns();  // LDS score words
  static constexpr bool strides_ok() {
    if (sstride(K - 1) != 1) return false;
    for (int i = 0; i < K - 1; ++i) {
      int s = 0;
      for (int j = i + 1; j < K; ++j) s += sstride(j);
      if (sstride(i) <= T * s) return false;
    }
    return true;
  }
  static_assert(strides_ok(), "LDS strides must give every cell of the tile its own word");
  static constexpr int dstride(int i) { return ipow(T, K - 1 - i); }
  static constexpr int pair_index(int i, int j) {  // i < j
    return i * (2 * K - i - 1) / 2 + (j - i - 1);
  }
  static constexpr int off(int b) {  // LDS offset of neighbour v - b
    int o = 0;
    for (int i = 0; i < K; ++i)
      if ((b >> i) & 1) o += sstride(i);
    return o;
  }
};

// Lane p of the sweep takes line v[p].  For k >= 4 the lines are in
// ascending order of their coordinate sum (ties by line index): a line with
// sum s is active in steps s .. s + T - 1, so a wave whose lines have nearly
// equal sums issues the step body in few more steps than one line needs,
// where consecutive line indices span a sum range of about 2T (129^4 fill
// 2.27 -> 1.89 ms).  For k <= 3 the fill is bound by the latency of its steps
// rather than by issue, and consecutive lines keep the LDS banks apart, so
// the order is the identity.
template <int K>
struct LineOrder {
  uint16_t v[Cfg<K>::L];
  constexpr LineOrder() : v() {
    constexpr int T = Cfg<K>::T, L = Cfg<K>::L, KL = K - 1;
    int p = 0;
    if (K <= 3) {
      for (int l = 0; l < L; ++l) v[l] = (uint16_t)l;
      return;
    }
    for (int s = 0; s <= KL * (T - 1); ++s)
      for (int l = 0; l < L; ++l) {
        int rem = l, sum = 0;
        for (int i = 0; i < KL; ++i) {
          sum += rem % T;
          rem /= T;
        }
        if (sum == s) v[p++] = (uint16_t)l;
      }
  }
};
template <int K>
__device__ const LineOrder<K> kLineOrder{};

template <int K>
struct Smem {
  int32_t S[Cfg<K>::NS];                                // tile keys with halo
  int32_t PT[Cfg<K>::NP * Cfg<K>::T * Cfg<K>::T];       // pair scores << k
  // substitution matrix << k: |sub| <= 127, so the values fit 16 bits for
  // every k <= 8 (the 2 KB saved let one more k = 3 or k = 4 tile
  // workgroup share a compute unit's LDS)
  int16_t SUB[kSubLds * kSubLds];
  uint8_t RES[K * Cfg<K>::T];                           // residues of the tile
  uint16_t LORD[K <= 3 ? 1 : Cfg<K>::L];                // LineOrder<K> (k >= 4)
  alignas(16) uint8_t DIRB[Cfg<K>::REGDIR ? 16 : Cfg<K>::DBS];  // staged direction bytes
};

__device__ inline int64_t wall_now() { return (int64_t)wall_clock64(); }

// Optional phase timestamps per tile (compile with -DMSA_TRACE): 8 int64 per
// tile, written by every lane of the wave (same value, no divergent branch):
// 0 start, 1 dependencies met, 2 halo loaded, 3 swept, 5 faces exported,
// 6 flag stored, 4 end (direction block stored), 7 the workgroup.
#ifdef MSA_TRACE
#define MSA_TRACE_POINT(jd, tile, j) \
  do { if ((jd).trace) (jd).trace[(int64_t)(tile) * 8 + (j)] = wall_now(); } while (0)
#else
#define MSA_TRACE_POINT(jd, tile, j) do { } while (0)
#endif

// Watchdog for dependency waits: 2 s of waiting while the wave runs
// (WaitClock: 100 MHz ticks, pauses of the queue excluded).
constexpr int64_t kWaitLimitTicks = 200000000;
// Longest pause between two polls of a dependency wait, in units of
// s_sleep 2 (about 128 clocks each).
#ifndef MSA_MAX_NAP
#define MSA_MAX_NAP 16
#endif
constexpr int kMaxNap = MSA_MAX_NAP;

// Face-plane accesses.  Face values are relaxed agent-scope atomics
// (device-coherent loads and stores that bypass the non-coherent per-XCD
// cache state); a tile's completion flag is stored only after the wave's face
// stores have completed (see process_tile), so a reader that has seen the
// flag reads the final face values.
__device__ inline int32_t face_load(const int32_t *p) {
  return __hip_atomic_load(const_cast<int32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void face_store(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tile coordinates of a (wave-uniform) row-major tile index: the digits in
// the mixed radix P, one division by tstride[i] per dimension, each a
// multiply-high with the job's constants (tdm, tdsh; exact for every 32-bit
// index), so they take scalar instructions.
template <int K>
__device__ __forceinline__ void tile_coords(const JobDev &jd, int tile, int (&c)[K]) {
  uint32_t rem = (uint32_t)tile;
#pragma unroll
  for (int i = 0; i < K - 1; ++i) {
    const uint32_t t = __umulhi(jd.tdm[i], rem);
    const uint32_t sh = jd.tdsh[i];
    const uint32_t q = (t + ((rem - t) >> (sh & 0xffu))) >> (sh >> 8);
    c[i] = (int)q;
    rem -= q * (uint32_t)jd.tstride[i];
  }
  c[K - 1] = (int)rem;
}

// Per-launch constant table into LDS (done once per persistent workgroup).
template <int K, int NT>
__device__ void load_tables(const JobDev &jd, int alpha, Smem<K> &sm) {
  const int tid = threadIdx.x;
  if (alpha <= kSubLds)
    for (int e = tid; e < alpha * alpha; e += NT)
      sm.SUB[(e / alpha) * kSubLds + e % alpha] = (int16_t)(((int32_t)jd.sub[e]) * (1 << K));
  if constexpr (K >= 4)
    for (int p = tid; p < Cfg<K>::L; p += NT) sm.LORD[p] = kLineOrder<K>.v[p];
}

// Appends one byte at the top of a little-endian register queue of NR words
// (the oldest byte leaves at the bottom).
template <int NR>
__device__ inline void shift_in(uint32_t (&d)[NR], uint32_t byte) {
#pragma unroll
  for (int r = 0; r < NR - 1; ++r) d[r] = (d[r] >> 8) | (d[r + 1] << 24);
  d[NR - 1] = (d[NR - 1] >> 8) | (byte << 24);
}

// The halo slots a lane fills: slot tid + it * NT of the (T+1)^(k-1) cells of
// one face layer, as its base-(T+1) digits (least significant first, HB bits
// each), with bit 31 set for slots beyond the layer.  They do not depend on
// the tile, so for up to four slots per lane (k <= 7) they are computed once
// per workgroup instead of by division in every tile; k = 8 (nine slots,
// every register taken) computes them per tile.
template <int K, int NT>
struct HaloSlots {
  static constexpr int E = Cfg<K>::E;
  static constexpr int CNT = ipow(E, K - 1);
  static constexpr int IT = (CNT + NT - 1) / NT;
  static constexpr int HB = bits_for(E - 1);
  static constexpr bool PRE = IT <= 4;
  static_assert((K - 1) * HB <= 31, "digits fit below bit 31");
  uint32_t d[PRE ? IT : 1];
  __device__ static uint32_t compute(int tid, int it) {
    const int idx = tid + it * NT;
    uint32_t w = idx < CNT ? 0u : 0x80000000u;
    int rem = idx;
#pragma unroll
    for (int q = 0; q < K - 1; ++q) {
      w |= (uint32_t)(rem % E) << (q * HB);
      rem /= E;
    }
    return w;
  }
  __device__ explicit HaloSlots(int tid) {
#pragma unroll
    for (int it = 0; it < (PRE ? IT : 1); ++it) d[it] = PRE ? compute(tid, it) : 0u;
  }
  __device__ static int digit(uint32_t w, int q) { return (int)((w >> (q * HB)) & ((1u << HB) - 1)); }
};

// ---------------------------------------------------------------------------
// One tile of the fill.
// ---------------------------------------------------------------------------
// coopt: co-optimal mode (plain path, k <= 3): the direction byte of a cell is
// its tie set, bit b - 1 for every mask b whose candidate reaches the maximum
// (the origin's is 0).
// egf: end-gap-free mode (plain path): tiles with some c_i = 0 hold the cells
// with some v_i = 0, which score 0 with no decision; tiles on a far face fold
// their far-face cells into *best as (score << 32 | row-major cell index).
// prune: pruned mode (plain path, k <= 6): only kept tiles (jd.keep) run; a
// tile waits for every kept lower-neighbour tile and takes the halo cells of
// the others as -infinity.
// own0: the tile's predecessor along dimension 0 was this workgroup's previous
// tile (column schedule), so its last layer is still in LDS: that halo face is
// copied inside LDS instead of loaded, and its flag is not polled.
// cols: column schedule; no tile reads a dimension-0 face plane, so none is
// exported.
// scores: near-optimal mode: every cell's score is stored as well, in the
// layout of the direction block (jd.scores + tile * DBS).
// wlim: the dependency-wait time-out (100 MHz ticks), read by the kernel
// once (a load in every wait would also wait for the tile's stores: one
// counter tracks both).
template <int K, int NT>
__device__ void process_tile(const JobDev &jd, int alpha, int gap, int tile, int epoch,
                             Ctrl *ctrl, int32_t *jstatus, Smem<K> &sm,
                             const HaloSlots<K, NT> &hs, bool egf = false,
                             int64_t *best_key = nullptr, bool coopt = false,
                             bool prune = false, bool own0 = false, bool cols = false,
                             bool scores = false, int64_t wlim = kWaitLimitTicks) {
  using C = Cfg<K>;
  constexpr int T = C::T;
  constexpr int E = C::E;
  constexpr int M = C::M;
  constexpr int KL = C::KL;
  // The thread index is made opaque here so that values derived from it are
  // recomputed per tile instead of being hoisted out of the persistent loop
  // (which keeps them live in registers across every phase).
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));

  int c[K], lo[K], ext[K];
  bool origin = true, corner = true, lowtile = false, fartile = false;
  tile_coords<K>(jd, tile, c);
#pragma unroll
  for (int i = 0; i < K; ++i) {
    lo[i] = c[i] == 0 ? 0 : (c[i] - 1) * T + 1;
    ext[i] = c[i] == 0 ? 1 : min(T, jd.n[i] - (c[i] - 1) * T);
    origin = origin && c[i] == 0;
    corner = corner && c[i] == jd.P[i] - 1;
    lowtile = lowtile || c[i] == 0;
    fartile = fartile || c[i] == jd.P[i] - 1;
  }
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x) >> 6;
  const bool zero_tile = egf && lowtile;  // every cell scores 0, no decision

  MSA_TRACE_POINT(jd, tile, 0);
  // ---- residues of this tile (v = lo + q; sequence index v - 1) ----
  // They do not depend on the predecessor tiles, so they and the pair tables
  // are prepared before the dependency wait.  Loads are issued
  // unconditionally from clamped in-range addresses; the values are selected
  // and checked afterwards.
  {
    int r[K];
    const bool any_seq = jd.total_len > 0;  // uniform: no sequence bytes at all
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int q = tid < T ? tid : 0;
      const int v = lo[i] + q;
      const bool use = tid < T && q < ext[i] && v >= 1;
      const int pos = use ? jd.seq_off[i] + v - 1 : 0;
      r[i] = any_seq ? (int)jd.seqs[pos] : 0;
      r[i] = use ? r[i] : 0;
    }
    bool bad = false;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      bad = bad || r[i] >= alpha;
      if (tid < T) sm.RES[i * T + tid] = (uint8_t)(r[i] >= alpha ? 0 : r[i]);
    }
    if (bad) atomicCAS(jstatus, ST_OK, ST_EINVAL);
  }
  __syncthreads();

  // ---- pair tables: PT[p][a][b] = sub(r_i(a), r_j(b)) << k ----
#pragma unroll
  for (int i = 0; i < K; ++i) {
#pragma unroll
    for (int j = i + 1; j < K; ++j) {
      constexpr int TT = T * T;
      int32_t *pt = sm.PT + C::pair_index(i, j) * TT;
      for (int idx = tid; idx < TT; idx += NT) {
        const int a = sm.RES[i * T + idx / T];
        const int b = sm.RES[j * T + idx % T];
        pt[idx] = alpha <= kSubLds ? (int32_t)sm.SUB[a * kSubLds + b]
                                   : ((int32_t)jd.sub[a * alpha + b]) * (1 << K);
      }
    }
  }

  // ---- kept lower-neighbour tiles (pruned mode): bit S for tile c - e_S ----
  uint64_t kbits = ~0ull;
  if constexpr (K <= kPruneMaxK) {
    if (prune) {
      const int S = tid & 63;
      bool ok = S >= 1 && S <= C::M;
      int tn = tile;
#pragma unroll
      for (int i = 0; i < K; ++i)
        if ((S >> i) & 1) {
          ok = ok && c[i] > 0;
          tn -= jd.tstride[i];
        }
      const int kv = jd.keep[ok ? tn : tile];
      kbits = __ballot(ok && kv != 0);
    }
  }

  // ---- column schedule: layer l_0 = 0 is the previous tile's last layer ----
  // (l_0 = its extent), still in LDS.  It is copied before the dependency
  // wait, so that the barrier after the wait orders every read and write of
  // the copy before the halo stores below, which rewrite words of both
  // layers (their l_i = 0 edges for i >= 1).
  if (own0) {
    using HS0 = HaloSlots<K, NT>;
    const int e0 = c[0] - 1 == 0 ? 1 : T;
#pragma unroll
    for (int it = 0; it < HS0::IT; ++it) {
      uint32_t w;
      if constexpr (HS0::PRE)
        w = hs.d[it];
      else
        w = HS0::compute(tid, it);
      int s = 0;
#pragma unroll
      for (int j = K - 1; j >= 1; --j) s += HS0::digit(w, K - 1 - j) * C::sstride(j);
      if ((w >> 31) == 0) sm.S[s] = sm.S[s + e0 * C::sstride(0)];
    }
  }

  // ---- wait for the k face predecessors (diagonal ones are implied) ----
  // (pruned mode: for every kept lower neighbour, lane S polling tile c - e_S)
  // Wave 0 polls: lane i reads the flag of tile c - e_i until it has seen it
  // (a flag never goes back within a launch), so satisfied lanes stop loading.
  // The loop condition is a wave vote and every exit test is wave-uniform, so
  // the wave never splits; the other waves wait at the barrier below.  Polls
  // back off exponentially up to kMaxNap sleeps: tiles popped far ahead of the
  // running wavefront would otherwise flood the memory system with
  // device-coherent loads and slow every tile's halo and face traffic.
  if (wave == 0) {
    const int32_t *f = jd.flags;
    bool need = false;
    if (K <= kPruneMaxK && prune) {
      need = ((kbits >> (tid & 63)) & 1) != 0;
      int tn = tile;
#pragma unroll
      for (int i = 0; i < K; ++i)
        if ((tid >> i) & 1) tn -= jd.tstride[i];
      f = jd.flags + (need ? tn : tile);
    } else {
#pragma unroll
      for (int i = 0; i < K; ++i) {
        if (tid == i && c[i] > 0 && !(own0 && i == 0)) {
          need = true;
          f = jd.flags + (tile - jd.tstride[i]);
        }
      }
    }
    WaitClock wc;
    int nap = 1;
    for (int it = 0;; ++it) {
      if (need) need = __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch;
      if (!__any(need)) break;
      if ((it & 7) == 7) {
        const int st = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&ctrl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (st == ST_EDEVICE) break;
        if (wc.tick() > wlim) {
          // all lanes: idempotent; the wave whose lane made the change
          // records the wait (every lane stores the same values)
          const int prev = atomicCAS(&ctrl->status, ST_OK, ST_EDEVICE);
          const uint64_t missing = __ballot(need);
          if (__any(prev == ST_OK)) {
            // the first missing predecessor: its tile and the flag it holds
            const int lm = missing ? (int)__builtin_ctzll(missing) : 0;
            const int64_t ptile =
                __shfl((int)(f - jd.flags), lm, 64);
            const int32_t pval = __shfl(
                __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), lm, 64);
            ctrl->wd[0] = jd.qbase;
            ctrl->wd[1] = tile;
            ctrl->wd[2] = (int64_t)missing;
            ctrl->wd[3] = ptile;
            ctrl->wd[4] = pval;
            ctrl->wd[5] = __hip_atomic_load(&ctrl->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          break;
        }
      }
      for (int z = 0; z < nap; ++z) __builtin_amdgcn_s_sleep(2);
      nap = nap < kMaxNap ? 2 * nap : kMaxNap;
    }
    wc.report(ctrl);
  }
  __syncthreads();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);

  MSA_TRACE_POINT(jd, tile, 1);
  // ---- halo: layer l_i = 0 along each dimension ----
  // Loads first, LDS stores after: for small k every face load of every
  // dimension is in flight at once (one memory round trip per tile).
  // The slot digits are made opaque here, like the thread index, so that
  // nothing derived from them is kept live across the persistent loop.
  using HS = HaloSlots<K, NT>;
  uint32_t hd[HS::PRE ? HS::IT : 1];
  if constexpr (HS::PRE) {
#pragma unroll
    for (int it = 0; it < HS::IT; ++it) {
      hd[it] = hs.d[it];
      asm volatile("" : "+v"(hd[it]));
    }
  }
  // slot word it: precomputed, or (k = 8) computed where it is used
  auto slot = [&](int it) -> uint32_t {
    if constexpr (HS::PRE)
      return hd[it];
    else
      return HS::compute(tid, it);
  };
  {
    constexpr int cnt = ipow(E, K - 1);
    constexpr int IT = (cnt + NT - 1) / NT;
    constexpr bool ALL = K * IT <= 48;
    constexpr int CH = ALL ? IT : (IT < 6 ? IT : 6);
    constexpr int DG = ALL ? K : 1;  // dimensions per pass
    for (int i0 = 0; i0 < K; i0 += DG) {
      for (int it0 = 0; it0 < IT; it0 += CH) {
        int32_t val[DG][CH];
        int sidx[DG][CH];
#pragma unroll
        for (int di = 0; di < DG; ++di) {
          const int i = i0 + di;
          // Byte address of the halo's first cell (v_j = lo_j - 1, j != i)
          // in the face plane of tile c - e_i: wave-uniform, in scalar
          // registers.  A slot adds sum_j l_j * fbstride[i][j] with 32 x 32 ->
          // 64-bit multiply-adds (digits l_j <= T, byte strides below 2^32).
          int64_t hb = 0;
          if (c[i] > 0) {
            hb = jd.face_off[i] + (int64_t)(c[i] - 1) * jd.fplane[i];
#pragma unroll
            for (int j = 0; j < K; ++j)
              if (j != i) hb += (int64_t)(lo[j] - 1) * (jd.fbstride[i][j] >> 2);
          }
          const uint64_t hbase = (uint64_t)jd.faces + 4 * (uint64_t)hb;
#pragma unroll
          for (int it = 0; it < CH; ++it) {
            const uint32_t w = slot(it0 + it);
            int s = 0, q = 0;
            bool valid = (w >> 31) == 0, neg = (c[i] == 0);
            uint64_t addr = hbase;
            int src = 1 << i;  // the cell lies in tile c - e_src
#pragma unroll
            for (int j = K - 1; j >= 0; --j) {
              if (j == i) continue;
              const int l = HS::digit(w, q++);
              valid = valid && l <= ext[j];
              s += l * C::sstride(j);
              neg = neg || lo[j] - 1 + l < 0;
              src |= (l == 0 ? 1 : 0) << j;
              addr += (uint64_t)(uint32_t)l * jd.fbstride[i][j];
            }
            valid = valid && !(own0 && i == 0);  // copied inside LDS above
            sidx[di][it] = valid ? s : -1;
            // a cell of a pruned tile was never computed: -infinity
            const bool take = valid && !neg && ((kbits >> (src & 63)) & 1) != 0;
            // unconditional load from a clamped in-range offset, then select
            const int32_t got =
                face_load(take ? reinterpret_cast<const int32_t *>(addr) : jd.faces);
            val[di][it] = take ? got : kNegKey;
          }
        }
#pragma unroll
        for (int di = 0; di < DG; ++di)
#pragma unroll
          for (int it = 0; it < CH; ++it)
            if (sidx[di][it] >= 0) sm.S[sidx[di][it]] = val[di][it];
      }
    }
  }
  __syncthreads();

  MSA_TRACE_POINT(jd, tile, 2);
  // ---- sweep ----
  // Lane l owns line l = (q_0 .. q_{k-2}) of the tile and computes its cell
  // (line, t) at local hyperplane h = q_0 + ... + q_{k-2} + t, one cell per
  // step, with a barrier between steps.  The cell's LDS word is idx0 + t, so
  // the 2^k - 1 neighbours are fixed offsets below it; consecutive lanes hold
  // consecutive lines, whose words fall in distinct banks (strides above).
  constexpr int L = C::L;
  constexpr int U = (L + NT - 1) / NT;  // lines per lane
  constexpr int NR = C::REGDIR ? T / 4 : 1;
  uint32_t dr[U][NR];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int r = 0; r < NR; ++r) dr[u][r] = 0;
  if (origin) {
    // every lane writes the same values (no lane-divergent branch)
    int s = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) s += C::sstride(i);
    sm.S[s] = 0;
    if constexpr (C::REGDIR)  // lane 0 holds line 0 (coordinate sum 0)
      dr[0][0] = tid == 0 ? (coopt ? 0u : (uint32_t)M) : 0u;  // mask 0 / empty tie set
    else
      sm.DIRB[0] = (uint8_t)(coopt ? 0 : M);
  } else {
    constexpr int ML = C::ML;
    constexpr int NPL = KL * (KL - 1) / 2;  // pairs within the line dimensions
    int hmax = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) hmax += ext[i] - 1;
    const int extL = ext[KL];
    int32_t gk[K + 1];
#pragma unroll
    for (int cb = 0; cb <= K; ++cb) gk[cb] = (gap * cb * (K - cb)) * (1 << K);

    // Per lane and line: the word of cell (line, t = 0), the line's coordinate
    // sum, and the pair-table rows of the pairs (i, k-1).  For k <= 5 the sums
    // of the pair scores within the line dimensions (fixed along the line) are
    // kept per neighbour mask b' over those dimensions; for larger k the pair
    // scores are read from LDS at every step.
    constexpr bool LREG = K <= 5;
    int idx0[U], sq[U], pto[U][KL], qv[U][KL];
    int ln[C::REGDIR ? 1 : U];  // the lanes' lines (staged direction bytes)
    bool lv[U];
    int32_t lsum[LREG ? U : 1][LREG ? ML + 1 : 1];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int pl = tid + u * NT;
      // the lane's line (k >= 4: coordinate-sum order; k <= 3: the identity)
      const int l = K <= 3 ? pl : pl < L ? (int)sm.LORD[pl] : L;
      if constexpr (!C::REGDIR) ln[u] = l;
      int rem = l;
#pragma unroll
      for (int i = KL - 1; i >= 0; --i) {
        qv[u][i] = rem % T;
        rem /= T;
      }
      bool ok = l < L;
      int s = 0, x = 1;
#pragma unroll
      for (int i = 0; i < KL; ++i) {
        ok = ok && qv[u][i] < ext[i];
        s += qv[u][i];
        x += (qv[u][i] + 1) * C::sstride(i);
        pto[u][i] = C::pair_index(i, KL) * T * T + qv[u][i] * T;
      }
      lv[u] = ok;
      sq[u] = s;
      idx0[u] = x;  // word of cell (line, t = 0)
      if constexpr (LREG) {
#pragma unroll
        for (int bp = 0; bp <= ML; ++bp) {
          int32_t cs = 0;
#pragma unroll
          for (int i = 0; i < KL; ++i)
#pragma unroll
            for (int j = i + 1; j < KL; ++j)
              if (((bp >> i) & 1) && ((bp >> j) & 1))
                cs += sm.PT[C::pair_index(i, j) * T * T + qv[u][i] * T + qv[u][j]];
          lsum[u][bp] = cs;
        }
      }
    }
    // prv[b'] = key of (line - b', t - 1); before the first step the t = -1
    // layer is the halo.
    int32_t prv[C::CARRY ? U : 1][C::CARRY ? ML + 1 : 1];
    if constexpr (C::CARRY) {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int bp = 0; bp <= ML; ++bp) prv[u][bp] = sm.S[idx0[u] - 1 - C::off(bp)];
    }

    for (int h = 0; h <= hmax; ++h) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int t = h - sq[u];
        if (!(lv[u] && (unsigned)t < (unsigned)extL)) continue;
        const int p = idx0[u] + t;
        int32_t pk[KL];
#pragma unroll
        for (int i = 0; i < KL; ++i) pk[i] = sm.PT[pto[u][i] + t];
        int32_t pvl[LREG ? 1 : (NPL > 0 ? NPL : 1)];
        if constexpr (!LREG) {
          int pi = 0;
#pragma unroll
          for (int i = 0; i < KL; ++i)
#pragma unroll
            for (int j = i + 1; j < KL; ++j)
              pvl[pi++] = sm.PT[C::pair_index(i, j) * T * T + qv[u][i] * T + qv[u][j]];
        }
        int32_t nowv[ML + 1];
        if constexpr (C::CARRY) {
#pragma unroll
          for (int bp = 1; bp <= ML; ++bp) nowv[bp] = sm.S[p - C::off(bp)];
        }
        int32_t best = INT32_MIN;
        int32_t cand[M <= 8 ? M + 1 : 1];  // kept for tie sets (k <= 3)
#pragma unroll
        for (int b = 1; b <= M; ++b) {
          const int bp = b & ML;
          const bool hasL = (b >> KL) & 1;
          // column score of candidate b (Section 2: sum over the pairs of the
          // column), gap term and tie-break bits; all pre-shifted by k
          int32_t col = gk[__builtin_popcount(b)] + (M - b);
          if constexpr (LREG) {
            if (__builtin_popcount(bp) >= 2) col += lsum[u][bp];
          } else {
            int pi = 0;
#pragma unroll
            for (int i = 0; i < KL; ++i)
#pragma unroll
              for (int j = i + 1; j < KL; ++j) {
                if (((bp >> i) & 1) && ((bp >> j) & 1)) col += pvl[pi];
                ++pi;
              }
          }
          if (hasL) {
#pragma unroll
            for (int i = 0; i < KL; ++i)
              if ((bp >> i) & 1) col += pk[i];
          }
          int32_t pred;
          if constexpr (C::CARRY)
            pred = hasL ? prv[u][bp] : nowv[bp];
          else
            pred = sm.S[p - C::off(b)];
          if constexpr (M <= 8) cand[b] = pred + col;
          best = max(best, pred + col);
          // large k: at most 32 neighbour reads in flight (register pressure)
          if constexpr (M > 63)
            if ((b & 31) == 31) asm volatile("" ::: "memory");
        }
        if (zero_tile) best = M;  // key 0; the byte decodes to mask 0
        const int32_t sv = best & ~M;
        uint32_t byte = (uint32_t)best & 0xFFu;
        if constexpr (M <= 8) {
          if (coopt) {  // tie set: every candidate with the maximal score
            byte = 0;
#pragma unroll
            for (int b = 1; b <= M; ++b)
              byte |= ((cand[b] & ~M) == sv ? 1u : 0u) << (b - 1);
          }
        }
        sm.S[p] = sv;
        if constexpr (C::CARRY) {
          prv[u][0] = sv;
#pragma unroll
          for (int bp = 1; bp <= ML; ++bp) prv[u][bp] = nowv[bp];
        }
        if constexpr (C::REGDIR)
          shift_in<NR>(dr[u], byte);
        else
          sm.DIRB[ln[u] * T + t] = (uint8_t)byte;
      }
      __syncthreads();
    }
    if constexpr (C::REGDIR) {
      // lines shorter than T: move byte t = 0 down to the first byte
      for (int s = extL; s < T; ++s)
#pragma unroll
        for (int u = 0; u < U; ++u) shift_in<NR>(dr[u], 0u);
    }
  }
  __syncthreads();

  // ---- end-gap-free: best far-face cell of this tile ----
  // Cell (line, t) is on the far face of dimension i when c_i is the last tile
  // coordinate and q_i = ext_i - 1.  Key: score << 32 | row-major index (the
  // index fits 32 bits, checked on the host); largest key wins.
  if (egf && fartile) {
    constexpr int L = C::L;
    constexpr int U = (L + NT - 1) / NT;
    int64_t cs[K];  // row-major strides of the (n_i + 1) tensor
    {
      int64_t acc = 1;
#pragma unroll
      for (int i = K - 1; i >= 0; --i) {
        cs[i] = acc;
        acc *= (int64_t)jd.n[i] + 1;
      }
    }
    int64_t mykey = INT64_MIN;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int l = tid + u * NT;
      int q[KL > 0 ? KL : 1];
      int rem = l;
#pragma unroll
      for (int i = KL - 1; i >= 0; --i) {
        q[i] = rem % T;
        rem /= T;
      }
      bool ok = l < L, whole = false;  // whole: every cell of the line is far
      int x = 1;
      int64_t lin = 0;
#pragma unroll
      for (int i = 0; i < KL; ++i) {
        ok = ok && q[i] < ext[i];
        whole = whole || (c[i] == jd.P[i] - 1 && q[i] == ext[i] - 1);
        x += (q[i] + 1) * C::sstride(i);
        lin += (int64_t)(lo[i] + q[i]) * cs[i];
      }
      const bool lastL = c[KL] == jd.P[KL] - 1;
      if (ok && (whole || lastL)) {
        for (int t = whole ? 0 : ext[KL] - 1; t < ext[KL]; ++t) {
          const int64_t key = ((int64_t)(sm.S[x + t] >> K) << 32) |
                              (int64_t)(uint32_t)(lin + (int64_t)(lo[KL] + t) * cs[KL]);
          mykey = key > mykey ? key : mykey;
        }
      }
    }
    if (mykey != INT64_MIN) atomicMax((long long *)best_key, (long long)mykey);
  }

  MSA_TRACE_POINT(jd, tile, 3);
  // ---- export upper faces (layer l_i = ext_i) for the successor along i ----
  // All LDS reads of a pass first (unconditional, clamped index), then the
  // predicated global stores, so the reads are not serialised against them.
  {
    constexpr int cnt = ipow(T, K - 1);
    constexpr int IT = (cnt + NT - 1) / NT;
    constexpr int DG = K * IT <= 32 ? K : 1;  // dimensions per pass
    for (int i0 = 0; i0 < K; i0 += DG) {
      int32_t val[DG][IT];
      uint64_t fo[DG][IT];  // byte addresses
      bool st[DG][IT];
#pragma unroll
      for (int di = 0; di < DG; ++di) {
        const int i = i0 + di;
        const bool has_succ = c[i] < jd.P[i] - 1 && !(cols && i == 0);
        // byte address of the face's first cell (v_j = lo_j) in plane c_i:
        // wave-uniform, as in the halo load
        int64_t eb = jd.face_off[i] + (int64_t)c[i] * jd.fplane[i];
#pragma unroll
        for (int j = 0; j < K; ++j)
          if (j != i) eb += (int64_t)lo[j] * (jd.fbstride[i][j] >> 2);
        const uint64_t ebase = (uint64_t)jd.faces + 4 * (uint64_t)eb;
#pragma unroll
        for (int it = 0; it < IT; ++it) {
          const int idx = tid + it * NT;
          int rem = idx;
          int sidx = ext[i] * C::sstride(i);
          bool valid = has_succ && idx < cnt;
          uint64_t addr = ebase;
#pragma unroll
          for (int j = K - 1; j >= 0; --j) {
            if (j == i) continue;
            const int qq = rem % T;
            rem /= T;
            valid = valid && qq < ext[j];
            sidx += (qq + 1) * C::sstride(j);
            addr += (uint64_t)(uint32_t)qq * jd.fbstride[i][j];
          }
          val[di][it] = sm.S[valid ? sidx : 0];
          fo[di][it] = addr;
          st[di][it] = valid;
        }
      }
#pragma unroll
      for (int di = 0; di < DG; ++di)
#pragma unroll
        for (int it = 0; it < IT; ++it)
          if (st[di][it]) face_store(reinterpret_cast<int32_t *>(fo[di][it]), val[di][it]);
    }
  }

  MSA_TRACE_POINT(jd, tile, 5);
  // ---- publish completion ----
  // Each wave makes its own stores visible, the barrier orders all waves before
  // wave 0 stores the flag.  All 64 lanes of wave 0 store the same value: a
  // lane-divergent branch next to the persistent loop's back edge lets the
  // compiler peel lanes off the loop.
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);  // the wave's face stores have completed
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (wave == 0)
    __hip_atomic_store(jd.flags + tile, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  MSA_TRACE_POINT(jd, tile, 6);
  // The score and the direction block are stored after the flag: only the
  // traceback, a later kernel, reads them, and the completion wait before the
  // flag then covers the face stores alone.
  if (corner) {  // all lanes store the same value
    int s = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) s += ext[i] * C::sstride(i);
    *jd.score_out = (int64_t)(sm.S[s] >> K);
  }

  // ---- direction block: cell (line, t) at byte line * T + t ----
  {
    uint8_t *blk = jd.dir + (int64_t)tile * C::DBS;
    if constexpr (C::REGDIR) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int pl = tid + u * NT;
        if (pl < L) {
          const int l = K <= 3 ? pl : (int)sm.LORD[pl];  // the line this lane swept
          if constexpr (NR % 4 == 0) {
            uint4 *dst = reinterpret_cast<uint4 *>(blk + l * T);
#pragma unroll
            for (int r = 0; r < NR / 4; ++r)
              dst[r] = make_uint4(dr[u][4 * r], dr[u][4 * r + 1], dr[u][4 * r + 2],
                                  dr[u][4 * r + 3]);
          } else if constexpr (NR == 2) {
            *reinterpret_cast<uint2 *>(blk + l * T) = make_uint2(dr[u][0], dr[u][1]);
          } else {
            uint32_t *dst = reinterpret_cast<uint32_t *>(blk + l * T);
#pragma unroll
            for (int r = 0; r < NR; ++r) dst[r] = dr[u][r];
          }
        }
      }
    } else {
      const uint4 *src = reinterpret_cast<const uint4 *>(sm.DIRB);
      uint4 *dst = reinterpret_cast<uint4 *>(blk);
      for (int idx = tid; idx < C::DBS / 16; idx += NT) dst[idx] = src[idx];
    }
  }

  // ---- near-optimal mode: cell scores, index sum_i q_i * T^(k-1-i) ----
  if (scores) {
    int32_t *dst = jd.scores + (int64_t)tile * C::DBS;
    constexpr int NC = ipow(T, K);
    for (int idx = tid; idx < NC; idx += NT) {
      int rem = idx, x = 0;
      bool ok = true;
#pragma unroll
      for (int i = K - 1; i >= 0; --i) {
        const int q = rem % T;
        rem /= T;
        ok = ok && q < ext[i];
        x += (q + 1) * C::sstride(i);
      }
      if (ok) dst[idx] = sm.S[x] >> K;
    }
  }

  MSA_TRACE_POINT(jd, tile, 4);
#ifdef MSA_TRACE
  if (jd.trace) jd.trace[(int64_t)tile * 8 + 7] = blockIdx.x;
#endif
}

// The plain fill's job descriptor for one tile: the kernel's first argument,
// read in the kernel-argument segment (explicit arguments start at its
// offset 0).  The descriptor's fields are loop-invariant, so the compiler
// would load them all before the persistent loop and, short of scalar
// registers, park them in vector register lanes, paying a v_readlane (a
// vector instruction) at every use in every tile.  Seen through a pointer
// into the segment (constant address space) that is opaque at each tile,
// they are reloaded per tile with scalar loads instead; the segment stays in
// the scalar cache.  (The parameter's own address would not do: taking it
// makes the compiler copy the argument to private memory.)  k = 8, whose
// tile code takes every vector register anyway, keeps the parameter: there
// the per-tile reloads made the compiler spill to scratch.
template <int K>
__device__ __forceinline__ const JobDev &job_arg(const JobDev &jd) {
  if constexpr (K >= 8) {
    return jd;
  } else {
    using CJob = const __attribute__((address_space(4))) JobDev;
    CJob *kp = (CJob *)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(kp));
    return *(const JobDev *)kp;
  }
}

// Plain path: one job, descriptor passed by value (first argument: job_arg
// reads it in place).
// pass (pruned mode): 1 = first pass, 2 = second pass, which runs only when
// the first missed its threshold; 0 otherwise.
template <int K, int NT>
__global__ __launch_bounds__(NT) void fill_kernel(JobDev jd, Ctrl *ctrl,
                                                  const int32_t *__restrict__ order, int pass) {
  __shared__ Smem<K> sm;
  if (pass == 2 && __builtin_amdgcn_readfirstlane(ctrl->redo) == 0) return;
  const int alpha = ctrl->alpha;
  const int gap = ctrl->gap;
  const int mode = __builtin_amdgcn_readfirstlane(ctrl->flags);
  const bool egf = (mode & kEndGapsFree) != 0;
  const bool coopt = (mode & kCoOptimal) != 0;
  const bool prune = (mode & kPrune) != 0;
  const bool nearopt = (mode & kNearOpt) != 0;
  // column schedule (not in pruned mode): a workgroup takes a column of tiles
  // along dimension 0 and computes it bottom up
  const bool cols = !prune && jd.ncols > 0;
  const int nq = prune ? __builtin_amdgcn_readfirstlane(ctrl->nqueue)
                       : cols ? jd.ncols : jd.ntiles;
  load_tables<K, NT>(jd, alpha, sm);
  const HaloSlots<K, NT> hs(threadIdx.x);
  const int epoch = __hip_atomic_load(&ctrl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  static_assert(NT % 64 == 0, "whole waves per workgroup");
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x) >> 6;
  __shared__ int32_t bcast;
  for (;;) {
    // Queue pop without a lane-divergent branch: wave 0's lanes all issue the
    // atomic, only lane 0 adds 1, lane 0's result is broadcast through LDS and
    // read back as a wave-uniform (SGPR) value, so the loop exit is uniform.
    if (wave == 0) {
      const int got = atomicAdd(&ctrl->head, threadIdx.x == 0 ? 1 : 0);
      bcast = __builtin_amdgcn_readfirstlane(got);
    }
    __syncthreads();
    const int qi = __builtin_amdgcn_readfirstlane(bcast);
    __syncthreads();
    if (qi >= nq) break;
    if (cols) {
      const int base = __builtin_amdgcn_readfirstlane(jd.corder[qi]);
      for (int c0 = 0; c0 < jd.P[0]; ++c0)
        process_tile<K, NT>(job_arg<K>(jd), alpha, gap, base + c0 * jd.tstride[0], epoch, ctrl,
                            &ctrl->status, sm, hs, egf, &ctrl->best, coopt, false, c0 > 0, true,
                            nearopt);
    } else {
      process_tile<K, NT>(job_arg<K>(jd), alpha, gap, __builtin_amdgcn_readfirstlane(order[qi]),
                          epoch, ctrl, &ctrl->status, sm, hs, egf, &ctrl->best, coopt, prune,
                          false, false, nearopt);
    }
  }
}

// ---------------------------------------------------------------------------
// Traceback: one workgroup of one wave.
// ---------------------------------------------------------------------------
// egf: end-gap-free mode; best is the fill's far-face key (score << 32 |
// row-major index of the end cell).  The walk then starts at that cell, stops
// at the first cell with some v_i = 0, and the unaligned suffixes and prefixes
// become one-residue columns (sequence 0 first in the output).
// coopt: the direction bytes are tie sets; the walk takes the lowest mask of
// each, which is the decision of the plain mode.
// The modes are template parameters so that the plain walk's step loop has
// no mode branches.
template <int K, bool egf = false, bool coopt = false>
__device__ void traceback_job(const JobDev &jd, int status_in, uint8_t *dirb,
                              int64_t best = 0) {
  using C = Cfg<K>;
  constexpr int T = C::T;
  constexpr int M = C::M;
  constexpr int NQ = C::DBS / 16;        // 16-byte chunks per direction block
  constexpr int CPL = (NQ + 63) / 64;    // chunks per lane
  // Blocks of the lower neighbour tiles are prefetched into registers on
  // entering a tile: all 2^k - 1 of them while that takes at most 128
  // registers, else the k face neighbours (other exits load on demand).
  constexpr bool ALLN = M * CPL * 4 <= 128;
  constexpr int NPF = ALLN ? M : K;
  const int tid = threadIdx.x;
  const int NT = blockDim.x;
  int status = __builtin_amdgcn_readfirstlane(status_in);

  int v[K], c[K], q[K];
  int Li = 0;                      // path length so far (sum n_i < 2^31)
  int pbuf = 0;  // path bytes L & ~63 .. L - 1, one per lane, flushed every 64
  auto emit = [&](int b) {
    pbuf = tid == (Li & 63) ? b : pbuf;
    ++Li;
    if ((Li & 63) == 0) jd.path[Li - 64 + tid] = (uint8_t)pbuf;
  };
  bool done = true;
  if constexpr (egf) {
    // end cell from its row-major index; the suffixes after it are emitted
    // first (the path is recorded end first): sequence k-1's, ..., sequence 0's
    int64_t lin = (int64_t)(uint32_t)best;
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
      v[i] = (int)(lin % ((int64_t)jd.n[i] + 1));
      lin /= (int64_t)jd.n[i] + 1;
    }
    bool anyz = false;
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
      for (int x = v[i]; x < jd.n[i]; ++x) emit(1 << i);
      anyz = anyz || v[i] == 0;
    }
    done = anyz;
  } else {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      v[i] = jd.n[i];
      done = done && v[i] == 0;
    }
  }
  if (status != ST_OK) done = true;
  u32x4 *const lds4 = reinterpret_cast<u32x4 *>(dirb);

  u32x4 pf[NPF > 0 ? NPF : 1][CPL];
  int64_t t = 0;
  if (!done) {
#pragma unroll
    for (int i = 0; i < K; ++i) {
      c[i] = v[i] == 0 ? 0 : (v[i] - 1) / T + 1;
      t += (int64_t)c[i] * jd.tstride[i];
    }
    const u32x4 *src = reinterpret_cast<const u32x4 *>(jd.dir + t * C::DBS);
    for (int idx = tid; idx < NQ; idx += 64) lds4[idx] = src[idx];
  }
  while (!done) {
    // position in the current tile (already in LDS)
    int d = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      q[i] = v[i] - (c[i] == 0 ? 0 : (c[i] - 1) * T + 1);
      d += q[i] * C::dstride(i);
    }
    // prefetch the neighbour blocks (an absent neighbour loads this tile)
#pragma unroll
    for (int s = 0; s < NPF; ++s) {
      const int S = ALLN ? s + 1 : 1 << s;
      int64_t tn = t;
      bool ok = true;
#pragma unroll
      for (int i = 0; i < K; ++i)
        if ((S >> i) & 1) {
          ok = ok && c[i] > 0;
          tn -= jd.tstride[i];
        }
      const u32x4 *src = reinterpret_cast<const u32x4 *>(jd.dir + (ok ? tn : t) * C::DBS);
#pragma unroll
      for (int x = 0; x < CPL; ++x) {
        const int idx = tid + x * 64;
        pf[s][x] = src[idx < NQ ? idx : NQ - 1];
      }
    }
    __syncthreads();
    // The walk inside the tile tracks only the tile position q and its byte
    // offset d; v = base + q follows when the walk leaves.  A cell with some
    // v_i = 0 (the end of the walk) lies only in a tile with c_i = 0, where
    // q_i = v_i; elsewhere the loop checks nothing but the mask and the exit.
    // Every step lowers sum(v) by at least one, so the walk takes at most
    // sum n_i steps (the path's capacity) before it ends or steps below some
    // v_i = 0, which the exit check below catches.
    int base[K];
    uint32_t zmask = 0;  // dimensions with c_i = 0
#pragma unroll
    for (int i = 0; i < K; ++i) {
      base[i] = c[i] == 0 ? 0 : (c[i] - 1) * T + 1;
      zmask |= (uint32_t)(c[i] == 0) << i;
    }
    bool bad = false;
    // k <= 6: lane l reads the byte of the cell mask l below the current one,
    // so the next step's byte is a register read (readlane by the decoded
    // mask), and the read for the step after it is issued before this step's
    // remaining work instead of after it.  A candidate outside the block
    // reads a clamped address and is never used: a step to it leaves the tile.
    // (k > 6: one uniform read per step.)
    constexpr bool CAND = M < 64;
    int loff = 0;
    if constexpr (CAND) {
#pragma unroll
      for (int i = 0; i < K; ++i) loff += ((tid & M) >> i & 1) * C::dstride(i);
    }
    int cand = CAND ? dirb[max(d - loff, 0)] : 0;
    int byte = CAND ? __builtin_amdgcn_readlane(cand, 0) : 0;
    for (;;) {
      // every lane walks the same path: keep the walk state wave-uniform
      if constexpr (!CAND) byte = __builtin_amdgcn_readfirstlane(dirb[d]);
      const int b = coopt ? (byte ? __builtin_ctz(byte) + 1 : 0) : M - (byte & M);
      if (b == 0) {  // corrupt decision data: a cell without a move
        bad = true;
        break;
      }
      int qor = 0;
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const int bi = (b >> i) & 1;
        q[i] -= bi;
        d -= bi * C::dstride(i);
        qor |= q[i];
      }
      if constexpr (CAND) {
        byte = __builtin_amdgcn_readlane(cand, b);  // the next cell's byte
        cand = dirb[max(d - loff, 0)];              // its successors' bytes
      }
      emit(b);
      if (qor < 0) break;  // left the tile
      if (zmask != 0) {
        // the end of the walk: every v_i = 0 (plain), some v_i = 0 (end gaps free)
        bool stop = !egf;
#pragma unroll
        for (int i = 0; i < K; ++i) {
          const bool z = ((zmask >> i) & 1) != 0 && q[i] == 0;
          stop = egf ? (stop || z) : (stop && z);
        }
        if (stop) {
          done = true;
          break;
        }
      }
    }
    // the step that left the tile may also have ended the walk
    bool allz = true, anyz = false;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      v[i] = base[i] + q[i];
      bad = bad || v[i] < 0;  // a step below v_i = 0: corrupt decision data
      allz = allz && v[i] == 0;
      anyz = anyz || v[i] == 0;
    }
    if (bad) {
      status = ST_EDEVICE;
      done = true;
    }
    done = done || (egf ? anyz : allz);
    if (done) break;
    // enter the next tile: its block was prefetched unless the walk left
    // through an edge or corner that is not in the prefetched set
    int S = 0;
    t = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int ci = v[i] == 0 ? 0 : (v[i] - 1) / T + 1;
      if (ci != c[i]) S |= 1 << i;
      c[i] = ci;
      t += (int64_t)ci * jd.tstride[i];
    }
    __syncthreads();
    bool hit = false;
#pragma unroll
    for (int s = 0; s < NPF; ++s) {
      const int Ss = ALLN ? s + 1 : 1 << s;
      if (Ss == S) {
#pragma unroll
        for (int x = 0; x < CPL; ++x) {
          const int idx = tid + x * 64;
          if (idx < NQ) lds4[idx] = pf[s][x];
        }
        hit = true;
      }
    }
    if (!hit) {
      const u32x4 *src = reinterpret_cast<const u32x4 *>(jd.dir + t * C::DBS);
      for (int idx = tid; idx < NQ; idx += 64) lds4[idx] = src[idx];
    }
  }
  if (egf && status == ST_OK) {
    // the unaligned prefixes before the start cell: sequence k-1's, ..., 0's
#pragma unroll
    for (int i = K - 1; i >= 0; --i)
      for (int x = 0; x < v[i]; ++x) emit(1 << i);
  }
  if ((Li & 63) != 0 && tid < (Li & 63)) jd.path[(Li & ~63) + tid] = (uint8_t)pbuf;
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  const int64_t L = status != ST_OK ? 0 : Li;

  // expand masks (path[L-1] is the first column) into gapped rows
  int cnt[K];
#pragma unroll
  for (int i = 0; i < K; ++i) cnt[i] = 0;
  for (int64_t c0 = 0; c0 < L; c0 += NT) {
    const int64_t col = c0 + tid;
    const int m = col < L ? jd.path[L - 1 - col] : 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int bit = (m >> i) & 1;
      // inclusive prefix sum over the workgroup (one wave)
      int incl = bit;
      for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(incl, d, 64);
        if ((tid & 63) >= d) incl += y;
      }
      const int pos = cnt[i] + incl - bit;
      if (col < L)
        jd.aln_out[(int64_t)i * jd.aln_cap + col] =
            bit ? jd.seqs[jd.seq_off[i] + pos] : (uint8_t)0xFF;
      cnt[i] += __shfl(incl, 63, 64);
    }
  }
  if (tid == 0) {
    *jd.aln_len_out = L;
    *jd.status_out = status;
    if (status != ST_OK)
      *jd.score_out = 0;
    else if (egf)
      *jd.score_out = best >> 32;
  }
}

template <int K>
__global__ __launch_bounds__(64) void traceback_kernel(JobDev jd, Ctrl *ctrl) {
  __shared__ alignas(16) uint8_t dirb[Cfg<K>::DBS];
  const bool egf = (ctrl->flags & kEndGapsFree) != 0;
  const bool coopt = (ctrl->flags & kCoOptimal) != 0;
  const int st = __hip_atomic_load(&ctrl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (egf)
    traceback_job<K, true, false>(
        jd, st, dirb, __hip_atomic_load(&ctrl->best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  else if (coopt)
    traceback_job<K, false, true>(jd, st, dirb);
  else
    traceback_job<K, false, false>(jd, st, dirb);
  __syncthreads();
  if (threadIdx.x == 0) {
    // ready the control block for the next launch on this workspace
    ctrl->head = 0;
    ctrl->status = ST_OK;
    ctrl->best = INT64_MIN;
    ctrl->epoch = ctrl->epoch + 1;
  }
}

// ---------------------------------------------------------------------------
// Co-optimal alignments (co-optimal mode, k <= 3): one wave walks depth first
// from the far corner along tie-set masks, trying the masks of each cell in
// ascending order.  Every such walk reaches the origin with the optimal score
// and every optimal alignment is one, so the alignments come in lexicographic
// order of their column masks read from the last column to the first (the
// first is the plain traceback's).  The stack of chosen masks lives in LDS
// (sum n_i <= kCoMaxTotal), each entry with a flag (kMoreTies) when that cell
// has tied masks above the one taken; after an alignment the walk jumps back
// to the deepest flagged level with one wave-wide scan of the stack instead of
// stepping back through the cells.  The direction block of the current cell's
// tile is cached in LDS.  Alignment p goes to aln_out + p * k * aln_cap.
// ---------------------------------------------------------------------------
constexpr int kMoreTies = 0x80;  // stack entry flag: the cell has tied masks above it
constexpr int kMaskBits = 0x7F;

template <int K>
__global__ __launch_bounds__(64) void coopt_kernel(JobDev jd, Ctrl *ctrl, int32_t max_paths,
                                                   uint8_t *aln_out, int64_t *len_out,
                                                   int32_t *npaths_out) {
  using C = Cfg<K>;
  constexpr int T = C::T;
  constexpr int M = C::M;
  constexpr int NQ = C::DBS / 16;
  __shared__ alignas(16) uint8_t dirb[C::DBS];
  __shared__ uint8_t path[kCoMaxTotal];
  const int tid = threadIdx.x;
  int status = __builtin_amdgcn_readfirstlane(
      __hip_atomic_load(&ctrl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  // the blocks hold tie sets only when the workspace was set up for them
  if (status == ST_OK && !(ctrl->flags & kCoOptimal)) status = ST_EINVAL;
  int v[K];
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = jd.n[i];
  int cur_t = -1;  // tile whose block is in dirb
  int d = 0, np = 0;
  int tried = 0;       // masks up to this one were tried at depth d
  int64_t steps = 0;
  const int64_t step_limit = (int64_t)max_paths * (2 * jd.total_len + 2) + 2;
  while (status == ST_OK) {
    bool origin = true;
#pragma unroll
    for (int i = 0; i < K; ++i) origin = origin && v[i] == 0;
    if (origin) {
      // emit path[0..d) (path[d-1] is the first column) as alignment np
      uint8_t *blk = aln_out + (int64_t)np * K * jd.aln_cap;
      int cnt[K];
#pragma unroll
      for (int i = 0; i < K; ++i) cnt[i] = 0;
      for (int c0 = 0; c0 < d; c0 += 64) {
        const int col = c0 + tid;
        const int m = col < d ? (path[d - 1 - col] & kMaskBits) : 0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
          const int bit = (m >> i) & 1;
          int incl = bit;
          for (int s = 1; s < 64; s <<= 1) {
            const int y = __shfl_up(incl, s, 64);
            if (tid >= s) incl += y;
          }
          const int pos = cnt[i] + incl - bit;
          if (col < d)
            blk[(int64_t)i * jd.aln_cap + col] = bit ? jd.seqs[jd.seq_off[i] + pos] : (uint8_t)0xFF;
          cnt[i] += __shfl(incl, 63, 64);
        }
      }
      if (tid == 0) len_out[np] = d;
      ++np;
      if (np == max_paths || d == 0) break;
      // back up to the deepest level whose cell has untried tied masks: scan
      // the stack 64 entries at a time (lane x reads level e - x), adding the
      // masks of the levels popped to v
      int e = d - 1, found = -1;
      int back[K];
#pragma unroll
      for (int i = 0; i < K; ++i) back[i] = 0;
      while (e >= 0) {
        const int lvl = e - tid;
        const int ent = lvl >= 0 ? path[lvl] : 0;
        const uint64_t flagged = __ballot((ent & kMoreTies) != 0);
        // levels e, e-1, ... up to and including the first flagged one
        const int upto = flagged ? __builtin_ctzll(flagged) : 63;
        const bool popped = tid <= upto && lvl >= 0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
          const uint64_t bits = __ballot(popped && ((ent >> i) & 1));
          back[i] += __builtin_popcountll(bits);
        }
        if (flagged) {
          found = e - upto;
          break;
        }
        e -= 64;
      }
      if (found < 0) break;  // every alignment has been produced
#pragma unroll
      for (int i = 0; i < K; ++i) v[i] += back[i];
      d = found;
      tried = path[d] & kMaskBits;
      continue;
    }
    if (++steps > step_limit) {  // corrupt tie data: never loop for ever
      status = ST_EDEVICE;
      break;
    }
    // tie set of cell v (its tile's block cached in LDS)
    int t = 0;  // tile index (fewer than 2^30 tiles)
    int dl = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int ci = v[i] == 0 ? 0 : (v[i] - 1) / T + 1;
      t += ci * jd.tstride[i];
      dl += (v[i] - (ci == 0 ? 0 : (ci - 1) * T + 1)) * C::dstride(i);
    }
    if (t != cur_t) {
      __syncthreads();
      const uint4 *src = reinterpret_cast<const uint4 *>(jd.dir + (int64_t)t * C::DBS);
      uint4 *dst = reinterpret_cast<uint4 *>(dirb);
      for (int idx = tid; idx < NQ; idx += 64) dst[idx] = src[idx];
      __syncthreads();
      cur_t = t;
    }
    // tie bits 0 .. M - 1 (bit b - 1 for mask b)
    const int ties = __builtin_amdgcn_readfirstlane(dirb[dl]) & ((1 << M) - 1);
    const int rest = ties & ~((1 << tried) - 1);  // masks above `tried`
    if (rest != 0) {
      const int b = __builtin_ctz(rest) + 1;
      bool bad = d >= jd.total_len;
#pragma unroll
      for (int i = 0; i < K; ++i) bad = bad || (((b >> i) & 1) && v[i] == 0);
      if (bad) {
        status = ST_EDEVICE;
        break;
      }
      // every lane stores the same byte; the one wave's LDS accesses stay in
      // program order, so no barrier is needed before path[d] is read back
      const bool more = (rest & ~((1 << b) - 1)) != 0;  // tied masks above b
      path[d] = (uint8_t)(b | (more ? kMoreTies : 0));
#pragma unroll
      for (int i = 0; i < K; ++i) v[i] -= (b >> i) & 1;
      ++d;
      tried = 0;
      continue;
    }
    if (ties == 0 && tried == 0) {  // a cell other than the origin with no tie
      status = ST_EDEVICE;
      break;
    }
    if (d == 0) break;  // every alignment has been produced
    --d;
    tried = path[d] & kMaskBits;
#pragma unroll
    for (int i = 0; i < K; ++i) v[i] += (tried >> i) & 1;
  }
  __syncthreads();
  if (tid == 0) {
    *npaths_out = status == ST_OK ? np : 0;
    *jd.status_out = status;
    if (status != ST_OK) *jd.score_out = 0;
    // ready the control block for the next launch on this workspace
    ctrl->head = 0;
    ctrl->status = ST_OK;
    ctrl->best = INT64_MIN;
    ctrl->epoch = ctrl->epoch + 1;
  }
}

template <int K>
static int launch_coopt_k(const JobDev &jd, Ctrl *ctrl, int32_t max_paths, uint8_t *aln_out,
                          int64_t *len_out, int32_t *npaths_out, hipStream_t s) {
  if constexpr (K <= 3) {
    launch_begin();
    hipLaunchKernelGGL((coopt_kernel<K>), dim3(1), dim3(64), 0, s, jd, ctrl, max_paths, aln_out,
                       len_out, npaths_out);
    return launch_end();
  } else {
    return -1;
  }
}

// ---------------------------------------------------------------------------
// Near-optimal alignments (near-optimal mode, k <= 6): every global alignment
// whose score is at least opt - delta (Section 6: alignments within a
// threshold of the optimum set by the user).  The fill has also stored every
// cell's score xi, laid out as the direction blocks.  One wave walks depth
// first from the far corner.  At cell v, with s the score of the columns
// taken so far, lane b - 1 tests mask b: v - b lies in the tensor and
// xi(v - b) + SP(col(v, b)) + s >= opt - delta.  xi(v - b) is the score of
// some path from the origin, so every step passing the test leads to at least
// one alignment at or above the threshold (the walk has no dead end), and
// every such alignment is walked.  The masks of a cell are taken in
// ascending order, so the list is sorted by the column masks read from the
// last column to the first, and delta = 0 gives the co-optimal list.  Per
// column the LDS stack keeps the mask taken, the set of masks that passed
// and the score so far (sum n_i <= kNoMaxTotal); after an alignment the walk
// jumps back to the deepest column with a passing mask left, found with one
// wave-wide scan of the stack.  Alignment p goes to aln_out + p * k *
// aln_cap, its score to scores_out[p].
// ---------------------------------------------------------------------------
template <int K>
__global__ __launch_bounds__(64) void nearopt_kernel(JobDev jd, Ctrl *ctrl, int64_t delta,
                                                     int32_t max_paths, int64_t *scores_out,
                                                     uint8_t *aln_out, int64_t *len_out,
                                                     int32_t *npaths_out) {
  using C = Cfg<K>;
  constexpr int T = C::T;
  constexpr int M = (1 << K) - 1;  // masks 1..M; lane b - 1 tests mask b
  static_assert(M <= 64, "one lane per mask");
  __shared__ uint64_t pass_set[kNoMaxTotal + 1];
  __shared__ int32_t sofar[kNoMaxTotal + 1];
  __shared__ uint8_t path[kNoMaxTotal + 1];
  const int tid = threadIdx.x;
  int status = __builtin_amdgcn_readfirstlane(
      __hip_atomic_load(&ctrl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  // the cell scores exist only when the workspace was set up for them
  if (status == ST_OK && !(ctrl->flags & kNearOpt)) status = ST_EINVAL;
  const int alpha = ctrl->alpha;
  const int gap = ctrl->gap;
  const int64_t threshold = *jd.score_out - delta;
  const int bl = tid + 1;  // this lane's mask
  // this lane's pair (pi, pj) for the pair scores of a cell (lane p < C(k,2))
  int pi = 0, pj = 0, so = 0;
  {
    int p = 0;
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
      for (int j = i + 1; j < K; ++j) {
        if (p == tid) {
          pi = i;
          pj = j;
        }
        ++p;
      }
#pragma unroll
    for (int i = 0; i < K; ++i) so = tid == i ? jd.seq_off[i] : so;
  }
  int v[K];
#pragma unroll
  for (int i = 0; i < K; ++i) v[i] = jd.n[i];
  int d = 0, np = 0;
  int tried = 0;      // masks up to this one were taken at depth d
  bool fresh = true;  // pass_set[d] not computed yet
  int64_t steps = 0;
  const int64_t step_limit = (int64_t)max_paths * (2 * jd.total_len + 2) + 2;
  sofar[0] = 0;  // every lane stores the same value
  while (status == ST_OK) {
    bool origin = true;
#pragma unroll
    for (int i = 0; i < K; ++i) origin = origin && v[i] == 0;
    if (origin) {
      // emit path[0..d) (path[d-1] is the first column) as alignment np
      uint8_t *blk = aln_out + (int64_t)np * K * jd.aln_cap;
      int cnt[K];
#pragma unroll
      for (int i = 0; i < K; ++i) cnt[i] = 0;
      for (int c0 = 0; c0 < d; c0 += 64) {
        const int col = c0 + tid;
        const int m = col < d ? path[d - 1 - col] : 0;
#pragma unroll
        for (int i = 0; i < K; ++i) {
          const int bit = (m >> i) & 1;
          int incl = bit;
          for (int sh = 1; sh < 64; sh <<= 1) {
            const int y = __shfl_up(incl, sh, 64);
            if (tid >= sh) incl += y;
          }
          const int pos = cnt[i] + incl - bit;
          if (col < d)
            blk[(int64_t)i * jd.aln_cap + col] = bit ? jd.seqs[jd.seq_off[i] + pos] : (uint8_t)0xFF;
          cnt[i] += __shfl(incl, 63, 64);
        }
      }
      if (tid == 0) {
        len_out[np] = d;
        scores_out[np] = sofar[d];
      }
      ++np;
      if (np == max_paths || d == 0) break;
      // back up to the deepest column with a passing mask above the one
      // taken: scan the stack 64 entries at a time (lane x reads level
      // e - x), adding the masks of the levels popped to v
      int e = d - 1, found = -1;
      int back[K];
#pragma unroll
      for (int i = 0; i < K; ++i) back[i] = 0;
      while (e >= 0) {
        const int lvl = e - tid;
        const int ent = lvl >= 0 ? path[lvl] : 0;
        const bool more = lvl >= 0 && (pass_set[lvl] >> ent) != 0;
        const uint64_t flagged = __ballot(more);
        const int upto = flagged ? __builtin_ctzll(flagged) : 63;
        const bool popped = tid <= upto && lvl >= 0;
#pragma unroll
        for (int i = 0; i < K; ++i)
          back[i] += __builtin_popcountll(__ballot(popped && ((ent >> i) & 1)));
        if (flagged) {
          found = e - upto;
          break;
        }
        e -= 64;
      }
      if (found < 0) break;  // every alignment has been produced
#pragma unroll
      for (int i = 0; i < K; ++i) v[i] += back[i];
      d = found;
      tried = path[d];
      fresh = false;
      continue;
    }
    if (++steps > step_limit) {  // inconsistent scores: never loop for ever
      status = ST_EDEVICE;
      break;
    }
    // residues of cell v (lane i < k loads r_i) and its pair scores (lane p)
    int vi = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) vi = tid == i ? v[i] : vi;
    int rown = 0;
    if (tid < K && vi >= 1) rown = jd.seqs[so + vi - 1];
    int r[K];
#pragma unroll
    for (int i = 0; i < K; ++i) r[i] = __shfl(rown, i, 64);
    int ri = 0, rj = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      ri = pi == i ? r[i] : ri;
      rj = pj == i ? r[i] : rj;
    }
    const int pown = tid < K * (K - 1) / 2 ? (int)jd.sub[ri * alpha + rj] : 0;
    // SP(col(v, b)) of this lane's mask: residue pairs, residue-gap pairs
    int32_t sp = 0;
    {
      int p = 0;
#pragma unroll
      for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = i + 1; j < K; ++j) {
          const int bi = (bl >> i) & 1, bj = (bl >> j) & 1;
          const int32_t ps = __shfl(pown, p, 64);
          sp += (bi && bj) ? ps : (bi ^ bj) ? gap : 0;
          ++p;
        }
    }
    if (fresh) {
      // xi(v - b) of this lane's mask, in the layout of the direction blocks
      bool ok = tid < M;
      int t = 0, dl = 0;
#pragma unroll
      for (int i = 0; i < K; ++i) {
        const int u = v[i] - ((bl >> i) & 1);
        ok = ok && u >= 0;
        const int uu = u < 0 ? 0 : u;
        const int ci = uu == 0 ? 0 : (uu - 1) / T + 1;
        t += ci * jd.tstride[i];
        dl += (uu - (ci == 0 ? 0 : (ci - 1) * T + 1)) * C::dstride(i);
      }
      const int32_t xi = ok ? jd.scores[(int64_t)t * C::DBS + dl] : 0;
      const bool pass = ok && (int64_t)xi + sp + sofar[d] >= threshold;
      const uint64_t set = __ballot(pass);
      if (set == 0) {  // a cell off the origin from which no alignment reaches the threshold
        status = ST_EDEVICE;
        break;
      }
      pass_set[d] = set;  // every lane stores the same value
      fresh = false;
    }
    const uint64_t set = pass_set[d];
    const uint64_t rest = set & ~((1ull << tried) - 1);  // masks above `tried`
    if (rest != 0) {
      const int b = __builtin_ctzll(rest) + 1;
      if (d >= jd.total_len) {  // a walk longer than any alignment
        status = ST_EDEVICE;
        break;
      }
      const int32_t spb = __shfl(sp, b - 1, 64);
      // every lane stores the same values; the one wave's LDS accesses stay
      // in program order, so no barrier is needed before they are read back
      path[d] = (uint8_t)b;
      sofar[d + 1] = sofar[d] + spb;
#pragma unroll
      for (int i = 0; i < K; ++i) v[i] -= (b >> i) & 1;
      ++d;
      tried = 0;
      fresh = true;
      continue;
    }
    if (d == 0) break;  // every alignment has been produced
    --d;
    tried = path[d];
#pragma unroll
    for (int i = 0; i < K; ++i) v[i] += (tried >> i) & 1;
    fresh = false;
  }
  __syncthreads();
  if (tid == 0) {
    *npaths_out = status == ST_OK ? np : 0;
    *jd.status_out = status;
    if (status != ST_OK) *jd.score_out = 0;
    // ready the control block for the next launch on this workspace
    ctrl->head = 0;
    ctrl->status = ST_OK;
    ctrl->best = INT64_MIN;
    ctrl->epoch = ctrl->epoch + 1;
  }
}

template <int K>
static int launch_nearopt_k(const JobDev &jd, Ctrl *ctrl, int64_t delta, int32_t max_paths,
                            int64_t *scores_out, uint8_t *aln_out, int64_t *len_out,
                            int32_t *npaths_out, hipStream_t s) {
  if constexpr (K <= kNoMaxK) {
    launch_begin();
    hipLaunchKernelGGL((nearopt_kernel<K>), dim3(1), dim3(64), 0, s, jd, ctrl, delta, max_paths,
                       scores_out, aln_out, len_out, npaths_out);
    return launch_end();
  } else {
    return -1;
  }
}

// Row-major decision tensor (mask b per cell) from the tile-major blocks.
template <int K>
// A co-optimal workspace exports the bytes as stored (the tie sets) instead
// of decoding them to the chosen mask.
__global__ void export_dirs_kernel(JobDev jd, const Ctrl *ctrl, uint8_t *out, int64_t ncell) {
  const bool raw = (ctrl->flags & kCoOptimal) != 0;
  using C = Cfg<K>;
  constexpr int T = C::T;
  for (int64_t lin = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; lin < ncell;
       lin += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = lin;
    int v[K];
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
      v[i] = (int)(rem % (jd.n[i] + 1));
      rem /= (jd.n[i] + 1);
    }
    int t = 0, d = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int ci = v[i] == 0 ? 0 : (v[i] - 1) / T + 1;
      const int loi = ci == 0 ? 0 : (ci - 1) * T + 1;
      t += ci * jd.tstride[i];
      d += (v[i] - loi) * C::dstride(i);
    }
    const int byte = jd.dir[(int64_t)t * C::DBS + d];
    out[lin] = raw ? (uint8_t)byte : (uint8_t)(C::M - (byte & C::M));
  }
}

// ---------------------------------------------------------------------------
// Batched path: many jobs (uneven k and lengths) in one persistent launch.
// ---------------------------------------------------------------------------

// Queue construction over tile columns along dimension 0: column t of job j
// (its c_0 = 0 tile, t = sum_{d>=1} c_d * tstride[d]) goes to slot wbase_j[w]
// (where the host placed job j's columns starting in wave w = sum c_d) + its
// rank among those columns in lexicographic order of (c_1..c_{k-1}).  Every
// job's columns appear in the order of their first tile's wave, which makes
// the queue a topological order of all dependencies.
__global__ void batch_queue_kernel(const BatchArgs *__restrict__ a,
                                   const JobDev *__restrict__ jobs) {
  const int njobs = a->njobs;
  const int64_t *__restrict__ jcols = a->jcols;
  int32_t *qjob = a->qjob;
  int32_t *qtile = a->qtile;
  const int64_t total = jcols[njobs];
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = njobs;  // jcols[lo] <= g < jcols[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (jcols[mid] <= g) lo = mid; else hi = mid;
    }
    const JobDev &jd = jobs[lo];
    const int t = (int)(g - jcols[lo]);
    int c[kMaxK];
    int w = 0;
    for (int d = 1; d < jd.k; ++d) {
      c[d] = (t / jd.tstride[d]) % jd.P[d];
      w += c[d];
    }
    int64_t rank = 0;
    int s = w;
    for (int d = 1; d < jd.k - 1; ++d) {
      for (int cc = 0; cc < c[d]; ++cc)
        if (s - cc >= 0) rank += jd.wcnt[(d + 1) * jd.nwaves + (s - cc)];
      s -= c[d];
    }
    const int64_t pos = jd.wbase[w] + rank;
    qjob[pos] = lo;
    qtile[pos] = t;
  }
}

template <int K>
constexpr size_t smem_bytes() { return sizeof(Smem<K>); }
template <int KLO, int KHI>
constexpr size_t batch_smem_bytes() {
  size_t m = 0;
  for (int k = KLO; k <= KHI; ++k) {
    const size_t b = k == 2 ? smem_bytes<2>() : k == 3 ? smem_bytes<3>() : k == 4 ? smem_bytes<4>()
                   : k == 5 ? smem_bytes<5>() : k == 6 ? smem_bytes<6>() : k == 7 ? smem_bytes<7>()
                   : smem_bytes<8>();
    m = b > m ? b : m;
  }
  return m;
}

// One tile of job `jd` with K = k; reloads the per-k cell table and the
// job's substitution matrix into LDS when they differ from the cached ones.
// The column of tiles base + c_0 * tstride[0], bottom up (see process_tile's
// own0 and cols).
template <int K, int NT>
__device__ void batch_column(const JobDev &jd, int base, int epoch, Ctrl *ctrl, void *smraw,
                             int &cur_k, const int8_t *&cur_sub, int64_t wlim) {
  Smem<K> &sm = *reinterpret_cast<Smem<K> *>(smraw);
  if (cur_k != K || cur_sub != jd.sub) {
    __syncthreads();
    load_tables<K, NT>(jd, jd.alpha, sm);
    __syncthreads();
    cur_k = K;
    cur_sub = jd.sub;
  }
  const HaloSlots<K, NT> hs(threadIdx.x);
  for (int c0 = 0; c0 < jd.P[0]; ++c0)
    process_tile<K, NT>(jd, jd.alpha, jd.gap, base + c0 * jd.tstride[0], epoch, ctrl,
                        jd.jstatus, sm, hs, false, nullptr, false, false, c0 > 0, true, false,
                        wlim);
}

// The job descriptors come as a kernel argument of their own (a fixed arena
// offset, so the captured launch stays valid): read through a restrict
// argument, the compiler proves that no store of the kernel reaches them and
// keeps their fields in scalar registers; read through a pointer loaded from
// the descriptor, every field would take vector registers.
// Waves per SIMD the batched fill is compiled for: as many workgroups as the
// k class's LDS allows (k = 2..4 and 5: five; k = 6: four; k = 7..8: one).
constexpr int batch_waves_per_eu(int klo, int khi) {
  return khi <= 5 ? 5 : khi == 6 ? 4 : 1;
}

template <int KLO, int KHI, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(batch_waves_per_eu(KLO, KHI))))
void batch_fill_kernel(const BatchArgs *__restrict__ a,
                                                        const JobDev *__restrict__ jobs,
                                                        Ctrl *ctrl) {
  __shared__ alignas(16) char smraw[batch_smem_bytes<KLO, KHI>()];
  const int32_t *__restrict__ qjob = a->qjob;
  const int32_t *__restrict__ qtile = a->qtile;
  const int32_t total = __builtin_amdgcn_readfirstlane((int32_t)a->cols);
  __shared__ int32_t bcast;
  const int epoch = __hip_atomic_load(&ctrl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // the launch's dependency-wait time-out (0: the default), read once
  const int64_t wl = __hip_atomic_load(&ctrl->wait_limit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int64_t wlim = wl > 0 ? wl : kWaitLimitTicks;
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x) >> 6;
  int cur_k = -1;
  const int8_t *cur_sub = nullptr;
  for (;;) {
    if (wave == 0) {  // see fill_kernel: no lane-divergent branch around the pop
      const int got = atomicAdd(&ctrl->head, threadIdx.x == 0 ? 1 : 0);
      bcast = __builtin_amdgcn_readfirstlane(got);
    }
    __syncthreads();
    const int q = __builtin_amdgcn_readfirstlane(bcast);
    __syncthreads();
    if (q >= total) break;
    const int j = __builtin_amdgcn_readfirstlane(qjob[q]);
    const int tile = __builtin_amdgcn_readfirstlane(qtile[q]);
    const JobDev &jd = jobs[j];
    switch (jd.k) {
      case 2: if constexpr (KLO <= 2 && 2 <= KHI) batch_column<2, NT>(jd, tile, epoch, ctrl, smraw, cur_k, cur_sub, wlim); break;
      case 3: if constexpr (KLO <= 3 && 3 <= KHI) batch_column<3, NT>(jd, tile, epoch, ctrl, smraw, cur_k, cur_sub, wlim); break;
      case 4: if constexpr (KLO <= 4 && 4 <= KHI) batch_column<4, NT>(jd, tile, epoch, ctrl, smraw, cur_k, cur_sub, wlim); break;
      case 5: if constexpr (KLO <= 5 && 5 <= KHI) batch_column<5, NT>(jd, tile, epoch, ctrl, smraw, cur_k, cur_sub, wlim); break;
      case 6: if constexpr (KLO <= 6 && 6 <= KHI) batch_column<6, NT>(jd, tile, epoch, ctrl, smraw, cur_k, cur_sub, wlim); break;
      case 7: if constexpr (KLO <= 7 && 7 <= KHI) batch_column<7, NT>(jd, tile, epoch, ctrl, smraw, cur_k, cur_sub, wlim); break;
      case 8: if constexpr (KLO <= 8 && 8 <= KHI) batch_column<8, NT>(jd, tile, epoch, ctrl, smraw, cur_k, cur_sub, wlim); break;
      default: break;
    }
  }
}

// One workgroup (one wave) per job at a time (jobs blockIdx.x, + gridDim.x,
// ...): walk, expand, write the outputs.
template <int KLO, int KHI>
__global__ __launch_bounds__(64) void batch_traceback_kernel(const BatchArgs *__restrict__ a,
                                                             const JobDev *__restrict__ jobs,
                                                             Ctrl *ctrl) {
  __shared__ alignas(16) uint8_t dirb[4096];
  const int njobs = __builtin_amdgcn_readfirstlane(a->njobs);
  const int gst = __hip_atomic_load(&ctrl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int j = blockIdx.x; j < njobs; j += gridDim.x) {
    const JobDev &jd = jobs[j];
    const int jst = __hip_atomic_load(jd.jstatus, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int st = gst != ST_OK ? gst : jst;
    switch (jd.k) {
      case 2: if constexpr (KLO <= 2 && 2 <= KHI) traceback_job<2>(jd, st, dirb); break;
      case 3: if constexpr (KLO <= 3 && 3 <= KHI) traceback_job<3>(jd, st, dirb); break;
      case 4: if constexpr (KLO <= 4 && 4 <= KHI) traceback_job<4>(jd, st, dirb); break;
      case 5: if constexpr (KLO <= 5 && 5 <= KHI) traceback_job<5>(jd, st, dirb); break;
      case 6: if constexpr (KLO <= 6 && 6 <= KHI) traceback_job<6>(jd, st, dirb); break;
      case 7: if constexpr (KLO <= 7 && 7 <= KHI) traceback_job<7>(jd, st, dirb); break;
      case 8: if constexpr (KLO <= 8 && 8 <= KHI) traceback_job<8>(jd, st, dirb); break;
      default: break;
    }
  }
}

// Clears the completion flags of a launch (a kernel, not a memset, so that the
// launch sequence can be captured in a graph).
__global__ void batch_zero_kernel(const BatchArgs *__restrict__ a) {
  int32_t *flags = a->flags;
  const int64_t n = a->tiles;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    flags[i] = 0;
}

// Reports the launch-wide status (MSA_EDEVICE after a dependency wait timed
// out) and the longest pause of a dependency wait, and readies the control
// block for the next launch on the same arena.
__global__ void batch_finish_kernel(const BatchArgs *__restrict__ a, Ctrl *ctrl) {
  if (threadIdx.x == 0) {
    a->gstatus[0] = ctrl->status;
    int64_t *g64 = reinterpret_cast<int64_t *>(a->gstatus + 2);
    g64[0] = ctrl->max_pause;
    for (int q = 0; q < 6; ++q) {
      g64[1 + q] = ctrl->wd[q];
      ctrl->wd[q] = 0;
    }
    g64[7] = a->cols;
    ctrl->max_pause = 0;
    ctrl->head = 0;
    ctrl->status = ST_OK;
    ctrl->epoch = ctrl->epoch + 1;
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from the ABI layer).
// ---------------------------------------------------------------------------
constexpr int kFillThreads = 256;  // four waves per tile

template <int K>
static int launch_fill_k(const JobDev &jd, Ctrl *ctrl, const int32_t *order, int grid,
                         int pass, hipStream_t s) {
  launch_begin();
  hipLaunchKernelGGL((fill_kernel<K, kFillThreads>), dim3(grid), dim3(kFillThreads), 0, s, jd,
                     ctrl, order, pass);
  return launch_end();
}

template <int K>
static int launch_traceback_k(const JobDev &jd, Ctrl *ctrl, hipStream_t s) {
  launch_begin();
  hipLaunchKernelGGL((traceback_kernel<K>), dim3(1), dim3(64), 0, s, jd, ctrl);
  return launch_end();
}

template <int K>
static int occupancy_k() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fill_kernel<K, kFillThreads>,
                                                   kFillThreads, 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

template <int K>
static int launch_export_k(const JobDev &jd, const Ctrl *ctrl, uint8_t *out, int64_t ncell,
                           hipStream_t s) {
  int64_t blocks = (ncell + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  launch_begin();
  hipLaunchKernelGGL((export_dirs_kernel<K>), dim3((unsigned)blocks), dim3(256), 0, s, jd, ctrl,
                     out, ncell);
  return launch_end();
}

#define MSA_DISPATCH_K(k, fn, ...)                 \
  switch (k) {                                     \
    case 2: return fn<2>(__VA_ARGS__);             \
    case 3: return fn<3>(__VA_ARGS__);             \
    case 4: return fn<4>(__VA_ARGS__);             \
    case 5: return fn<5>(__VA_ARGS__);             \
    case 6: return fn<6>(__VA_ARGS__);             \
    case 7: return fn<7>(__VA_ARGS__);             \
    case 8: return fn<8>(__VA_ARGS__);             \
    default: return -1;                            \
  }

int launch_fill(const JobDev &jd, Ctrl *ctrl, const int32_t *order, int grid, int pass,
                hipStream_t s) {
  MSA_DISPATCH_K(jd.k, launch_fill_k, jd, ctrl, order, grid, pass, s);
}

int launch_traceback(const JobDev &jd, Ctrl *ctrl, hipStream_t s) {
  MSA_DISPATCH_K(jd.k, launch_traceback_k, jd, ctrl, s);
}

int fill_occupancy(int k) { MSA_DISPATCH_K(k, occupancy_k); }

int launch_coopt(const JobDev &jd, Ctrl *ctrl, int32_t max_paths, uint8_t *aln_out,
                 int64_t *len_out, int32_t *npaths_out, hipStream_t s) {
  MSA_DISPATCH_K(jd.k, launch_coopt_k, jd, ctrl, max_paths, aln_out, len_out, npaths_out, s);
}

int launch_nearopt(const JobDev &jd, Ctrl *ctrl, int64_t delta, int32_t max_paths,
                   int64_t *scores_out, uint8_t *aln_out, int64_t *len_out, int32_t *npaths_out,
                   hipStream_t s) {
  MSA_DISPATCH_K(jd.k, launch_nearopt_k, jd, ctrl, delta, max_paths, scores_out, aln_out,
                 len_out, npaths_out, s);
}

int launch_export(const JobDev &jd, const Ctrl *ctrl, uint8_t *out, int64_t ncell,
                  hipStream_t s) {
  MSA_DISPATCH_K(jd.k, launch_export_k, jd, ctrl, out, ncell, s);
}

}  // namespace msa

// ---------------------------------------------------------------------------
// Batched launches: k class 0 covers k = 2..4, 1 is k = 5, 2 is k = 6, 3 covers
// k = 7..8.
// ---------------------------------------------------------------------------
namespace msa {

constexpr int kBatchThreads = 256;
// Fixed grids of the launch sequence (it is replayed from a graph for every
// batch): the flag-clearing and queue kernels stride over the tiles and
// columns, the traceback over the jobs, one wave per job at a time.
constexpr int kBatchAuxGrid = 1024;
constexpr int kBatchTraceGrid = 4096;

template <int KLO, int KHI>
static int launch_batch_k(const BatchArgs *d_args, const JobDev *d_jobs, Ctrl *ctrl, int grid,
                          hipStream_t s) {
  launch_begin();
  hipLaunchKernelGGL(batch_zero_kernel, dim3(kBatchAuxGrid), dim3(256), 0, s, d_args);
  hipLaunchKernelGGL(batch_queue_kernel, dim3(kBatchAuxGrid), dim3(256), 0, s, d_args, d_jobs);
  hipLaunchKernelGGL((batch_fill_kernel<KLO, KHI, kBatchThreads>), dim3(grid),
                     dim3(kBatchThreads), 0, s, d_args, d_jobs, ctrl);
  hipLaunchKernelGGL((batch_traceback_kernel<KLO, KHI>), dim3(kBatchTraceGrid), dim3(64), 0, s,
                     d_args, d_jobs, ctrl);
  hipLaunchKernelGGL(batch_finish_kernel, dim3(1), dim3(64), 0, s, d_args, ctrl);
  return launch_end();
}

int launch_batch(int kclass, const BatchArgs *d_args, const JobDev *d_jobs, Ctrl *ctrl, int grid,
                 hipStream_t s) {
  switch (kclass) {
    case 0: return launch_batch_k<2, 4>(d_args, d_jobs, ctrl, grid, s);
    case 1: return launch_batch_k<5, 5>(d_args, d_jobs, ctrl, grid, s);
    case 2: return launch_batch_k<6, 6>(d_args, d_jobs, ctrl, grid, s);
    default: return launch_batch_k<7, 8>(d_args, d_jobs, ctrl, grid, s);
  }
}

template <int KLO, int KHI>
static int batch_occupancy_k() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_fill_kernel<KLO, KHI, kBatchThreads>,
                                                   kBatchThreads, 0) != hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

int batch_occupancy(int kclass) {
  switch (kclass) {
    case 0: return batch_occupancy_k<2, 4>();
    case 1: return batch_occupancy_k<5, 5>();
    case 2: return batch_occupancy_k<6, 6>();
    default: return batch_occupancy_k<7, 8>();
  }
}

}  // namespace msa
