// msa_internal.h -- structures shared by the host core and the HIP kernels of
// the library (not part of the public ABI).
//
// Tiling (Section 3 of the paper: hypercube partitions of edge S that overlap
// their lower neighbours by one layer, scheduled in computation waves of
// equal distance from the origin).  Here a tile has edge T = S - 1 interior
// cells plus a one-cell halo.  Along dimension i the tile coordinate c runs
// over [0, P_i) with P_i = 1 + ceil(n_i / T):
//   c = 0      : the one-cell-thick initial-gap layer v_i = 0;
//   c >= 1     : cells v_i in [(c-1)T + 1, min(cT, n_i)].
// The halo of a tile along i is the layer v_i = lo_i - 1, i.e. the last layer
// of tile c - 1 (or, for c = 0, a virtual layer of -infinity).  Every cell
// belongs to exactly one tile, so the fill needs no special boundary code:
// an out-of-range neighbour reads -infinity and never wins.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msa {

// HIP keeps one last-error code per host thread until it is read.  A
// launcher clears it right before its launches, so that what it reads
// afterwards comes from those launches and not from an earlier call of the
// same thread: launch_begin() ... launch_end() (0 or -1).
inline void launch_begin() { (void)hipGetLastError(); }
inline int launch_end() { return hipGetLastError() == hipSuccess ? 0 : -1; }

constexpr int kMaxK = 8;
constexpr int kNegKey = -(1 << 30);  // "-infinity" key; see range check

// Device-visible description of one alignment job.  Lives in the workspace
// (plain path) or in the batch descriptor array (batched / served paths).
struct JobDev {
  int32_t k, T, alpha, gap;
  int32_t n[kMaxK];            // sequence lengths
  int32_t P[kMaxK];            // tiles per dimension (incl. the v_i = 0 layer)
  int32_t tstride[kMaxK];      // row-major tile strides (last dim fastest)
  // division by tstride[i] as a multiply-high (see udiv_magic, msa_plan.cpp):
  // multiplier, and the two shifts in the low and the next byte
  uint32_t tdm[kMaxK];
  uint32_t tdsh[kMaxK];
  int32_t ntiles;
  int32_t nwaves;              // sum(P) - k + 1
  int32_t dbs;                 // direction block stride (T^k rounded to 16)
  int32_t seq_off[kMaxK];      // offsets of each sequence in the seq buffer
  int64_t face_off[kMaxK];     // element offset of face array i in `faces`
  int64_t fplane[kMaxK];       // elements per face plane of dimension i
  uint32_t fbstride[kMaxK][kMaxK];  // face-plane strides in bytes: fbstride[i][j],
                                    // j != i (below 2^32, checked by the plan)
  int64_t total_len;           // sum of lengths (traceback path capacity)
  // device pointers (filled per call for the plain path)
  const uint8_t *seqs;         // concatenated sequences
  const int8_t *sub;           // alpha x alpha
  int32_t *faces;              // face planes (int32 keys)
  uint8_t *dir;                // tile-major direction blocks
  int32_t *flags;              // per-tile completion epoch
  uint8_t *path;               // traceback masks, end first
  int64_t *score_out;
  uint8_t *aln_out;
  int64_t aln_cap;
  int64_t *aln_len_out;
  int32_t *status_out;
  const uint8_t *keep;        // pruned mode: per-tile keep flags (else null)
  const int32_t *corder;      // column schedule: first tile of each column, in order
  int32_t ncols;              // columns along dimension 0 (0: tile queue instead)
  int64_t *trace;             // optional per-tile phase timestamps (debug builds)
  int32_t *scores;            // near-optimal mode: every cell's score, laid out as `dir`
  // batched path only
  int32_t *jstatus;           // per-job status (bad residue code)
  const int32_t *wcnt;        // (k+1) x nwaves: tuples (c_d..c_{k-1}) summing to s
  const int64_t *wbase;       // nwaves: queue slot of this job's first tile of wave w
  int64_t qbase;              // first tile of this job in the launch's tile numbering
};

// Control block of one persistent launch (in device memory).
struct Ctrl {
  int32_t head;     // next queue slot
  int32_t epoch;    // flags equal to epoch mean "tile done in this launch"
  int32_t status;   // MSA_OK, MSA_EINVAL (bad code), MSA_EDEVICE (watchdog)
  int32_t alpha;    // scoring fixed at set-up (plain path)
  int32_t gap;
  int32_t flags;    // kEndGapsFree / kCoOptimal (plain path, set at set-up)
  int64_t best;     // end-gap-free: max of (score << 32 | row-major cell index)
                    // over the far faces; INT64_MIN between launches
  // pruned mode (tile bounds): U = sum of pairwise optima, the threshold of
  // the last pass, tiles kept by it and the number of passes run
  int64_t prune_U, prune_L, prune_kept, prune_passes;
  int64_t lo;       // closed-form lower bound of every score (set-up)
  int64_t prune_c;  // C(k,2) * max(|gap|, max |sub|) (set-up)
  int32_t nqueue;   // tiles in the pruned queue
  int32_t redo;     // 1 when the first pruned pass missed its threshold
  int64_t max_pause;  // longest pause seen inside a dependency wait (ticks of
                      // the 100 MHz clock, see WaitClock); batched launches
                      // report and clear it
  int64_t wd[6];      // the first dependency wait that timed out: the job's
                      // first tile in the launch's numbering (JobDev::qbase),
                      // the tile, the mask of the predecessor dimensions
                      // still missing, the first missing predecessor tile,
                      // the value its flag held, and the queue head then
                      // (batched launches report it)
  int64_t wait_limit;  // batched launches: dependency-wait time-out in 100 MHz
                       // ticks (0: 2 s)
  int32_t pad[26];
};
static_assert(sizeof(Ctrl) == 256, "control block is one 256-byte slot");
constexpr int64_t kBatchWaitTicks = 25000000;  // 250 ms: batched launches' time-out

// Time a dependency wait has spent waiting, for its watchdog.  The 100 MHz
// wall clock is read at every check of the wait, and only gaps shorter than
// kPauseTicks between two checks count: a running wave checks every few
// microseconds, so a longer gap means the wave did not run (its queue was
// preempted, for one), which is no sign of a missing dependency.  The longest
// such gap is kept for the launch's report.
constexpr int64_t kPauseTicks = 100000;  // 1 ms
struct WaitClock {
  int64_t last;
  int64_t waited = 0;
  int64_t pause = 0;
  __device__ WaitClock() : last((int64_t)wall_clock64()) {}
  // Takes a clock reading; returns the time waited so far (ticks).
  __device__ int64_t tick() {
    const int64_t now = (int64_t)wall_clock64();
    const int64_t d = now - last;
    last = now;
    if (d < kPauseTicks)
      waited += d;
    else if (d > pause)
      pause = d;
    return waited;
  }
  __device__ void report(Ctrl *ctrl) const {
    if (pause > 0)
      __hip_atomic_fetch_max(&ctrl->max_pause, pause, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
};

// Alignment mode bits (same values as MSA_END_GAPS_FREE / MSA_COOPTIMAL in
// the C ABI).
constexpr int32_t kEndGapsFree = 1;
constexpr int32_t kCoOptimal = 2;
constexpr int32_t kPrune = 4;
// Pruned mode: the dependency wait covers all 2^k - 1 lower neighbour tiles
// with one lane each (k <= 6), and the pairwise tables keep one row of
// boundary values per band of rows in a wave's registers (n_i < kPruneMaxLen).
constexpr int kPruneMinK = 3;
constexpr int kPruneMaxK = 6;
constexpr int kPruneMaxLen = 16384;
constexpr int kMaxPairs = kPruneMaxK * (kPruneMaxK - 1) / 2;

// Device descriptor of the pruning kernels (pairwise tables, tile bounds,
// tile selection and compaction).
struct PruneDev {
  int32_t k, npairs, T;
  int32_t ntiles;
  int32_t n[kMaxK], P[kMaxK], tstride[kMaxK], seq_off[kMaxK];
  int32_t pi[kMaxPairs], pj[kMaxPairs];  // pair p = (pi[p], pj[p]), pi < pj
  int64_t tab_off[kMaxPairs];  // int32 offset of pair p's prefix table (suffix follows)
  int64_t bm_off[kMaxPairs];   // int32 offset of pair p's block-maximum table
  int32_t nblocks;             // selection blocks of kSelBlock tiles
  const uint8_t *seqs;
  const int8_t *sub;
  int32_t alpha, gap;
  int32_t *tabs;               // pairwise tables (column-major, see the kernels)
  int32_t *bm;                 // block maxima of prefix + suffix per tile pair
  uint8_t *keep;               // per tile (row-major tile index): kept in the last pass
  const int32_t *order;        // tiles in computation-wave order
  int32_t *korder;             // kept tiles in the same order
  int32_t *bcnt;               // kept tiles per selection block, then their offsets
  const int64_t *score;        // the fill's end score
};
constexpr int kSelBlock = 1024;

// Near-optimal mode (alignments within a threshold of the optimum): one wave
// tests the 2^k - 1 masks of a cell at once (k <= 6), and the walk keeps its
// stack (mask, masks passing the threshold and score so far per column, at
// most sum n_i) in LDS.
constexpr int32_t kNearOpt = 8;
constexpr int kNoMaxK = 6;
constexpr int kNoMaxTotal = 4096;

// Co-optimal mode: tie sets fit a byte for k <= 3, and the enumeration keeps
// its stack of masks (one per column, at most sum n_i) in LDS.
constexpr int kCoMaxK = 3;
constexpr int kCoMaxTotal = 32768;

// Streaming fill of k = 3 (msa_sweep3.hip): a workgroup owns kSwRows rows
// (dimension 0) x 64 lanes (dimension 1) of lines along dimension 2 and
// sweeps the whole length; neighbouring workgroups exchange their boundary
// lines through tagged values in two exchange regions of the workspace.
constexpr int kSwNW = 8;           // compute waves per workgroup
constexpr int kSwRPW = 3;          // rows per compute wave
constexpr int kSwRows = kSwNW * kSwRPW;  // rows per workgroup
constexpr int kSwLanes = 64;       // lanes (dimension-1 cells) per wave
constexpr int kSwSeqMax = 16384;   // longest third sequence (kept in LDS)
constexpr int kSwSubMax = 32;      // largest alphabet (matrix kept in LDS)

// Parameters of one batched launch, written into the launch's arena with its
// inputs.  The launch sequence then takes only fixed arguments (this
// descriptor's address, the job descriptors' address, the control block,
// fixed grids), so it is captured once per arena in a graph and replayed for
// every batch.
struct BatchArgs {
  const int64_t *jcols;       // njobs + 1: tile columns before job i
  int32_t *qjob, *qtile;      // the column queue: job index and first tile
  int32_t *flags;             // per-tile completion flags of all jobs
  int32_t *gstatus;           // output: the launch-wide status at its end
                              // ([0]), the longest pause of a dependency wait
                              // (int64 at [2], 100 MHz ticks) and the first
                              // timed-out wait (Ctrl::wd, int64 at [4..9])
  int64_t tiles;              // tiles of all jobs
  int64_t cols;               // columns of all jobs (queue length)
  int32_t njobs;
  int32_t pad;
};

// One entry of the batched tile queue: (job index, tile linear index).
struct QItem {
  int32_t job;
  int32_t tile;
};

// Tile edge per k (LDS footprint (T+1)^k * 4 bytes for the score tile).
constexpr int tile_edge_for_k(int k) {
  return k == 2 ? 32 : k == 3 ? 16 : k == 4 ? 8 : k == 5 ? 4 : k == 6 ? 3 : 2;
}

constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

constexpr int bits_for(int x) {  // bits to hold values 0..x
  return x <= 1 ? 1 : 1 + bits_for(x >> 1);
}

}  // namespace msa
