// msa_plan.h -- host core: validation, closed-form score bounds, tile grid,
// hyperplane cell tables, tile schedule and workspace layout.
#pragma once
#include <stdint.h>

#include <vector>

#include "msa_internal.h"

namespace msa {

// Validated shape + derived geometry of one alignment.
struct Plan {
  int k = 0, T = 0;
  int32_t n[kMaxK] = {};
  int32_t P[kMaxK] = {};
  int32_t tstride[kMaxK] = {};
  int64_t ntiles = 0;
  int32_t nwaves = 0;
  int32_t dbs = 0;
  int64_t ncell = 0;         // prod(n_i + 1)
  int64_t nu = 0;            // neighbour updates prod(2n_i+1) - prod(n_i+1)
  int64_t total_len = 0;     // sum n_i
  int64_t face_off[kMaxK] = {};
  int64_t fplane[kMaxK] = {};
  int64_t fstride[kMaxK][kMaxK] = {};
  int64_t face_elems = 0;
  // workspace layout (byte offsets from the workspace base)
  int64_t off_ctrl = 0, off_sub = 0, off_order = 0, off_flags = 0, off_path = 0,
          off_faces = 0, off_dir = 0, bytes = 0;
  int64_t ncols = 0, off_corder = 0;  // tile columns along dimension 0 and their order
  int64_t max_wave = 0;      // tiles in the widest computation wave
  // pruned mode (3 <= k <= 6, every n_i < kPruneMaxLen): pairwise tables,
  // block maxima, keep flags, the kept-tile queue and selection block counts
  bool prunable = false;
  int npairs = 0;
  int32_t pi[kMaxPairs] = {}, pj[kMaxPairs] = {};
  int64_t tab_off[kMaxPairs] = {}, bm_off[kMaxPairs] = {};  // int32 elements
  int32_t nblocks = 0;
  int64_t off_ptab = 0, off_pbm = 0, off_keep = 0, off_korder = 0, off_bcnt = 0;
  // streaming fill of k = 3: workgroup grid and the two exchange regions,
  // X0 (last row of each workgroup row, by diagonal d = v1 + v2) and X1 (last
  // lane of each workgroup column)
  int32_t sw_nb0 = 0, sw_nb1 = 0;
  int64_t x0_plane = 0, x1_plane = 0;  // int32 elements per boundary
  int64_t off_x0 = 0, off_x1 = 0, x_bytes = 0;
};

// The streaming k = 3 fill runs the plain mode (flags 0) of a k = 3 plan
// whose alphabet and third sequence fit its LDS tables.
bool sweep3_eligible(const Plan &p, int alpha, int32_t flags);

constexpr int64_t kSubBytes = 255 * 255;
constexpr int64_t kMaxTiles = (int64_t)1 << 30;

// Fills geometry and layout; returns 0 or a negative status.
int make_plan(const int32_t *lens, int32_t k, Plan *p);

// Tiles ordered by computation wave (sum of tile coordinates).
void make_tile_order(const Plan &p, std::vector<int32_t> *order);

// Tile columns along dimension 0 (the tiles with equal c_1..c_{k-1}), given
// by their c_0 = 0 tile, ordered by the wave of that tile.
void make_column_order(const Plan &p, std::vector<int32_t> *order);

// Validation of scoring inputs (matrix symmetric, alpha range) and the
// device integer range check.  Returns 0 or a negative status.
int check_scoring(const int32_t *lens, int32_t k, const int8_t *submat, int32_t alpha,
                  int32_t gap);

int score_bounds(const int32_t *lens, int32_t k, const int8_t *submat, int32_t alpha,
                 int32_t gap, int64_t *lo, int64_t *hi);

// check_scoring plus the range the mode `flags` needs (the pruned mode's
// -infinity chains).  Returns 0 or a negative status.
int check_scoring_mode(const int32_t *lens, int32_t k, const int8_t *submat, int32_t alpha,
                       int32_t gap, uint32_t flags);

// Near-optimal mode: bytes of the cell-score region that follows the plan's
// layout (at offset p.bytes), one int32 per cell laid out as the direction
// blocks.
int64_t nearopt_bytes(const Plan &p);
// Division by an invariant (tile strides): multiplier and shifts, and the
// quotient they give (the kernels' formula, for host checks).
void udiv_magic(uint32_t d, uint32_t *m, uint32_t *sh);
uint32_t udiv_apply(uint32_t n, uint32_t m, uint32_t sh);

// Device descriptor for a plan placed at workspace base `ws`.
void fill_jobdev(const Plan &p, char *ws, int alpha, int gap, JobDev *jd);

// Pruning descriptor for a prunable plan at workspace base `ws`.
void fill_prunedev(const Plan &p, char *ws, const uint8_t *d_seqs, int64_t *d_score,
                   PruneDev *pd);

}  // namespace msa
