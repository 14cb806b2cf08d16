// msa_runtime.h -- device-side runtime of the library: workspace set-up and
// launches of the plain path.
#pragma once
#include <hip/hip_runtime.h>

#include "msa_plan.h"

namespace msa {

// kernels (msa_kernels.hip)
// pass: 0 plain; 1, 2 the passes of the pruned mode (2 runs only after a miss)
int launch_fill(const JobDev &jd, Ctrl *ctrl, const int32_t *order, int grid, int pass,
                hipStream_t s);
int launch_traceback(const JobDev &jd, Ctrl *ctrl, hipStream_t s);
int launch_export(const JobDev &jd, const Ctrl *ctrl, uint8_t *out, int64_t ncell,
                  hipStream_t s);
int launch_nearopt(const JobDev &jd, Ctrl *ctrl, int64_t delta, int32_t max_paths,
                   int64_t *scores_out, uint8_t *aln_out, int64_t *len_out, int32_t *npaths_out,
                   hipStream_t s);
int launch_coopt(const JobDev &jd, Ctrl *ctrl, int32_t max_paths, uint8_t *aln_out,
                 int64_t *len_out, int32_t *npaths_out, hipStream_t s);
int fill_occupancy(int k);
// pruning kernels (msa_prune.hip)
int launch_prune_bounds(const PruneDev &pd, Ctrl *ctrl, hipStream_t s);
int launch_prune_select(const PruneDev &pd, Ctrl *ctrl, int pass, hipStream_t s);
int launch_prune_check(const PruneDev &pd, Ctrl *ctrl, hipStream_t s);
// The batched launch sequence (flag clearing, queue, fill, traceback, control
// block reset) for the batch described by d_args; grid workgroups for the
// persistent fill.  Fixed arguments only, so it can be captured in a graph.
int launch_batch(int kclass, const BatchArgs *d_args, const JobDev *d_jobs, Ctrl *ctrl, int grid,
                 hipStream_t s);
int batch_occupancy(int kclass);
// streaming k = 3 fill (msa_sweep3.hip), for plans with sweep3_eligible
int launch_sweep3(const Plan &p, char *ws, const JobDev &jd, Ctrl *ctrl, int32_t flags,
                  hipStream_t s);

// runtime (msa_runtime.cpp)
int device_cu_count();
// drops what prepare_workspace recorded for `ws` (before its memory is freed)
void forget_workspace(const char *ws);
// mode flags given to prepare_workspace for the workspace at `ws` (0 if none)
int32_t workspace_flags(const char *ws);
// MSA_OK when `ws` was prepared for the shape of `p` (and its alphabet size
// in *alpha when alpha is not null), else MSA_EINVAL
int check_workspace(const Plan &p, const char *ws, int32_t *alpha);
int prepare_workspace(const Plan &p, char *ws, const int8_t *submat, int alpha, int gap,
                      int32_t flags, hipStream_t s);
// which: 1 = fill only, 2 = traceback only, 3 = both
int run_plain(const Plan &p, char *ws, const uint8_t *d_seqs, int64_t *d_score, uint8_t *d_aln,
              int64_t aln_cap, int64_t *d_aln_len, int32_t *d_status, hipStream_t s,
              int which = 3);
// run_plain on a workspace whose set-up the caller guarantees (plain mode,
// no registry check): the allocation-free entry point sets its static
// workspace up on the device itself.
int run_plain_set_up(const Plan &p, char *ws, int alpha, const uint8_t *d_seqs,
                     int64_t *d_score, uint8_t *d_aln, int64_t aln_cap, int64_t *d_aln_len,
                     int32_t *d_status, hipStream_t s, int which = 3);
int export_dirs(const Plan &p, char *ws, uint8_t *out, hipStream_t s);
// pruned mode: keep flags of the last pass (ntiles bytes, row-major tile
// index) and {U, threshold, tiles kept, passes} of the last fill
int export_prune(const Plan &p, char *ws, uint8_t *keep_out, int64_t *info_out,
                 hipStream_t s);
// fill, then up to max_paths co-optimal alignments (workspace prepared with
// the co-optimal flag)
// Near-optimal mode: the fill (cell scores kept) and the walk of the
// alignments scoring at least opt - delta.
int run_nearopt(const Plan &p, char *ws, const uint8_t *d_seqs, int64_t delta, int32_t max_paths,
                int64_t *d_score, int64_t *d_scores, uint8_t *d_aln, int64_t aln_cap,
                int64_t *d_aln_len, int32_t *d_npaths, int32_t *d_status, hipStream_t s);

int run_coopt(const Plan &p, char *ws, const uint8_t *d_seqs, int32_t max_paths, int64_t *d_score,
              uint8_t *d_aln, int64_t aln_cap, int64_t *d_aln_len, int32_t *d_npaths,
              int32_t *d_status, hipStream_t s);

}  // namespace msa
