/*
 * msa_dp.h -- C ABI of an MI355X (gfx950) library for optimal multiple
 * sequence alignment by full k-dimensional dynamic programming.
 *
 * Method (Helal et al., "Parallelizing Optimal Multiple Sequence Alignment by
 * Dynamic Programming"):
 *   - Section 2, Eq. 1 and the paragraph after it: k sequences of lengths n_i
 *     span a k-dimensional tensor of shape (n_i + 1); every cell takes the
 *     maximum over its 2^k - 1 lower neighbours v - b (b a nonempty subset of
 *     the sequences) of  score(v - b) + column score(v, b).
 *   - Section 5.2: the column score is the sum over sequence pairs of
 *     sub(x, y) for two residues, `gap` for a residue and a gap, 0 for two gaps.
 *   - Section 4 (scoring of a cell): the initial cell is initialised (to 0).
 *   - Section 2 (traceback): the alignment is read back from the end of the
 *     tensor to the origin following the optimal choices.
 *   - Section 3 (partitions of edge S grouped in computation waves of equal
 *     distance from the origin; Eqs. 2-3, Tables 1-2): the GPU fill cuts the
 *     tensor into hypercube tiles and schedules them by the same wave order.
 * Readings where the paper is silent: global alignment (walk starts at the
 * far corner); out-of-range neighbours are not candidates; ties go to the
 * lowest neighbour mask b (bit i = sequence i contributes a residue).
 *
 * Conventions for every entry point:
 *   - Residues are codes in [0, alpha), alpha <= 255; `submat` is alpha x alpha
 *     int8, row-major, and must be symmetric.
 *   - `gap` is ADDED per residue-gap pair (penalties are negative).
 *   - 2 <= k <= MSA_MAX_K; lengths >= 0 (empty sequences allowed).
 *   - An alignment is k rows of `aln_cap` bytes (row i at offset i*aln_cap);
 *     row i is sequence i with gaps written as MSA_GAP_CODE; columns run from
 *     the origin to the end; aln_cap must be >= sum of the lengths.
 *   - All arithmetic is exact integer arithmetic (int32 on the device after
 *     a closed-form range check, MSA_ERANGE if it cannot be guaranteed).
 *   - Return value: MSA_OK (0) or a negative status.  On error no output is
 *     written (for the asynchronous device entry points: see each call).
 *   - The library keeps no caller pointer after a call returns, except where
 *     stated (server jobs).
 */
#ifndef MSA_DP_H
#define MSA_DP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSA_MAX_K 8          /* a direction byte holds the 2^k - 1 masks */
#define MSA_GAP_CODE 0xFF    /* gap symbol in alignment rows */

enum {
  MSA_OK = 0,
  MSA_EINVAL = -1,     /* bad argument (k, lengths, codes, matrix, capacity) */
  MSA_ERANGE = -2,     /* score range does not fit the device integer width */
  MSA_ENOMEM = -3,     /* workspace larger than the device or the budget */
  MSA_EDEVICE = -4,    /* HIP error or device watchdog timeout */
  MSA_EAGAIN = -5,     /* server: result not ready yet */
  MSA_ESHUTDOWN = -6   /* server: handle is shutting down */
};

/* Alignment mode flags (the _ex entry points). */
#define MSA_END_GAPS_FREE 1u /* end-gap-free alignment, see msa_dp_align_ex */
#define MSA_COOPTIMAL 2u     /* tie sets kept for msa_dp_align_coopt */
#define MSA_PRUNE 4u         /* exact tile pruning, see msa_dp_align_ex */
#define MSA_NEAROPT 8u       /* cell scores kept for msa_dp_nearopt_dev */

/* ------------------------------------------------------------------------
 * Launch-configuration tuner.  Per (architecture of the current device,
 * kind, k, length bucket) a table holds the fill variant and the number of
 * workgroups per compute unit that later calls use; every configuration
 * computes the same bytes, only the time differs.  Buckets: the plain path
 * keys by k and ceil(log2(longest length + 1)); the batched path by k class
 * (k = 2..4, 5, 6, 7..8).  Thread-safe; the table lives for the process.
 *   kind    : MSA_TUNE_PLAIN or MSA_TUNE_BATCH
 *   variant : plain path: 0 the built-in rule, 1 the streaming k = 3 fill
 *             (used only where it applies), 2 the tile fill; batched: 0
 *   wpc     : workgroups per compute unit of the tile fill or the batched
 *             fill (capped at what fits); 0 the built-in rule
 * msa_dp_tune_set stores a choice, msa_dp_tune_get reads it ((0, 0) when
 * none is stored) into choice_out[2], msa_dp_tune_clear empties the table.
 * msa_dp_tune_candidates writes up to cap / 2 (variant, wpc) pairs the tuner
 * tries for that key and returns their number.
 * msa_dp_autotune times the fill of every candidate on a device workspace of
 * the given shape and scoring (seeded residues; `reps` timed fills each,
 * median, HIP events), stores the fastest and returns it in choice_out[2]
 * (and its time in *best_ms_out when not NULL).  It allocates a workspace of
 * msa_dp_workspace_bytes(lens, k) bytes for the duration of the call.
 * msa_dp_autotune_batch runs msa_dp_align_batch on the jobs of each k class
 * present with every candidate workgroup count (`reps` timed runs each,
 * median wall time) and stores the fastest; wpc_out[4] receives the choice
 * per k class (0 for classes not present).
 * Errors: MSA_EINVAL for bad arguments, the errors of msa_dp_align /
 * msa_dp_align_batch, MSA_EDEVICE.
 * ---------------------------------------------------------------------- */
#define MSA_TUNE_PLAIN 0
#define MSA_TUNE_BATCH 1
int msa_dp_tune_set(int32_t kind, int32_t k, int32_t max_len, int32_t variant, int32_t wpc);
int msa_dp_tune_get(int32_t kind, int32_t k, int32_t max_len, int32_t *choice_out);
void msa_dp_tune_clear(void);
int msa_dp_tune_candidates(int32_t kind, int32_t k, int32_t max_len, int32_t *out,
                           int32_t cap);
int msa_dp_autotune(const int32_t *lens, int32_t k, const int8_t *submat, int32_t alpha,
                    int32_t gap, int32_t reps, int32_t *choice_out, float *best_ms_out);

/* Human-readable text for a status code (static storage). */
const char *msa_strerror(int status);

/* ------------------------------------------------------------------------
 * Plain path, host buffers.
 * Aligns k sequences: seqs[i] points to lens[i] host bytes.  Device memory
 * is managed internally (a per-thread cache keyed by the shape, reused by
 * later calls of the same shape).  Synchronous.
 *   score_out   : optimal sum-of-pairs score
 *   aln_out     : k rows of aln_cap bytes (host)
 *   aln_len_out : number of alignment columns L
 * Errors: MSA_EINVAL, MSA_ERANGE, MSA_ENOMEM, MSA_EDEVICE.
 * ---------------------------------------------------------------------- */
int msa_dp_align(const uint8_t *const *seqs, const int32_t *lens, int32_t k,
                 const int8_t *submat, int32_t alpha, int32_t gap,
                 int64_t *score_out, uint8_t *aln_out, int64_t aln_cap,
                 int64_t *aln_len_out);

/* ------------------------------------------------------------------------
 * msa_dp_align_ex: msa_dp_align with mode flags (flags = 0 is msa_dp_align).
 *
 * MSA_END_GAPS_FREE: end-gap-free alignment, the reading of Section 2's
 *   traceback start (the best-scoring cell of the far boundary) for k
 *   sequences.  Cells with some v_i = 0 score 0 (unaligned prefixes are
 *   free); the score is the maximum over the cells with some v_i = n_i
 *   (unaligned suffixes are free), the largest row-major cell index on ties;
 *   the walk goes back from that cell to the first cell with some v_i = 0.
 *   Output columns: the unaligned prefixes (sequence 0 first, one residue per
 *   column), the walked columns, the unaligned suffixes (sequence 0 first,
 *   one residue per column); the score is the sum-of-pairs score of the
 *   walked columns.  Requires prod(lens[i] + 1) <= 2^32 (else MSA_ERANGE).
 * MSA_COOPTIMAL: the fill keeps every maximising mask of each cell (its tie
 *   set, bit b - 1 for mask b); the alignment returned is the same as with
 *   flags = 0.  Requires k <= 3 and sum(lens) <= 32768 (MSA_EINVAL /
 *   MSA_ERANGE otherwise); not combinable with MSA_END_GAPS_FREE (MSA_EINVAL).
 * MSA_PRUNE: exact search-space reduction, Section 6's computation of only
 *   the partitions (tiles) where an optimal alignment can lie, made exact
 *   with the pairwise bound of Carrillo and Lipman: every cell v of an
 *   alignment with score S has S <= sum_{i<j} F_ij(v_i, v_j) + G_ij(v_i, v_j)
 *   (optimal pairwise scores of the prefixes and of the suffixes), so a tile
 *   whose bound, the sum over pairs of the maximum of F_ij + G_ij over the
 *   tile, is below a lower bound L of the optimum is not computed.  Pass 1
 *   uses L1 = U - ceil(|U|/16) - C(k,2) * max(|gap|, max|sub|), U the sum of
 *   the pairwise optima; its result is exact when its score reaches L1,
 *   otherwise pass 2 runs with L2 = that score (a real path's score, else no
 *   pruning).  Score and alignment equal those of flags = 0 (the decisions
 *   along optimal alignments are unchanged); the decision bytes of other
 *   cells may differ or be unwritten.  Requires 3 <= k <= 6 (else
 *   MSA_EINVAL) and every length < 16384 (else MSA_ERANGE); combinable with
 *   MSA_COOPTIMAL, not with MSA_END_GAPS_FREE (MSA_EINVAL).
 * Other flag bits: MSA_EINVAL.  Errors otherwise as msa_dp_align.
 * ---------------------------------------------------------------------- */
int msa_dp_align_ex(const uint8_t *const *seqs, const int32_t *lens, int32_t k,
                    const int8_t *submat, int32_t alpha, int32_t gap, uint32_t flags,
                    int64_t *score_out, uint8_t *aln_out, int64_t aln_cap,
                    int64_t *aln_len_out);

/* ------------------------------------------------------------------------
 * msa_dp_align_coopt: up to max_paths co-optimal alignments (every global
 * alignment with the optimal score): Section 6 proposes a traceback that
 * branches wherever several choices tie.  Synchronous, host
 * buffers, same device-memory cache as msa_dp_align.
 *   max_paths   : >= 1
 *   score_out   : the optimal score
 *   aln_out     : max_paths blocks of k rows of aln_cap bytes; alignment p
 *                 is at aln_out + p * k * aln_cap (layout as msa_dp_align)
 *   aln_len_out : max_paths int64, the column count of each alignment
 *   npaths_out  : number of alignments written; fewer than max_paths means
 *                 every co-optimal alignment was written
 * Order: the walk from the far corner tries the tied masks of each cell in
 * ascending order, so alignment 0 is msa_dp_align's and the list is sorted
 * by the column masks read from the last column to the first.
 * k <= 3 keeps a tie set per cell (sum(lens) <= 32768); 4 <= k <= 6 runs
 * the walk of msa_dp_align_nearopt with delta = 0, which lists the same
 * alignments in the same order (sum(lens) <= 4096).  Errors as msa_dp_align,
 * and MSA_EINVAL for k > 6 or max_paths < 1, MSA_ERANGE for longer inputs.
 * ---------------------------------------------------------------------- */
int msa_dp_align_coopt(const uint8_t *const *seqs, const int32_t *lens, int32_t k,
                       const int8_t *submat, int32_t alpha, int32_t gap, int32_t max_paths,
                       int64_t *score_out, uint8_t *aln_out, int64_t aln_cap,
                       int64_t *aln_len_out, int32_t *npaths_out);

/* ------------------------------------------------------------------------
 * msa_dp_align_nearopt: up to max_paths near-optimal alignments, every global
 * alignment whose sum-of-pairs score is at least opt - delta (Section 6: the
 * alignments within a threshold of the optimum set by the user).  The fill
 * also keeps every cell's score xi; a walk from the far corner then takes a
 * step v -> v - b only when xi(v - b) + SP(col(v, b)) plus the score of the
 * columns already taken reaches opt - delta, which some alignment through
 * that step does, so the walk has no dead end.  Synchronous, host buffers,
 * same device-memory cache as msa_dp_align.
 *   delta       : >= 0
 *   max_paths   : >= 1
 *   score_out   : the optimal score
 *   scores_out  : max_paths int64, the score of each alignment written
 *   aln_out     : max_paths blocks of k rows of aln_cap bytes (as
 *                 msa_dp_align_coopt)
 *   aln_len_out : max_paths int64 column counts
 *   npaths_out  : number of alignments written; fewer than max_paths means
 *                 every alignment at or above the threshold was written
 * Order: the masks of each cell are tried in ascending order, so the list is
 * sorted by the column masks read from the last column to the first;
 * delta = 0 gives msa_dp_align_coopt's list.  Requires k <= 6 and
 * sum(lens) <= 4096; the workspace needs 4 more bytes per cell (padded like
 * the direction blocks, msa_dp_workspace_bytes_ex).  Errors as msa_dp_align,
 * and MSA_EINVAL for k > 6, delta < 0 or max_paths < 1, MSA_ERANGE for
 * longer inputs.
 * ---------------------------------------------------------------------- */
int msa_dp_align_nearopt(const uint8_t *const *seqs, const int32_t *lens, int32_t k,
                         const int8_t *submat, int32_t alpha, int32_t gap, int64_t delta,
                         int32_t max_paths, int64_t *score_out, int64_t *scores_out,
                         uint8_t *aln_out, int64_t aln_cap, int64_t *aln_len_out,
                         int32_t *npaths_out);

/* Device-buffer form of msa_dp_align_nearopt on a workspace of at least
 * msa_dp_workspace_bytes_ex(lens, k, MSA_NEAROPT) bytes prepared with
 * msa_dp_prepare_ex(..., MSA_NEAROPT, ...): enqueues the fill and the walk on
 * hip_stream (asynchronous).  d_scores holds max_paths int64, the other
 * outputs as msa_dp_coopt_dev; d_status MSA_EINVAL when the workspace was not
 * prepared with MSA_NEAROPT (d_npaths and d_score then read 0).  Returns
 * MSA_EINVAL / MSA_ERANGE at once, enqueuing nothing, for the argument errors
 * of msa_dp_align_nearopt or those of msa_dp_align_dev. */
int msa_dp_nearopt_dev(void *d_workspace, int64_t ws_bytes, const uint8_t *d_seqs,
                       const int32_t *lens, int32_t k, int64_t delta, int32_t max_paths,
                       int64_t *d_score, int64_t *d_scores, uint8_t *d_aln, int64_t aln_cap,
                       int64_t *d_aln_len, int32_t *d_npaths, int32_t *d_status,
                       void *hip_stream);

/* Device-buffer form of msa_dp_align_coopt on a workspace prepared with
 * msa_dp_prepare_ex(..., MSA_COOPTIMAL, ...): enqueues the fill and the
 * enumeration on hip_stream (asynchronous).  d_aln holds max_paths * k rows
 * of aln_cap bytes, d_aln_len max_paths int64, d_npaths one int32; d_status
 * as msa_dp_align_dev, and MSA_EINVAL when the workspace was not prepared
 * with MSA_COOPTIMAL (d_npaths and d_score read 0 when it is not MSA_OK).
 * Returns MSA_EINVAL / MSA_ERANGE at once, enqueuing nothing, for k > 3,
 * sum(lens) > 32768, max_paths < 1 or the errors of msa_dp_align_dev. */
int msa_dp_coopt_dev(void *d_workspace, int64_t ws_bytes, const uint8_t *d_seqs,
                     const int32_t *lens, int32_t k, int32_t max_paths, int64_t *d_score,
                     uint8_t *d_aln, int64_t aln_cap, int64_t *d_aln_len,
                     int32_t *d_npaths, int32_t *d_status, void *hip_stream);

/* ------------------------------------------------------------------------
 * Plain path, device-resident buffers (the form the benchmark times).
 *
 * msa_dp_workspace_bytes: device workspace needed for one alignment of the
 *   given lengths (tile edge chosen by the library for k).  Returns the byte
 *   count (> 0) or a negative status (MSA_EINVAL / MSA_ENOMEM on overflow).
 *
 * msa_dp_prepare: one-time set-up of a caller-allocated workspace for the
 *   given shape and scoring: validates, checks the score range, writes the
 *   tile schedule and the substitution matrix into the workspace (host to
 *   device copies on `hip_stream`).  Must be called before the first
 *   msa_dp_align_dev on that workspace and again whenever lens, k, submat,
 *   alpha or gap change.  d_workspace must be 256-byte aligned and hold
 *   msa_dp_workspace_bytes(lens, k) bytes.
 *
 * msa_dp_align_dev: enqueue one alignment on `hip_stream` (a hipStream_t,
 *   NULL = default stream).  Asynchronous: returns after launching.
 *   d_seqs      : device bytes, the k sequences concatenated (sum lens)
 *   d_score     : device int64, optimal score
 *   d_aln       : device, k rows of aln_cap bytes
 *   d_aln_len   : device int64, L
 *   d_status    : device int32, MSA_OK or MSA_EINVAL (a residue code
 *                 >= alpha) or MSA_EDEVICE (watchdog); outputs are
 *                 meaningful only when it reads MSA_OK
 *   Host-detectable errors (bad k/lens/cap, unprepared or mismatched
 *   workspace, launch failure) are returned immediately and nothing is
 *   enqueued.  Calls on one workspace must be stream-ordered.
 * ---------------------------------------------------------------------- */
int64_t msa_dp_workspace_bytes(const int32_t *lens, int32_t k);

/* msa_dp_workspace_bytes for a workspace to be prepared with mode `flags`
 * (msa_dp_prepare_ex): MSA_NEAROPT adds one int32 cell score per cell
 * (padded like the direction blocks); the other modes need no more than
 * msa_dp_workspace_bytes.  Same returns, and MSA_EINVAL / MSA_ERANGE for
 * flags the shape does not allow. */
int64_t msa_dp_workspace_bytes_ex(const int32_t *lens, int32_t k, uint32_t flags);

int msa_dp_prepare(void *d_workspace, int64_t ws_bytes, const int32_t *lens,
                   int32_t k, const int8_t *submat, int32_t alpha,
                   int32_t gap, void *hip_stream);

/* msa_dp_prepare with mode flags (see msa_dp_align_ex); the mode is kept in
 * the workspace and applies to every later msa_dp_align_dev,
 * msa_dp_fill_dev / msa_dp_traceback_dev on it.  flags = 0 is
 * msa_dp_prepare. */
int msa_dp_prepare_ex(void *d_workspace, int64_t ws_bytes, const int32_t *lens,
                      int32_t k, const int8_t *submat, int32_t alpha,
                      int32_t gap, uint32_t flags, void *hip_stream);

int msa_dp_align_dev(void *d_workspace, int64_t ws_bytes,
                     const uint8_t *d_seqs, const int32_t *lens, int32_t k,
                     int64_t *d_score, uint8_t *d_aln, int64_t aln_cap,
                     int64_t *d_aln_len, int32_t *d_status, void *hip_stream);

/* msa_dp_align_static: msa_dp_align_dev without a caller workspace, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The call allocates
 * nothing: the workspace is a file-scope device array of 32 MiB that each
 * device the library runs on holds until the process ends, and its set-up
 * (control block, matrix, column schedule, cleared flags) is a kernel whose
 * inputs come by value, so the call only enqueues kernels on hip_stream
 * (asynchronous).  Arguments as msa_dp_align_dev, plus the scoring of
 * msa_dp_prepare (submat is a host pointer read during the call).
 * Limits: alpha <= 32 and a workspace (msa_dp_workspace_bytes) of at most
 * 32 MiB -- MSA_EINVAL / MSA_ENOMEM otherwise, returned at once with nothing
 * enqueued; the other errors as msa_dp_align_dev.  Plain mode only.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (the set-up rewrites what must start cleared): calls that
 * overlap on one device race and must be ordered by the caller (one stream,
 * or events between streams). */
int msa_dp_align_static(const uint8_t *d_seqs, const int32_t *lens, int32_t k,
                        const int8_t *submat, int32_t alpha, int32_t gap,
                        int64_t *d_score, uint8_t *d_aln, int64_t aln_cap,
                        int64_t *d_aln_len, int32_t *d_status, void *hip_stream);

/* The two launches of msa_dp_align_dev, for callers that time or overlap them
 * separately.  msa_dp_fill_dev scores every cell and writes the optimal score
 * to d_score; msa_dp_traceback_dev then writes the alignment, its length and
 * the status (and resets d_score to 0 on error).  Same arguments and rules as
 * msa_dp_align_dev; the traceback must follow the fill on the same stream:
 * it re-arms the workspace's work counter, so a second fill without the
 * traceback in between finds no work left and returns without scoring. */
int msa_dp_fill_dev(void *d_workspace, int64_t ws_bytes, const uint8_t *d_seqs,
                    const int32_t *lens, int32_t k, int64_t *d_score, void *hip_stream);

int msa_dp_traceback_dev(void *d_workspace, int64_t ws_bytes, const uint8_t *d_seqs,
                         const int32_t *lens, int32_t k, int64_t *d_score,
                         uint8_t *d_aln, int64_t aln_cap, int64_t *d_aln_len,
                         int32_t *d_status, void *hip_stream);

/* Copy the decision tensor of the last alignment run on `d_workspace` into
 * d_dir_out: prod(lens[i] + 1) bytes, row-major with the last sequence's
 * index fastest, byte = chosen neighbour mask b (0 at the origin); on a
 * workspace prepared with MSA_COOPTIMAL, byte = the cell's tie set (bit b - 1
 * for each maximising mask b, 0 at the origin).  For verification.
 * Asynchronous on hip_stream. */
int msa_dp_export_dirs(void *d_workspace, int64_t ws_bytes,
                       const int32_t *lens, int32_t k, uint8_t *d_dir_out,
                       void *hip_stream);

/* For a workspace prepared with MSA_PRUNE, after a fill: d_keep_out (may be
 * NULL) receives one byte per tile, 1 if the last pass computed it, in
 * row-major order of the tile coordinates (tiles along dimension i: one for
 * v_i = 0, then ceil(n_i / msa_dp_tile_edge(k)) of that edge); d_info_out
 * (may be NULL) receives 4 int64: U, the last pass's threshold L (INT64_MIN
 * for no pruning), the tiles it computed, and the passes run (1 or 2).
 * Device buffers; asynchronous on hip_stream.  MSA_EINVAL if the workspace
 * was not prepared with MSA_PRUNE. */
int msa_dp_export_prune(void *d_workspace, int64_t ws_bytes, const int32_t *lens,
                        int32_t k, uint8_t *d_keep_out, int64_t *d_info_out,
                        void *hip_stream);

/* ------------------------------------------------------------------------
 * Batched path: many independent alignments (uneven k and lengths) through
 * one persistent kernel per group of jobs whose workspaces fit
 * `hbm_budget_bytes` (0 = a default fraction of free device memory).
 * Synchronous.  Job inputs are host pointers read during the call.
 * results[i].aln must point to k * results[i].aln_cap host bytes; the call
 * writes status, score and aln_len of every result.  Returns MSA_OK when
 * the batch ran (per-job errors are in results[i].status), or a negative
 * status for a whole-call failure.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t k;
  const uint8_t *seqs[MSA_MAX_K];  /* host, lens[i] bytes each */
  int32_t lens[MSA_MAX_K];
  const int8_t *submat;            /* host, alpha x alpha */
  int32_t alpha;
  int32_t gap;
} msa_job;

typedef struct {
  int32_t status;    /* MSA_OK or a negative status for this job */
  int64_t score;
  uint8_t *aln;      /* caller-owned, k rows of aln_cap bytes */
  int64_t aln_cap;
  int64_t aln_len;
} msa_result;

int msa_dp_align_batch(const msa_job *jobs, int32_t njobs,
                       msa_result *results, int64_t hbm_budget_bytes);

/* The batched half of the tuner (see msa_dp_autotune above). */
int msa_dp_autotune_batch(const msa_job *jobs, int32_t njobs, int32_t reps, int32_t *wpc_out);

/* ------------------------------------------------------------------------
 * Served path: a request loop that admits jobs as device memory (the HBM
 * budget) and launch slots free up, keeps their state on the device and runs
 * several persistent launches at once (continuous batching).  Small launches
 * overlap on the device; a launch of 32 jobs or more runs alone (it waits for
 * the launches in flight and later ones wait for it, on the device).
 *
 * msa_server_create: hbm_budget_bytes (0 = default), max_inflight = maximum
 *   launches in flight (launch slots, each with its share of the budget),
 *   max_jobs_per_launch.  NULL on failure.
 * msa_server_submit: copies the job's inputs; *ticket identifies it.
 *   MSA_EINVAL / MSA_ERANGE for invalid jobs, MSA_ENOMEM when the job alone
 *   exceeds the whole budget, MSA_ESHUTDOWN after destroy started.
 * msa_server_poll: MSA_EAGAIN while running; otherwise fills *out (out->aln
 *   and out->aln_cap supplied by the caller), returns the job status and
 *   forgets the ticket.  MSA_EINVAL for an unknown ticket.
 * msa_server_wait: like poll but blocks up to timeout_us (< 0 = forever);
 *   MSA_EAGAIN on timeout.
 * msa_server_destroy: waits for in-flight launches, frees everything.
 * Thread-safe: submit/poll/wait may be called from several threads.
 * ---------------------------------------------------------------------- */
typedef struct msa_server msa_server;

msa_server *msa_server_create(int64_t hbm_budget_bytes, int32_t max_inflight,
                              int32_t max_jobs_per_launch);
int msa_server_submit(msa_server *srv, const msa_job *job, uint64_t *ticket);
int msa_server_poll(msa_server *srv, uint64_t ticket, msa_result *out);
int msa_server_wait(msa_server *srv, uint64_t ticket, msa_result *out,
                    int64_t timeout_us);
void msa_server_destroy(msa_server *srv);

/* msa_server_stats: counters of the server so far, for measurement.  Writes
 * the first n of: [0] launches completed, [1] jobs completed, [2] device
 * busy time in microseconds (the union of the completed launches' device
 * intervals, each from its input copy to its output copy, measured with HIP
 * events), [3] span in microseconds from the first launch's start to the
 * last launch's end, [4] jobs queued and not yet admitted, [5] jobs that
 * ended with a status other than MSA_OK, [6] the last such status (MSA_OK if
 * none), [7] the longest pause in microseconds that a launch's fill saw
 * between two checks of a dependency wait, that is a time its queue did not
 * run (0 if none; such pauses do not count towards the wait's time-out,
 * 250 ms in a batched launch),
 * [8] jobs queued again because their launch's dependency wait timed out
 * (each job is re-run at most once; a second time-out returns MSA_EDEVICE).
 * Returns MSA_OK or MSA_EINVAL. */
int msa_server_stats(msa_server *srv, int64_t *out, int32_t n);

/* msa_server_debug_wait_limit: the next `launches` launches of the server
 * (in admission order) give up a dependency wait after `ticks` ticks of the
 * 100 MHz clock instead of 250 ms, so that a test can exercise the time-out
 * path from the host (every kernel still exits normally; the launch reports
 * MSA_EDEVICE and the server re-runs its jobs once).  Returns MSA_OK or
 * MSA_EINVAL (ticks < 1, launches < 0). */
int msa_server_debug_wait_limit(msa_server *srv, int64_t ticks, int32_t launches);

/* ------------------------------------------------------------------------
 * Host-side helpers (no device needed), exposed for tests and tools.
 * ---------------------------------------------------------------------- */

/* Closed-form bounds on every cell score (any alignment of prefixes):
 * for gap <= 0, lo = gap*(k-1)*sum(n_i) (all single-residue columns) and
 * hi = max(0, max sub) * sum_{i<j} min(n_i, n_j); otherwise
 * +-sum(n_i)*C(k,2)*max(|gap|, max|sub|).  Returns MSA_OK or MSA_EINVAL. */
int msa_dp_score_bounds(const int32_t *lens, int32_t k, const int8_t *submat,
                        int32_t alpha, int32_t gap, int64_t *lo, int64_t *hi);

/* Validation of a shape, scoring and mode flags without a device: the
 * checks msa_dp_prepare_ex makes before touching the workspace (k, lengths,
 * flags, symmetric matrix, and the closed-form range check of every key the
 * fill can form in that mode; for MSA_PRUNE that includes the -infinity keys
 * that travel through kept tiles whose lower neighbours were pruned, along a
 * monotone path of up to sum(n_i) cells).  Returns MSA_OK, MSA_EINVAL or
 * MSA_ERANGE. */
int msa_dp_check_scoring(const int32_t *lens, int32_t k, const int8_t *submat,
                         int32_t alpha, int32_t gap, uint32_t flags);

/* Tile edge (interior cells per dimension) the library uses for k. */
int32_t msa_dp_tile_edge(int32_t k);

/* Tile grid of a shape: tiles_per_dim[i] = 1 + ceil(n_i / T) (the extra tile
 * is the one-cell-thick initial-gap layer v_i = 0); returns the number of
 * tile waves (sum of tiles_per_dim - k + 1), or a negative status. */
int32_t msa_dp_tile_grid(const int32_t *lens, int32_t k, int32_t tile_edge,
                         int32_t *tiles_per_dim);

/* Number of tiles in each computation wave (tiles whose coordinates sum to
 * w) of a grid with p[i] tiles along dimension i (Section 3.1-3.2, Eqs. 2-3,
 * Tables 1-2).  Writes counts[0 .. waves-1] and returns the wave count
 * sum(p) - k + 1, or a negative status (cap too small / bad input). */
int32_t msa_dp_wave_counts(const int32_t *p, int32_t k, int64_t *counts,
                           int32_t cap);

#ifdef __cplusplus
}
#endif
#endif /* MSA_DP_H */
