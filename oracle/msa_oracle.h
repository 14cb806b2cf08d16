/*
 * msa_oracle.h -- reference (oracle) implementation of optimal k-sequence
 * alignment by full dynamic programming.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may call this.  It shares no code, header,
 * table or helper with the GPU library; neither side includes the other.
 *
 * What it computes (Helal et al., "Parallelizing Optimal Multiple Sequence
 * Alignment by Dynamic Programming"):
 *   - Section 2, Eq. 1: the pairwise recurrence max over three neighbours of
 *     (neighbour score + substitution score or gap score);
 *   - Section 2 (text after Eq. 1): its generalisation to k sequences, where a
 *     cell of the k-dimensional tensor of shape (n_i + 1) takes the maximum over
 *     its 2^k - 1 lower neighbours;
 *   - Section 5.2: the sum-of-pairs column score (residue-residue pairs use the
 *     substitution score, residue-gap pairs score the gap value, gap-gap pairs
 *     score 0);
 *   - Section 2 (traceback): the optimal alignment is recovered by walking
 *     back from the end of the tensor to the origin along optimal choices.
 *
 * Readings taken where the paper is silent (all listed in the design notes):
 *   - global alignment: the walk starts at the far corner (n_0, ..., n_{k-1});
 *   - the origin scores 0, and a neighbour outside the tensor is not a
 *     candidate;
 *   - ties go to the lowest neighbour bitmask b, where bit i of b set means
 *     "sequence i contributes its residue to this column";
 *   - the gap value is added per residue-gap pair (a penalty is negative).
 *
 * Exact integer arithmetic (int64); no rounding anywhere.
 */
#ifndef MSA_ORACLE_H
#define MSA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSA_ORACLE_GAP 0xFF /* gap symbol in the returned alignment rows */
#define MSA_ORACLE_MAX_K 8

/*
 * Align k sequences (2 <= k <= 8).
 *   seqs[i]    : lens[i] residue codes in [0, alpha)
 *   sub        : alpha x alpha substitution scores, row-major, symmetric
 *   gap        : score added for each residue-gap pair in a column
 *   score_out  : optimal sum-of-pairs score
 *   dir_out    : optional (may be NULL); prod(lens[i] + 1) bytes, row-major
 *                with the last sequence's index fastest; dir_out[v] is the
 *                chosen neighbour mask b at cell v (0 at the origin)
 *   aln_out    : k rows of aln_cap bytes; row i is sequence i with gaps
 *                written as MSA_ORACLE_GAP, columns from origin to end
 *   aln_len_out: number of columns L
 * Returns 0, or -1 on invalid input / allocation failure (outputs untouched).
 */
int msa_oracle_align(int32_t k, const int32_t *lens, const uint8_t *const *seqs,
                     int32_t alpha, const int32_t *sub, int32_t gap,
                     int64_t *score_out, uint8_t *dir_out,
                     uint8_t *aln_out, int64_t aln_cap, int64_t *aln_len_out);

/*
 * End-gap-free variant.  Section 2 starts the traceback at the best-scoring
 * cell of the tensor's far boundary; read for k sequences as:
 *   - every cell with some v_i = 0 scores 0 and has no decision (dir 0): any
 *     prefixes may be left unaligned for free;
 *   - every other cell follows the same recurrence as msa_oracle_align (all of
 *     its 2^k - 1 neighbours exist);
 *   - the score is the maximum over the cells with some v_i = n_i (the rest of
 *     every sequence is left unaligned for free); among equal maxima the cell
 *     with the largest row-major index ends the alignment;
 *   - the walk goes back from that cell until it reaches a cell with some
 *     v_i = 0;
 *   - output columns: the unaligned prefixes (sequence 0 first, one residue
 *     per column), then the walked columns, then the unaligned suffixes
 *     (sequence 0 first, one residue per column).
 * core_begin_out / core_end_out (may be NULL) receive the column range of the
 * walked part; the score is the sum-of-pairs score of those columns.
 * Other arguments and the return value as msa_oracle_align.
 */
int msa_oracle_align_egf(int32_t k, const int32_t *lens, const uint8_t *const *seqs,
                         int32_t alpha, const int32_t *sub, int32_t gap,
                         int64_t *score_out, uint8_t *dir_out,
                         uint8_t *aln_out, int64_t aln_cap, int64_t *aln_len_out,
                         int64_t *core_begin_out, int64_t *core_end_out);

/*
 * Co-optimal alignments (the paper's remark that the approach can also return
 * co-optimal alignments, Section 6): the same global fill, but every cell
 * keeps its tie set T(v) = { b : candidate b reaches the maximum }.  Every
 * walk from the far corner that only steps along tie-set masks reaches the
 * origin with the optimal score, and every optimal alignment is such a walk.
 * They are enumerated depth first, the masks of each cell tried in ascending
 * order, so alignments come in lexicographic order of their column masks read
 * from the last column to the first; the first one is msa_oracle_align's.
 *   max_paths   : at most this many alignments are returned (>= 1)
 *   aln_out     : max_paths blocks of k rows of aln_cap bytes
 *   aln_len_out : max_paths column counts
 *   npaths_out  : number returned; fewer than max_paths means these are all
 *   tie_out     : optional (may be NULL); prod(lens[i] + 1) bytes, bit b - 1
 *                 set when mask b is in T(v) (k <= 8 uses the low bits of one
 *                 byte; k <= 3 only, larger k is rejected)
 * Returns 0, or -1 on invalid input (k > 3 included) / allocation failure.
 */
int msa_oracle_coopt(int32_t k, const int32_t *lens, const uint8_t *const *seqs,
                     int32_t alpha, const int32_t *sub, int32_t gap, int32_t max_paths,
                     int64_t *score_out, uint8_t *tie_out, uint8_t *aln_out,
                     int64_t aln_cap, int64_t *aln_len_out, int32_t *npaths_out);

/*
 * Near-optimal alignments (Section 6: the alignments whose score lies within
 * a threshold set by the user of the optimum): every global alignment with
 * sum-of-pairs score >= opt - delta.  xi(u), the optimal score of a path from
 * the origin to u, is reached by some path; so a walk from the far corner that
 * has collected the suffix score s on reaching cell v can still end at or
 * above the threshold through mask b exactly when
 *     xi(v - b) + SP(col(v, b)) + s >= opt - delta.
 * Walking only such steps enumerates exactly the near-optimal alignments,
 * with no dead end.  Depth first, the masks of each cell tried in ascending
 * order, as msa_oracle_coopt: alignments come in lexicographic order of their
 * column masks read from the last column to the first, and with delta = 0 the
 * list is msa_oracle_coopt's.
 *   delta       : >= 0
 *   max_paths   : at most this many alignments are returned (>= 1)
 *   score_out   : the optimal score
 *   scores_out  : max_paths int64, the score of each alignment returned
 *   aln_out, aln_len_out, npaths_out : as msa_oracle_coopt
 * Any k in 2..8.  Returns 0, or -1 on invalid input / allocation failure.
 */
int msa_oracle_nearopt(int32_t k, const int32_t *lens, const uint8_t *const *seqs,
                       int32_t alpha, const int32_t *sub, int32_t gap, int64_t delta,
                       int32_t max_paths, int64_t *score_out, int64_t *scores_out,
                       uint8_t *aln_out, int64_t aln_cap, int64_t *aln_len_out,
                       int32_t *npaths_out);

/*
 * Score every cell: writes the full int64 score tensor (prod(lens[i]+1)
 * entries, same layout as dir_out) without a traceback.  Returns 0 or -1.
 */
int msa_oracle_fill(int32_t k, const int32_t *lens, const uint8_t *const *seqs,
                    int32_t alpha, const int32_t *sub, int32_t gap,
                    int64_t *score_tensor_out, uint8_t *dir_out);

#ifdef __cplusplus
}
#endif
#endif
