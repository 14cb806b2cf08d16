/*
 * msa_oracle.c -- plain, slow, single-threaded reference for optimal
 * k-sequence alignment by dynamic programming.  TEST INFRASTRUCTURE ONLY:
 * called by the test suite, the smoke check and the benchmark's CPU-baseline
 * leg, never by the GPU library.  Shares no code with the GPU path.
 *
 * Every step follows the definition in the paper (Helal et al.):
 *   cell tensor   : shape (n_i + 1), the "+1" being the initial gap character
 *                   (Section 3.2, the (8,8,8,8) -> (9,9,9,9), 6561-cell example)
 *   recurrence    : Eq. 1 (Section 2) for two sequences, generalised to the
 *                   2^k - 1 lower neighbours of a cell (Section 2)
 *   column score  : sum of pairs, gap-gap = 0 (Section 5.2)
 *   initial cell  : initialised, here to 0 (Section 4, scoring of a cell)
 *   traceback     : walk from the end of the tensor back to the origin
 *                   following the optimal choices (Section 2)
 * No blocking, fusion or reordering: cells are visited in row-major order
 * (every lower neighbour v - b precedes v in that order), each candidate is
 * scored by building its column and summing its pairs.
 */
#include "msa_oracle.h"

#include <stdlib.h>
#include <string.h>

#define GAP_SYM (-1)

/* Score of one pair of column entries (Section 5.2 scheme, Eq. 1 terms). */
static int64_t pair_score(int x, int y, int32_t alpha, const int32_t *sub,
                          int32_t gap) {
  if (x == GAP_SYM && y == GAP_SYM) return 0;          /* gap-gap pair */
  if (x == GAP_SYM || y == GAP_SYM) return gap;        /* residue-gap pair */
  return sub[(int64_t)x * alpha + y];                  /* sub(a_i, b_j) */
}

/* Column produced when stepping into cell v from v - b: sequence i
 * contributes residue s_i[v_i - 1] when bit i of b is set, a gap otherwise. */
static void build_column(int32_t k, const int64_t *v, int b,
                         const uint8_t *const *seqs, int *col) {
  for (int i = 0; i < k; ++i)
    col[i] = ((b >> i) & 1) ? (int)seqs[i][v[i] - 1] : GAP_SYM;
}

/* Sum-of-pairs score of a column. */
static int64_t sp_score(int32_t k, const int *col, int32_t alpha,
                        const int32_t *sub, int32_t gap) {
  int64_t s = 0;
  for (int i = 0; i < k; ++i)
    for (int j = i + 1; j < k; ++j) s += pair_score(col[i], col[j], alpha, sub, gap);
  return s;
}

static int validate(int32_t k, const int32_t *lens, const uint8_t *const *seqs,
                    int32_t alpha, const int32_t *sub) {
  if (k < 2 || k > MSA_ORACLE_MAX_K || !lens || !seqs || !sub) return -1;
  if (alpha < 1 || alpha > 255) return -1;
  for (int i = 0; i < k; ++i) {
    if (lens[i] < 0) return -1;
    if (lens[i] > 0 && !seqs[i]) return -1;
    for (int32_t t = 0; t < lens[i]; ++t)
      if (seqs[i][t] >= alpha) return -1;
  }
  return 0;
}

/* Full fill: score tensor xi (int64) and decision tensor D (lowest
 * maximising mask).  Row-major strides, last sequence fastest. */
static int fill(int32_t k, const int32_t *lens, const uint8_t *const *seqs,
                int32_t alpha, const int32_t *sub, int32_t gap, int64_t *xi,
                uint8_t *D) {
  int64_t stride[MSA_ORACLE_MAX_K];
  int64_t ncell = 1;
  for (int i = k - 1; i >= 0; --i) {
    stride[i] = ncell;
    ncell *= (int64_t)lens[i] + 1;
  }
  int64_t v[MSA_ORACLE_MAX_K];
  int col[MSA_ORACLE_MAX_K];
  const int nmask = 1 << k;
  for (int64_t lin = 0; lin < ncell; ++lin) {
    /* coordinates of cell lin */
    int64_t rem = lin;
    for (int i = 0; i < k; ++i) {
      v[i] = rem / stride[i];
      rem -= v[i] * stride[i];
    }
    if (lin == 0) { /* initial cell */
      xi[0] = 0;
      D[0] = 0;
      continue;
    }
    int have = 0;
    int64_t best = 0;
    int bestb = 0;
    for (int b = 1; b < nmask; ++b) {
      /* neighbour v - b must lie inside the tensor */
      int ok = 1;
      int64_t pred = lin;
      for (int i = 0; i < k; ++i) {
        if ((b >> i) & 1) {
          if (v[i] == 0) { ok = 0; break; }
          pred -= stride[i];
        }
      }
      if (!ok) continue;
      build_column(k, v, b, seqs, col);
      int64_t cand = xi[pred] + sp_score(k, col, alpha, sub, gap);
      /* strictly greater: among equal candidates the first (lowest b) stays */
      if (!have || cand > best) {
        best = cand;
        bestb = b;
        have = 1;
      }
    }
    xi[lin] = best;
    D[lin] = (uint8_t)bestb;
  }
  return 0;
}

int msa_oracle_fill(int32_t k, const int32_t *lens, const uint8_t *const *seqs,
                    int32_t alpha, const int32_t *sub, int32_t gap,
                    int64_t *score_tensor_out, uint8_t *dir_out) {
  if (validate(k, lens, seqs, alpha, sub) != 0 || !score_tensor_out) return -1;
  int64_t ncell = 1;
  for (int i = 0; i < k; ++i) ncell *= (int64_t)lens[i] + 1;
  uint8_t *D = dir_out ? dir_out : (uint8_t *)malloc((size_t)ncell);
  if (!D) return -1;
  fill(k, lens, seqs, alpha, sub, gap, score_tensor_out, D);
  if (!dir_out) free(D);
  return 0;
}

int msa_oracle_align(int32_t k, const int32_t *lens, const uint8_t *const *seqs,
                     int32_t alpha, const int32_t *sub, int32_t gap,
                     int64_t *score_out, uint8_t *dir_out, uint8_t *aln_out,
                     int64_t aln_cap, int64_t *aln_len_out) {
  if (validate(k, lens, seqs, alpha, sub) != 0) return -1;
  if (!score_out || !aln_out || !aln_len_out) return -1;
  int64_t total = 0;
  for (int i = 0; i < k; ++i) total += lens[i];
  if (aln_cap < total) return -1;

  int64_t stride[MSA_ORACLE_MAX_K];
  int64_t ncell = 1;
  for (int i = k - 1; i >= 0; --i) {
    stride[i] = ncell;
    ncell *= (int64_t)lens[i] + 1;
  }
  int64_t *xi = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
  uint8_t *D = dir_out ? dir_out : (uint8_t *)malloc((size_t)ncell);
  /* columns are emitted end-first during the walk, then reversed */
  uint8_t *rev = (uint8_t *)malloc((size_t)(total > 0 ? total : 1) * (size_t)k);
  if (!xi || !D || !rev) {
    free(xi);
    if (!dir_out) free(D);
    free(rev);
    return -1;
  }
  fill(k, lens, seqs, alpha, sub, gap, xi, D);

  /* traceback from the far corner to the origin */
  int64_t v[MSA_ORACLE_MAX_K];
  int64_t lin = 0;
  for (int i = 0; i < k; ++i) {
    v[i] = lens[i];
    lin += v[i] * stride[i];
  }
  int64_t L = 0;
  while (lin != 0) {
    int b = D[lin];
    for (int i = 0; i < k; ++i) {
      if ((b >> i) & 1) {
        rev[L * k + i] = seqs[i][v[i] - 1];
        v[i] -= 1;
        lin -= stride[i];
      } else {
        rev[L * k + i] = MSA_ORACLE_GAP;
      }
    }
    ++L;
  }
  for (int64_t c = 0; c < L; ++c)
    for (int i = 0; i < k; ++i) aln_out[i * aln_cap + c] = rev[(L - 1 - c) * k + i];
  *score_out = xi[ncell - 1];
  *aln_len_out = L;
  free(xi);
  if (!dir_out) free(D);
  free(rev);
  return 0;
}

/* End-gap-free fill: cells with some v_i = 0 score 0 and carry no decision;
 * every other cell takes the maximum over all 2^k - 1 neighbours (they all
 * exist), lowest mask on ties. */
static void fill_egf(int32_t k, const int32_t *lens, const uint8_t *const *seqs,
                     int32_t alpha, const int32_t *sub, int32_t gap, int64_t *xi,
                     uint8_t *D) {
  int64_t stride[MSA_ORACLE_MAX_K];
  int64_t ncell = 1;
  for (int i = k - 1; i >= 0; --i) {
    stride[i] = ncell;
    ncell *= (int64_t)lens[i] + 1;
  }
  int64_t v[MSA_ORACLE_MAX_K];
  int col[MSA_ORACLE_MAX_K];
  const int nmask = 1 << k;
  for (int64_t lin = 0; lin < ncell; ++lin) {
    int64_t rem = lin;
    int on_lower = 0;
    for (int i = 0; i < k; ++i) {
      v[i] = rem / stride[i];
      rem -= v[i] * stride[i];
      if (v[i] == 0) on_lower = 1;
    }
    if (on_lower) { /* free unaligned prefixes */
      xi[lin] = 0;
      D[lin] = 0;
      continue;
    }
    int64_t best = 0;
    int bestb = 0;
    for (int b = 1; b < nmask; ++b) {
      int64_t pred = lin;
      for (int i = 0; i < k; ++i)
        if ((b >> i) & 1) pred -= stride[i];
      build_column(k, v, b, seqs, col);
      int64_t cand = xi[pred] + sp_score(k, col, alpha, sub, gap);
      if (b == 1 || cand > best) {
        best = cand;
        bestb = b;
      }
    }
    xi[lin] = best;
    D[lin] = (uint8_t)bestb;
  }
}

int msa_oracle_align_egf(int32_t k, const int32_t *lens, const uint8_t *const *seqs,
                         int32_t alpha, const int32_t *sub, int32_t gap,
                         int64_t *score_out, uint8_t *dir_out, uint8_t *aln_out,
                         int64_t aln_cap, int64_t *aln_len_out,
                         int64_t *core_begin_out, int64_t *core_end_out) {
  if (validate(k, lens, seqs, alpha, sub) != 0) return -1;
  if (!score_out || !aln_out || !aln_len_out) return -1;
  int64_t total = 0;
  for (int i = 0; i < k; ++i) total += lens[i];
  if (aln_cap < total) return -1;

  int64_t stride[MSA_ORACLE_MAX_K];
  int64_t ncell = 1;
  for (int i = k - 1; i >= 0; --i) {
    stride[i] = ncell;
    ncell *= (int64_t)lens[i] + 1;
  }
  int64_t *xi = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
  uint8_t *D = dir_out ? dir_out : (uint8_t *)malloc((size_t)ncell);
  uint8_t *rev = (uint8_t *)malloc((size_t)(total > 0 ? total : 1) * (size_t)k);
  if (!xi || !D || !rev) {
    free(xi);
    if (!dir_out) free(D);
    free(rev);
    return -1;
  }
  fill_egf(k, lens, seqs, alpha, sub, gap, xi, D);

  /* end cell: best score among cells with some v_i = n_i; ties -> largest
   * row-major index (the scan is ascending, so >= keeps the last one) */
  int64_t v[MSA_ORACLE_MAX_K];
  int64_t end = -1, best = 0;
  for (int64_t lin = 0; lin < ncell; ++lin) {
    int64_t rem = lin;
    int on_upper = 0;
    for (int i = 0; i < k; ++i) {
      v[i] = rem / stride[i];
      rem -= v[i] * stride[i];
      if (v[i] == lens[i]) on_upper = 1;
    }
    if (!on_upper) continue;
    if (end < 0 || xi[lin] >= best) {
      best = xi[lin];
      end = lin;
    }
  }
  int64_t e[MSA_ORACLE_MAX_K];
  {
    int64_t rem = end;
    for (int i = 0; i < k; ++i) {
      e[i] = rem / stride[i];
      rem -= e[i] * stride[i];
      v[i] = e[i];
    }
  }
  /* walk back while every v_i >= 1 */
  int64_t lin = end, W = 0;
  for (;;) {
    int on_lower = 0;
    for (int i = 0; i < k; ++i)
      if (v[i] == 0) on_lower = 1;
    if (on_lower) break;
    int b = D[lin];
    for (int i = 0; i < k; ++i) {
      if ((b >> i) & 1) {
        rev[W * k + i] = seqs[i][v[i] - 1];
        v[i] -= 1;
        lin -= stride[i];
      } else {
        rev[W * k + i] = MSA_ORACLE_GAP;
      }
    }
    ++W;
  }
  /* assemble: prefixes v_i (start cell), walked columns, suffixes from e_i */
  int64_t L = 0;
  for (int i = 0; i < k; ++i)
    for (int64_t t = 0; t < v[i]; ++t, ++L)
      for (int j = 0; j < k; ++j)
        aln_out[j * aln_cap + L] = (j == i) ? seqs[i][t] : MSA_ORACLE_GAP;
  const int64_t core_begin = L;
  for (int64_t c = 0; c < W; ++c, ++L)
    for (int j = 0; j < k; ++j) aln_out[j * aln_cap + L] = rev[(W - 1 - c) * k + j];
  const int64_t core_end = L;
  for (int i = 0; i < k; ++i)
    for (int64_t t = e[i]; t < lens[i]; ++t, ++L)
      for (int j = 0; j < k; ++j)
        aln_out[j * aln_cap + L] = (j == i) ? seqs[i][t] : MSA_ORACLE_GAP;

  *score_out = best;
  *aln_len_out = L;
  if (core_begin_out) *core_begin_out = core_begin;
  if (core_end_out) *core_end_out = core_end;
  free(xi);
  if (!dir_out) free(D);
  free(rev);
  return 0;
}

/* Global fill that keeps, per cell, the set of maximising masks (bit b - 1
 * for mask b); same recurrence and candidates as fill(). */
static void fill_ties(int32_t k, const int32_t *lens, const uint8_t *const *seqs,
                      int32_t alpha, const int32_t *sub, int32_t gap, int64_t *xi,
                      uint8_t *TS) {
  int64_t stride[MSA_ORACLE_MAX_K];
  int64_t ncell = 1;
  for (int i = k - 1; i >= 0; --i) {
    stride[i] = ncell;
    ncell *= (int64_t)lens[i] + 1;
  }
  int64_t v[MSA_ORACLE_MAX_K];
  int col[MSA_ORACLE_MAX_K];
  int64_t cand[256];
  int valid[256];
  const int nmask = 1 << k;
  for (int64_t lin = 0; lin < ncell; ++lin) {
    int64_t rem = lin;
    for (int i = 0; i < k; ++i) {
      v[i] = rem / stride[i];
      rem -= v[i] * stride[i];
    }
    if (lin == 0) {
      xi[0] = 0;
      TS[0] = 0;
      continue;
    }
    int have = 0;
    int64_t best = 0;
    for (int b = 1; b < nmask; ++b) {
      valid[b] = 1;
      int64_t pred = lin;
      for (int i = 0; i < k; ++i)
        if ((b >> i) & 1) {
          if (v[i] == 0) valid[b] = 0;
          pred -= stride[i];
        }
      if (!valid[b]) continue;
      build_column(k, v, b, seqs, col);
      cand[b] = xi[pred] + sp_score(k, col, alpha, sub, gap);
      if (!have || cand[b] > best) best = cand[b];
      have = 1;
    }
    uint8_t t = 0;
    for (int b = 1; b < nmask; ++b)
      if (valid[b] && cand[b] == best) t |= (uint8_t)(1u << (b - 1));
    xi[lin] = best;
    TS[lin] = t;
  }
}

int msa_oracle_coopt(int32_t k, const int32_t *lens, const uint8_t *const *seqs,
                     int32_t alpha, const int32_t *sub, int32_t gap, int32_t max_paths,
                     int64_t *score_out, uint8_t *tie_out, uint8_t *aln_out,
                     int64_t aln_cap, int64_t *aln_len_out, int32_t *npaths_out) {
  if (validate(k, lens, seqs, alpha, sub) != 0 || k > 3 || max_paths < 1) return -1;
  if (!score_out || !aln_out || !aln_len_out || !npaths_out) return -1;
  int64_t total = 0;
  for (int i = 0; i < k; ++i) total += lens[i];
  if (aln_cap < total) return -1;
  int64_t stride[MSA_ORACLE_MAX_K];
  int64_t ncell = 1;
  for (int i = k - 1; i >= 0; --i) {
    stride[i] = ncell;
    ncell *= (int64_t)lens[i] + 1;
  }
  int64_t *xi = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
  uint8_t *TS = tie_out ? tie_out : (uint8_t *)malloc((size_t)ncell);
  int *path = (int *)malloc((size_t)(total + 1) * sizeof(int)); /* mask per depth */
  if (!xi || !TS || !path) {
    free(xi);
    if (!tie_out) free(TS);
    free(path);
    return -1;
  }
  fill_ties(k, lens, seqs, alpha, sub, gap, xi, TS);

  /* depth-first walk from the far corner: path[d] is the mask taken at depth
   * d, from the cell reached after the first d steps */
  int64_t lin = ncell - 1;
  int64_t d = 0;
  int32_t np = 0;
  path[0] = 0; /* next mask to try is the lowest one above path[d] */
  for (;;) {
    if (lin == 0) { /* reached the origin: emit the alignment of path[0..d) */
      uint8_t *blk = aln_out + (int64_t)np * k * aln_cap;
      int64_t pos[MSA_ORACLE_MAX_K];
      for (int i = 0; i < k; ++i) pos[i] = 0;
      for (int64_t c = 0; c < d; ++c) { /* columns origin first */
        const int b = path[d - 1 - c];
        for (int i = 0; i < k; ++i)
          blk[i * aln_cap + c] = ((b >> i) & 1) ? seqs[i][pos[i]++] : MSA_ORACLE_GAP;
      }
      aln_len_out[np] = d;
      if (++np == max_paths) break;
      /* back up one step and try the next tied mask there */
      if (d == 0) break;
      --d;
      for (int i = 0; i < k; ++i)
        if ((path[d] >> i) & 1) lin += stride[i];
    }
    /* next mask of T(cell) above path[d] */
    const uint8_t t = TS[lin];
    int b = path[d] + 1;
    while (b < (1 << k) && !((t >> (b - 1)) & 1)) ++b;
    if (b < (1 << k)) {
      path[d] = b;
      for (int i = 0; i < k; ++i)
        if ((b >> i) & 1) lin -= stride[i];
      ++d;
      path[d] = 0;
      continue;
    }
    /* no mask left here: back up */
    if (d == 0) break;
    --d;
    for (int i = 0; i < k; ++i)
      if ((path[d] >> i) & 1) lin += stride[i];
  }
  *score_out = xi[ncell - 1];
  *npaths_out = np;
  free(xi);
  if (!tie_out) free(TS);
  free(path);
  return 0;
}

int msa_oracle_nearopt(int32_t k, const int32_t *lens, const uint8_t *const *seqs,
                       int32_t alpha, const int32_t *sub, int32_t gap, int64_t delta,
                       int32_t max_paths, int64_t *score_out, int64_t *scores_out,
                       uint8_t *aln_out, int64_t aln_cap, int64_t *aln_len_out,
                       int32_t *npaths_out) {
  if (validate(k, lens, seqs, alpha, sub) != 0 || delta < 0 || max_paths < 1) return -1;
  if (!score_out || !scores_out || !aln_out || !aln_len_out || !npaths_out) return -1;
  int64_t total = 0;
  for (int i = 0; i < k; ++i) total += lens[i];
  if (aln_cap < total) return -1;
  int64_t stride[MSA_ORACLE_MAX_K];
  int64_t ncell = 1;
  for (int i = k - 1; i >= 0; --i) {
    stride[i] = ncell;
    ncell *= (int64_t)lens[i] + 1;
  }
  int64_t *xi = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
  uint8_t *D = (uint8_t *)malloc((size_t)ncell);
  int *path = (int *)malloc((size_t)(total + 1) * sizeof(int));           /* mask per depth */
  int64_t *sfx = (int64_t *)malloc((size_t)(total + 1) * sizeof(int64_t)); /* score so far */
  if (!xi || !D || !path || !sfx) {
    free(xi);
    free(D);
    free(path);
    free(sfx);
    return -1;
  }
  fill(k, lens, seqs, alpha, sub, gap, xi, D);
  const int64_t threshold = xi[ncell - 1] - delta;
  const int nmask = 1 << k;

  /* depth-first walk from the far corner: path[d] is the mask taken at depth
   * d, sfx[d] the score of the columns taken before depth d */
  int64_t lin = ncell - 1;
  int64_t d = 0;
  int32_t np = 0;
  path[0] = 0;
  sfx[0] = 0;
  int64_t v[MSA_ORACLE_MAX_K];
  int col[MSA_ORACLE_MAX_K];
  for (;;) {
    if (lin == 0) { /* reached the origin: emit the alignment of path[0..d) */
      uint8_t *blk = aln_out + (int64_t)np * k * aln_cap;
      int64_t pos[MSA_ORACLE_MAX_K];
      for (int i = 0; i < k; ++i) pos[i] = 0;
      for (int64_t c = 0; c < d; ++c) { /* columns origin first */
        const int b = path[d - 1 - c];
        for (int i = 0; i < k; ++i)
          blk[i * aln_cap + c] = ((b >> i) & 1) ? seqs[i][pos[i]++] : MSA_ORACLE_GAP;
      }
      aln_len_out[np] = d;
      scores_out[np] = sfx[d];
      if (++np == max_paths) break;
      if (d == 0) break;
      --d; /* back up one step and try the next mask there */
      for (int i = 0; i < k; ++i)
        if ((path[d] >> i) & 1) lin += stride[i];
    }
    /* coordinates of the current cell */
    int64_t rem = lin;
    for (int i = 0; i < k; ++i) {
      v[i] = rem / stride[i];
      rem -= v[i] * stride[i];
    }
    /* the next mask above path[d] whose step can still end at or above the
     * threshold */
    int taken = 0;
    for (int b = path[d] + 1; b < nmask && !taken; ++b) {
      int ok = 1;
      int64_t pred = lin;
      for (int i = 0; i < k; ++i) {
        if ((b >> i) & 1) {
          if (v[i] == 0) { ok = 0; break; }
          pred -= stride[i];
        }
      }
      if (!ok) continue;
      build_column(k, v, b, seqs, col);
      const int64_t s = sp_score(k, col, alpha, sub, gap);
      if (xi[pred] + s + sfx[d] >= threshold) {
        path[d] = b;
        sfx[d + 1] = sfx[d] + s;
        lin = pred;
        ++d;
        path[d] = 0;
        taken = 1;
      }
    }
    if (taken) continue;
    /* no mask left here: back up */
    if (d == 0) break;
    --d;
    for (int i = 0; i < k; ++i)
      if ((path[d] >> i) & 1) lin += stride[i];
  }
  *score_out = xi[ncell - 1];
  *npaths_out = np;
  free(xi);
  free(D);
  free(path);
  free(sfx);
  return 0;
}
