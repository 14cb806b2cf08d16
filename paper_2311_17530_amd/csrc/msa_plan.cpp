// msa_plan.cpp -- host core of the library (no device calls).
#include "msa_plan.h"

#include <string.h>

#include <algorithm>

#include "../../include/msa_dp.h"

namespace msa {

static int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

static bool mul_ok(int64_t a, int64_t b, int64_t lim) { return a == 0 || b <= lim / a; }

int make_plan(const int32_t *lens, int32_t k, Plan *p) {
  if (!lens || !p || k < 2 || k > kMaxK) return MSA_EINVAL;
  Plan q;
  q.k = k;
  q.T = tile_edge_for_k(k);
  const int64_t lim = (int64_t)1 << 50;
  q.ncell = 1;
  int64_t a = 1;
  for (int i = 0; i < k; ++i) {
    if (lens[i] < 0 || lens[i] > (1 << 24)) return MSA_EINVAL;
    q.n[i] = lens[i];
    q.P[i] = 1 + (lens[i] + q.T - 1) / q.T;
    if (!mul_ok(q.ncell, (int64_t)lens[i] + 1, lim)) return MSA_ENOMEM;
    q.ncell *= (int64_t)lens[i] + 1;
    if (!mul_ok(a, 2 * (int64_t)lens[i] + 1, lim)) return MSA_ENOMEM;
    a *= 2 * (int64_t)lens[i] + 1;
    q.total_len += lens[i];
  }
  q.nu = a - q.ncell;
  q.ntiles = 1;
  for (int i = k - 1; i >= 0; --i) {
    q.tstride[i] = (int32_t)q.ntiles;
    if (!mul_ok(q.ntiles, q.P[i], kMaxTiles)) return MSA_ENOMEM;
    q.ntiles *= q.P[i];
  }
  q.nwaves = 1 - k;
  for (int i = 0; i < k; ++i) q.nwaves += q.P[i];
  // tiles per wave: coefficients of prod_i (1 + x + ... + x^(P_i - 1))
  {
    std::vector<int64_t> cnt(q.nwaves + 1, 0), nxt(q.nwaves + 1, 0);
    cnt[0] = 1;
    int top = 0;
    for (int i = 0; i < k; ++i) {
      std::fill(nxt.begin(), nxt.end(), 0);
      int64_t run = 0;  // sliding window sum of cnt[w - P_i + 1 .. w]
      for (int w = 0; w <= top + q.P[i] - 1; ++w) {
        if (w <= top) run += cnt[w];
        if (w - q.P[i] >= 0) run -= cnt[w - q.P[i]];
        nxt[w] = run;
      }
      top += q.P[i] - 1;
      std::swap(cnt, nxt);
    }
    q.max_wave = *std::max_element(cnt.begin(), cnt.end());
  }
  const int64_t nc = ipow(q.T, k);
  q.dbs = (int32_t)((nc + 15) / 16 * 16);
  // face planes: dimension i keeps P_i - 1 planes over the other dimensions
  q.face_elems = 0;
  for (int i = 0; i < k; ++i) {
    int64_t plane = 1;
    for (int j = k - 1; j >= 0; --j) {
      if (j == i) continue;
      // the kernels form face addresses from 32-bit byte strides (a stride
      // of 2^30 words needs a face plane of at least 2^31 words, 8 GiB)
      if (plane >= ((int64_t)1 << 30)) return MSA_ENOMEM;
      q.fstride[i][j] = plane;
      if (!mul_ok(plane, (int64_t)q.n[j] + 1, lim)) return MSA_ENOMEM;
      plane *= (int64_t)q.n[j] + 1;
    }
    q.fplane[i] = plane;
    q.face_off[i] = q.face_elems;
    if (!mul_ok(plane, (int64_t)q.P[i] - 1, lim)) return MSA_ENOMEM;
    q.face_elems += plane * (q.P[i] - 1);
  }
  // workspace layout
  int64_t o = 0;
  q.off_ctrl = o;   o = align256(o + (int64_t)sizeof(Ctrl));
  q.off_sub = o;    o = align256(o + kSubBytes);
  q.off_order = o;  o = align256(o + q.ntiles * 4);
  q.ncols = q.ntiles / q.P[0];
  q.off_corder = o; o = align256(o + q.ncols * 4);
  q.off_flags = o;  o = align256(o + q.ntiles * 4);
  q.off_path = o;   o = align256(o + std::max<int64_t>(q.total_len, 1));
  q.off_faces = o;
  if (!mul_ok(q.face_elems, 4, lim)) return MSA_ENOMEM;
  // at least one block, so a clamped (unconditional) read at offset 0 is in range
  o = align256(o + std::max<int64_t>(q.face_elems * 4, 256));
  q.off_dir = o;
  if (!mul_ok(q.ntiles, q.dbs, lim)) return MSA_ENOMEM;
  o = align256(o + q.ntiles * q.dbs);
  q.prunable = k >= kPruneMinK && k <= kPruneMaxK;
  for (int i = 0; i < k; ++i) q.prunable = q.prunable && q.n[i] < kPruneMaxLen;
  if (q.prunable) {
    int64_t tab = 0, bm = 0;
    for (int i = 0; i < k; ++i)
      for (int j = i + 1; j < k; ++j) {
        const int p = q.npairs++;
        q.pi[p] = i;
        q.pj[p] = j;
        q.tab_off[p] = tab;
        tab += 2 * ((int64_t)q.n[i] + 1) * ((int64_t)q.n[j] + 1);
        q.bm_off[p] = bm;
        bm += (int64_t)q.P[i] * q.P[j];
      }
    q.nblocks = (int32_t)((q.ntiles + kSelBlock - 1) / kSelBlock);
    q.off_ptab = o;   o = align256(o + tab * 4);
    q.off_pbm = o;    o = align256(o + bm * 4);
    q.off_keep = o;   o = align256(o + q.ntiles);
    q.off_korder = o; o = align256(o + q.ntiles * 4);
    q.off_bcnt = o;   o = align256(o + (int64_t)q.nblocks * 4);
  }
  if (k == 3) {
    q.sw_nb0 = (q.n[0] + 1 + kSwRows - 1) / kSwRows;
    q.sw_nb1 = (q.n[1] + 1 + kSwLanes - 1) / kSwLanes;
    q.x0_plane = ((int64_t)q.n[1] + q.n[2] + 1) * ((int64_t)q.n[1] + 1);
    q.x1_plane = ((int64_t)q.n[0] + 1) * ((int64_t)q.n[2] + kSwNW);  // X1[e = v2 + w][v0]
    q.off_x0 = o;
    o = align256(o + std::max<int64_t>((q.sw_nb0 - 1) * q.x0_plane * 4, 256));
    q.off_x1 = o;
    o = align256(o + std::max<int64_t>((q.sw_nb1 - 1) * q.x1_plane * 4, 256));
    q.x_bytes = o - q.off_x0;
  }
  q.bytes = o;
  *p = q;
  return MSA_OK;
}

// The streaming k = 3 fill covers the plain and the end-gap-free modes.
bool sweep3_eligible(const Plan &p, int alpha, int32_t flags) {
  // the loader keeps each exchange element's offset within its window of
  // n2 + 1 steps as 32 bits: n2 steps of n1 + 1 (X0) or n0 + 1 (X1) words
  const int64_t wmax = (int64_t)p.n[2] * ((int64_t)std::max(p.n[0], p.n[1]) + 1);
  return p.k == 3 && (flags & ~kEndGapsFree) == 0 && alpha >= 1 && alpha <= kSwSubMax &&
         p.n[2] <= kSwSeqMax && wmax < ((int64_t)1 << 31);
}

void make_tile_order(const Plan &p, std::vector<int32_t> *order) {
  std::vector<int64_t> count(p.nwaves + 1, 0);
  auto wave = [&](int64_t t) {
    int s = 0;
    for (int i = 0; i < p.k; ++i) s += (int)((t / p.tstride[i]) % p.P[i]);
    return s;
  };
  for (int64_t t = 0; t < p.ntiles; ++t) count[wave(t) + 1]++;
  for (int w = 0; w < p.nwaves; ++w) count[w + 1] += count[w];
  order->assign(p.ntiles, 0);
  for (int64_t t = 0; t < p.ntiles; ++t) (*order)[count[wave(t)]++] = (int32_t)t;
}

void make_column_order(const Plan &p, std::vector<int32_t> *order) {
  std::vector<int32_t> all;
  make_tile_order(p, &all);
  order->clear();
  order->reserve(p.ncols);
  for (int32_t t : all)
    if (t / p.tstride[0] == 0) order->push_back(t);  // c_0 = 0: first tile of a column
}

int score_bounds(const int32_t *lens, int32_t k, const int8_t *submat, int32_t alpha,
                 int32_t gap, int64_t *lo, int64_t *hi) {
  if (!lens || !submat || !lo || !hi || k < 2 || k > kMaxK || alpha < 1 || alpha > 255)
    return MSA_EINVAL;
  int64_t sum = 0;
  for (int i = 0; i < k; ++i) {
    if (lens[i] < 0) return MSA_EINVAL;
    sum += lens[i];
  }
  int smax = -128, sabs = 0;
  for (int i = 0; i < alpha * alpha; ++i) {
    smax = std::max<int>(smax, submat[i]);
    sabs = std::max<int>(sabs, submat[i] < 0 ? -submat[i] : submat[i]);
  }
  if (gap <= 0) {
    *lo = (int64_t)gap * (k - 1) * sum;
    int64_t pairs = 0;
    for (int i = 0; i < k; ++i)
      for (int j = i + 1; j < k; ++j) pairs += std::min(lens[i], lens[j]);
    *hi = (int64_t)std::max(0, smax) * pairs;
  } else {
    const int64_t m = std::max<int64_t>(gap, sabs);
    *hi = sum * (int64_t)(k * (k - 1) / 2) * m;
    *lo = -*hi;
  }
  return MSA_OK;
}

int check_scoring(const int32_t *lens, int32_t k, const int8_t *submat, int32_t alpha,
                  int32_t gap) {
  if (!submat || alpha < 1 || alpha > 255) return MSA_EINVAL;
  for (int a = 0; a < alpha; ++a)
    for (int b = a + 1; b < alpha; ++b)
      if (submat[a * alpha + b] != submat[b * alpha + a]) return MSA_EINVAL;
  int64_t lo = 0, hi = 0;
  int rc = score_bounds(lens, k, submat, alpha, gap, &lo, &hi);
  if (rc) return rc;
  // largest |column score|: C(k,2) * max(|gap|, max|sub|)
  int sabs = 0;
  for (int i = 0; i < alpha * alpha; ++i)
    sabs = std::max<int>(sabs, submat[i] < 0 ? -submat[i] : submat[i]);
  const int64_t g = gap < 0 ? -(int64_t)gap : gap;
  const int64_t colmax = (int64_t)(k * (k - 1) / 2) * std::max<int64_t>(g, sabs);
  const int64_t span = (lo < 0 ? -lo : lo) + (hi < 0 ? -hi : hi) + 2 * colmax + 1;
  // keys are score * 2^k; the -infinity key is -2^30 (see kNegKey)
  if (span > (((int64_t)1 << 30) >> k)) return MSA_ERANGE;
  return MSA_OK;
}

int check_scoring_mode(const int32_t *lens, int32_t k, const int8_t *submat, int32_t alpha,
                       int32_t gap, uint32_t flags) {
  int rc = check_scoring(lens, k, submat, alpha, gap);
  if (rc || !(flags & kPrune)) return rc;
  // Pruned mode: a kept tile whose lower neighbours were pruned starts from
  // -infinity halo keys, and such values can travel along a monotone path of
  // up to sum(n_i) cells through kept tiles, each step adding one column score
  // (|column score| <= colmax).  They must stay below every real key (real
  // scores are >= lo) and above the int32 minimum:
  //   -2^30 + 2^k * sum(n) * colmax < 2^k * (lo - 1)
  //   -2^30 - 2^k * sum(n) * colmax >= -2^31.
  int64_t lo = 0, hi = 0;
  rc = score_bounds(lens, k, submat, alpha, gap, &lo, &hi);
  if (rc) return rc;
  int64_t sum = 0;
  for (int i = 0; i < k; ++i) sum += lens[i];
  int sabs = 0;
  for (int i = 0; i < alpha * alpha; ++i)
    sabs = std::max<int>(sabs, submat[i] < 0 ? -submat[i] : submat[i]);
  const int64_t g = gap < 0 ? -(int64_t)gap : gap;
  const int64_t colmax = (int64_t)(k * (k - 1) / 2) * std::max<int64_t>(g, sabs);
  const int64_t chain = sum * colmax;
  const int64_t need = chain + (lo < 0 ? -lo : lo) + 1;
  if (need >= (((int64_t)1 << 30) >> k)) return MSA_ERANGE;
  return MSA_OK;
}

int64_t nearopt_bytes(const Plan &p) { return align256(p.ntiles * (int64_t)p.dbs * 4); }

// Unsigned division of any 32-bit n by an invariant d >= 1 as
// q = (t + ((n - t) >> s1)) >> s2 with t = mulhi(m, n), after Granlund and
// Montgomery, "Division by invariant integers using multiplication" (1994):
// l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1, s1 = min(l, 1),
// s2 = max(l - 1, 0).  The kernels use it for tile coordinates, which then
// take scalar instructions instead of a division on the vector unit.
void udiv_magic(uint32_t d, uint32_t *m, uint32_t *sh) {
  int l = 0;
  while (l < 32 && ((uint64_t)1 << l) < d) ++l;
  *m = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
  *sh = (uint32_t)std::min(l, 1) | ((uint32_t)std::max(l - 1, 0) << 8);
}

uint32_t udiv_apply(uint32_t n, uint32_t m, uint32_t sh) {
  const uint32_t t = (uint32_t)(((uint64_t)m * n) >> 32);
  return (t + ((n - t) >> (sh & 0xff))) >> (sh >> 8);
}

void fill_jobdev(const Plan &p, char *ws, int alpha, int gap, JobDev *jd) {
  memset(jd, 0, sizeof(*jd));
  jd->k = p.k;
  jd->T = p.T;
  jd->alpha = alpha;
  jd->gap = gap;
  int32_t off = 0;
  for (int i = 0; i < p.k; ++i) {
    jd->n[i] = p.n[i];
    jd->P[i] = p.P[i];
    jd->tstride[i] = p.tstride[i];
    udiv_magic((uint32_t)p.tstride[i], &jd->tdm[i], &jd->tdsh[i]);
    jd->seq_off[i] = off;
    off += p.n[i];
    jd->face_off[i] = p.face_off[i];
    jd->fplane[i] = p.fplane[i];
    for (int j = 0; j < p.k; ++j) jd->fbstride[i][j] = (uint32_t)(4 * p.fstride[i][j]);
  }
  jd->ntiles = (int32_t)p.ntiles;
  jd->nwaves = p.nwaves;
  jd->dbs = p.dbs;
  jd->total_len = p.total_len;
  jd->sub = reinterpret_cast<const int8_t *>(ws + p.off_sub);
  jd->faces = reinterpret_cast<int32_t *>(ws + p.off_faces);
  jd->dir = reinterpret_cast<uint8_t *>(ws + p.off_dir);
  jd->flags = reinterpret_cast<int32_t *>(ws + p.off_flags);
  jd->corder = reinterpret_cast<const int32_t *>(ws + p.off_corder);
  jd->ncols = (int32_t)p.ncols;
  jd->path = reinterpret_cast<uint8_t *>(ws + p.off_path);
  jd->scores = ws ? reinterpret_cast<int32_t *>(ws + p.bytes) : nullptr;
}

}  // namespace msa

namespace msa {

void fill_prunedev(const Plan &p, char *ws, const uint8_t *d_seqs, int64_t *d_score,
                   PruneDev *pd) {
  memset(pd, 0, sizeof(*pd));
  pd->k = p.k;
  pd->npairs = p.npairs;
  pd->T = p.T;
  pd->ntiles = (int32_t)p.ntiles;
  int32_t off = 0;
  for (int i = 0; i < p.k; ++i) {
    pd->n[i] = p.n[i];
    pd->P[i] = p.P[i];
    pd->tstride[i] = p.tstride[i];
    pd->seq_off[i] = off;
    off += p.n[i];
  }
  for (int q = 0; q < p.npairs; ++q) {
    pd->pi[q] = p.pi[q];
    pd->pj[q] = p.pj[q];
    pd->tab_off[q] = p.tab_off[q];
    pd->bm_off[q] = p.bm_off[q];
  }
  pd->nblocks = p.nblocks;
  pd->seqs = d_seqs;
  pd->sub = reinterpret_cast<const int8_t *>(ws + p.off_sub);
  pd->tabs = reinterpret_cast<int32_t *>(ws + p.off_ptab);
  pd->bm = reinterpret_cast<int32_t *>(ws + p.off_pbm);
  pd->keep = reinterpret_cast<uint8_t *>(ws + p.off_keep);
  pd->order = reinterpret_cast<const int32_t *>(ws + p.off_order);
  pd->korder = reinterpret_cast<int32_t *>(ws + p.off_korder);
  pd->bcnt = reinterpret_cast<int32_t *>(ws + p.off_bcnt);
  pd->score = d_score;
}

}  // namespace msa
