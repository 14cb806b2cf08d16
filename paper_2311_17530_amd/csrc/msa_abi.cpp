// msa_abi.cpp -- C ABI of the library: plain (host and device buffer) paths,
// host-side helpers.  The batched and served paths live in msa_batch.cpp.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/msa_dp.h"
#include "msa_plan.h"
#include "msa_runtime.h"

using namespace msa;

extern "C" const char *msa_strerror(int status) {
  switch (status) {
    case MSA_OK: return "ok";
    case MSA_EINVAL: return "invalid argument";
    case MSA_ERANGE: return "score range exceeds the device integer width";
    case MSA_ENOMEM: return "workspace exceeds the device memory or the budget";
    case MSA_EDEVICE: return "device error or watchdog timeout";
    case MSA_EAGAIN: return "result not ready";
    case MSA_ESHUTDOWN: return "server is shutting down";
    default: return "unknown status";
  }
}

extern "C" int msa_dp_score_bounds(const int32_t *lens, int32_t k, const int8_t *submat,
                                   int32_t alpha, int32_t gap, int64_t *lo, int64_t *hi) {
  return score_bounds(lens, k, submat, alpha, gap, lo, hi);
}

extern "C" int32_t msa_dp_tile_edge(int32_t k) {
  if (k < 2 || k > MSA_MAX_K) return MSA_EINVAL;
  return tile_edge_for_k(k);
}

extern "C" int32_t msa_dp_tile_grid(const int32_t *lens, int32_t k, int32_t tile_edge,
                                    int32_t *tiles_per_dim) {
  if (!lens || !tiles_per_dim || k < 2 || k > MSA_MAX_K || tile_edge < 1) return MSA_EINVAL;
  int32_t waves = 1 - k;
  for (int i = 0; i < k; ++i) {
    if (lens[i] < 0) return MSA_EINVAL;
    tiles_per_dim[i] = 1 + (lens[i] + tile_edge - 1) / tile_edge;
    waves += tiles_per_dim[i];
  }
  return waves;
}

extern "C" int32_t msa_dp_wave_counts(const int32_t *p, int32_t k, int64_t *counts,
                                      int32_t cap) {
  if (!p || !counts || k < 1 || k > MSA_MAX_K) return MSA_EINVAL;
  int32_t waves = 1 - k;
  for (int i = 0; i < k; ++i) {
    if (p[i] < 1) return MSA_EINVAL;
    waves += p[i];
  }
  if (cap < waves) return MSA_EINVAL;
  // polynomial product  prod_i (1 + x + ... + x^{p_i - 1}): coefficient w
  // counts the tiles whose coordinates sum to w
  std::vector<int64_t> poly(1, 1);
  for (int i = 0; i < k; ++i) {
    std::vector<int64_t> nxt(poly.size() + p[i] - 1, 0);
    for (size_t a = 0; a < poly.size(); ++a)
      for (int b = 0; b < p[i]; ++b) nxt[a + b] += poly[a];
    poly.swap(nxt);
  }
  for (int32_t w = 0; w < waves; ++w) counts[w] = poly[w];
  return waves;
}

static int validate_shape(const int32_t *lens, int32_t k) {
  if (!lens || k < 2 || k > MSA_MAX_K) return MSA_EINVAL;
  for (int i = 0; i < k; ++i)
    if (lens[i] < 0) return MSA_EINVAL;
  return MSA_OK;
}

extern "C" int64_t msa_dp_workspace_bytes(const int32_t *lens, int32_t k) {
  int rc = validate_shape(lens, k);
  if (rc) return rc;
  Plan p;
  rc = make_plan(lens, k, &p);
  if (rc) return rc;
  return p.bytes;
}

// Mode flags.  The end-gap-free end-cell key holds the row-major cell index
// in 32 bits; a co-optimal tie set fits a byte for k <= 3 and its walk keeps
// one mask per column on chip.
// The pruned mode needs 3 <= k <= 6 and lengths below kPruneMaxLen (its
// pairwise bounds assume the global alignment's start and end).
static int check_flags(const Plan &p, uint32_t flags) {
  if (flags & ~(uint32_t)(MSA_END_GAPS_FREE | MSA_COOPTIMAL | MSA_PRUNE | MSA_NEAROPT))
    return MSA_EINVAL;
  if (flags & MSA_NEAROPT) {  // a mode of its own: the plain fill plus cell scores
    if (flags != MSA_NEAROPT || p.k > kNoMaxK) return MSA_EINVAL;
    if (p.total_len > kNoMaxTotal) return MSA_ERANGE;
  }
  if ((flags & MSA_END_GAPS_FREE) && (flags & (MSA_COOPTIMAL | MSA_PRUNE))) return MSA_EINVAL;
  if (flags & MSA_PRUNE) {
    if (p.k < kPruneMinK || p.k > kPruneMaxK) return MSA_EINVAL;
    if (!p.prunable) return MSA_ERANGE;
  }
  if ((flags & MSA_END_GAPS_FREE) && p.ncell > ((int64_t)1 << 32)) return MSA_ERANGE;
  if (flags & MSA_COOPTIMAL) {
    if (p.k > kCoMaxK) return MSA_EINVAL;
    if (p.total_len > kCoMaxTotal) return MSA_ERANGE;
  }
  return MSA_OK;
}

// Workspace bytes for a mode: the near-optimal mode's cell scores follow
// the plain layout.
static int64_t ws_need(const Plan &p, uint32_t flags) {
  return p.bytes + ((flags & MSA_NEAROPT) ? nearopt_bytes(p) : 0);
}

extern "C" int64_t msa_dp_workspace_bytes_ex(const int32_t *lens, int32_t k, uint32_t flags) {
  int rc = validate_shape(lens, k);
  if (rc) return rc;
  Plan p;
  rc = make_plan(lens, k, &p);
  if (rc) return rc;
  rc = check_flags(p, flags);
  if (rc) return rc;
  return ws_need(p, flags);
}

extern "C" int msa_dp_check_scoring(const int32_t *lens, int32_t k, const int8_t *submat,
                                    int32_t alpha, int32_t gap, uint32_t flags) {
  int rc = validate_shape(lens, k);
  if (rc) return rc;
  Plan p;
  rc = make_plan(lens, k, &p);
  if (rc) return rc;
  rc = check_flags(p, flags);
  if (rc) return rc;
  return check_scoring_mode(lens, k, submat, alpha, gap, flags);
}

extern "C" int msa_dp_prepare_ex(void *d_workspace, int64_t ws_bytes, const int32_t *lens,
                                 int32_t k, const int8_t *submat, int32_t alpha, int32_t gap,
                                 uint32_t flags, void *hip_stream) {
  int rc = validate_shape(lens, k);
  if (rc) return rc;
  if (!d_workspace || ((uintptr_t)d_workspace & 255)) return MSA_EINVAL;
  Plan p;
  rc = make_plan(lens, k, &p);
  if (rc) return rc;
  rc = check_flags(p, flags);
  if (rc) return rc;
  rc = check_scoring_mode(lens, k, submat, alpha, gap, flags);
  if (rc) return rc;
  if (ws_bytes < ws_need(p, flags)) return MSA_EINVAL;
  return prepare_workspace(p, (char *)d_workspace, submat, alpha, gap, (int32_t)flags,
                           (hipStream_t)hip_stream);
}

extern "C" int msa_dp_prepare(void *d_workspace, int64_t ws_bytes, const int32_t *lens,
                              int32_t k, const int8_t *submat, int32_t alpha, int32_t gap,
                              void *hip_stream) {
  return msa_dp_prepare_ex(d_workspace, ws_bytes, lens, k, submat, alpha, gap, 0u, hip_stream);
}

extern "C" int msa_dp_align_dev(void *d_workspace, int64_t ws_bytes, const uint8_t *d_seqs,
                                const int32_t *lens, int32_t k, int64_t *d_score,
                                uint8_t *d_aln, int64_t aln_cap, int64_t *d_aln_len,
                                int32_t *d_status, void *hip_stream) {
  int rc = validate_shape(lens, k);
  if (rc) return rc;
  if (!d_workspace || ((uintptr_t)d_workspace & 255) || !d_score || !d_aln_len || !d_status)
    return MSA_EINVAL;
  Plan p;
  rc = make_plan(lens, k, &p);
  if (rc) return rc;
  if (ws_bytes < p.bytes || aln_cap < p.total_len || (p.total_len > 0 && !d_aln) ||
      (p.total_len > 0 && !d_seqs))
    return MSA_EINVAL;
  return run_plain(p, (char *)d_workspace, d_seqs, d_score, d_aln, aln_cap, d_aln_len,
                   d_status, (hipStream_t)hip_stream);
}

extern "C" int msa_dp_fill_dev(void *d_workspace, int64_t ws_bytes, const uint8_t *d_seqs,
                               const int32_t *lens, int32_t k, int64_t *d_score,
                               void *hip_stream) {
  int rc = validate_shape(lens, k);
  if (rc) return rc;
  if (!d_workspace || ((uintptr_t)d_workspace & 255) || !d_score) return MSA_EINVAL;
  Plan p;
  rc = make_plan(lens, k, &p);
  if (rc) return rc;
  if (ws_bytes < p.bytes || (p.total_len > 0 && !d_seqs)) return MSA_EINVAL;
  return run_plain(p, (char *)d_workspace, d_seqs, d_score, nullptr, 0, nullptr, nullptr,
                   (hipStream_t)hip_stream, 1);
}

extern "C" int msa_dp_traceback_dev(void *d_workspace, int64_t ws_bytes, const uint8_t *d_seqs,
                                    const int32_t *lens, int32_t k, int64_t *d_score,
                                    uint8_t *d_aln, int64_t aln_cap, int64_t *d_aln_len,
                                    int32_t *d_status, void *hip_stream) {
  int rc = validate_shape(lens, k);
  if (rc) return rc;
  if (!d_workspace || ((uintptr_t)d_workspace & 255) || !d_score || !d_aln_len || !d_status)
    return MSA_EINVAL;
  Plan p;
  rc = make_plan(lens, k, &p);
  if (rc) return rc;
  if (ws_bytes < p.bytes || aln_cap < p.total_len || (p.total_len > 0 && !d_aln) ||
      (p.total_len > 0 && !d_seqs))
    return MSA_EINVAL;
  return run_plain(p, (char *)d_workspace, d_seqs, d_score, d_aln, aln_cap, d_aln_len,
                   d_status, (hipStream_t)hip_stream, 2);
}

extern "C" int msa_dp_export_dirs(void *d_workspace, int64_t ws_bytes, const int32_t *lens,
                                  int32_t k, uint8_t *d_dir_out, void *hip_stream) {
  int rc = validate_shape(lens, k);
  if (rc) return rc;
  if (!d_workspace || !d_dir_out) return MSA_EINVAL;
  Plan p;
  rc = make_plan(lens, k, &p);
  if (rc) return rc;
  if (ws_bytes < p.bytes) return MSA_EINVAL;
  return export_dirs(p, (char *)d_workspace, d_dir_out, (hipStream_t)hip_stream);
}

extern "C" int msa_dp_export_prune(void *d_workspace, int64_t ws_bytes, const int32_t *lens,
                                   int32_t k, uint8_t *d_keep_out, int64_t *d_info_out,
                                   void *hip_stream) {
  int rc = validate_shape(lens, k);
  if (rc) return rc;
  if (!d_workspace || (!d_keep_out && !d_info_out)) return MSA_EINVAL;
  Plan p;
  rc = make_plan(lens, k, &p);
  if (rc) return rc;
  if (ws_bytes < p.bytes) return MSA_EINVAL;
  return export_prune(p, (char *)d_workspace, d_keep_out, d_info_out, (hipStream_t)hip_stream);
}

extern "C" int msa_dp_coopt_dev(void *d_workspace, int64_t ws_bytes, const uint8_t *d_seqs,
                                const int32_t *lens, int32_t k, int32_t max_paths,
                                int64_t *d_score, uint8_t *d_aln, int64_t aln_cap,
                                int64_t *d_aln_len, int32_t *d_npaths, int32_t *d_status,
                                void *hip_stream) {
  int rc = validate_shape(lens, k);
  if (rc) return rc;
  if (!d_workspace || ((uintptr_t)d_workspace & 255) || !d_score || !d_aln_len || !d_npaths ||
      !d_status || !d_aln || max_paths < 1)
    return MSA_EINVAL;
  Plan p;
  rc = make_plan(lens, k, &p);
  if (rc) return rc;
  rc = check_flags(p, MSA_COOPTIMAL);
  if (rc) return rc;
  if (ws_bytes < p.bytes || aln_cap < p.total_len || (p.total_len > 0 && !d_seqs))
    return MSA_EINVAL;
  return run_coopt(p, (char *)d_workspace, d_seqs, max_paths, d_score, d_aln, aln_cap,
                   d_aln_len, d_npaths, d_status, (hipStream_t)hip_stream);
}

extern "C" int msa_dp_nearopt_dev(void *d_workspace, int64_t ws_bytes, const uint8_t *d_seqs,
                                  const int32_t *lens, int32_t k, int64_t delta,
                                  int32_t max_paths, int64_t *d_score, int64_t *d_scores,
                                  uint8_t *d_aln, int64_t aln_cap, int64_t *d_aln_len,
                                  int32_t *d_npaths, int32_t *d_status, void *hip_stream) {
  int rc = validate_shape(lens, k);
  if (rc) return rc;
  if (!d_workspace || ((uintptr_t)d_workspace & 255) || !d_score || !d_scores || !d_aln_len ||
      !d_npaths || !d_status || !d_aln || max_paths < 1 || delta < 0)
    return MSA_EINVAL;
  Plan p;
  rc = make_plan(lens, k, &p);
  if (rc) return rc;
  rc = check_flags(p, MSA_NEAROPT);
  if (rc) return rc;
  if (ws_bytes < ws_need(p, MSA_NEAROPT) || aln_cap < p.total_len ||
      (p.total_len > 0 && !d_seqs))
    return MSA_EINVAL;
  return run_nearopt(p, (char *)d_workspace, d_seqs, delta, max_paths, d_score, d_scores, d_aln,
                     aln_cap, d_aln_len, d_npaths, d_status, (hipStream_t)hip_stream);
}

// ---------------------------------------------------------------------------
// Host-buffer convenience path: a per-thread cache of device buffers.
// ---------------------------------------------------------------------------
namespace {
struct HostCache {
  int device = -1;
  void *ws = nullptr;
  int64_t ws_bytes = 0;
  uint8_t *io = nullptr;  // seqs | aln | score | len | status
  int64_t io_bytes = 0;
  // signature of the prepared workspace
  int32_t k = 0, lens[MSA_MAX_K] = {}, alpha = 0, gap = 0;
  uint32_t flags = 0;
  std::vector<int8_t> sub;
  hipStream_t stream = nullptr;
  ~HostCache() {
    // process exit: the runtime may already be torn down; leak rather than fault
  }
};
thread_local HostCache g_cache;
}  // namespace

// Validates a host-buffer call and readies the per-thread cache: a workspace
// prepared for (lens, scoring, flags), `io_need` bytes of device I/O buffers,
// and the sequences copied to the start of the I/O buffer (enqueued).
static int host_call_setup(const uint8_t *const *seqs, const int32_t *lens, int32_t k,
                           const int8_t *submat, int32_t alpha, int32_t gap, uint32_t flags,
                           const Plan &p, int64_t io_need) {
  const int64_t wsb = ws_need(p, flags);
  for (int i = 0; i < k; ++i)
    if (lens[i] > 0 && !seqs[i]) return MSA_EINVAL;
  for (int i = 0; i < k; ++i)
    for (int32_t t = 0; t < lens[i]; ++t)
      if (seqs[i][t] >= alpha) return MSA_EINVAL;
  int rc = check_scoring_mode(lens, k, submat, alpha, gap, flags);
  if (rc) return rc;

  HostCache &c = g_cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MSA_EDEVICE;
  if (c.device != dev) {
    c = HostCache();
    c.device = dev;
    if (hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking) != hipSuccess)
      return MSA_EDEVICE;
  }
  if (c.ws_bytes < wsb) {
    if (c.ws) (void)hipFree(c.ws);
    c.ws = nullptr;
    c.ws_bytes = 0;
    c.k = 0;
    if (hipMalloc(&c.ws, wsb) != hipSuccess) {
      c.ws = nullptr;
      return MSA_ENOMEM;
    }
    c.ws_bytes = wsb;
  }
  if (c.io_bytes < io_need) {
    if (c.io) (void)hipFree(c.io);
    c.io = nullptr;
    c.io_bytes = 0;
    if (hipMalloc(&c.io, io_need) != hipSuccess) {
      c.io = nullptr;
      return MSA_ENOMEM;
    }
    c.io_bytes = io_need;
  }
  bool same = c.k == k && c.alpha == alpha && c.gap == gap && c.flags == flags &&
              (int64_t)c.sub.size() == (int64_t)alpha * alpha &&
              memcmp(c.sub.data(), submat, (size_t)alpha * alpha) == 0;
  for (int i = 0; same && i < k; ++i) same = c.lens[i] == lens[i];
  if (!same) {
    rc = prepare_workspace(p, (char *)c.ws, submat, alpha, gap, (int32_t)flags, c.stream);
    if (rc) {
      c.k = 0;
      return rc;
    }
    c.k = k;
    c.alpha = alpha;
    c.gap = gap;
    c.flags = flags;
    for (int i = 0; i < k; ++i) c.lens[i] = lens[i];
    c.sub.assign(submat, submat + (size_t)alpha * alpha);
  }
  int64_t off = 0;
  for (int i = 0; i < k; ++i) {
    if (lens[i] > 0 &&
        hipMemcpyAsync(c.io + off, seqs[i], lens[i], hipMemcpyHostToDevice, c.stream) !=
            hipSuccess)
      return MSA_EDEVICE;
    off += lens[i];
  }
  return MSA_OK;
}

extern "C" int msa_dp_align_ex(const uint8_t *const *seqs, const int32_t *lens, int32_t k,
                               const int8_t *submat, int32_t alpha, int32_t gap, uint32_t flags,
                               int64_t *score_out, uint8_t *aln_out, int64_t aln_cap,
                               int64_t *aln_len_out) {
  int rc = validate_shape(lens, k);
  if (rc) return rc;
  if (!seqs || !score_out || !aln_len_out) return MSA_EINVAL;
  Plan p;
  rc = make_plan(lens, k, &p);
  if (rc) return rc;
  rc = check_flags(p, flags);
  if (rc) return rc;
  if (aln_cap < p.total_len || (p.total_len > 0 && !aln_out)) return MSA_EINVAL;
  const int64_t io_need = ((p.total_len + 255) & ~255LL) + k * ((aln_cap + 255) & ~255LL) + 256;
  rc = host_call_setup(seqs, lens, k, submat, alpha, gap, flags, p, io_need);
  if (rc) return rc;
  HostCache &c = g_cache;
  uint8_t *d_seqs = c.io;
  uint8_t *d_aln = d_seqs + ((p.total_len + 255) & ~255LL);
  int64_t *d_misc = (int64_t *)(d_aln + k * ((aln_cap + 255) & ~255LL));
  rc = run_plain(p, (char *)c.ws, d_seqs, d_misc, d_aln, aln_cap, d_misc + 1,
                 (int32_t *)(d_misc + 2), c.stream);
  if (rc) return rc;
  int64_t misc[3] = {0, 0, 0};
  if (hipMemcpyAsync(misc, d_misc, sizeof(misc), hipMemcpyDeviceToHost, c.stream) !=
      hipSuccess)
    return MSA_EDEVICE;
  if (hipStreamSynchronize(c.stream) != hipSuccess) return MSA_EDEVICE;
  const int32_t st = (int32_t)(misc[2] & 0xffffffff);
  if (st != MSA_OK) return st;
  const int64_t L = misc[1];
  if (L > 0) {
    if (hipMemcpy2DAsync(aln_out, aln_cap, d_aln, aln_cap, L, k, hipMemcpyDeviceToHost,
                         c.stream) != hipSuccess)
      return MSA_EDEVICE;
    if (hipStreamSynchronize(c.stream) != hipSuccess) return MSA_EDEVICE;
  }
  *score_out = misc[0];
  *aln_len_out = L;
  return MSA_OK;
}

extern "C" int msa_dp_align(const uint8_t *const *seqs, const int32_t *lens, int32_t k,
                            const int8_t *submat, int32_t alpha, int32_t gap,
                            int64_t *score_out, uint8_t *aln_out, int64_t aln_cap,
                            int64_t *aln_len_out) {
  return msa_dp_align_ex(seqs, lens, k, submat, alpha, gap, 0u, score_out, aln_out, aln_cap,
                         aln_len_out);
}

extern "C" int msa_dp_align_coopt(const uint8_t *const *seqs, const int32_t *lens, int32_t k,
                                  const int8_t *submat, int32_t alpha, int32_t gap,
                                  int32_t max_paths, int64_t *score_out, uint8_t *aln_out,
                                  int64_t aln_cap, int64_t *aln_len_out, int32_t *npaths_out) {
  int rc = validate_shape(lens, k);
  if (rc) return rc;
  if (k > kCoMaxK && k <= kNoMaxK) {
    // tie sets need more than a byte: the near-optimal walk at delta = 0
    // lists the same alignments in the same order
    if (max_paths < 1) return MSA_EINVAL;
    std::vector<int64_t> sc((size_t)max_paths);
    return msa_dp_align_nearopt(seqs, lens, k, submat, alpha, gap, 0, max_paths, score_out,
                                sc.data(), aln_out, aln_cap, aln_len_out, npaths_out);
  }
  if (!seqs || !score_out || !aln_len_out || !npaths_out || !aln_out || max_paths < 1)
    return MSA_EINVAL;
  Plan p;
  rc = make_plan(lens, k, &p);
  if (rc) return rc;
  rc = check_flags(p, MSA_COOPTIMAL);
  if (rc) return rc;
  if (aln_cap < p.total_len) return MSA_EINVAL;
  // device I/O: seqs | max_paths blocks of k rows | lengths | score, npaths, status
  const int64_t seq_b = (p.total_len + 255) & ~255LL;
  const int64_t blk = (int64_t)k * aln_cap;
  if (blk > 0 && max_paths > (INT64_MAX / 4) / blk) return MSA_ENOMEM;
  const int64_t aln_b = ((int64_t)max_paths * blk + 255) & ~255LL;
  const int64_t len_b = ((int64_t)max_paths * 8 + 255) & ~255LL;
  const int64_t io_need = seq_b + aln_b + len_b + 256;
  rc = host_call_setup(seqs, lens, k, submat, alpha, gap, MSA_COOPTIMAL, p, io_need);
  if (rc) return rc;
  HostCache &c = g_cache;
  uint8_t *d_seqs = c.io;
  uint8_t *d_aln = d_seqs + seq_b;
  int64_t *d_len = (int64_t *)(d_aln + aln_b);
  int64_t *d_misc = (int64_t *)((char *)d_len + len_b);  // score | npaths | status
  rc = run_coopt(p, (char *)c.ws, d_seqs, max_paths, d_misc, d_aln, aln_cap, d_len,
                 (int32_t *)(d_misc + 1), (int32_t *)(d_misc + 2), c.stream);
  if (rc) return rc;
  int64_t misc[3] = {0, 0, 0};
  if (hipMemcpyAsync(misc, d_misc, sizeof(misc), hipMemcpyDeviceToHost, c.stream) !=
      hipSuccess)
    return MSA_EDEVICE;
  if (hipStreamSynchronize(c.stream) != hipSuccess) return MSA_EDEVICE;
  const int32_t st = (int32_t)(misc[2] & 0xffffffff);
  if (st != MSA_OK) return st;
  const int32_t np = (int32_t)(misc[1] & 0xffffffff);
  if (np < 1 || np > max_paths) return MSA_EDEVICE;
  if (hipMemcpyAsync(aln_len_out, d_len, (size_t)np * 8, hipMemcpyDeviceToHost, c.stream) !=
          hipSuccess ||
      (blk > 0 && hipMemcpyAsync(aln_out, d_aln, (size_t)(np * blk), hipMemcpyDeviceToHost,
                                 c.stream) != hipSuccess))
    return MSA_EDEVICE;
  if (hipStreamSynchronize(c.stream) != hipSuccess) return MSA_EDEVICE;
  *score_out = misc[0];
  *npaths_out = np;
  return MSA_OK;
}

extern "C" int msa_dp_align_nearopt(const uint8_t *const *seqs, const int32_t *lens, int32_t k,
                                    const int8_t *submat, int32_t alpha, int32_t gap,
                                    int64_t delta, int32_t max_paths, int64_t *score_out,
                                    int64_t *scores_out, uint8_t *aln_out, int64_t aln_cap,
                                    int64_t *aln_len_out, int32_t *npaths_out) {
  int rc = validate_shape(lens, k);
  if (rc) return rc;
  if (!seqs || !score_out || !scores_out || !aln_len_out || !npaths_out || !aln_out ||
      max_paths < 1 || delta < 0)
    return MSA_EINVAL;
  Plan p;
  rc = make_plan(lens, k, &p);
  if (rc) return rc;
  rc = check_flags(p, MSA_NEAROPT);
  if (rc) return rc;
  if (aln_cap < p.total_len) return MSA_EINVAL;
  // device I/O: seqs | max_paths blocks of k rows | lengths | scores | score, npaths, status
  const int64_t seq_b = (p.total_len + 255) & ~255LL;
  const int64_t blk = (int64_t)k * aln_cap;
  if (blk > 0 && max_paths > (INT64_MAX / 4) / blk) return MSA_ENOMEM;
  const int64_t aln_b = ((int64_t)max_paths * blk + 255) & ~255LL;
  const int64_t len_b = ((int64_t)max_paths * 8 + 255) & ~255LL;
  const int64_t io_need = seq_b + aln_b + 2 * len_b + 256;
  rc = host_call_setup(seqs, lens, k, submat, alpha, gap, MSA_NEAROPT, p, io_need);
  if (rc) return rc;
  HostCache &c = g_cache;
  uint8_t *d_seqs = c.io;
  uint8_t *d_aln = d_seqs + seq_b;
  int64_t *d_len = (int64_t *)(d_aln + aln_b);
  int64_t *d_sc = (int64_t *)((char *)d_len + len_b);
  int64_t *d_misc = (int64_t *)((char *)d_sc + len_b);  // score | npaths | status
  rc = run_nearopt(p, (char *)c.ws, d_seqs, delta, max_paths, d_misc, d_sc, d_aln, aln_cap,
                   d_len, (int32_t *)(d_misc + 1), (int32_t *)(d_misc + 2), c.stream);
  if (rc) return rc;
  int64_t misc[3] = {0, 0, 0};
  if (hipMemcpyAsync(misc, d_misc, sizeof(misc), hipMemcpyDeviceToHost, c.stream) !=
      hipSuccess)
    return MSA_EDEVICE;
  if (hipStreamSynchronize(c.stream) != hipSuccess) return MSA_EDEVICE;
  const int32_t st = (int32_t)(misc[2] & 0xffffffff);
  if (st != MSA_OK) return st;
  const int32_t np = (int32_t)(misc[1] & 0xffffffff);
  if (np < 1 || np > max_paths) return MSA_EDEVICE;
  if (hipMemcpyAsync(aln_len_out, d_len, (size_t)np * 8, hipMemcpyDeviceToHost, c.stream) !=
          hipSuccess ||
      hipMemcpyAsync(scores_out, d_sc, (size_t)np * 8, hipMemcpyDeviceToHost, c.stream) !=
          hipSuccess ||
      (blk > 0 && hipMemcpyAsync(aln_out, d_aln, (size_t)(np * blk), hipMemcpyDeviceToHost,
                                 c.stream) != hipSuccess))
    return MSA_EDEVICE;
  if (hipStreamSynchronize(c.stream) != hipSuccess) return MSA_EDEVICE;
  *score_out = misc[0];
  *npaths_out = np;
  return MSA_OK;
}
