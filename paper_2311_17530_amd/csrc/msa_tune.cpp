// msa_tune.cpp -- launch-configuration tuner (see msa_tune.h) and its C ABI:
// a table keyed by (architecture of the current device, kind, k, length
// bucket), filled by measured runs (msa_dp_autotune, msa_dp_autotune_batch)
// or set explicitly (msa_dp_tune_set).
#include "msa_tune.h"

#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/msa_dp.h"
#include "msa_launch.h"
#include "msa_plan.h"
#include "msa_runtime.h"

namespace msa {

namespace {
std::mutex g_tmu;
std::map<std::tuple<std::string, int, int, int>, TuneChoice> g_table;

// "gfx950" from the current device's architecture name (features dropped);
// "none" without a device.
std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "none";
  std::string a(prop.gcnArchName);
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}
}  // namespace

int length_bucket(const int32_t *n, int k) {
  int32_t m = 0;
  for (int i = 0; i < k; ++i) m = std::max(m, n[i]);
  int b = 0;
  while ((int64_t)1 << b < (int64_t)m + 1) ++b;
  return b;
}

bool tune_get(int kind, int k, int bucket, TuneChoice *c) {
  const auto key = std::make_tuple(device_arch(), kind, k, bucket);
  std::lock_guard<std::mutex> lk(g_tmu);
  auto it = g_table.find(key);
  if (it == g_table.end()) return false;
  *c = it->second;
  return true;
}

void tune_set(int kind, int k, int bucket, const TuneChoice &c) {
  const auto key = std::make_tuple(device_arch(), kind, k, bucket);
  std::lock_guard<std::mutex> lk(g_tmu);
  g_table[key] = c;
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_tmu);
  g_table.clear();
}

}  // namespace msa

using namespace msa;

static int tune_key(int32_t kind, int32_t k, int32_t max_len, int *kk, int *bucket) {
  if (kind == kTunePlain) {
    if (k < 2 || k > kMaxK || max_len < 0) return MSA_EINVAL;
    *kk = k;
    *bucket = length_bucket(&max_len, 1);
    return MSA_OK;
  }
  if (kind == kTuneBatch) {
    if (k < 2 || k > kMaxK) return MSA_EINVAL;
    *kk = kclass_of(k);
    *bucket = 0;
    return MSA_OK;
  }
  return MSA_EINVAL;
}

extern "C" int msa_dp_tune_set(int32_t kind, int32_t k, int32_t max_len, int32_t variant,
                               int32_t wpc) {
  int kk = 0, b = 0;
  int rc = tune_key(kind, k, max_len, &kk, &b);
  if (rc) return rc;
  if (variant < 0 || variant > 2 || wpc < 0 || wpc > 64) return MSA_EINVAL;
  if (kind == kTuneBatch && variant != 0) return MSA_EINVAL;
  TuneChoice c;
  c.variant = variant;
  c.wpc = wpc;
  tune_set(kind, kk, b, c);
  return MSA_OK;
}

extern "C" int msa_dp_tune_get(int32_t kind, int32_t k, int32_t max_len, int32_t *choice_out) {
  int kk = 0, b = 0;
  int rc = tune_key(kind, k, max_len, &kk, &b);
  if (rc) return rc;
  if (!choice_out) return MSA_EINVAL;
  TuneChoice c;
  tune_get(kind, kk, b, &c);  // none stored: the built-in rule (0, 0)
  choice_out[0] = c.variant;
  choice_out[1] = c.wpc;
  return MSA_OK;
}

extern "C" void msa_dp_tune_clear(void) { tune_clear(); }

static std::vector<TuneChoice> candidates(int kind, int k, int32_t max_len) {
  std::vector<TuneChoice> cs;
  if (kind == kTunePlain) {
    if (k == 3 && max_len <= kSwSeqMax) cs.push_back(TuneChoice{1, 0});
    const int occ = std::max(fill_occupancy(k), 1);
    for (int w = 1; w <= occ; ++w) cs.push_back(TuneChoice{2, w});
  } else {
    const int occ = std::max(batch_occupancy(kclass_of(k)), 1);
    for (int w = 1; w <= occ; ++w) cs.push_back(TuneChoice{0, w});
  }
  return cs;
}

extern "C" int msa_dp_tune_candidates(int32_t kind, int32_t k, int32_t max_len, int32_t *out,
                                      int32_t cap) {
  int kk = 0, b = 0;
  int rc = tune_key(kind, k, max_len, &kk, &b);
  if (rc) return rc;
  const std::vector<TuneChoice> cs = candidates(kind, k, max_len);
  for (int i = 0; out && i < (int)cs.size() && 2 * i + 1 < cap; ++i) {
    out[2 * i] = cs[i].variant;
    out[2 * i + 1] = cs[i].wpc;
  }
  return (int)cs.size();
}

static float median_of(std::vector<float> v) {
  std::sort(v.begin(), v.end());
  return v.empty() ? 0.f : v[v.size() / 2];
}

extern "C" int msa_dp_autotune(const int32_t *lens, int32_t k, const int8_t *submat,
                               int32_t alpha, int32_t gap, int32_t reps, int32_t *choice_out,
                               float *best_ms_out) {
  if (!lens || !submat || !choice_out || k < 2 || k > kMaxK || reps < 1 || reps > 100)
    return MSA_EINVAL;
  Plan p;
  int rc = make_plan(lens, k, &p);
  if (rc) return rc;
  rc = check_scoring(lens, k, submat, alpha, gap);
  if (rc) return rc;
  int32_t max_len = 0;
  for (int i = 0; i < k; ++i) max_len = std::max(max_len, lens[i]);
  const int bucket = length_bucket(lens, k);
  const std::vector<TuneChoice> cs = candidates(kTunePlain, k, max_len);
  // a workspace of this shape with seeded residues (the fill's time does
  // not depend on their values)
  const int64_t cap = std::max<int64_t>(p.total_len, 1);
  std::vector<uint8_t> seqs((size_t)cap);
  uint32_t x = 12345u;
  for (auto &c : seqs) {
    x = x * 1664525u + 1013904223u;
    c = (uint8_t)((x >> 16) % (uint32_t)alpha);
  }
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  char *ws = nullptr, *io = nullptr;
  const int64_t io_b = cap + (int64_t)k * cap + 256;
  bool ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
            hipMalloc(&ws, p.bytes) == hipSuccess && hipMalloc(&io, io_b) == hipSuccess;
  uint8_t *d_seqs = reinterpret_cast<uint8_t *>(io);
  uint8_t *d_aln = d_seqs + cap;
  int64_t *d_misc = reinterpret_cast<int64_t *>(io + ((cap + (int64_t)k * cap + 7) & ~7LL));
  ok = ok && hipMemcpyAsync(d_seqs, seqs.data(), (size_t)cap, hipMemcpyHostToDevice, s) ==
                 hipSuccess;
  ok = ok && prepare_workspace(p, ws, submat, alpha, gap, 0, s) == MSA_OK;
  float best = 0.f;
  TuneChoice bestc;
  for (size_t ci = 0; ok && ci < cs.size(); ++ci) {
    tune_set(kTunePlain, k, bucket, cs[ci]);
    auto whole = [&](int which) {
      return run_plain(p, ws, d_seqs, d_misc, d_aln, cap, d_misc + 1, (int32_t *)(d_misc + 2), s,
                       which) == MSA_OK;
    };
    ok = whole(3);  // warm-up
    std::vector<float> t;
    for (int r = 0; ok && r < reps; ++r) {
      ok = hipEventRecord(e0, s) == hipSuccess && whole(1) &&
           hipEventRecord(e1, s) == hipSuccess && whole(2) &&
           hipEventSynchronize(e1) == hipSuccess;
      float ms = 0.f;
      ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
      t.push_back(ms);
    }
    const float m = median_of(t);
    if (ok && (ci == 0 || m < best)) {
      best = m;
      bestc = cs[ci];
    }
  }
  if (s) (void)hipStreamSynchronize(s);
  if (ws) {
    forget_workspace(ws);
    (void)hipFree(ws);
  }
  if (io) (void)hipFree(io);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (!ok) {
    tune_set(kTunePlain, k, bucket, TuneChoice{});
    return MSA_EDEVICE;
  }
  tune_set(kTunePlain, k, bucket, bestc);
  choice_out[0] = bestc.variant;
  choice_out[1] = bestc.wpc;
  if (best_ms_out) *best_ms_out = best;
  return MSA_OK;
}

extern "C" int msa_dp_autotune_batch(const msa_job *jobs, int32_t njobs, int32_t reps,
                                     int32_t *wpc_out) {
  if (!jobs || njobs < 1 || !wpc_out || reps < 1 || reps > 100) return MSA_EINVAL;
  for (int i = 0; i < njobs; ++i)
    if (validate_job(jobs[i]) != MSA_OK) return MSA_EINVAL;
  for (int c = 0; c < 4; ++c) wpc_out[c] = 0;
  for (int kc = 0; kc < 4; ++kc) {
    std::vector<msa_job> cls;
    for (int i = 0; i < njobs; ++i)
      if (kclass_of(jobs[i].k) == kc) cls.push_back(jobs[i]);
    if (cls.empty()) continue;
    std::vector<std::vector<uint8_t>> bufs(cls.size());
    std::vector<msa_result> res(cls.size());
    for (size_t i = 0; i < cls.size(); ++i) {
      int64_t total = 0;
      for (int d = 0; d < cls[i].k; ++d) total += cls[i].lens[d];
      const int64_t cap = std::max<int64_t>(total, 1);
      bufs[i].resize((size_t)(cap * cls[i].k));
      memset(&res[i], 0, sizeof(res[i]));
      res[i].aln = bufs[i].data();
      res[i].aln_cap = cap;
    }
    const std::vector<TuneChoice> cs = candidates(kTuneBatch, cls[0].k, 0);
    float best = 0.f;
    int bestw = 0;
    for (size_t ci = 0; ci < cs.size(); ++ci) {
      tune_set(kTuneBatch, kc, 0, cs[ci]);
      int rc = msa_dp_align_batch(cls.data(), (int32_t)cls.size(), res.data(), 0);  // warm-up
      if (rc) return rc;
      std::vector<float> t;
      for (int r = 0; r < reps; ++r) {
        const auto a = std::chrono::steady_clock::now();
        rc = msa_dp_align_batch(cls.data(), (int32_t)cls.size(), res.data(), 0);
        const auto b = std::chrono::steady_clock::now();
        if (rc) return rc;
        t.push_back(std::chrono::duration<float, std::milli>(b - a).count());
      }
      const float m = median_of(t);
      if (ci == 0 || m < best) {
        best = m;
        bestw = cs[ci].wpc;
      }
    }
    tune_set(kTuneBatch, kc, 0, TuneChoice{0, bestw});
    wpc_out[kc] = bestw;
  }
  return MSA_OK;
}
