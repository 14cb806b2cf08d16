// msa_batch.cpp -- msa_dp_align_batch: many independent alignments through
// batched persistent launches (one per group of jobs of one k class whose
// arena fits the HBM budget).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "../../include/msa_dp.h"
#include "msa_launch.h"

using namespace msa;

namespace msa {

// Default HBM budget: 60% of the free device memory, at most 96 GiB.
int64_t default_budget() {
  size_t freeb = 0, totalb = 0;
  if (hipMemGetInfo(&freeb, &totalb) != hipSuccess) return (int64_t)8 << 30;
  int64_t b = (int64_t)(freeb * 0.6);
  return std::min<int64_t>(b, (int64_t)96 << 30);
}

// Orders jobs by k class, then k, then scoring, so that consecutive tiles of a
// launch share the per-k cell table and the substitution matrix in LDS.
void sort_for_launch(const msa_job *jobs, std::vector<int> *idx) {
  std::stable_sort(idx->begin(), idx->end(), [&](int a, int b) {
    const msa_job &x = jobs[a], &y = jobs[b];
    if (kclass_of(x.k) != kclass_of(y.k)) return kclass_of(x.k) < kclass_of(y.k);
    if (x.k != y.k) return x.k < y.k;
    if (x.alpha != y.alpha) return x.alpha < y.alpha;
    return std::memcmp(x.submat, y.submat, (size_t)x.alpha * x.alpha) < 0;
  });
}

}  // namespace msa

namespace {
// Per-thread launch arena, reused by later calls and kept for the life of the
// process (never destroyed at exit, when the HIP runtime may be gone).
thread_local Launch *g_launch = nullptr;
thread_local int64_t g_launch_bytes = 0;
}  // namespace

extern "C" int msa_dp_align_batch(const msa_job *jobs, int32_t njobs, msa_result *results,
                                  int64_t hbm_budget_bytes) {
  if (njobs < 0 || (njobs > 0 && (!jobs || !results))) return MSA_EINVAL;
  if (njobs == 0) return MSA_OK;
  std::vector<int> valid;
  for (int i = 0; i < njobs; ++i) {
    int rc = validate_job(jobs[i]);
    int64_t total = 0;
    for (int d = 0; rc == MSA_OK && d < jobs[i].k; ++d) total += jobs[i].lens[d];
    if (rc == MSA_OK && (results[i].aln_cap < total || (total > 0 && !results[i].aln)))
      rc = MSA_EINVAL;
    results[i].status = rc;
    results[i].score = 0;
    results[i].aln_len = 0;
    if (rc == MSA_OK) valid.push_back(i);
  }
  if (valid.empty()) return MSA_OK;
  const int64_t budget = hbm_budget_bytes > 0 ? hbm_budget_bytes : default_budget();
  sort_for_launch(jobs, &valid);

  if (!g_launch) g_launch = new Launch();
  Launch &L = *g_launch;
  if (g_launch_bytes < budget) {
    int rc = L.init(budget);
    if (rc) return rc;
    g_launch_bytes = budget;
  } else {
    int rc = L.init(g_launch_bytes);
    if (rc) return rc;
  }
  const int64_t cap = L.capacity();

  size_t pos = 0;
  while (pos < valid.size()) {
    // greedy group: one k class, within the arena
    std::vector<const msa_job *> grp;
    std::vector<int> gidx;
    const int kc = kclass_of(jobs[valid[pos]].k);
    int64_t used = 0, tiles = 0;
    while (pos < valid.size()) {
      const msa_job &j = jobs[valid[pos]];
      if (kclass_of(j.k) != kc) break;
      const int64_t b = job_arena_bytes(j);
      Plan p;
      make_plan(j.lens, j.k, &p);
      const int64_t need = used + b + Launch::overhead_bytes((int)grp.size() + 1, tiles + p.ntiles);
      if (need > cap || grp.size() >= 65536 || tiles + p.ntiles >= ((int64_t)1 << 30)) {
        if (grp.empty()) {  // this job alone exceeds the budget
          results[valid[pos]].status = MSA_ENOMEM;
          ++pos;
          continue;
        }
        break;
      }
      used += b;
      tiles += p.ntiles;
      grp.push_back(&j);
      gidx.push_back(valid[pos]);
      ++pos;
    }
    if (grp.empty()) continue;
    int rc = L.start(grp);
    if (rc == MSA_OK) rc = L.wait();
    for (size_t g = 0; g < gidx.size(); ++g) {
      if (rc != MSA_OK) {
        results[gidx[g]].status = rc;
        continue;
      }
      L.fill_result((int)g, &results[gidx[g]]);
    }
    L.release();
    if (rc == MSA_EDEVICE) return rc;
  }
  return MSA_OK;
}
