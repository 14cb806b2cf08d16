// msa_runtime.cpp -- workspace set-up and plain-path launches.
#include "msa_runtime.h"

#include <string.h>

#include <stdlib.h>

#include <algorithm>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/msa_dp.h"
#include "msa_tune.h"

namespace msa {

namespace {
std::mutex g_mu;
// What each prepared workspace (by device address) was prepared for: its
// shape, so that a launch on it with other lengths is refused, and its mode
// flags, so that a launch knows its kernel sequence without reading the
// device control block.
struct WsSig {
  int32_t k = 0;
  int32_t n[kMaxK] = {};
  int64_t bytes = 0;
  int32_t flags = 0;
  int32_t alpha = 0;
};
std::unordered_map<uintptr_t, WsSig> g_ws;
int g_cu[64] = {};
int g_occ[64][kMaxK + 1] = {};
}  // namespace

int device_cu_count() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_cu[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n < 1)
      n = 1;
    g_cu[dev] = n;
  }
  return g_cu[dev];
}

void forget_workspace(const char *ws) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_ws.erase((uintptr_t)ws);
}

int32_t workspace_flags(const char *ws) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ws.find((uintptr_t)ws);
  return it == g_ws.end() ? 0 : it->second.flags;
}

int check_workspace(const Plan &p, const char *ws, int32_t *alpha) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ws.find((uintptr_t)ws);
  if (it == g_ws.end()) return MSA_EINVAL;  // never prepared
  const WsSig &w = it->second;
  if (w.k != p.k || w.bytes != p.bytes) return MSA_EINVAL;
  for (int i = 0; i < p.k; ++i)
    if (w.n[i] != p.n[i]) return MSA_EINVAL;
  if (alpha) *alpha = w.alpha;
  return MSA_OK;
}

static int occupancy(int k) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_occ[dev][k]) g_occ[dev][k] = fill_occupancy(k);
  return g_occ[dev][k] > 0 ? g_occ[dev][k] : 1;
}

int prepare_workspace(const Plan &p, char *ws, const int8_t *submat, int alpha, int gap,
                      int32_t flags,
                      hipStream_t s) {
  std::vector<int32_t> order;
  make_tile_order(p, &order);
  Ctrl ctrl;
  memset(&ctrl, 0, sizeof(ctrl));
  ctrl.epoch = 1;
  ctrl.alpha = alpha;
  ctrl.gap = gap;
  ctrl.flags = flags;
  ctrl.best = INT64_MIN;
  // pruned mode: the closed-form score floor and the first threshold's margin
  int64_t lo = 0, hi = 0;
  if (score_bounds(p.n, p.k, submat, alpha, gap, &lo, &hi) != 0) return MSA_EINVAL;
  ctrl.lo = lo;
  int cmax = gap < 0 ? -gap : gap;
  for (int x = 0; x < alpha * alpha; ++x) cmax = std::max(cmax, std::abs((int)submat[x]));
  ctrl.prune_c = (int64_t)(p.k * (p.k - 1) / 2) * cmax;
  bool ok = true;
  ok = ok && hipMemcpyAsync(ws + p.off_ctrl, &ctrl, sizeof(ctrl), hipMemcpyHostToDevice, s) ==
                 hipSuccess;
  ok = ok && hipMemcpyAsync(ws + p.off_sub, submat, (size_t)alpha * alpha,
                            hipMemcpyHostToDevice, s) == hipSuccess;
  ok = ok && hipMemcpyAsync(ws + p.off_order, order.data(), order.size() * 4,
                            hipMemcpyHostToDevice, s) == hipSuccess;
  std::vector<int32_t> corder;
  make_column_order(p, &corder);
  ok = ok && hipMemcpyAsync(ws + p.off_corder, corder.data(), corder.size() * 4,
                            hipMemcpyHostToDevice, s) == hipSuccess;
  ok = ok && hipMemsetAsync(ws + p.off_flags, 0, (size_t)p.ntiles * 4, s) == hipSuccess;
  // the streaming k = 3 fill's exchange regions: tag 0, never a launch's tag
  if (p.k == 3)
    ok = ok && hipMemsetAsync(ws + p.off_x0, 0, (size_t)p.x_bytes, s) == hipSuccess;
  ok = ok && hipStreamSynchronize(s) == hipSuccess;
  std::lock_guard<std::mutex> lk(g_mu);
  if (ok) {
    WsSig w;
    w.k = p.k;
    for (int i = 0; i < p.k; ++i) w.n[i] = p.n[i];
    w.bytes = p.bytes;
    w.flags = flags;
    w.alpha = alpha;
    g_ws[(uintptr_t)ws] = w;
  } else {
    g_ws.erase((uintptr_t)ws);  // a failed set-up leaves the workspace unprepared
  }
  return ok ? MSA_OK : MSA_EDEVICE;
}

#ifdef MSA_TRACE
// debug builds only: per-tile phase timestamps of the next fills
static int64_t *g_trace_buf = nullptr;
extern "C" void msa_dp_debug_set_trace(int64_t *d_buf) { g_trace_buf = d_buf; }
#endif

static int fill_grid(const Plan &p, int wpc) {
  // Persistent workgroups: as many tiles as the widest wave holds, rounded
  // down to whole compute units, at least one per unit and at most what
  // fits.  Beyond the widest wave extra workgroups only wait, and tiles that
  // share a compute unit slow each other's sweep, which is the critical path.
  // A tuned choice (wpc > 0) fixes the workgroups per compute unit instead.
  const int64_t cu = device_cu_count();
  int64_t grid = p.max_wave / cu * cu;
  if (grid < cu) grid = cu;
  if (wpc > 0) grid = cu * wpc;
  if (grid > cu * occupancy(p.k)) grid = cu * occupancy(p.k);
  if (grid > p.ntiles) grid = p.ntiles;
  if (grid < 1) grid = 1;
  return (int)grid;
}

// The fill of a prepared workspace: one launch, or in pruned mode (the mode
// is known to the host from the plan and flags cached at set-up) the bound,
// selection and two-pass sequence of msa_prune.hip.
static int run_fill(const Plan &p, char *ws, JobDev &jd, hipStream_t s, int alpha) {
  Ctrl *ctrl = reinterpret_cast<Ctrl *>(ws + p.off_ctrl);
  TuneChoice tc;
  tune_get(kTunePlain, p.k, length_bucket(p.n, p.k), &tc);
  if (tc.variant != 2 && sweep3_eligible(p, alpha, workspace_flags(ws)))
    return launch_sweep3(p, ws, jd, ctrl, workspace_flags(ws), s);
  const int32_t *order = reinterpret_cast<const int32_t *>(ws + p.off_order);
  int grid = fill_grid(p, tc.variant == 2 ? tc.wpc : 0);
  if (jd.ncols > 0 && grid > jd.ncols) grid = jd.ncols;
  if (!(workspace_flags(ws) & kPrune)) return launch_fill(jd, ctrl, order, grid, 0, s);
  PruneDev pd;
  fill_prunedev(p, ws, jd.seqs, jd.score_out, &pd);
  jd.keep = pd.keep;
  const int32_t *korder = pd.korder;
  if (launch_prune_bounds(pd, ctrl, s) != 0) return -1;
  for (int pass = 1; pass <= 2; ++pass) {
    if (launch_prune_select(pd, ctrl, pass, s) != 0) return -1;
    if (launch_fill(jd, ctrl, korder, grid, pass, s) != 0) return -1;
    if (pass == 1 && launch_prune_check(pd, ctrl, s) != 0) return -1;
  }
  return 0;
}

int run_plain(const Plan &p, char *ws, const uint8_t *d_seqs, int64_t *d_score, uint8_t *d_aln,
              int64_t aln_cap, int64_t *d_aln_len, int32_t *d_status, hipStream_t s,
              int which) {
  int32_t alpha = 0;
  if (check_workspace(p, ws, &alpha) != MSA_OK) return MSA_EINVAL;
  return run_plain_set_up(p, ws, alpha, d_seqs, d_score, d_aln, aln_cap, d_aln_len, d_status, s,
                          which);
}

int run_plain_set_up(const Plan &p, char *ws, int alpha, const uint8_t *d_seqs,
                     int64_t *d_score, uint8_t *d_aln, int64_t aln_cap, int64_t *d_aln_len,
                     int32_t *d_status, hipStream_t s, int which) {
  JobDev jd;
  fill_jobdev(p, ws, 0, 0, &jd);  // alpha and gap are read from the control block
  jd.seqs = d_seqs;
  jd.score_out = d_score;
  jd.aln_out = d_aln;
  jd.aln_cap = aln_cap;
  jd.aln_len_out = d_aln_len;
  jd.status_out = d_status;
#ifdef MSA_TRACE
  jd.trace = g_trace_buf;
#endif
  Ctrl *ctrl = reinterpret_cast<Ctrl *>(ws + p.off_ctrl);
  if ((which & 1) && run_fill(p, ws, jd, s, alpha) != 0) return MSA_EDEVICE;
  if ((which & 2) && launch_traceback(jd, ctrl, s) != 0) return MSA_EDEVICE;
  return MSA_OK;
}

int run_coopt(const Plan &p, char *ws, const uint8_t *d_seqs, int32_t max_paths, int64_t *d_score,
              uint8_t *d_aln, int64_t aln_cap, int64_t *d_aln_len, int32_t *d_npaths,
              int32_t *d_status, hipStream_t s) {
  int32_t alpha = 0;
  if (check_workspace(p, ws, &alpha) != MSA_OK) return MSA_EINVAL;
  JobDev jd;
  fill_jobdev(p, ws, 0, 0, &jd);
  jd.seqs = d_seqs;
  jd.score_out = d_score;
  jd.aln_cap = aln_cap;
  jd.status_out = d_status;
  Ctrl *ctrl = reinterpret_cast<Ctrl *>(ws + p.off_ctrl);
  if (run_fill(p, ws, jd, s, alpha) != 0) return MSA_EDEVICE;
  if (launch_coopt(jd, ctrl, max_paths, d_aln, d_aln_len, d_npaths, s) != 0) return MSA_EDEVICE;
  return MSA_OK;
}

int run_nearopt(const Plan &p, char *ws, const uint8_t *d_seqs, int64_t delta, int32_t max_paths,
                int64_t *d_score, int64_t *d_scores, uint8_t *d_aln, int64_t aln_cap,
                int64_t *d_aln_len, int32_t *d_npaths, int32_t *d_status, hipStream_t s) {
  int32_t alpha = 0;
  if (check_workspace(p, ws, &alpha) != MSA_OK) return MSA_EINVAL;
  JobDev jd;
  fill_jobdev(p, ws, 0, 0, &jd);
  jd.seqs = d_seqs;
  jd.score_out = d_score;
  jd.aln_cap = aln_cap;
  jd.status_out = d_status;
  Ctrl *ctrl = reinterpret_cast<Ctrl *>(ws + p.off_ctrl);
  if (run_fill(p, ws, jd, s, alpha) != 0) return MSA_EDEVICE;
  if (launch_nearopt(jd, ctrl, delta, max_paths, d_scores, d_aln, d_aln_len, d_npaths, s) != 0)
    return MSA_EDEVICE;
  return MSA_OK;
}

int export_dirs(const Plan &p, char *ws, uint8_t *out, hipStream_t s) {
  if (check_workspace(p, ws, nullptr) != MSA_OK) return MSA_EINVAL;
  JobDev jd;
  fill_jobdev(p, ws, 0, 0, &jd);
  const Ctrl *ctrl = reinterpret_cast<const Ctrl *>(ws + p.off_ctrl);
  return launch_export(jd, ctrl, out, p.ncell, s) == 0 ? MSA_OK : MSA_EDEVICE;
}

}  // namespace msa

namespace msa {

int export_prune(const Plan &p, char *ws, uint8_t *keep_out, int64_t *info_out,
                 hipStream_t s) {
  if (check_workspace(p, ws, nullptr) != MSA_OK) return MSA_EINVAL;
  if (!p.prunable || !(workspace_flags(ws) & kPrune)) return MSA_EINVAL;
  const Ctrl *ctrl = reinterpret_cast<const Ctrl *>(ws + p.off_ctrl);
  bool ok = true;
  if (keep_out)
    ok = ok && hipMemcpyAsync(keep_out, ws + p.off_keep, (size_t)p.ntiles,
                              hipMemcpyDeviceToDevice, s) == hipSuccess;
  if (info_out)  // prune_U, prune_L, prune_kept, prune_passes are contiguous
    ok = ok && hipMemcpyAsync(info_out, &ctrl->prune_U, 4 * sizeof(int64_t),
                              hipMemcpyDeviceToDevice, s) == hipSuccess;
  return ok ? MSA_OK : MSA_EDEVICE;
}

}  // namespace msa
