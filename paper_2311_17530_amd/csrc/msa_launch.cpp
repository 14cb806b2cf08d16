// msa_launch.cpp -- staging and running one batched persistent launch.
#include "msa_launch.h"

#include <string.h>

#include <algorithm>
#include <map>

#include "msa_runtime.h"
#include "msa_tune.h"

namespace msa {

static int64_t a256(int64_t x) { return (x + 255) & ~(int64_t)255; }

// The batch descriptor sits right after the control block in every arena, and
// the job descriptors right after it: both addresses are fixed per arena, so
// a captured launch sequence stays valid for every batch the arena holds.
constexpr int64_t kArgsOff = 256;
constexpr int64_t kJobsOff = 512;
static_assert(sizeof(Ctrl) <= kArgsOff, "control block first");
static_assert(kArgsOff + (int64_t)sizeof(BatchArgs) <= kJobsOff, "descriptor before the jobs");

int validate_job(const msa_job &j, int64_t) {
  if (j.k < 2 || j.k > MSA_MAX_K) return MSA_EINVAL;
  if (!j.submat || j.alpha < 1 || j.alpha > 255) return MSA_EINVAL;
  for (int i = 0; i < j.k; ++i) {
    if (j.lens[i] < 0) return MSA_EINVAL;
    if (j.lens[i] > 0 && !j.seqs[i]) return MSA_EINVAL;
    for (int32_t t = 0; t < j.lens[i]; ++t)
      if (j.seqs[i][t] >= j.alpha) return MSA_EINVAL;
  }
  Plan p;
  int rc = make_plan(j.lens, j.k, &p);
  if (rc) return rc;
  return check_scoring(j.lens, j.k, j.submat, j.alpha, j.gap);
}

namespace {
struct JobSizes {
  Plan p;
  int64_t cap = 0;       // alignment row capacity
  int64_t nw = 0;        // waves
  int64_t small = 0;     // host-initialised bytes
  int64_t big = 0;       // device-only bytes (path, faces, dir)
  int64_t out = 0;       // output rows
};

int sizes_of(const msa_job &j, JobSizes *s) {
  int rc = make_plan(j.lens, j.k, &s->p);
  if (rc) return rc;
  const Plan &p = s->p;
  s->cap = std::max<int64_t>(1, p.total_len);
  s->nw = p.nwaves;
  s->small = a256(std::max<int64_t>(p.total_len, 1)) +        // sequences
             a256((int64_t)(j.k + 1) * p.nwaves * 4) +        // wave counts
             a256((int64_t)p.nwaves * 8) +                    // wave queue slots
             256;                                             // job status
  s->big = a256(std::max<int64_t>(p.total_len, 1)) +          // traceback path
           a256(std::max<int64_t>(p.face_elems * 4, 256)) +   // face planes
           a256(p.ntiles * p.dbs);                            // direction blocks
  s->out = a256((int64_t)j.k * s->cap);
  return MSA_OK;
}
}  // namespace

int64_t job_arena_bytes(const msa_job &j) {
  JobSizes s;
  if (sizes_of(j, &s)) return -1;
  return s.small + s.big + s.out + 12 * s.p.ntiles + (int64_t)sizeof(JobDev) + 64;
}

int64_t Launch::overhead_bytes(int njobs, int64_t ntiles_total) {
  int64_t tables = 0;
  for (int k = 2; k <= kMaxK; ++k) {
    const int T = tile_edge_for_k(k);
    tables += a256((int64_t)ipow(T, k) * 4) + a256((int64_t)(k * (T - 1) + 2) * 4);
  }
  return 768 + tables + a256((int64_t)njobs * sizeof(JobDev)) + a256((int64_t)(njobs + 1) * 8) +
         a256((int64_t)njobs * 24) + 3 * a256(ntiles_total * 4) + 255 * 255 * 4 + 4096;
}

Launch::~Launch() {
  if (busy_) wait();
  drop_graphs();
  if (d_) (void)hipFree(d_);
  if (h_in_) (void)hipHostFree(h_in_);
  if (h_out_) (void)hipHostFree(h_out_);
  if (done_) (void)hipEventDestroy(done_);
  if (start_) (void)hipEventDestroy(start_);
  if (stream_ && own_stream_) (void)hipStreamDestroy(stream_);
}

int Launch::init(int64_t bytes, hipStream_t shared) {
  if (hipGetDevice(&device_) != hipSuccess) return MSA_EDEVICE;
  if (!stream_ && shared) {
    stream_ = shared;
    own_stream_ = false;
  }
  if (!stream_ && hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking) != hipSuccess)
    return MSA_EDEVICE;
  if (!done_ && hipEventCreateWithFlags(&done_, hipEventDefault) != hipSuccess)
    return MSA_EDEVICE;
  if (!start_ && hipEventCreateWithFlags(&start_, hipEventDefault) != hipSuccess)
    return MSA_EDEVICE;
  if (cap_ < bytes) {
    drop_graphs();  // they hold addresses inside the old arena
    if (d_) (void)hipFree(d_);
    d_ = nullptr;
    cap_ = 0;
    if (hipMalloc(&d_, bytes) != hipSuccess) {
      d_ = nullptr;
      return MSA_ENOMEM;
    }
    cap_ = bytes;
  }
  // Pinned staging and the four k classes' launch graphs are made here, once
  // per arena, so that launches under load (a server's slots) allocate and
  // instantiate nothing while other slots' persistent fills run.
  int rc = ensure_host(1 << 20, 1 << 20);
  if (rc) return rc;
  for (int kc = 0; kc < 4; ++kc) (void)ensure_graph(kc, batch_grid(kc));
  // The stream's first kernel and its first copies each way make the runtime
  // create the hardware queues behind them; doing it here keeps that out of
  // the time when other slots' persistent fills run (the queue list changes
  // then, and running queues are preempted).
  if (hipMemsetAsync(d_, 0, 256, stream_) != hipSuccess ||
      hipMemcpyAsync(d_, h_in_, 256, hipMemcpyHostToDevice, stream_) != hipSuccess ||
      hipMemcpyAsync(h_out_, d_, 256, hipMemcpyDeviceToHost, stream_) != hipSuccess ||
      hipStreamSynchronize(stream_) != hipSuccess)
    return MSA_EDEVICE;
  return MSA_OK;
}

// Persistent workgroups of the batched fill: every one that fits, or the
// tuned count per CU.
int Launch::batch_grid(int kc) const {
  int wpc = batch_occupancy(kc);
  TuneChoice tc;
  if (tune_get(kTuneBatch, kc, 0, &tc) && tc.wpc > 0) wpc = std::min(wpc, (int)tc.wpc);
  const int grid = device_cu_count() * wpc;
  return grid < 1 ? 1 : grid;
}

void Launch::drop_graphs() {
  for (int kc = 0; kc < 4; ++kc) {
    if (graph_[kc]) (void)hipGraphExecDestroy(graph_[kc]);
    graph_[kc] = nullptr;
    graph_failed_[kc] = false;
  }
}

// Captures the launch sequence of k class kc on this arena.  Returns 0 when
// a graph is ready; otherwise the caller launches the kernels directly.
int Launch::ensure_graph(int kc, int grid) {
  if (graph_[kc] && graph_grid_[kc] != grid) {  // another tuned grid: capture again
    (void)hipGraphExecDestroy(graph_[kc]);
    graph_[kc] = nullptr;
  }
  if (graph_[kc]) return 0;
  if (graph_failed_[kc]) return -1;
  graph_grid_[kc] = grid;
  hipGraph_t g = nullptr;
  bool ok = hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    const int rc = launch_batch(kc, reinterpret_cast<const BatchArgs *>(d_ + kArgsOff),
                                reinterpret_cast<const JobDev *>(d_ + kJobsOff),
                                reinterpret_cast<Ctrl *>(d_), grid, stream_);
    ok = hipStreamEndCapture(stream_, &g) == hipSuccess && rc == 0 && g;
  }
  ok = ok && hipGraphInstantiate(&graph_[kc], g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (!ok) {
    graph_[kc] = nullptr;
    graph_failed_[kc] = true;
    (void)hipGetLastError();  // clear a capture error; the direct launches follow
    return -1;
  }
  return 0;
}

int Launch::ensure_host(int64_t in_bytes, int64_t out_bytes) {
  if (h_in_cap_ < in_bytes) {
    if (h_in_) (void)hipHostFree(h_in_);
    h_in_ = nullptr;
    h_in_cap_ = 0;
    const int64_t want = std::max<int64_t>(in_bytes, 1 << 20);
    if (hipHostMalloc((void **)&h_in_, want, hipHostMallocDefault) != hipSuccess) return MSA_ENOMEM;
    h_in_cap_ = want;
  }
  if (h_out_cap_ < out_bytes) {
    if (h_out_) (void)hipHostFree(h_out_);
    h_out_ = nullptr;
    h_out_cap_ = 0;
    const int64_t want = std::max<int64_t>(out_bytes, 1 << 20);
    if (hipHostMalloc((void **)&h_out_, want, hipHostMallocDefault) != hipSuccess)
      return MSA_ENOMEM;
    h_out_cap_ = want;
  }
  return MSA_OK;
}

int Launch::start(const std::vector<const msa_job *> &jobs,
                  const std::vector<hipEvent_t> &after) {
  if (busy_ || jobs.empty()) return MSA_EINVAL;
  const int nj = (int)jobs.size();
  const int kc = kclass_of(jobs[0]->k);
  std::vector<JobSizes> sz(nj);
  int64_t tiles = 0, small = 0, big = 0, outb = 0;
  for (int i = 0; i < nj; ++i) {
    if (kclass_of(jobs[i]->k) != kc) return MSA_EINVAL;
    if (sizes_of(*jobs[i], &sz[i])) return MSA_EINVAL;
    tiles += sz[i].p.ntiles;
    small += sz[i].small;
    big += sz[i].big;
    outb += sz[i].out;
  }
  if (tiles >= ((int64_t)1 << 31) - 1) return MSA_ENOMEM;

  // ---- layout: [inputs (one host-to-device copy)][outputs][device only] ----
  int64_t o = 0;
  const int64_t off_ctrl = o;  o += 256;
  const int64_t off_args = o;  o = a256(o + (int64_t)sizeof(BatchArgs));
  const int64_t off_jobs = o;  o = a256(o + (int64_t)nj * sizeof(JobDev));
  if (off_args != kArgsOff || off_jobs != kJobsOff) return MSA_EINVAL;
  const int64_t off_jt = o;    o = a256(o + (int64_t)(nj + 1) * 8);
  const int64_t off_jc = o;    o = a256(o + (int64_t)(nj + 1) * 8);
  // substitution matrices, deduplicated by content
  std::map<std::string, int64_t> subs;
  std::vector<int64_t> sub_off(nj);
  for (int i = 0; i < nj; ++i) {
    const msa_job &j = *jobs[i];
    std::string key((const char *)j.submat, (size_t)j.alpha * j.alpha);
    key.push_back((char)j.alpha);
    auto it = subs.find(key);
    if (it == subs.end()) {
      it = subs.emplace(key, o).first;
      o = a256(o + (int64_t)j.alpha * j.alpha);
    }
    sub_off[i] = it->second;
  }
  std::vector<int64_t> job_small(nj);
  for (int i = 0; i < nj; ++i) {
    job_small[i] = o;
    o += sz[i].small;
  }
  const int64_t in_bytes = o;
  // outputs
  const int64_t off_out = o;
  const int64_t off_score = o;  o = a256(o + (int64_t)nj * 8);
  const int64_t off_len = o;    o = a256(o + (int64_t)nj * 8);
  const int64_t off_stat = o;   o = a256(o + (int64_t)nj * 4);
  const int64_t off_gst = o;    o = a256(o + 72);
  std::vector<int64_t> job_out(nj);
  for (int i = 0; i < nj; ++i) {
    job_out[i] = o;
    o += sz[i].out;
  }
  const int64_t out_bytes = o - off_out;
  // device only
  const int64_t off_qjob = o;  o = a256(o + tiles * 4);
  const int64_t off_qtile = o; o = a256(o + tiles * 4);
  const int64_t off_flags = o; o = a256(o + tiles * 4);
  std::vector<int64_t> job_big(nj);
  for (int i = 0; i < nj; ++i) {
    job_big[i] = o;
    o += sz[i].big;
  }
  if (o > cap_) return MSA_ENOMEM;
  int rc = ensure_host(in_bytes, out_bytes);
  if (rc) return rc;

  // ---- host image of the input region ----
  char *h = h_in_;
  memset(h, 0, (size_t)in_bytes);
  Ctrl ctrl;
  memset(&ctrl, 0, sizeof(ctrl));
  ctrl.epoch = 1;
  // A batched dependency wait is bounded by one job's tile chain (a few ms
  // even for large jobs), so a launch gives up after 250 ms instead of the
  // plain fill's 2 s: a launch that times out is re-run sooner.
  ctrl.wait_limit = wait_limit_ > 0 ? wait_limit_ : kBatchWaitTicks;
  memcpy(h + off_ctrl, &ctrl, sizeof(ctrl));
  for (auto &kv : subs)
    memcpy(h + kv.second, kv.first.data(), kv.first.size() - 1);
  int64_t *jt = reinterpret_cast<int64_t *>(h + off_jt);
  int64_t *jc = reinterpret_cast<int64_t *>(h + off_jc);  // columns before job i
  jt[0] = 0;
  jc[0] = 0;
  meta_.assign(nj, Meta());
  std::vector<const int32_t *> wave_cnt(nj);
  std::vector<int64_t *> wave_base(nj);
  JobDev *jd_all = reinterpret_cast<JobDev *>(h + off_jobs);
  for (int i = 0; i < nj; ++i) {
    const msa_job &j = *jobs[i];
    const Plan &p = sz[i].p;
    jt[i + 1] = jt[i] + p.ntiles;
    jc[i + 1] = jc[i] + p.ncols;
    JobDev jd;
    fill_jobdev(p, nullptr, j.alpha, j.gap, &jd);
    // small region of this job
    int64_t so = job_small[i];
    char *hs_base = h + so;
    int64_t pos = 0;
    for (int d = 0; d < j.k; ++d) {
      if (j.lens[d] > 0) memcpy(hs_base + pos, j.seqs[d], (size_t)j.lens[d]);
      pos += j.lens[d];
    }
    const int64_t o_seq = so;
    so += a256(std::max<int64_t>(p.total_len, 1));
    const int64_t o_wcnt = so;
    int32_t *wc = reinterpret_cast<int32_t *>(h + so);
    const int nw = p.nwaves;
    // wc[d][s]: coordinate tuples (c_d..c_{k-1}) with sum s
    for (int s = 0; s < nw; ++s) wc[j.k * nw + s] = (s == 0);
    for (int d = j.k - 1; d >= 0; --d)
      for (int s = 0; s < nw; ++s) {
        int64_t acc = 0;
        for (int c = 0; c < p.P[d] && c <= s; ++c) acc += wc[(d + 1) * nw + (s - c)];
        wc[d * nw + s] = (int32_t)acc;
      }
    so += a256((int64_t)(j.k + 1) * nw * 4);
    const int64_t o_wst = so;
    wave_cnt[i] = wc + nw;  // row 1: columns by the wave of their first tile
    wave_base[i] = reinterpret_cast<int64_t *>(h + so);
    so += a256((int64_t)nw * 8);
    const int64_t o_jst = so;
    // device pointers
    jd.seqs = reinterpret_cast<const uint8_t *>(d_ + o_seq);
    jd.sub = reinterpret_cast<const int8_t *>(d_ + sub_off[i]);
    jd.wcnt = reinterpret_cast<const int32_t *>(d_ + o_wcnt);
    jd.wbase = reinterpret_cast<const int64_t *>(d_ + o_wst);
    jd.jstatus = reinterpret_cast<int32_t *>(d_ + o_jst);
    jd.qbase = jt[i];
    jd.flags = reinterpret_cast<int32_t *>(d_ + off_flags) + jt[i];
    int64_t bo = job_big[i];
    jd.path = reinterpret_cast<uint8_t *>(d_ + bo);
    bo += a256(std::max<int64_t>(p.total_len, 1));
    jd.faces = reinterpret_cast<int32_t *>(d_ + bo);
    bo += a256(std::max<int64_t>(p.face_elems * 4, 256));
    jd.dir = reinterpret_cast<uint8_t *>(d_ + bo);
    jd.score_out = reinterpret_cast<int64_t *>(d_ + off_score) + i;
    jd.aln_len_out = reinterpret_cast<int64_t *>(d_ + off_len) + i;
    jd.status_out = reinterpret_cast<int32_t *>(d_ + off_stat) + i;
    jd.aln_out = reinterpret_cast<uint8_t *>(d_ + job_out[i]);
    jd.aln_cap = sz[i].cap;
    jd.trace = nullptr;
    memcpy(&jd_all[i], &jd, sizeof(JobDev));
    meta_[i].k = j.k;
    meta_[i].cap = sz[i].cap;
    meta_[i].aln_off = job_out[i] - off_out;
    meta_[i].qbase = jt[i];
  }

  // The queue holds tile columns along dimension 0 (a workgroup computes a
  // column bottom up, as in the plain fill) in wave-major order across jobs:
  // every job's columns starting in wave 0, then every job's columns starting
  // in wave 1, ...  The persistent workgroups so work on all jobs' wavefronts
  // at once instead of waiting on one job's dependency chain at a time; a
  // column depends only on columns of its job that start in earlier waves,
  // so the order is topological.
  {
    int wmax = 0;
    for (int i = 0; i < nj; ++i) wmax = std::max(wmax, sz[i].p.nwaves);
    std::vector<int64_t> slot(wmax, 0);  // next free slot of wave w
    std::vector<int64_t> tot(wmax, 0);
    for (int i = 0; i < nj; ++i)
      for (int w = 0; w < sz[i].p.nwaves; ++w) tot[w] += wave_cnt[i][w];
    int64_t acc = 0;
    for (int w = 0; w < wmax; ++w) {
      slot[w] = acc;
      acc += tot[w];
    }
    for (int i = 0; i < nj; ++i)
      for (int w = 0; w < sz[i].p.nwaves; ++w) {
        wave_base[i][w] = slot[w];
        slot[w] += wave_cnt[i][w];
      }
  }

  // ---- batch descriptor (read by the launch sequence) ----
  BatchArgs args;
  memset(&args, 0, sizeof(args));
  args.jcols = reinterpret_cast<const int64_t *>(d_ + off_jc);
  args.qjob = reinterpret_cast<int32_t *>(d_ + off_qjob);
  args.qtile = reinterpret_cast<int32_t *>(d_ + off_qtile);
  args.flags = reinterpret_cast<int32_t *>(d_ + off_flags);
  args.gstatus = reinterpret_cast<int32_t *>(d_ + off_gst);
  args.tiles = tiles;
  args.cols = jc[nj];
  args.njobs = nj;
  memcpy(h + off_args, &args, sizeof(args));

  // ---- enqueue: inputs, the launch sequence (a graph replay), outputs ----
  const int grid = batch_grid(kc);
  const bool graph = ensure_graph(kc, grid) == 0;
  bool ok = true;
  for (hipEvent_t e : after) ok = ok && hipStreamWaitEvent(stream_, e, 0) == hipSuccess;
  ok = ok && hipEventRecord(start_, stream_) == hipSuccess;
  ok = ok && hipMemcpyAsync(d_, h, (size_t)in_bytes, hipMemcpyHostToDevice, stream_) == hipSuccess;
  if (graph)
    ok = ok && hipGraphLaunch(graph_[kc], stream_) == hipSuccess;
  else
    ok = ok && launch_batch(kc, reinterpret_cast<const BatchArgs *>(d_ + off_args),
                            reinterpret_cast<const JobDev *>(d_ + off_jobs),
                            reinterpret_cast<Ctrl *>(d_ + off_ctrl), grid, stream_) == 0;
  ok = ok && hipMemcpyAsync(h_out_, d_ + off_out, (size_t)out_bytes, hipMemcpyDeviceToHost,
                            stream_) == hipSuccess;
  ok = ok && hipEventRecord(done_, stream_) == hipSuccess;
  out_bytes_ = out_bytes;
  out_off_ = off_out;
  (void)off_score;
  busy_ = true;
  launch_status_ = ok ? MSA_OK : MSA_EDEVICE;
  return launch_status_;
}

bool Launch::ready() {
  if (!busy_) return true;
  return hipEventQuery(done_) != hipErrorNotReady;
}

int Launch::wait() {
  if (!busy_) return MSA_OK;
  if (hipEventSynchronize(done_) != hipSuccess) launch_status_ = MSA_EDEVICE;
  return launch_status_;
}

bool Launch::interval_ms(hipEvent_t ref, float *t0, float *t1) const {
  return hipEventElapsedTime(t0, ref, start_) == hipSuccess &&
         hipEventElapsedTime(t1, ref, done_) == hipSuccess;
}

int32_t Launch::device_status() const {
  const int nj = (int)meta_.size();
  const int64_t off_gst = 2 * a256((int64_t)nj * 8) + a256((int64_t)nj * 4);
  return *reinterpret_cast<const int32_t *>(h_out_ + off_gst);
}

int64_t Launch::device_max_pause_us() const {
  const int nj = (int)meta_.size();
  const int64_t off_gst = 2 * a256((int64_t)nj * 8) + a256((int64_t)nj * 4);
  return *reinterpret_cast<const int64_t *>(h_out_ + off_gst + 8) / 100;  // 100 MHz ticks
}

bool Launch::device_timeout(int *job, int64_t *tile, int64_t *missing, int64_t more[4]) const {
  const int nj = (int)meta_.size();
  const int64_t off_gst = 2 * a256((int64_t)nj * 8) + a256((int64_t)nj * 4);
  const int64_t *w = reinterpret_cast<const int64_t *>(h_out_ + off_gst + 16);
  if (device_status() == MSA_OK) return false;
  *job = -1;
  for (int i = 0; i < nj; ++i)
    if (meta_[i].qbase == w[0]) *job = i;
  *tile = w[1];
  *missing = w[2];
  if (more)
    for (int q = 0; q < 4; ++q) more[q] = w[3 + q];
  return true;
}

void Launch::result(int i, LaunchResult *out) const {
  const int nj = (int)meta_.size();
  const int64_t off_len = a256((int64_t)nj * 8);
  const int64_t off_stat = off_len + a256((int64_t)nj * 8);
  const int64_t *scores = reinterpret_cast<const int64_t *>(h_out_);
  const int64_t *lens = reinterpret_cast<const int64_t *>(h_out_ + off_len);
  const int32_t *stats = reinterpret_cast<const int32_t *>(h_out_ + off_stat);
  out->k = meta_[i].k;
  out->cap = meta_[i].cap;
  out->status = launch_status_ != MSA_OK ? launch_status_ : stats[i];
  out->score = out->status == MSA_OK ? scores[i] : 0;
  out->aln_len = out->status == MSA_OK ? lens[i] : 0;
  const uint8_t *rows = reinterpret_cast<const uint8_t *>(h_out_ + meta_[i].aln_off);
  out->aln.assign(rows, rows + (size_t)meta_[i].k * meta_[i].cap);
}

void Launch::fill_result(int i, msa_result *out) const {
  const int nj = (int)meta_.size();
  const int64_t off_len = a256((int64_t)nj * 8);
  const int64_t off_stat = off_len + a256((int64_t)nj * 8);
  const int64_t *scores = reinterpret_cast<const int64_t *>(h_out_);
  const int64_t *lens = reinterpret_cast<const int64_t *>(h_out_ + off_len);
  const int32_t *stats = reinterpret_cast<const int32_t *>(h_out_ + off_stat);
  const int st = launch_status_ != MSA_OK ? launch_status_ : stats[i];
  out->status = st;
  out->score = st == MSA_OK ? scores[i] : 0;
  out->aln_len = st == MSA_OK ? lens[i] : 0;
  if (st == MSA_OK && out->aln && out->aln_len > 0) {
    const uint8_t *rows = reinterpret_cast<const uint8_t *>(h_out_ + meta_[i].aln_off);
    for (int r = 0; r < meta_[i].k; ++r)
      memcpy(out->aln + (int64_t)r * out->aln_cap, rows + (int64_t)r * meta_[i].cap,
             (size_t)out->aln_len);
  }
}

}  // namespace msa
