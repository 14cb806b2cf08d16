// msa_server.cpp -- served path: a request loop with continuous batching.
//
// Jobs are submitted at any time.  A worker thread keeps up to `max_inflight`
// batched persistent launches in flight, each slot on a stream of its own;
// whenever a slot is free it admits the oldest queued jobs (of one k class)
// that fit the slot's share of the HBM budget, so requests that arrive while
// others run start as soon as a slot and its memory free up.  Small launches
// (the latency regime) overlap on the device.  A large launch (kLargeLaunch
// jobs or more, the saturated regime) runs alone: its stream waits for every
// launch in flight, and every later launch waits for it, through events, so
// the host still stages ahead.  Large persistent fills running side by side
// on several hardware queues had those queues preempted, and now and then a
// dependency wait of one of them timed out; one at a time they were also
// faster.  Finished results wait in a table until polled.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/msa_dp.h"
#include "msa_launch.h"

namespace msa {
int64_t default_budget();
}
using namespace msa;

namespace {

struct Pending {
  uint64_t ticket = 0;
  msa_job job{};
  std::vector<uint8_t> seqbuf;
  std::vector<int8_t> sub;
  int64_t bytes = 0;
  int64_t ntiles = 0;
  int retries = 0;  // launches re-run after a dependency-wait time-out
};

struct Done {
  int32_t status = MSA_OK;
  int64_t score = 0;
  int64_t aln_len = 0;
  int k = 0;
  int64_t cap = 0;
  std::vector<uint8_t> aln;
};

// Launches of at least this many jobs run alone on the device.
constexpr int kLargeLaunch = 32;

struct Slot {
  std::unique_ptr<Launch> launch;
  bool large = false;  // the launch in flight is a large one
  std::vector<uint64_t> tickets;
  std::vector<std::unique_ptr<Pending>> jobs;  // inputs stay alive while staged
};

}  // namespace

struct msa_server {
  std::mutex mu;
  std::condition_variable cv_work;  // worker wake-up
  std::condition_variable cv_done;  // results available
  int device = 0;
  int64_t budget = 0;
  int64_t slot_bytes = 0;
  int max_inflight = 1;
  int max_jobs = 256;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<std::unique_ptr<Pending>> queue;
  std::map<uint64_t, Done> done;
  std::map<uint64_t, int> running;  // ticket -> slot
  std::vector<Slot> slots;
  std::thread worker;
  int init_status = MSA_OK;
  // statistics: launches and jobs completed, and each launch's device
  // interval (ms after `ref`, recorded at creation) for the busy time
  hipEvent_t ref = nullptr;
  int64_t n_launches = 0, n_jobs = 0;
  // jobs that ended with a status other than MSA_OK, and the last such status
  int64_t n_failed = 0;
  int32_t last_failure = MSA_OK;
  // longest pause a launch's fill saw inside a dependency wait (its queue
  // not running), microseconds
  int64_t max_pause_us = 0;
  int n_timeouts = 0;  // time-outs reported on stderr so far
  int64_t n_rerun = 0;  // jobs queued again after their launch timed out
  // msa_server_debug_wait_limit: launches left with a short wait limit
  int64_t dbg_wait_ticks = 0;
  int dbg_launches = 0;
  std::vector<std::pair<float, float>> intervals;

  void run();
  bool admit(Slot &s, int free_slots);
  void collect(Slot &s);
  void note_failure(int32_t status, int64_t jobs, const char *where);
};

// Failed jobs are counted (msa_server_stats) and the first few failures are
// reported on stderr with where they arose, so that a failure seen under
// load can be told apart from the others.
void msa_server::note_failure(int32_t status, int64_t jobs, const char *where) {
  n_failed += jobs;
  last_failure = status;
  if (n_failed - jobs < 8)
    fprintf(stderr, "msa server: %lld job(s) ended with status %d (%s)\n", (long long)jobs,
            (int)status, where);
}

bool msa_server::admit(Slot &s, int free_slots) {
  // FIFO admission: the oldest job fixes the k class; later jobs of the same
  // class join while they fit the slot's arena and the launch's share of the
  // queue: the queued jobs split evenly over the free slots (at most
  // max_jobs each), so a short queue gives small launches that finish soon
  // and a burst spreads over every free slot instead of filling one.
  if (queue.empty()) return false;
  const int kc = kclass_of(queue.front()->job.k);
  const int64_t share = ((int64_t)queue.size() + free_slots - 1) / std::max(1, free_slots);
  const int limit = (int)std::min<int64_t>(max_jobs, std::max<int64_t>(1, share));
  std::vector<const msa_job *> grp;
  int64_t used = 0, tiles = 0;
  for (auto it = queue.begin(); it != queue.end() && (int)grp.size() < limit;) {
    Pending &p = **it;
    if (kclass_of(p.job.k) != kc) {
      ++it;
      continue;
    }
    const int64_t need =
        used + p.bytes + Launch::overhead_bytes((int)grp.size() + 1, tiles + p.ntiles);
    if (need > s.launch->capacity()) {
      if (grp.empty()) {  // cannot happen: oversized jobs are rejected at submit
        done[p.ticket].status = MSA_ENOMEM;
        it = queue.erase(it);
        cv_done.notify_all();
        continue;
      }
      break;
    }
    used += p.bytes;
    tiles += p.ntiles;
    grp.push_back(&p.job);
    s.tickets.push_back(p.ticket);
    s.jobs.push_back(std::move(*it));
    it = queue.erase(it);
  }
  if (grp.empty()) return false;
  // debug: the next dbg_launches launches take a short dependency-wait limit
  s.launch->set_wait_limit(dbg_launches > 0 ? dbg_wait_ticks : 0);
  if (dbg_launches > 0) --dbg_launches;
  // device order: a large launch after every launch in flight, any launch
  // after a large one in flight
  s.large = (int)grp.size() >= kLargeLaunch;
  std::vector<hipEvent_t> after;
  for (auto &o : slots)
    if (&o != &s && o.launch->busy() && (s.large || o.large)) after.push_back(o.launch->done_event());
  const int rc = s.launch->start(grp, after);
  for (uint64_t t : s.tickets) running[t] = 0;
  if (rc != MSA_OK) {
    note_failure(rc, (int64_t)s.tickets.size(), "launch set-up");
    for (uint64_t t : s.tickets) {
      done[t].status = rc;
      running.erase(t);
    }
    s.tickets.clear();
    s.jobs.clear();
    s.launch->release();
    cv_done.notify_all();
    return false;
  }
  return true;
}

void msa_server::collect(Slot &s) {
  s.launch->wait();
  float t0 = 0.f, t1 = 0.f;
  if (ref && s.launch->interval_ms(ref, &t0, &t1)) intervals.emplace_back(t0, t1);
  ++n_launches;
  max_pause_us = std::max(max_pause_us, s.launch->device_max_pause_us());
  int jb = -1;
  int64_t tile = 0, missing = 0, more[4] = {};
  const bool timed_out = s.launch->device_timeout(&jb, &tile, &missing, more);
  {
    if (timed_out && n_timeouts < 4) {
      ++n_timeouts;
      fprintf(stderr, "msa server: a launch of %zu jobs timed out in a dependency wait: job %d",
              s.tickets.size(), jb);
      if (jb >= 0 && jb < (int)s.jobs.size()) {
        const msa_job &j = s.jobs[jb]->job;
        fprintf(stderr, " (k = %d, lengths", j.k);
        for (int d = 0; d < j.k; ++d) fprintf(stderr, " %lld", (long long)j.lens[d]);
        fprintf(stderr, ")");
      }
      fprintf(stderr,
              ", tile %lld, missing predecessor dimensions 0x%llx (tile %lld, flag %lld), "
              "queue head %lld of %lld\n",
              (long long)tile, (unsigned long long)missing, (long long)more[0],
              (long long)more[1], (long long)more[2], (long long)more[3]);
    }
  }
  // A launch whose dependency wait timed out is re-run once: its jobs go back
  // to the front of the queue (the result of a re-run is the same exact
  // alignment); a job whose second launch times out too returns the status.
  std::vector<std::unique_ptr<Pending>> again;
  for (size_t i = 0; i < s.tickets.size(); ++i) {
    LaunchResult r;
    s.launch->result((int)i, &r);
    if (timed_out && r.status == MSA_EDEVICE && s.jobs[i]->retries == 0) {
      ++s.jobs[i]->retries;
      running.erase(s.tickets[i]);
      again.push_back(std::move(s.jobs[i]));
      continue;
    }
    Done &d = done[s.tickets[i]];
    d.status = r.status;
    if (r.status != MSA_OK)
      note_failure(r.status, 1,
                   s.launch->device_status() != MSA_OK ? "launch result: dependency wait timed out"
                                                       : "launch result: job status");
    d.score = r.score;
    d.aln_len = r.aln_len;
    d.k = r.k;
    d.cap = r.cap;
    d.aln.swap(r.aln);
    running.erase(s.tickets[i]);
  }
  n_jobs += (int64_t)(s.tickets.size() - again.size());
  n_rerun += (int64_t)again.size();
  for (auto it = again.rbegin(); it != again.rend(); ++it) queue.push_front(std::move(*it));
  s.tickets.clear();
  s.jobs.clear();
  s.launch->release();
  cv_done.notify_all();
}

void msa_server::run() {
  if (hipSetDevice(device) != hipSuccess) {
    std::lock_guard<std::mutex> lk(mu);
    init_status = MSA_EDEVICE;
    return;
  }
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    bool progress = false;
    for (auto &s : slots) {
      if (s.launch->busy() && s.launch->ready()) {
        collect(s);
        progress = true;
      }
    }
    int free_slots = 0;
    for (auto &s : slots) free_slots += s.launch->busy() ? 0 : 1;
    for (auto &s : slots) {
      if (!s.launch->busy() && !queue.empty() && !stop) {
        progress |= admit(s, free_slots);
        --free_slots;
      }
    }
    bool any_busy = false;
    for (auto &s : slots) any_busy |= s.launch->busy();
    if (stop && !any_busy) break;
    if (!progress) {
      if (any_busy)  // poll the device for finished launches
        cv_work.wait_for(lk, std::chrono::microseconds(50));
      else
        cv_work.wait(lk, [&] { return stop || !queue.empty(); });
    }
  }
  // shutting down: jobs never admitted are reported as such
  for (auto &p : queue) done[p->ticket].status = MSA_ESHUTDOWN;
  queue.clear();
  cv_done.notify_all();
}

extern "C" msa_server *msa_server_create(int64_t hbm_budget_bytes, int32_t max_inflight,
                                         int32_t max_jobs_per_launch) {
  if (max_inflight < 1 || max_inflight > 16 || max_jobs_per_launch < 1) return nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  std::unique_ptr<msa_server> s(new msa_server());
  s->device = dev;
  s->budget = hbm_budget_bytes > 0 ? hbm_budget_bytes : default_budget();
  s->max_inflight = max_inflight;
  s->max_jobs = max_jobs_per_launch;
  s->slot_bytes = s->budget / max_inflight;
  s->slots.resize(max_inflight);
  for (auto &sl : s->slots) {
    sl.launch.reset(new Launch());
    if (sl.launch->init(s->slot_bytes) != MSA_OK) return nullptr;
  }
  if (hipEventCreate(&s->ref) != hipSuccess || hipEventRecord(s->ref, nullptr) != hipSuccess ||
      hipEventSynchronize(s->ref) != hipSuccess)
    return nullptr;
  s->worker = std::thread([p = s.get()] { p->run(); });
  return s.release();
}

extern "C" int msa_server_submit(msa_server *srv, const msa_job *job, uint64_t *ticket) {
  if (!srv || !job || !ticket) return MSA_EINVAL;
  int rc = validate_job(*job);
  if (rc) return rc;
  std::unique_ptr<Pending> p(new Pending());
  int64_t total = 0;
  for (int d = 0; d < job->k; ++d) total += job->lens[d];
  p->seqbuf.resize((size_t)std::max<int64_t>(total, 1));
  p->sub.assign(job->submat, job->submat + (size_t)job->alpha * job->alpha);
  p->job = *job;
  int64_t off = 0;
  for (int d = 0; d < job->k; ++d) {
    if (job->lens[d] > 0) std::memcpy(p->seqbuf.data() + off, job->seqs[d], (size_t)job->lens[d]);
    p->job.seqs[d] = p->seqbuf.data() + off;
    off += job->lens[d];
  }
  p->job.submat = p->sub.data();
  p->bytes = job_arena_bytes(p->job);
  Plan pl;
  make_plan(job->lens, job->k, &pl);
  p->ntiles = pl.ntiles;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->stop) return MSA_ESHUTDOWN;
  if (srv->init_status != MSA_OK) return srv->init_status;
  if (p->bytes + Launch::overhead_bytes(1, p->ntiles) > srv->slot_bytes) return MSA_ENOMEM;
  p->ticket = srv->next_ticket++;
  *ticket = p->ticket;
  srv->queue.push_back(std::move(p));
  srv->cv_work.notify_all();
  return MSA_OK;
}

static int take_result(msa_server *srv, uint64_t ticket, msa_result *out) {
  auto it = srv->done.find(ticket);
  if (it == srv->done.end()) return MSA_EAGAIN;
  Done &d = it->second;
  out->status = d.status;
  out->score = d.status == MSA_OK ? d.score : 0;
  out->aln_len = d.status == MSA_OK ? d.aln_len : 0;
  if (d.status == MSA_OK && d.aln_len > 0) {
    if (!out->aln || out->aln_cap < d.aln_len) {
      out->status = MSA_EINVAL;
      srv->done.erase(it);
      return MSA_EINVAL;
    }
    for (int r = 0; r < d.k; ++r)
      std::memcpy(out->aln + (int64_t)r * out->aln_cap, d.aln.data() + (int64_t)r * d.cap,
                  (size_t)d.aln_len);
  }
  const int st = d.status;
  srv->done.erase(it);
  return st;
}

static bool known_ticket(msa_server *srv, uint64_t ticket) {
  if (srv->done.count(ticket) || srv->running.count(ticket)) return true;
  for (auto &p : srv->queue)
    if (p->ticket == ticket) return true;
  return false;
}

extern "C" int msa_server_poll(msa_server *srv, uint64_t ticket, msa_result *out) {
  if (!srv || !out) return MSA_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (!known_ticket(srv, ticket)) return MSA_EINVAL;
  return take_result(srv, ticket, out);
}

extern "C" int msa_server_wait(msa_server *srv, uint64_t ticket, msa_result *out,
                               int64_t timeout_us) {
  if (!srv || !out) return MSA_EINVAL;
  std::unique_lock<std::mutex> lk(srv->mu);
  if (!known_ticket(srv, ticket)) return MSA_EINVAL;
  auto ready = [&] { return srv->done.count(ticket) > 0; };
  if (timeout_us < 0)
    srv->cv_done.wait(lk, ready);
  else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
    return MSA_EAGAIN;
  return take_result(srv, ticket, out);
}

extern "C" int msa_server_stats(msa_server *srv, int64_t *out, int32_t n) {
  if (!srv || !out || n < 1) return MSA_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  // union of the launches' device intervals: time with at least one launch
  // of this server on the device
  std::vector<std::pair<float, float>> iv = srv->intervals;
  std::sort(iv.begin(), iv.end());
  double busy = 0.0, lo = 0.0, hi = 0.0, first = 0.0, last = 0.0;
  bool open = false;
  for (auto &x : iv) {
    if (!open) {
      lo = x.first;
      hi = x.second;
      first = x.first;
      open = true;
    } else if (x.first > hi) {
      busy += hi - lo;
      lo = x.first;
      hi = x.second;
    } else if (x.second > hi) {
      hi = x.second;
    }
    last = std::max(last, (double)x.second);
  }
  if (open) busy += hi - lo;
  const int64_t v[9] = {srv->n_launches, srv->n_jobs, (int64_t)(busy * 1000.0),
                        open ? (int64_t)((last - first) * 1000.0) : 0,
                        (int64_t)srv->queue.size(), srv->n_failed, srv->last_failure,
                        srv->max_pause_us, srv->n_rerun};
  for (int i = 0; i < n && i < 9; ++i) out[i] = v[i];
  return MSA_OK;
}

extern "C" int msa_server_debug_wait_limit(msa_server *srv, int64_t ticks, int32_t launches) {
  if (!srv || ticks < 1 || launches < 0) return MSA_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  srv->dbg_wait_ticks = ticks;
  srv->dbg_launches = launches;
  return MSA_OK;
}

extern "C" void msa_server_destroy(msa_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    srv->cv_work.notify_all();
  }
  if (srv->worker.joinable()) srv->worker.join();
  if (srv->ref) (void)hipEventDestroy(srv->ref);
  delete srv;
}
