// msa_launch.h -- one batched persistent launch: a device arena holding many
// jobs (descriptors, sequences, tile queue, flags, face planes, direction
// blocks, outputs), staged from host jobs and run asynchronously on a stream.
// Used by the batched call and by the server.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/msa_dp.h"
#include "msa_plan.h"

namespace msa {

// Validation of one host job; returns MSA_OK or a status.
int validate_job(const msa_job &j, int64_t aln_cap_needed_check = -1);

// k class of the batched kernels: 0 for k = 2..4, 1 for k = 5, 2 for k = 6,
// 3 for k = 7..8.  A batched kernel takes the registers of its largest k, so
// k = 5 and 6 get kernels of their own (k = 5 alone: 3 workgroups per CU
// instead of 1 beside k = 8).
inline int kclass_of(int k) { return k <= 4 ? 0 : k == 5 ? 1 : k == 6 ? 2 : 3; }

// Device bytes one job needs inside a launch arena.
int64_t job_arena_bytes(const msa_job &j);

struct LaunchResult {
  int32_t status = MSA_OK;
  int64_t score = 0;
  int64_t aln_len = 0;
  std::vector<uint8_t> aln;  // k rows of `cap` bytes
  int64_t cap = 0;
  int k = 0;
};

class Launch {
 public:
  Launch() = default;
  ~Launch();
  Launch(const Launch &) = delete;
  Launch &operator=(const Launch &) = delete;

  // Arena and stream set-up on the current device; arena of `bytes`.  With
  // `shared`, the launch runs on that stream (owned by the caller) instead of
  // one of its own.
  int init(int64_t bytes, hipStream_t shared = nullptr);
  int64_t capacity() const { return cap_; }

  // Fixed bytes of a launch besides the jobs (control block, tables, queue).
  static int64_t overhead_bytes(int njobs, int64_t ntiles_total);

  // Stages the given valid jobs (all of one k class) and enqueues the launch,
  // on the device after the events in `after` (other launches' done events).
  // Returns MSA_OK, MSA_ENOMEM if they do not fit, or MSA_EDEVICE.
  int start(const std::vector<const msa_job *> &jobs,
            const std::vector<hipEvent_t> &after = {});
  // Recorded after the launch's output copy (a later launch may wait on it).
  hipEvent_t done_event() const { return done_; }
  bool busy() const { return busy_; }
  bool ready();            // launch finished (non-blocking)
  int wait();              // block until finished
  // After ready()/wait(): result of the i-th staged job.
  void result(int i, LaunchResult *out) const;
  void fill_result(int i, msa_result *out) const;
  // After ready()/wait(): the launch-wide device status (MSA_EDEVICE when a
  // dependency wait of the fill timed out; a job's own status can also be
  // MSA_EDEVICE when its traceback met inconsistent decisions).
  int32_t device_status() const;
  // After ready()/wait(): the longest pause (microseconds) a dependency wait
  // of the fill saw between two of its checks, that is a time the fill did
  // not run (its queue preempted); such pauses do not count towards the
  // wait's time-out.  0 when there was none.
  int64_t device_max_pause_us() const;
  // After ready()/wait() of a launch whose device status is not MSA_OK: the
  // first dependency wait that timed out, as the index of its job among the
  // staged ones (-1 if not found), its tile and the mask of the predecessor
  // dimensions it still missed; `more` (if not null) receives the first
  // missing predecessor tile, the value its flag held, the queue head then and
  // the queue length.  False when the launch did not time out.
  bool device_timeout(int *job, int64_t *tile, int64_t *missing,
                      int64_t more[4] = nullptr) const;
  int njobs() const { return (int)meta_.size(); }
  // After ready()/wait(): the launch's device interval (from its first copy
  // to its last) in milliseconds after `ref`, an event recorded earlier on
  // the same device.  False if the events cannot be read.
  bool interval_ms(hipEvent_t ref, float *t0, float *t1) const;
  void release() { busy_ = false; meta_.clear(); }
  // Dependency-wait time-out of the next launches, in 100 MHz ticks (0: the
  // batched default, kBatchWaitTicks); a host-side way to exercise time-out
  // handling.
  void set_wait_limit(int64_t ticks) { wait_limit_ = ticks; }

 private:
  struct Meta {
    int k = 0;
    int64_t cap = 0;
    int64_t aln_off = 0;  // offset of the rows in the host output image
    int64_t qbase = 0;    // first tile of the job in the launch's numbering
  };
  int device_ = -1;
  hipStream_t stream_ = nullptr;
  bool own_stream_ = true;
  hipEvent_t start_ = nullptr;  // before the input copy (timing)
  hipEvent_t done_ = nullptr;   // after the output copy (timing)
  char *d_ = nullptr;
  int64_t cap_ = 0;
  char *h_in_ = nullptr;  // pinned staging (inputs)
  int64_t h_in_cap_ = 0;
  char *h_out_ = nullptr;  // pinned outputs
  int64_t h_out_cap_ = 0;
  int64_t out_bytes_ = 0;
  int64_t out_off_ = 0;
  std::vector<Meta> meta_;
  bool busy_ = false;
  int launch_status_ = MSA_OK;
  int64_t wait_limit_ = 0;
  // The launch sequence of each k class, captured once on this arena (its
  // arguments are the arena's fixed batch descriptor and control block) and
  // replayed for every batch; dropped when the arena is reallocated.
  hipGraphExec_t graph_[4] = {};
  int graph_grid_[4] = {};  // the fill grid each graph was captured with
  bool graph_failed_[4] = {};
  int ensure_host(int64_t in_bytes, int64_t out_bytes);
  int batch_grid(int kc) const;
  int ensure_graph(int kc, int grid);
  void drop_graphs();
};

}  // namespace msa
