// msa_static.hip -- msa_dp_align_static: the plain path (fill + traceback)
// on a workspace that lives in a file-scope device array, for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The array `scratch` holds one workspace of the plain path (control block,
// substitution matrix, column schedule, completion flags, traceback path,
// face planes, direction blocks), laid out by make_plan exactly as a caller's
// workspace would be.  Its set-up, which msa_dp_prepare does with host copies,
// is done here by one kernel whose inputs come by value in its arguments, so
// a call issues kernels only: no allocation, no host-to-device copy, no
// memset.  Each device the library runs on holds its own copy of the array
// (kStaticScratchBytes) until the process ends; every call on a device shares
// it, so calls that overlap on one device (different streams, or threads
// without ordering) race and must be serialised by the caller.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>

#include "../../include/msa_dp.h"
#include "msa_plan.h"
#include "msa_runtime.h"

namespace msa {

constexpr int64_t kStaticScratchBytes = (int64_t)32 << 20;  // 32 MiB per device
constexpr int kStaticSubMax = 32;                          // alpha <= 32 (by value)
constexpr int kStaticWaveTable = 8192;                     // (k + 1) * waves ints

static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

namespace {

struct StaticArgs {
  int32_t alpha, gap;
  int64_t lo;                              // closed-form score floor
  int8_t sub[kStaticSubMax * kStaticSubMax];
};

std::mutex g_static_mu;
void *g_static_ptr[64] = {};  // device address of `scratch`, per device

// The address of this device's copy of `scratch` (looked up once per device
// with that device current); nullptr on failure.
void *static_ptr(int dev) {
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_static_ptr[dev] = ptr;
  }
  return g_static_ptr[dev];
}

}  // namespace

// Set-up of the workspace at `ws` (one workgroup): control block, matrix,
// zeroed completion flags, and the column schedule -- the tile columns along
// dimension 0 (c_0 = 0 tiles, index t < ncols) in order of their wave
// w = c_1 + ... + c_{k-1}, ties by t, the order make_column_order writes.
// wc[d][s] counts the tuples (c_d .. c_{k-1}) with sum s; a column's slot is
// the number of columns of smaller wave plus its rank among its wave's
// columns in lexicographic order of (c_1 .. c_{k-1}).
__global__ __launch_bounds__(256) void static_setup_kernel(JobDev jd, Ctrl *ctrl, uint8_t *sub,
                                                           int32_t *flags, int32_t *corder,
                                                           StaticArgs a) {
  __shared__ int32_t wc[kStaticWaveTable];
  __shared__ int64_t wbase_s[kStaticWaveTable / 3];
  const int tid = threadIdx.x;
  const int k = jd.k;
  const int nw = jd.nwaves;
  if (tid == 0) {
    Ctrl c;
    memset(&c, 0, sizeof(c));
    c.epoch = 1;
    c.alpha = a.alpha;
    c.gap = a.gap;
    c.best = INT64_MIN;
    c.lo = a.lo;
    *ctrl = c;
  }
  for (int e = tid; e < a.alpha * a.alpha; e += blockDim.x) sub[e] = (uint8_t)a.sub[e];
  for (int64_t t = tid; t < jd.ntiles; t += blockDim.x) flags[t] = 0;
  if (tid == 0) {
    for (int s = 0; s < nw; ++s) wc[k * nw + s] = s == 0;
    for (int d = k - 1; d >= 1; --d)
      for (int s = 0; s < nw; ++s) {
        int acc = 0;
        for (int c = 0; c < jd.P[d] && c <= s; ++c) acc += wc[(d + 1) * nw + s - c];
        wc[d * nw + s] = acc;
      }
    int64_t acc = 0;
    for (int s = 0; s < nw; ++s) {
      wbase_s[s] = acc;
      acc += wc[1 * nw + s];
    }
  }
  __syncthreads();
  for (int t = tid; t < jd.ncols; t += blockDim.x) {
    int c[kMaxK];
    int w = 0;
    for (int d = 1; d < k; ++d) {
      c[d] = (t / jd.tstride[d]) % jd.P[d];
      w += c[d];
    }
    int64_t rank = 0;
    int s = w;
    for (int d = 1; d < k - 1; ++d) {
      for (int cc = 0; cc < c[d]; ++cc)
        if (s - cc >= 0) rank += wc[(d + 1) * nw + (s - cc)];
      s -= c[d];
    }
    corder[wbase_s[w] + rank] = t;
  }
}

// Clears `n` int32 words (the streaming k = 3 fill's exchange regions: tag 0
// is never a launch's tag).
__global__ __launch_bounds__(256) void static_zero_kernel(int32_t *p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

}  // namespace msa

using namespace msa;

extern "C" int msa_dp_align_static(const uint8_t *d_seqs, const int32_t *lens, int32_t k,
                                   const int8_t *submat, int32_t alpha, int32_t gap,
                                   int64_t *d_score, uint8_t *d_aln, int64_t aln_cap,
                                   int64_t *d_aln_len, int32_t *d_status, void *hip_stream) {
  if (!lens || k < 2 || k > MSA_MAX_K || !submat || !d_score || !d_aln_len || !d_status)
    return MSA_EINVAL;
  for (int i = 0; i < k; ++i)
    if (lens[i] < 0) return MSA_EINVAL;
  if (alpha < 1 || alpha > kStaticSubMax) return MSA_EINVAL;
  Plan p;
  int rc = make_plan(lens, k, &p);
  if (rc) return rc;
  if (aln_cap < p.total_len || (p.total_len > 0 && (!d_aln || !d_seqs))) return MSA_EINVAL;
  rc = check_scoring_mode(lens, k, submat, alpha, gap, 0u);
  if (rc) return rc;
  // the workspace must fit the static array, and the wave tables the set-up
  // kernel's LDS
  if (p.bytes > kStaticScratchBytes || (int64_t)(k + 1) * p.nwaves > kStaticWaveTable ||
      p.nwaves > kStaticWaveTable / 3)
    return MSA_ENOMEM;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return MSA_EDEVICE;
  char *ws = static_cast<char *>(static_ptr(dev));
  if (!ws) return MSA_EDEVICE;
  StaticArgs a;
  memset(&a, 0, sizeof(a));
  a.alpha = alpha;
  a.gap = gap;
  int64_t lo = 0, hi = 0;
  if (score_bounds(lens, k, submat, alpha, gap, &lo, &hi) != 0) return MSA_EINVAL;
  a.lo = lo;
  memcpy(a.sub, submat, (size_t)alpha * alpha);
  JobDev jd;
  fill_jobdev(p, ws, alpha, gap, &jd);
  hipStream_t s = (hipStream_t)hip_stream;
  launch_begin();
  hipLaunchKernelGGL(static_setup_kernel, dim3(1), dim3(256), 0, s, jd,
                     reinterpret_cast<Ctrl *>(ws + p.off_ctrl),
                     reinterpret_cast<uint8_t *>(ws + p.off_sub),
                     reinterpret_cast<int32_t *>(ws + p.off_flags),
                     reinterpret_cast<int32_t *>(ws + p.off_corder), a);
  if (k == 3) {
    const int64_t words = p.x_bytes / 4;
    hipLaunchKernelGGL(static_zero_kernel, dim3((unsigned)std::min<int64_t>(1024, words / 256 + 1)),
                       dim3(256), 0, s, reinterpret_cast<int32_t *>(ws + p.off_x0), words);
  }
  if (launch_end() != 0) return MSA_EDEVICE;
  return run_plain_set_up(p, ws, alpha, d_seqs, d_score, d_aln, aln_cap, d_aln_len, d_status, s);
}
