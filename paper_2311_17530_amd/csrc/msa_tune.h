// msa_tune.h -- launch-configuration tuner: for each (GPU architecture, k,
// length bucket) the fill variant and workgroups per compute unit that a
// measured run found fastest.  Every configuration computes the same bytes;
// only the time differs.
#pragma once
#include <stdint.h>

namespace msa {

constexpr int kTunePlain = 0;  // plain path: k, bucket of the longest sequence
constexpr int kTuneBatch = 1;  // batched fill: k class, bucket 0

// variant (plain path): 0 the built-in rule, 1 the streaming k = 3 fill,
// 2 the tile fill.  wpc: workgroups per compute unit of the tile fill
// (plain) or of the persistent batched fill; 0 the built-in rule.
struct TuneChoice {
  int32_t variant = 0;
  int32_t wpc = 0;
};

// ceil(log2(max n_i + 1)): sequences within a factor of two share a bucket.
int length_bucket(const int32_t *n, int k);
// The stored choice for the current device's architecture (false: none).
bool tune_get(int kind, int k, int bucket, TuneChoice *c);
void tune_set(int kind, int k, int bucket, const TuneChoice &c);
void tune_clear();

}  // namespace msa
