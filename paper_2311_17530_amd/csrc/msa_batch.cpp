// msa_batch.cpp -- batched path (placeholder until the persistent batch kernel lands).
#include <hip/hip_runtime.h>

#include "../../include/msa_dp.h"

extern "C" int msa_dp_align_batch(const msa_job *jobs, int32_t njobs, msa_result *results,
                                  int64_t hbm_budget_bytes) {
  (void)jobs; (void)njobs; (void)results; (void)hbm_budget_bytes;
  return MSA_EDEVICE;
}
