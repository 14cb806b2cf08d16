// msa_server.cpp -- served path (placeholder).
#include <hip/hip_runtime.h>

#include "../../include/msa_dp.h"

extern "C" msa_server *msa_server_create(int64_t, int32_t, int32_t) { return nullptr; }
extern "C" int msa_server_submit(msa_server *, const msa_job *, uint64_t *) { return MSA_EDEVICE; }
extern "C" int msa_server_poll(msa_server *, uint64_t, msa_result *) { return MSA_EDEVICE; }
extern "C" int msa_server_wait(msa_server *, uint64_t, msa_result *, int64_t) { return MSA_EDEVICE; }
extern "C" void msa_server_destroy(msa_server *) {}
