// Job server of the C ABI: whole simplification jobs admitted by HBM budget,
// kept resident on the device and stepped by a server thread.
#pragma once

#include "adr.h"

namespace adr {

struct JobServer;

JobServer* jobs_create(adr_ctx* ctx, int device, uint64_t budget);
void jobs_destroy(JobServer* s);
adr_status jobs_submit(JobServer* s, const adr_job_desc* d, uint64_t* id, char* msg, size_t n);
adr_status jobs_poll(JobServer* s, uint64_t id, adr_job_status* st, adr_job_result* out, char* msg,
                     size_t n);

}  // namespace adr
