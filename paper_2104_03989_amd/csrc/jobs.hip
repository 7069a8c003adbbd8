// Job server (not yet implemented: every submit reports ADR_E_UNIMPL).
#include <stdio.h>

#include "jobs.h"

namespace adr {

struct JobServer {
  int device;
};

JobServer* jobs_create(adr_ctx*, int device, uint64_t) { return new JobServer{device}; }
void jobs_destroy(JobServer* s) { delete s; }
adr_status jobs_submit(JobServer*, const adr_job_desc*, uint64_t*, char* msg, size_t n) {
  snprintf(msg, n, "job server not implemented");
  return ADR_E_UNIMPL;
}
adr_status jobs_poll(JobServer*, uint64_t, adr_job_status*, adr_job_result*, char* msg, size_t n) {
  snprintf(msg, n, "unknown job");
  return ADR_E_NOTFOUND;
}

}  // namespace adr
