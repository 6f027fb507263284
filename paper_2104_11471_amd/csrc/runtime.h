// Internal runtime interface shared by the C ABI (tcfft.cpp) and the serving
// scheduler (serve.cpp).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tcfft.h"

namespace tcfft {

// One transform job: `batch` transforms (<= the plan's batch) of plan's size
// and precision, read from `in`, written to `out`, with workspace `ws` (at
// least tcfft_internal_plan_ws_bytes(plan, batch) bytes; may be null when
// that is 0).
struct Job {
  tcfft_plan plan;
  const void* in;
  void* out;
  int64_t batch;
  void* ws;
};

}  // namespace tcfft

// Grouped mixed-size launch of `njobs` jobs on stream `s` (see tcfft_exec_many).
tcfft_status tcfft_internal_exec_jobs(const tcfft::Job* jobs, int njobs, hipStream_t s);
size_t tcfft_internal_plan_ws_bytes(const tcfft_plan_s* p, int64_t batch);
int64_t tcfft_internal_plan_batch(const tcfft_plan_s* p);
int64_t tcfft_internal_plan_points(const tcfft_plan_s* p);
int tcfft_internal_plan_prec(const tcfft_plan_s* p);
