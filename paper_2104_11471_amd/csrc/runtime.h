// Internal runtime interface shared by the C ABI (tcfft.cpp) and the serving
// scheduler (serve.cpp).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>

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

// Instantiated graphs of grouped launches, keyed by the sequence of kernel
// variants of a batch (owned by one stream / descriptor arena).
struct GraphCache {
  std::map<std::string, void*> execs;  // hipGraphExec_t
  std::map<std::string, int> seen;     // batches seen per sequence before capturing
  int capture_after = 3;               // capture a sequence on its 3rd occurrence
  ~GraphCache();
};

}  // namespace tcfft

// Grouped mixed-size launch of `njobs` jobs on stream `s` (see tcfft_exec_many).
// With desc_arena (device, arena_cap bytes, owned by this stream) the
// descriptor tables go there instead of a stream-ordered allocation; with
// graphs as well, the launch sequence is captured once per variant sequence
// and replayed as a HIP graph.
// arg_upload: the tables are written by kernels from their arguments instead
// of a copy from pinned host memory (no host or device allocation).
tcfft_status tcfft_internal_exec_jobs(const tcfft::Job* jobs, int njobs, hipStream_t s,
                                      void* desc_arena, size_t arena_cap,
                                      tcfft::GraphCache* graphs, bool arg_upload = false);
// Descriptor arena bytes that always suffice for a batch of max_jobs jobs.
size_t tcfft_internal_desc_bytes(int max_jobs);
size_t tcfft_internal_plan_ws_bytes(const tcfft_plan_s* p, int64_t batch);
int64_t tcfft_internal_plan_batch(const tcfft_plan_s* p);
int64_t tcfft_internal_plan_points(const tcfft_plan_s* p);
int tcfft_internal_plan_prec(const tcfft_plan_s* p);
