// Compiled variants: row kernels with the real-input epilogue (forward,
// real == 1) or prologue (inverse, real == 2), one line of M = L points per
// real transform of 2L values.
#include "pass_kernels.h"

namespace tcfft {

// Grouped launch of the split real variants: one tile per workgroup, the grid
// being the group's tile count.  Inside the persistent loop of
// row_kernel_multi these spilled (44-328 bytes per lane: the split last stage
// holds 128 result registers across the epilogue's barrier, on top of the
// loop's state).
template <int L, int R0, int NT, int RK>
__global__ __launch_bounds__(NT, 1) void row_kernel_multi_one(const GroupHdr* __restrict__ hdr) {
  extern __shared__ uint32_t lds[];
  CGroupHdr* h = (CGroupHdr*)hdr;
  CKParams* jobs = (CKParams*)h->jobs;
  CInt64* prefix = (CInt64*)h->prefix;
  const int njobs = (int)h->njobs;
  const int64_t total = njobs > 0 ? prefix[njobs] : 0;
  const int64_t w = blockIdx.x;
  if (w >= total) return;
  const int j = find_job(prefix, njobs, w);
  const KParams kp = load_job(jobs, j);
  row_body<L, R0, NT, true, false, RK>(kp, w - prefix[j], lds);
}

#define ROWKR1(L_, R_, N_, RK_)                                                      \
  if (k.kind == K_ROW && k.L == L_ && k.R0 == R_ && k.NT == N_ && !k.tstore &&       \
      k.real == RK_ && k.C == 0) {                                                   \
    if (k.split) {                                                                   \
      out->single = (KernelFn)row_kernel<L_, R_, N_, true, false, RK_>;              \
      out->multi = (MultiFn)row_kernel_multi_one<L_, R_, N_, RK_>;                   \
      out->multi_one = true;                                                         \
    } else {                                                                        \
      out->single = (KernelFn)row_kernel<L_, R_, N_, false, false, RK_>;             \
      out->multi = (MultiFn)row_kernel_multi<L_, R_, N_, false, false, RK_>;         \
    }                                                                                \
    out->persistent = false;                                                         \
    return true;                                                                     \
  }
#define ROWKR(L_, R_, N_) ROWKR1(L_, R_, N_, 1) ROWKR1(L_, R_, N_, 2)

bool find_real_row_kernels(const KernelKey& k, KernelFns* out) {
  ROWKR(64, 4, 256)
  ROWKR(128, 8, 256)
  ROWKR(256, 1, 256)
  ROWKR(512, 2, 256)
  ROWKR(1024, 4, 256)
  ROWKR(2048, 8, 256)
  ROWKR(4096, 1, 256)
  ROWKR(8192, 2, 256)
  ROWKR(16384, 4, 256)
  return false;
}

}  // namespace tcfft
