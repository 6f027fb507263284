// Compiled variants: row kernels with the real-input epilogue (forward,
// real == 1) or prologue (inverse, real == 2), one line of M = L points per
// real transform of 2L values.
#include "pass_kernels.h"

namespace tcfft {

#define ROWKR1(L_, R_, N_, RK_)                                                      \
  if (k.kind == K_ROW && k.L == L_ && k.R0 == R_ && k.NT == N_ && !k.tstore &&       \
      k.real == RK_ && k.C == 0) {                                                   \
    if (k.split) {                                                                   \
      out->single = (KernelFn)row_kernel<L_, R_, N_, true, false, RK_>;              \
      out->multi = (MultiFn)row_kernel_multi<L_, R_, N_, true, false, RK_>;          \
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
