// Compiled variants: column kernels, L <= 128.
#include "pass_kernels.h"

namespace tcfft {

#define ROWK(L_, R_, N_)                                                             \
  if (k.kind == K_ROW && k.L == L_ && k.R0 == R_ && k.NT == N_) {                    \
    if (k.split) {                                                                   \
      out->single = (KernelFn)row_kernel<L_, R_, N_, true>;                          \
      out->multi = (MultiFn)row_kernel_multi<L_, R_, N_, true>;                      \
    } else {                                                                        \
      out->single = (KernelFn)row_kernel<L_, R_, N_, false>;                         \
      out->multi = (MultiFn)row_kernel_multi<L_, R_, N_, false>;                     \
    }                                                                                \
    return true;                                                                     \
  }

#define COLK4(L_, R_, C_, N_, X_, T_)                                                \
  if (k.kind == K_COL && k.L == L_ && k.R0 == R_ && k.C == C_ && k.NT == N_ &&       \
      k.xtw == X_ && k.tstore == T_) {                                               \
    if (k.split) {                                                                   \
      out->single = (KernelFn)col_kernel<L_, R_, C_, N_, true, X_, T_>;              \
      out->multi = (MultiFn)col_kernel_multi<L_, R_, C_, N_, true, X_, T_>;          \
    } else {                                                                        \
      out->single = (KernelFn)col_kernel<L_, R_, C_, N_, false, X_, T_>;             \
      out->multi = (MultiFn)col_kernel_multi<L_, R_, C_, N_, false, X_, T_>;         \
      out->persistent = ColPipe<ColGeom<L_, R_, C_, N_>, false, T_>::value;          \
    }                                                                                \
    return true;                                                                     \
  }
#define COLK(L_, R_, C_, N_)                                                         \
  COLK4(L_, R_, C_, N_, false, false) COLK4(L_, R_, C_, N_, true, false)             \
  COLK4(L_, R_, C_, N_, true, true)

bool find_col_kernels_small(const KernelKey& k, KernelFns* out) {
  COLK(16, 1, 64, 64)
  COLK(32, 2, 64, 128)
  COLK(64, 4, 64, 256)
  COLK(128, 8, 64, 256)
  COLK(16, 1, 16, 64)
  COLK(32, 2, 16, 64)
  COLK(64, 4, 16, 64)
  COLK(128, 8, 16, 128)
  COLK(16, 1, 32, 64)
  COLK(32, 2, 32, 64)
  COLK(64, 4, 32, 128)
  COLK(128, 8, 32, 256)
  return false;
}

}  // namespace tcfft
