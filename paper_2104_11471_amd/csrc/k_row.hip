// Compiled variants: row kernels.
#include "pass_kernels.h"

namespace tcfft {

#define ROWK(L_, R_, N_)                                                             \
  if (k.kind == K_ROW && k.L == L_ && k.R0 == R_ && k.NT == N_ && !k.tstore && !k.real &&  \
      k.C == 0) {                                                                    \
    if (k.split) {                                                                   \
      out->single = (KernelFn)row_kernel<L_, R_, N_, true>;                          \
      out->multi = (MultiFn)row_kernel_multi<L_, R_, N_, true>;                      \
      out->persistent = RowPipe<RowGeom<L_, R_, N_>, true>::value;                   \
    } else {                                                                        \
      out->single = (KernelFn)row_kernel<L_, R_, N_, false>;                         \
      out->multi = (MultiFn)row_kernel_multi<L_, R_, N_, false>;                     \
      out->persistent = RowPipe<RowGeom<L_, R_, N_>, false>::value;                  \
    }                                                                                \
    return true;                                                                     \
  }

// 8192 points per workgroup (KernelKey.C = 8192; FP16 and split, 256 threads).
#define ROWKH(L_, R_)                                                                \
  if (k.kind == K_ROW && k.L == L_ && k.R0 == R_ && k.NT == 256 && k.C == 8192 &&     \
      !k.tstore && !k.real) {                                                        \
    if (k.split) {                                                                   \
      out->single = (KernelFn)row_kernel<L_, R_, 256, true, false, 0, 8192>;         \
      out->multi = (MultiFn)row_kernel_multi<L_, R_, 256, true, false, 0, 8192>;     \
    } else {                                                                        \
      out->single = (KernelFn)row_kernel<L_, R_, 256, false, false, 0, 8192>;        \
      out->multi = (MultiFn)row_kernel_multi<L_, R_, 256, false, false, 0, 8192>;    \
    }                                                                                \
    out->persistent = false;                                                         \
    return true;                                                                     \
  }

// Transposed-store variants (second pass of a four-step transform).
#define ROWKT(L_, R_, N_)                                                            \
  if (k.kind == K_ROW && k.L == L_ && k.R0 == R_ && k.NT == N_ && k.tstore && !k.real &&   \
      k.C == 0) {                                                                    \
    if (k.split) {                                                                   \
      out->single = (KernelFn)row_kernel<L_, R_, N_, true, true>;                    \
      out->multi = (MultiFn)row_kernel_multi<L_, R_, N_, true, true>;                \
    } else {                                                                        \
      out->single = (KernelFn)row_kernel<L_, R_, N_, false, true>;                   \
      out->multi = (MultiFn)row_kernel_multi<L_, R_, N_, false, true>;               \
    }                                                                                \
    out->persistent = false;                                                         \
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
    }                                                                                \
    return true;                                                                     \
  }
#define COLK(L_, R_, C_, N_)                                                         \
  COLK4(L_, R_, C_, N_, false, false) COLK4(L_, R_, C_, N_, true, false)             \
  COLK4(L_, R_, C_, N_, true, true)

bool find_row_kernels(const KernelKey& k, KernelFns* out) {
  ROWK(16, 1, 256)
  ROWK(32, 2, 256)
  ROWK(64, 4, 256)
  ROWK(128, 8, 256)
  ROWK(256, 1, 256)
  ROWK(512, 2, 256)
  ROWK(1024, 4, 256)
  ROWK(2048, 8, 256)
  ROWK(4096, 1, 256)
  ROWK(8192, 2, 256)
  ROWK(16384, 4, 256)
  ROWK(8192, 2, 512)
  ROWK(16384, 4, 512)
  ROWKH(256, 1)
  ROWKH(512, 2)
  ROWKH(1024, 4)
  ROWKH(2048, 8)
  ROWKH(4096, 1)
  ROWKH(8192, 2)
  ROWKT(256, 1, 256)
  ROWKT(512, 2, 256)
  ROWKT(1024, 4, 256)
  return false;
}

}  // namespace tcfft
