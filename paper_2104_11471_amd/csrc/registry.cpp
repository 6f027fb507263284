// Variant registry and per-variant sizes.
#include "kernels.h"

namespace tcfft {

bool find_kernels(const KernelKey& k, KernelFns* out) {
  return find_row_kernels(k, out) || find_col_kernels_small(k, out) ||
         find_col_kernels_256(k, out) || find_col_kernels_large(k, out) ||
         find_big_kernels(k, out) || find_real_row_kernels(k, out) || find_plane_kernels(k, out);
}

KernelFn find_kernel(const KernelKey& k) {
  KernelFns f;
  return find_kernels(k, &f) ? f.single : nullptr;
}

size_t kernel_lds_bytes(const KernelKey& k) {
  if (k.kind == K_BIG) return 16384 * 4;  // 4 sub-transforms of 4096 at a time
  const int64_t pts = kernel_points_per_wg(k);
  return (size_t)pts * 4 * (k.split ? 2 : 1);
}

int64_t kernel_points_per_wg(const KernelKey& k) {
  if (k.kind == K_ROW) {
    const int64_t wgp = k.C > 0 ? k.C : 16384;  // C: points per workgroup of a row pass
    return k.L >= wgp ? k.L : wgp;
  }
  if (k.kind == K_PLANE) return 16384;
  if (k.kind == K_BIG) return k.L;
  return (int64_t)k.L * k.C;
}

}  // namespace tcfft
