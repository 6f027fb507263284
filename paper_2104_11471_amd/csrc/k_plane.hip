// Plane pass kernels of a 3D (or 2D 16384-point) transform; the pass itself
// is described in plane_body.h.
#include "plane_body.h"

namespace tcfft {

template <int NZ, int R0Z, int NY, int R0Y, int NT, bool SPLIT>
__global__ __launch_bounds__(NT) void plane_kernel(KParams kp) {
  extern __shared__ uint32_t lds[];
  plane_body<NZ, R0Z, NY, R0Y, NT, SPLIT>(kp, blockIdx.x, lds);
}

template <int NZ, int R0Z, int NY, int R0Y, int NT, bool SPLIT>
__global__ __launch_bounds__(NT) void plane_kernel_multi(const GroupHdr* __restrict__ hdr) {
  extern __shared__ uint32_t lds[];
  CGroupHdr* h = (CGroupHdr*)hdr;
  CKParams* jobs = (CKParams*)h->jobs;
  CInt64* prefix = (CInt64*)h->prefix;
  const int njobs = (int)h->njobs;
  const int64_t total = njobs > 0 ? prefix[njobs] : 0;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int j = find_job(prefix, njobs, w);
    const KParams kp = load_job(jobs, j);
    plane_body<NZ, R0Z, NY, R0Y, NT, SPLIT>(kp, w - prefix[j], lds);
    __syncthreads();  // the next plane's first stage rewrites LDS
  }
}

#define PLANEK(NZ_, RZ_, NY_, RY_)                                                   \
  if (k.kind == K_PLANE && k.L == NZ_ && k.C == NY_ && k.NT == 256) {                \
    if (k.split) {                                                                   \
      if constexpr (NZ_ * NY_ == 16384) {                                            \
        out->single = (KernelFn)plane_kernel<NZ_, RZ_, NY_, RY_, 256, true>;         \
        out->multi = (MultiFn)plane_kernel_multi<NZ_, RZ_, NY_, RY_, 256, true>;     \
      } else {                                                                      \
        return false; /* several planes per workgroup: FP16 only */                 \
      }                                                                              \
    } else {                                                                        \
      out->single = (KernelFn)plane_kernel<NZ_, RZ_, NY_, RY_, 256, false>;          \
      out->multi = (MultiFn)plane_kernel_multi<NZ_, RZ_, NY_, RY_, 256, false>;      \
    }                                                                                \
    out->persistent = false;                                                         \
    return true;                                                                     \
  }

bool find_plane_kernels(const KernelKey& k, KernelFns* out) {
  PLANEK(64, 4, 256, 1)
  PLANEK(128, 8, 128, 8)
  PLANEK(256, 1, 64, 4)
  PLANEK(512, 2, 32, 2)
  PLANEK(1024, 4, 16, 1)
  PLANEK(64, 4, 64, 4)    // 4 planes per workgroup (FP16)
  PLANEK(128, 8, 32, 2)
  PLANEK(64, 4, 128, 8)   // 2 planes per workgroup (FP16)
  PLANEK(128, 8, 64, 4)
  PLANEK(256, 1, 32, 2)
  return false;
}

}  // namespace tcfft
