// Plane pass of a 3D transform: one workgroup computes the 2D DFT of NPL
// [ny][nz] planes (NPL ny nz = 16384 points, nz contiguous) entirely in LDS.
//
// The 3D DFT is separable (Eq. 1 over three indices): the row half runs the
// nz-point row stages of the row kernel over the plane's ny lines, its last
// stage leaving the results in natural order in LDS (position y nz + z); the
// column half then runs the ny-point column stages of the column kernel on
// that LDS block (element (y, z) at y C + z with C = nz), its first stage
// reading LDS instead of HBM, and its last stage writes the plane to HBM.  The
// data cross HBM once for both dimensions; the nx-point column pass over the
// planes follows as a separate pass.  With several planes per workgroup (FP16
// only: split data keep their lo plane 16384 words above the hi plane, the
// column stages expect it one plane above) the column half runs plane after
// plane on consecutive LDS blocks.
//
// Parameters: kp.tw = W_nz, kp.r0scale = the row half's radix-R0 scale;
// kp.xtw_lo = W_ny, kp.r0scale2 = the column half's; kp.ntrans = lines
// (planes x ny); kp.s_out = nz (row stride of the output plane).
#include "pass_kernels.h"

namespace tcfft {

template <int NZ, int R0Z, int NY, int R0Y, int NT, bool SPLIT>
__device__ __forceinline__ void plane_body(const KParams& kp, int64_t wg, uint32_t* lds) {
  constexpr int PL = NY * NZ, NPL = 16384 / PL;
  static_assert(NPL * PL == 16384 && (NPL == 1 || !SPLIT), "whole planes per workgroup");
  using CG = ColGeom<NY, R0Y, NZ, NT>;
  // the column half starts from LDS: a radix-16 or a stand-alone radix-R0
  // stage (the fused radix-R0 + radix-16 column stage reads HBM)
  static_assert(!ColFused<CG>::value, "column half must start from LDS");
  row_body<NZ, R0Z, NT, SPLIT, false, 3>(kp, wg, lds);  // rows: natural order in LDS
  __syncthreads();
  KParams kc = kp;
  kc.tw = kp.xtw_lo;
  kc.r0scale = kp.r0scale2;
  const FOps f = load_fops<SPLIT>(kp.fimg);
  // planes of this workgroup that exist (the batch may end inside it)
  const int64_t left = kp.ntrans / NY - wg * NPL;
  const int vp = left < NPL ? (int)left : NPL;
  for (int pl = 0; pl < vp; ++pl) {
    if (pl > 0) __syncthreads();
    ColCtx cx;
    cx.outer = wg * NPL + pl;
    cx.i0 = 0;
    cx.in_base = cx.outer * (int64_t)PL;
    cx.out_base = cx.in_base;
    cx.lds_off = pl * PL;  // the row half wrote plane pl at positions pl PL + y nz + z
    if constexpr (R0Y > 1) {
      col_stage_r0<CG, SPLIT, true>(kc, lds, cx);
      __syncthreads();
      col_stages_from<CG, CG::S - 1, SPLIT, false, false>(kc, lds, cx, f);
    } else {
      col_stages_from<CG, CG::S - 1, SPLIT, false, false>(kc, lds, cx, f);
    }
  }
}

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
