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
#pragma once
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

}  // namespace tcfft
