// Single-pass 65536-point 1D transform: one 512-thread workgroup per transform.
//
// Eq. 3 with N1 = 16, N2 = 4096 (Sec. 2.1), decimation in frequency: the
// radix-16 stage over the top digit d (stride 4096) runs straight from HBM
// into registers, giving for every column n in [0, 4096) the 16 values
//   y_k[n] = W_N^{k n} * sum_d x[d 4096 + n] W_16^{d k},      k in [0, 16),
// and X[k + 16 k'] is the 4096-point DFT of y_k at k' (Sec. 3.2: merging
// processes combined inside one block).  The 16 sub-transforms run 4 at a time
// through 64 KB of LDS with the row-pass stages (radix 16 at strides 256, 16,
// 1); every result stays in the registers its inputs came from.  The lane
// that ends up holding X[k + 16 k'] for k = 4s..4s+3 at one k' writes them as
// one 16-byte group; the results go out through LDS in four pieces of 16384
// consecutive outputs, so each wave stores 1 KB runs.  HBM traffic is one read
// and one write of the data (the two-pass plan moves it twice).
//
// Registers: 128 data words per lane (65536 points / 512 lanes) plus the stage
// working set; LDS: 64 KB.  The W_N table (kp.tw, 65536 entries) serves the
// first stage and kp.xtw_hi holds W_4096 for the sub-transforms.
#include "pass_kernels.h"

namespace tcfft {

namespace big {
constexpr int N = 65536;
constexpr int L = 4096;  // sub-transform length
constexpr int NT = 512;
using G = RowGeom<L, 1, NT>;  // 4 sub-transforms of 4096, 8 waves, 2 quads per wave
static_assert(G::TPB == 4 && G::QPW == 2 && G::PTS == 16384, "sub-transform geometry");
}  // namespace big

__device__ __forceinline__ void big_body(const KParams& kp, int64_t wg, uint32_t* lds) {
  using namespace big;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int64_t g0 = wg * (int64_t)N;
  const FOps f = load_fops<false>(kp.fimg);

  // ---- stage 1: rows d = 4g+i of columns n0..n0+3, 8 column quads per lane.
  u4 D[8][4];  // [slot][t]: data words, 4 per u4
  {
    u4 R[8][4];
#pragma unroll
    for (int qq = 0; qq < 8; ++qq) {
      const int n0 = 4 * c16 + 64 * (wave * 8 + qq);
#pragma unroll
      for (int i = 0; i < 4; ++i) R[qq][i] = gld4(kp.in + g0 + (int64_t)(4 * g + i) * L + n0);
    }
    // W_N^{(4g+j)(n0+t)} = W_N^{(4g+j) n0} * W_N^{(4g+j) t}
    const TwB B = load_twb(kp.tw, g, 1);
#pragma unroll
    for (int qq = 0; qq < 8; ++qq) {
      const int n0 = 4 * c16 + 64 * (wave * 8 + qq);
      float2 a[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) a[j] = tld(kp.tw, (4 * g + j) * n0);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        u4 xh;
#pragma unroll
        for (int i = 0; i < 4; ++i) xh[i] = R[qq][i][t];
        f4 yr, yi;
        mfma_dft16(xh, f.rh, f.ih, yr, yi);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float2 z =
              cmul(make_float2(yr[j], yi[j]), t == 0 ? a[j] : cmul(a[j], B.b[j][t - 1]));
          D[qq][t][j] = pack(z.x, z.y);
        }
      }
    }
  }

  // ---- stages 2-4: the 16 sub-transforms, group jg = {k = 4s + jg : s < 4}.
  // Lane (g, ...) holds y_{4g+jg} at its columns: it writes sub-transform s = g.
  KParams ks = kp;
  ks.tw = kp.xtw_hi;  // W_4096
#pragma unroll
  for (int jg = 0; jg < 4; ++jg) {
    if (jg > 0) __syncthreads();  // the previous group's last stage has read LDS
#pragma unroll
    for (int qq = 0; qq < 8; ++qq) {
      const int n0 = 4 * c16 + 64 * (wave * 8 + qq);
      lds_st4(lds, g * L + n0, u4{D[qq][0][jg], D[qq][1][jg], D[qq][2][jg], D[qq][3][jg]});
    }
    __syncthreads();
    row_stage16<G, 256, false, false>(ks, lds, G::TPB, 0, f);
    __syncthreads();
    row_stage16<G, 16, false, false>(ks, lds, G::TPB, 0, f);
    __syncthreads();
    // last radix-16 stage: natural output k' = klow + 256 (4g + j) of
    // sub-transform tau, kept in the slots this group freed
#pragma unroll
    for (int qq = 0; qq < 2; ++qq) {
      const int col0 = 4 * c16 + 64 * (wave * 2 + qq);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = col0 + t;
        const int p = (col >> 8) * L + posrev_hi<1, 3>(col & 255) * 16 + 4 * g;
        const u4 xh = lds_ld4(lds, p);
        f4 yr, yi;
        mfma_dft16(xh, f.rh, f.ih, yr, yi);
#pragma unroll
        for (int j = 0; j < 4; ++j) D[qq * 4 + j][t][jg] = pack(yr[j], yi[j]);
      }
    }
  }

  // ---- output: slot (qq*4 + j, t) holds X[4s + jg + 16 k'] for jg = 0..3 with
  // s = col >> 8, k' = (col & 255) + 256 (4g + j).  Piece pc = k' >> 10 = g.
#pragma unroll
  for (int pc = 0; pc < 4; ++pc) {
    __syncthreads();
    if (g == pc) {
#pragma unroll
      for (int qq = 0; qq < 2; ++qq) {
        const int col0 = 4 * c16 + 64 * (wave * 2 + qq);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int col = col0 + t;
#pragma unroll
          for (int j = 0; j < 4; ++j)
            lds_st4(lds, 4 * (col >> 8) + 16 * ((col & 255) + 256 * j), D[qq * 4 + j][t]);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int q4 = (int)threadIdx.x + NT * r;  // 16-byte group of the piece
      gst4(kp.out + g0 + pc * 16384 + 4 * q4, lds_ld4(lds, 4 * q4));
    }
  }
}

__global__ __launch_bounds__(512) void big_kernel(KParams kp) {
  extern __shared__ uint32_t lds[];
  big_body(kp, blockIdx.x, lds);
}

__global__ __launch_bounds__(512) void big_kernel_multi(const GroupHdr* __restrict__ hdr) {
  extern __shared__ uint32_t lds[];
  CGroupHdr* h = (CGroupHdr*)hdr;
  CKParams* jobs = (CKParams*)h->jobs;
  CInt64* prefix = (CInt64*)h->prefix;
  const int njobs = (int)h->njobs;
  const int64_t total = njobs > 0 ? prefix[njobs] : 0;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int j = find_job(prefix, njobs, w);
    const KParams kp = load_job(jobs, j);
    big_body(kp, w - prefix[j], lds);
    __syncthreads();  // the next tile's first LDS write
  }
}

bool find_big_kernels(const KernelKey& k, KernelFns* out) {
  if (k.kind == K_BIG && k.L == 65536 && k.R0 == 1 && k.NT == 512 && !k.split && !k.xtw &&
      !k.tstore) {
    out->single = (KernelFn)big_kernel;
    out->multi = (MultiFn)big_kernel_multi;
    out->persistent = false;
    return true;
  }
  return false;
}

}  // namespace tcfft
