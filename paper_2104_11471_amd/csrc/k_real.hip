// Real-input transforms on top of the complex path.
//
// An N-point real sequence x is read as M = N/2 complex points
// z[m] = x[2m] + i x[2m+1] (the FP16 storage of N reals is exactly M complex
// words).  With Z = DFT_M(z), the even and odd halves of x have
//   E[k] = (Z[k] + conj(Z[M-k])) / 2,    O[k] = (Z[k] - conj(Z[M-k])) / (2i),
// and X[k] = E[k] + W_N^k O[k] for k = 0..M (Z[M] = Z[0]): the first M + 1
// bins of the N-point DFT (Eq. 2 with N1 = 2, applied to a real input; the
// rest follow by Hermitian symmetry).  The inverse runs the same relations
// backwards: Z'[k] = (X[k] + conj(X[M-k])) + i (X[k] - conj(X[M-k])) W_N^{-k}
// for k < M, then the inverse M-point transform gives 2M (x[2m] + i x[2m+1])
// -- N times the real sequence, the unnormalised convention of the complex
// path.  Both passes are elementwise (FP32 arithmetic on FP16 data, FP64-made
// FP32 twiddles W_N^k, k <= M) and bound by HBM traffic.  These stand-alone
// passes serve the sizes whose complex transform is not one row pass (M = 16,
// 32 and the multi-pass M > 16384); the others run the same step inside the
// row pass (real_post / real_pre).
#include "pass_kernels.h"

namespace tcfft {

namespace {

template <bool SPLIT>
__device__ __forceinline__ float2 rd(const uint32_t* p, int64_t plane, int64_t i) {
  if constexpr (SPLIT) return value<true>(p[i], p[plane + i]);
  return value<false>(p[i], 0u);
}
template <bool SPLIT>
__device__ __forceinline__ void wr(uint32_t* p, int64_t plane, int64_t i, float2 v) {
  uint32_t h = 0, l = 0;
  emit<SPLIT>(v.x, v.y, h, l);
  gst1(p + i, h);
  if constexpr (SPLIT) gst1(p + plane + i, l);
}

// Forward post-pass: Z (batch x M words) -> X (batch x (M + 1) words).
// Thread (b, j), j in [0, M/2]: X[j] and X[M-j] from Z[j] and Z[M-j] (one
// twiddle product for the pair, see real_spec); j = M/2 pairs with itself.
// Every input word is read once.
template <bool SPLIT>
__global__ __launch_bounds__(256) void r2c_post_kernel(const uint32_t* __restrict__ z,
                                                       uint32_t* __restrict__ x,
                                                       const float2* __restrict__ tw, int64_t M,
                                                       int64_t batch, int64_t zplane, int64_t xplane) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t H = M / 2 + 1;
  if (i >= H * batch) return;
  const int64_t b = i / H, j = i - b * H;
  const uint32_t* zb = z + b * M;
  const float2 a = rd<SPLIT>(zb, zplane, j);
  const float2 c = rd<SPLIT>(zb, zplane, j == 0 ? 0 : M - j);
  float2 xk, xm;
  real_spec(a, c, tld(tw, j), xk, xm);
  wr<SPLIT>(x + b * (M + 1), xplane, j, xk);
  if (j != M - j) wr<SPLIT>(x + b * (M + 1), xplane, M - j, xm);  // j = 0: X[M]
}

// Inverse pre-pass: X (batch x (M + 1) words) -> Z' (batch x M words).
// Thread (b, j), j in [0, M/2]: Z'[j] and Z'[M-j] from X[j] and X[M-j] (see
// real_zpre); `tw` holds W_N^{-k}.  X[0] and X[M] count by their real parts
// (a real input's DFT has them real); Z'[M] does not exist.
template <bool SPLIT>
__global__ __launch_bounds__(256) void c2r_pre_kernel(const uint32_t* __restrict__ x,
                                                      uint32_t* __restrict__ z,
                                                      const float2* __restrict__ tw, int64_t M,
                                                      int64_t batch, int64_t xplane, int64_t zplane) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t H = M / 2 + 1;
  if (i >= H * batch) return;
  const int64_t b = i / H, j = i - b * H;
  const uint32_t* xb = x + b * (M + 1);
  float2 a = rd<SPLIT>(xb, xplane, j);
  float2 c = rd<SPLIT>(xb, xplane, M - j);
  if (j == 0) {
    a.y = 0.f;
    c.y = 0.f;
  }
  float2 zk, zm;
  real_zpre(a, c, tld(tw, j), zk, zm);
  wr<SPLIT>(z + b * M, zplane, j, zk);
  if (j != 0 && j != M - j) wr<SPLIT>(z + b * M, zplane, M - j, zm);
}

}  // namespace

void launch_r2c_post(const void* z, void* x, const float2* tw, int64_t M, int64_t batch,
                     bool split, hipStream_t s) {
  const int64_t n = (M / 2 + 1) * batch;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (split)
    hipLaunchKernelGGL(r2c_post_kernel<true>, grid, dim3(256), 0, s, (const uint32_t*)z,
                       (uint32_t*)x, tw, M, batch, M * batch, (M + 1) * batch);
  else
    hipLaunchKernelGGL(r2c_post_kernel<false>, grid, dim3(256), 0, s, (const uint32_t*)z,
                       (uint32_t*)x, tw, M, batch, (int64_t)0, (int64_t)0);
}

void launch_c2r_pre(const void* x, void* z, const float2* tw, int64_t M, int64_t batch,
                    bool split, hipStream_t s) {
  const int64_t n = (M / 2 + 1) * batch;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (split)
    hipLaunchKernelGGL(c2r_pre_kernel<true>, grid, dim3(256), 0, s, (const uint32_t*)x,
                       (uint32_t*)z, tw, M, batch, (M + 1) * batch, M * batch);
  else
    hipLaunchKernelGGL(c2r_pre_kernel<false>, grid, dim3(256), 0, s, (const uint32_t*)x,
                       (uint32_t*)z, tw, M, batch, (int64_t)0, (int64_t)0);
}

}  // namespace tcfft
