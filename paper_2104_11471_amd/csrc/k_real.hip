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
// FP32 twiddles W_N^k, k <= M) and bound by HBM traffic.
#include "pass_kernels.h"

namespace tcfft {

namespace {

__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

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
// Thread (b, k), k in [0, M]: X[k] = 0.5 (Z[k] + conj(Z[M-k])) + W_N^k * 0.5 (Z[k] - conj(Z[M-k])) / i
template <bool SPLIT>
__global__ __launch_bounds__(256) void r2c_post_kernel(const uint32_t* __restrict__ z,
                                                       uint32_t* __restrict__ x,
                                                       const float2* __restrict__ tw, int64_t M,
                                                       int64_t batch, int64_t zplane, int64_t xplane) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t per = M + 1;
  if (i >= per * batch) return;
  const int64_t b = i / per, k = i - b * per;
  const uint32_t* zb = z + b * M;
  const float2 a = rd<SPLIT>(zb, zplane, k == M ? 0 : k);
  const float2 c = cconj(rd<SPLIT>(zb, zplane, k == 0 ? 0 : M - k));
  const float2 e = cadd(a, c);                 // 2 E[k]
  const float2 d = csub(a, c);                 // 2 i O[k]
  const float2 o = make_float2(d.y, -d.x);     // 2 O[k] = d / i
  const float2 w = tld(tw, k);                 // W_N^k
  const float2 v = cadd(e, cmul(w, o));
  wr<SPLIT>(x + b * per, xplane, k, make_float2(0.5f * v.x, 0.5f * v.y));
}

// Inverse pre-pass: X (batch x (M + 1) words) -> Z' (batch x M words),
// Z'[k] = (X[k] + conj(X[M-k])) + i (X[k] - conj(X[M-k])) W_N^{-k}.
// `tw` holds W_N^{-k} (the inverse table).  X[0] and X[M] count by their real
// parts (a real input's DFT has them real).
template <bool SPLIT>
__global__ __launch_bounds__(256) void c2r_pre_kernel(const uint32_t* __restrict__ x,
                                                      uint32_t* __restrict__ z,
                                                      const float2* __restrict__ tw, int64_t M,
                                                      int64_t batch, int64_t xplane, int64_t zplane) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= M * batch) return;
  const int64_t b = i / M, k = i - b * M;
  const uint32_t* xb = x + b * (M + 1);
  float2 a = rd<SPLIT>(xb, xplane, k);
  float2 c = rd<SPLIT>(xb, xplane, M - k);
  if (k == 0) {  // X[0] and X[M] are real
    a.y = 0.f;
    c.y = 0.f;
  }
  c = cconj(c);
  const float2 e = cadd(a, c);
  const float2 d = cmul(csub(a, c), tld(tw, k));
  wr<SPLIT>(z + b * M, zplane, k, make_float2(e.x - d.y, e.y + d.x));  // e + i d
}

}  // namespace

void launch_r2c_post(const void* z, void* x, const float2* tw, int64_t M, int64_t batch,
                     bool split, hipStream_t s) {
  const int64_t n = (M + 1) * batch;
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
  const int64_t n = M * batch;
  const dim3 grid((unsigned)((n + 255) / 256));
  if (split)
    hipLaunchKernelGGL(c2r_pre_kernel<true>, grid, dim3(256), 0, s, (const uint32_t*)x,
                       (uint32_t*)z, tw, M, batch, (M + 1) * batch, M * batch);
  else
    hipLaunchKernelGGL(c2r_pre_kernel<false>, grid, dim3(256), 0, s, (const uint32_t*)x,
                       (uint32_t*)z, tw, M, batch, (int64_t)0, (int64_t)0);
}

}  // namespace tcfft
