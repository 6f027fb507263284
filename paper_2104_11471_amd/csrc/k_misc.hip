// FP32 radix-2 comparator and FP64 table generators.
#include "common.h"
#include "kernels.h"

namespace tcfft {

// ===========================================================================
// FP32 radix-2 Stockham comparator: one launch per stage, 16 B/point each way.
// ===========================================================================
__global__ __launch_bounds__(256) void radix2_stage_kernel(const float2* __restrict__ in,
                                                           float2* __restrict__ out, int64_t n,
                                                           int64_t ns, int64_t total,
                                                           const float2* __restrict__ tw) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= total) return;
  const int64_t half = n >> 1;
  const int64_t b = gid / half, j = gid - b * half;
  const float2* x = in + b * n;
  float2* y = out + b * n;
  const int64_t k = j & (ns - 1);
  const float2 a = x[j];
  const float2 c = cmul(x[j + half], tw[k * (n / (2 * ns))]);  // W_{2ns}^k
  const int64_t o = ((j - k) << 1) + k;
  y[o] = make_float2(a.x + c.x, a.y + c.y);
  y[o + ns] = make_float2(a.x - c.x, a.y - c.y);
}

void launch_radix2_stage(const float2* in, float2* out, int64_t n, int64_t ns, int64_t batch,
                         const float2* tw, hipStream_t s) {
  const int64_t total = batch * (n / 2);
  const int64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL(radix2_stage_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n, ns,
                     total, tw);
}

// ===========================================================================
// FP64 table generation on the device.
// ===========================================================================
__global__ void gen_twiddles_kernel(float2* tw, int64_t count, int64_t modulus, int64_t mult,
                                    double sgn) {
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (m >= count) return;
  const int64_t e = (int64_t)(((unsigned __int128)m * (unsigned __int128)mult) % (unsigned __int128)modulus);
  double sn, cs;
  sincospi(2.0 * (double)e / (double)modulus, &sn, &cs);
  tw[m] = make_float2((float)cs, (float)(sgn * sn));
}

void launch_gen_twiddles(float2* tw, int64_t count, int64_t modulus, int64_t mult, double sgn,
                         hipStream_t s) {
  hipLaunchKernelGGL(gen_twiddles_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                     tw, count, modulus, mult, sgn);
}

// Lane = 16 g + m holds row m of the A operand, K entries of input rows
// r = 4g..4g+3.  Entry (m, r) is F_16[m][r] W_{16 R}^{k r} = W_{16 R}^{r (R m + k)}
// (an input twiddle; R = 1, k = 0: the plain radix-16 matrix), or with P > 0
// W_{16 P}^{m lo} F_16[m][r] = W_{16 P}^{m (P r + lo)} (an output twiddle).
__global__ void gen_fimg_kernel(h8* img, double sgn, double scale, int R, int k, int P, int lo) {
  const int lane = threadIdx.x;  // 64 lanes
  const int g = lane >> 4, m = lane & 15;
  h8 rh, ih, rl, il;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = 4 * g + i;
    const int mod = 16 * (P > 0 ? P : R);
    const int e = P > 0 ? (m * (P * r + lo)) % mod : (r * (R * m + k)) % mod;
    double sn, cs;
    sincospi(2.0 * (double)e / (double)mod, &sn, &cs);
    const double fr = cs * scale, fi = sgn * sn * scale;
    // Yr row: [Fr, -Fi]; Yi row: [Fi, Fr]  (pairs = re/im halves of input row r)
    const double vr[2] = {fr, -fi}, vi[2] = {fi, fr};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      _Float16 a = (_Float16)vr[h];
      _Float16 b = (_Float16)vi[h];
      rh[2 * i + h] = a;
      ih[2 * i + h] = b;
      rl[2 * i + h] = (_Float16)((vr[h] - (double)a) * 2048.0);
      il[2 * i + h] = (_Float16)((vi[h] - (double)b) * 2048.0);
    }
  }
  img[lane] = rh;
  img[64 + lane] = ih;
  img[128 + lane] = rl;
  img[192 + lane] = il;
}

void launch_gen_fimg(void* img, double sgn, double scale, hipStream_t s) {
  hipLaunchKernelGGL(gen_fimg_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<h8*>(img), sgn,
                     scale, 1, 0, 0, 0);
}

void launch_gen_fimg_r(void* img, int R, double sgn, double scale, hipStream_t s) {
  for (int slot = 0; slot < R; ++slot) {
    // inverse plans: slot k' holds A_k with k = (R - k') mod R (the kernels
    // follow the forward sign, whose W^{k' d} is the inverse W^{k d})
    const int k = sgn > 0 ? (R - slot) % R : slot;
    hipLaunchKernelGGL(gen_fimg_kernel, dim3(1), dim3(64), 0, s,
                       reinterpret_cast<h8*>(img) + 256 * slot, sgn, scale, R, k, 0, 0);
  }
}

void launch_gen_fimg_tw(void* img, int P, double sgn, double scale, hipStream_t s) {
  for (int lo = 0; lo < P; ++lo)
    hipLaunchKernelGGL(gen_fimg_kernel, dim3(1), dim3(64), 0, s,
                       reinterpret_cast<h8*>(img) + 256 * lo, sgn, scale, 1, 0, P, lo);
}

// Autotuner scratch data: FP16 complex words with re, im in [-1, 1) from a
// hash of the word index (timing on zeros would run at unrepresentative power).
__global__ void fill_pattern_kernel(uint32_t* p, int64_t nwords) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= nwords) return;
  uint32_t h = (uint32_t)i * 0x9E3779B1u;
  h ^= h >> 15;
  h *= 0x85EBCA77u;
  h ^= h >> 13;
  const float re = (float)(h & 0xFFFF) * (1.0f / 32768.0f) - 1.0f;
  const float im = (float)(h >> 16) * (1.0f / 32768.0f) - 1.0f;
  p[i] = pack(re, im);
}

void launch_fill_pattern(void* p, int64_t nwords, hipStream_t s) {
  hipLaunchKernelGGL(fill_pattern_kernel, dim3((unsigned)((nwords + 255) / 256)), dim3(256), 0, s,
                     (uint32_t*)p, nwords);
}

}  // namespace tcfft
