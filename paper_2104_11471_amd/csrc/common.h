// Shared device-side definitions of the tcFFT-on-MFMA kernels (gfx950 only).
//
// Storage: one complex FP16 value = one 32-bit word, real part in the low half,
// imaginary part in the high half (interleaved (re, im) in memory).
//
// Matrix-core DFT block (paper Sec. 2.1, Eq. 3: X_out = F_N1 . (T (.) X_in), and
// Sec. 3.2's radix-16 sub-merge): a radix-16 DFT applied to 16 columns at once is
// one complex 16x16 by 16x16 product.  It runs as two real products
// v_mfma_f32_16x16x32_f16 (D[16x16] += A[16x32] . B[32x16], FP32 accumulate):
//   Yr = [Fr | -Fi] . [Xr ; Xi]      Yi = [Fi | Fr] . [Xr ; Xi]
// with the K = 32 axis holding the 16 inputs' real and imaginary halves.  The
// K order is ours to choose as long as A and B agree, so lane l = 16 g + c holds
// its 8 B-operand halves as the interleaved words of rows 4g..4g+3 of column c:
// interleaved complex data feeds the matrix core with no de-interleave.  The
// accumulator D has lane l holding rows 4g..4g+3 of column c, so the real and
// imaginary outputs of an element land in the same lane and register slot, and
// the twiddle multiply runs on them in FP32 (the MI355X form of Alg. 2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tcfft {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }
constexpr int pow16(int e) { return e == 0 ? 1 : 16 * pow16(e - 1); }

__device__ __forceinline__ float2 unpack(uint32_t v) {
  h2 h = __builtin_bit_cast(h2, v);
  return make_float2((float)h.x, (float)h.y);
}

// FP32 -> FP16 with round-to-nearest-even (v_cvt_pk_f16_f32).
__device__ __forceinline__ uint32_t pack(float re, float im) {
  h2 h = {(_Float16)re, (_Float16)im};
  return __builtin_bit_cast(uint32_t, h);
}

// Complex product with its fused multiply-adds written out: the library is
// built with -ffp-contract=off, so every kernel instantiation (single and
// grouped launches) performs exactly these roundings and gives the same bits.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}

// Split hi+lo encoding of an FP32 value v: hi = fp16(v), lo = fp16((v - hi) * 2^11).
__device__ __forceinline__ void split2(float re, float im, uint32_t& hi, uint32_t& lo) {
  h2 h = {(_Float16)re, (_Float16)im};
  float rr = (re - (float)h.x) * 2048.0f;
  float ri = (im - (float)h.y) * 2048.0f;
  hi = __builtin_bit_cast(uint32_t, h);
  lo = pack(rr, ri);
}

// Radix-16 DFT of 16 columns on the matrix core.  b = the lane's 4 complex
// inputs (rows 4g..4g+3 of its column), fr/fi = the lane's A operands.
__device__ __forceinline__ void mfma_dft16(u4 b, h8 fr, h8 fi, f4& yr, f4& yi) {
  h8 bh = __builtin_bit_cast(h8, b);
  f4 z = {0.f, 0.f, 0.f, 0.f};
  yr = __builtin_amdgcn_mfma_f32_16x16x32_f16(fr, bh, z, 0, 0, 0);
  yi = __builtin_amdgcn_mfma_f32_16x16x32_f16(fi, bh, z, 0, 0, 0);
}

// Compensated form for split hi+lo data and matrix (lo parts pre-scaled by 2^11):
//   Y = Fhi.Xhi + 2^-11 (Fhi.Xlo + Flo.Xhi); the lo.lo term is dropped.
__device__ __forceinline__ void mfma_dft16_split(u4 bhi, u4 blo, h8 frh, h8 fih, h8 frl,
                                                 h8 fil, f4& yr, f4& yi) {
  h8 xh = __builtin_bit_cast(h8, bhi);
  h8 xl = __builtin_bit_cast(h8, blo);
  f4 z = {0.f, 0.f, 0.f, 0.f};
  f4 mr = __builtin_amdgcn_mfma_f32_16x16x32_f16(frh, xh, z, 0, 0, 0);
  f4 mi = __builtin_amdgcn_mfma_f32_16x16x32_f16(fih, xh, z, 0, 0, 0);
  f4 cr = __builtin_amdgcn_mfma_f32_16x16x32_f16(frh, xl, z, 0, 0, 0);
  f4 ci = __builtin_amdgcn_mfma_f32_16x16x32_f16(fih, xl, z, 0, 0, 0);
  cr = __builtin_amdgcn_mfma_f32_16x16x32_f16(frl, xh, cr, 0, 0, 0);
  ci = __builtin_amdgcn_mfma_f32_16x16x32_f16(fil, xh, ci, 0, 0, 0);
  const float s = 1.0f / 2048.0f;
  yr = mr + cr * s;
  yi = mi + ci * s;
}

// Small DFTs on the vector ALU for the radix-2/4/8 remainder (paper Sec. 3.1:
// radices 2 and 4 whose matrices hold only 0, +-1, +-i, run off the matrix
// unit).  Decimation in frequency; v[k] holds output k on return.  sgn = -1
// forward, +1 inverse (W_R = exp(sgn * 2 pi i / R)).
__device__ __forceinline__ float2 mul_i(float2 a, float sgn) {  // a * (sgn * i)
  return make_float2(-sgn * a.y, sgn * a.x);
}

template <int R>
__device__ __forceinline__ void small_dft(float2 (&v)[R], float sgn);

template <>
__device__ __forceinline__ void small_dft<1>(float2 (&)[1], float) {}

template <>
__device__ __forceinline__ void small_dft<2>(float2 (&v)[2], float) {
  float2 a = v[0], b = v[1];
  v[0] = make_float2(a.x + b.x, a.y + b.y);
  v[1] = make_float2(a.x - b.x, a.y - b.y);
}

template <>
__device__ __forceinline__ void small_dft<4>(float2 (&v)[4], float sgn) {
  float2 a0 = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
  float2 a2 = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
  float2 a1 = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
  float2 a3 = mul_i(make_float2(v[1].x - v[3].x, v[1].y - v[3].y), sgn);
  v[0] = make_float2(a0.x + a1.x, a0.y + a1.y);
  v[2] = make_float2(a0.x - a1.x, a0.y - a1.y);
  v[1] = make_float2(a2.x + a3.x, a2.y + a3.y);
  v[3] = make_float2(a2.x - a3.x, a2.y - a3.y);
}

template <>
__device__ __forceinline__ void small_dft<8>(float2 (&v)[8], float sgn) {
  const float h = 0.70710678118654752440f;
  float2 a[4], b[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    a[j] = make_float2(v[j].x + v[j + 4].x, v[j].y + v[j + 4].y);
    b[j] = make_float2(v[j].x - v[j + 4].x, v[j].y - v[j + 4].y);
  }
  // b[j] *= W_8^j
  b[1] = cmul(b[1], make_float2(h, sgn * h));
  b[2] = mul_i(b[2], sgn);
  b[3] = cmul(b[3], make_float2(-h, sgn * h));
  small_dft<4>(a, sgn);
  small_dft<4>(b, sgn);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[2 * k] = a[k];
    v[2 * k + 1] = b[k];
  }
}

}  // namespace tcfft
