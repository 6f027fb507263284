// FP64 matrix-core variant: batched 1D complex FFT of L = R0 * 16^S <= 4096
// points in double precision, the radix-16 DFT blocks on
// v_mfma_f64_16x16x4f64 (the method of Sec. 3 carried to a wider matrix
// datatype, the generalisation named as future work in Sec. 7).
//
// The stages are those of the FP16 path (decimation in frequency, Eq. 3 with
// N1 = R0 then 16): for a sub-transform of Q = 16 P points at stride P,
//   y_k1[lo] = W_Q^{lo k1} * sum_r x[r P + lo] W_16^{r k1},
// stored at position k1 P + lo; a first radix-R0 stage (R0 in {2, 4, 8}) does
// the same with R0 in place of 16 on the vector ALU.  After all stages output
// k sits at position (k mod R0) 16^S + rev16(k div R0), the S base-16 digits
// of k div R0 in reverse order.
//
// A tile is 4096 points (4096 / L transforms, 64 KB of LDS as double2): a
// coalesced copy from HBM into LDS, the stages in place in LDS, and a
// coalesced copy out that reads the digit-reversed positions.  Two resident
// workgroups (256 threads) per CU stride over the tiles, each loading its next
// tile into registers while the current one runs its stages; lengths with a
// radix-8 first stage (128, 2048) run one tile per workgroup (the held-over
// tile would not fit their registers).  The radix-16
// block of 16 columns is the complex product Y = F X of the DFT matrix with 16
// columns, as three real products (T1 = Fr Xr, T2 = Fi Xi, T3 = (Fr + Fi)
// (Xr + Xi); Yr = T1 - T2, Yi = T3 - T1 - T2), each in four K = 4 slices (12
// MFMAs instead of the 16 of the four-product form), with the v_mfma_f64_16x16x4f64
// layouts: A[i][k] in lane i + 16 k, B[k][j] in lane j + 16 k, D[l / 16 + 4 r][l % 16]
// in element r of lane l (rows interleaved by 4, unlike the FP32-accumulator
// layout of the FP16 instructions).  Twiddles come from an FP64 table W_L^m (sincospi
// in FP64) and are applied to the FP64 accumulators.  No scaling: FP64 has the
// range for any size here.
#include <algorithm>

#include "kernels.h"

namespace tcfft {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int F64_PTS = 4096;  // points per workgroup
constexpr int F64_NT = 256;

constexpr int pow16c(int e) { return e == 0 ? 1 : 16 * pow16c(e - 1); }

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(__builtin_fma(a.x, b.x, -(a.y * b.y)), __builtin_fma(a.x, b.y, a.y * b.x));
}

// LDS index of position p (double2 units): the low 4 bits are XOR-ed with the
// next 4, so 16 lanes at stride 16 positions hit different banks.
__device__ __forceinline__ int sw(int p) { return p ^ ((p >> 4) & 15); }

template <int R0, int S>
__device__ __forceinline__ int out_pos(int k) {
  const int k0 = k % R0;
  int rest = k / R0, rev = 0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    rev = rev * 16 + (rest & 15);
    rest >>= 4;
  }
  constexpr int PS = pow16c(S);
  return k0 * PS + rev;
}

template <int L, int R0>
__global__ __launch_bounds__(F64_NT, R0 <= 4 ? 2 : 1) void f64_row_kernel(const double2* __restrict__ in,
                                                           double2* __restrict__ out,
                                                           int64_t ntrans,
                                                           const double2* __restrict__ tw) {
  constexpr int S = (__builtin_ctz(L) - __builtin_ctz(R0)) / 4;
  static_assert(R0 * pow16c(S) == L && L <= F64_PTS, "L = R0 * 16^S <= 4096");
  constexpr int TPB = F64_PTS / L;
  constexpr int PER = F64_PTS / F64_NT;  // points a thread copies in and out
  __shared__ double2 lds[F64_PTS];
  const int tid = threadIdx.x;
  const int64_t ntiles = (ntrans + TPB - 1) / TPB;
  auto valid_of = [&](int64_t w) {
    const int64_t rem = ntrans - w * TPB;
    return rem < TPB ? (int)rem : TPB;
  };
  // next tile's inputs, loaded while the current tile runs its stages
  double2 pf[PER];
  auto load_tile = [&](int64_t w) {
    const int valid = valid_of(w);
    const int64_t g0 = w * (int64_t)F64_PTS;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int p = tid + i * F64_NT;
      pf[i] = p / L < valid ? in[g0 + p] : make_double2(0.0, 0.0);  // lines past the batch: zeros
    }
  };
  // radix-16 A operands: F[k1 = c16][r = 4 kb + g] = W_16^{k1 r}, and Fr + Fi
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  double fr[4], fi[4], fs[4];
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    const double2 w = tw[((c16 * (4 * kb + g)) & 15) * (L / 16)];
    fr[kb] = w.x;
    fi[kb] = w.y;
    fs[kb] = w.x + w.y;
  }
  // persistent with the prefetch where it fits the register budget of two
  // workgroups per CU (all but the radix-8 first stages); otherwise one tile
  // per workgroup
  constexpr bool PREF = R0 <= 4;
  int64_t w = blockIdx.x;
  if (w >= ntiles) return;
  if constexpr (PREF) load_tile(w);
  for (; w < ntiles; w += PREF ? gridDim.x : ntiles) {
    const int valid = valid_of(w);
    const int64_t g0 = w * (int64_t)F64_PTS;
    if constexpr (!PREF) load_tile(w);
#pragma unroll
    for (int i = 0; i < PER; ++i) lds[sw(tid + i * F64_NT)] = pf[i];
    __syncthreads();
    if constexpr (PREF)
      if (w + gridDim.x < ntiles) load_tile(w + gridDim.x);

    // radix-R0 stage on the vector ALU: item (line, lo), lo < L / R0
    if constexpr (R0 > 1) {
      constexpr int P0 = L / R0, ITEMS = F64_PTS / R0;
      double2 wr[R0];  // W_R0^m
#pragma unroll
      for (int m = 0; m < R0; ++m) wr[m] = tw[m * (L / R0)];
#pragma unroll 1
      for (int i = 0; i < ITEMS / F64_NT; ++i) {
        const int it = tid + i * F64_NT;
        const int line = it / P0, lo = it % P0;
        const int base = line * L + lo;
        double2 x[R0];
#pragma unroll
        for (int d = 0; d < R0; ++d) x[d] = lds[sw(base + d * P0)];
#pragma unroll
        for (int k = 0; k < R0; ++k) {
          double2 y = x[0];
#pragma unroll
          for (int d = 1; d < R0; ++d) {
            const double2 v = zmul(x[d], wr[(d * k) % R0]);  // W_R0^{d k}
            y.x += v.x;
            y.y += v.y;
          }
          lds[sw(base + k * P0)] = zmul(y, tw[k * lo]);  // W_L^{k lo}
        }
      }
      __syncthreads();
    }

    // radix-16 stages on the matrix core; the complex product in three real
    // products: T1 = Fr Xr, T2 = Fi Xi, T3 = (Fr + Fi)(Xr + Xi), then
    // Yr = T1 - T2 and Yi = T3 - T1 - T2 (12 MFMAs per tile instead of 16)
#pragma unroll
    for (int s = 1; s <= S; ++s) {
      const int P = 1 << (4 * (S - s)), Q = 16 * P;
#pragma unroll 1
      for (int tt = 0; tt < F64_PTS / 16 / 16 / 4; ++tt) {
        const int c = 16 * (wave * (F64_PTS / 16 / 16 / 4) + tt) + c16;  // column of the stage
        const int lo = c % P, base = (c / P) * Q + lo;
        double xr[4], xi[4], xs[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          const double2 v = lds[sw(base + (4 * kb + g) * P)];
          xr[kb] = v.x;
          xi[kb] = v.y;
          xs[kb] = v.x + v.y;
        }
        d4 t1 = {0.0, 0.0, 0.0, 0.0}, t2 = t1, t3 = t1;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
          t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(fr[kb], xr[kb], t1, 0, 0, 0);
          t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(fi[kb], xi[kb], t2, 0, 0, 0);
          t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(fs[kb], xs[kb], t3, 0, 0, 0);
        }
        // every lane of the column has read its rows before any writes (one wave)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k1 = g + 4 * r;
          double2 y = make_double2(t1[r] - t2[r], t3[r] - t1[r] - t2[r]);
          if (P > 1) y = zmul(y, tw[lo * k1 * (L / Q)]);  // W_Q^{lo k1}
          lds[sw(base + k1 * P)] = y;
        }
      }
      __syncthreads();
    }

    // copy out in natural order
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int p = tid + i * F64_NT;
      const int line = p / L;
      if (line < valid) out[g0 + p] = lds[sw(line * L + out_pos<R0, S>(p % L))];
    }
    __syncthreads();  // the next tile rewrites LDS
  }
}

__global__ void gen_tw_f64(double2* tw, int64_t count, int64_t modulus, double sgn) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= count) return;
  double s, c;
  sincospi(2.0 * (double)m / (double)modulus, &s, &c);
  tw[m] = make_double2(c, sgn * s);
}

}  // namespace

void launch_gen_twiddles_f64(double2* tw, int64_t count, int64_t modulus, double sgn,
                             hipStream_t s) {
  hipLaunchKernelGGL(gen_tw_f64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, tw,
                     count, modulus, sgn);
}

hipError_t launch_f64_row(const double2* in, double2* out, int L, int64_t batch,
                          const double2* tw, hipStream_t s) {
  // persistent grid for the prefetching variants: two resident workgroups per
  // CU (64 KB of LDS each) stride over the tiles
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      ncu <= 0)
    return hipErrorInvalidDevice;
  const int tpb = F64_PTS / L;
  const int64_t ntiles = (batch + tpb - 1) / tpb;
  const bool pref = L != 128 && L != 2048;  // R0 <= 4: the persistent kernels
  const dim3 grid((unsigned)(pref ? std::min<int64_t>(ntiles, 2 * (int64_t)ncu) : ntiles)),
      block(F64_NT);
  switch (L) {
#define F64K(L_, R_) \
  case L_: hipLaunchKernelGGL((f64_row_kernel<L_, R_>), grid, block, 0, s, in, out, batch, tw); break;
    F64K(16, 1)
    F64K(32, 2)
    F64K(64, 4)
    F64K(128, 8)
    F64K(256, 1)
    F64K(512, 2)
    F64K(1024, 4)
    F64K(2048, 8)
    F64K(4096, 1)
#undef F64K
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tcfft
