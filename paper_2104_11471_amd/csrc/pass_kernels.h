// Pass kernels of the FP16 matrix-core FFT (gfx950).
//
// A pass computes, for every line of its input, an L-point DFT with
// L = R0 * 16^S, as the chain of merging processes of the paper (Sec. 2.1,
// Eq. 3; Sec. 3.2, Alg. 1): an optional radix-R0 stage (R0 in {2, 4, 8}) on the
// vector ALU, then S radix-16 stages on the matrix core.  The stages are
// decimation in frequency and in place (Sec. 4.2: in-place merging with a
// changing data order): stage s turns input digit d_s into output digit k_s at
// the same LDS position, then multiplies by the twiddle W_{Ls}^{k_s * r} of
// the remaining lower index r.  The twiddle runs in FP32 on the accumulator,
// before the single rounding to FP16 of that stage.  Position order at the end
// is digit-reversed; the last stage writes natural order straight from its
// registers.
//
// Exchange scopes (Sec. 3.2, "combine multiple mergings"): the first stage
// reads HBM directly into matrix-core operands, every later stage exchanges
// through LDS with one workgroup barrier, and passes exchange through HBM.
//
// Two kernel families:
//   row kernel  -- contiguous lines: TPB consecutive lines of L points per
//                  workgroup (1D transforms, 2D row pass).
//   col kernel  -- strided lines: C adjacent columns of an [L][inner] block per
//                  workgroup, so every HBM access moves C*4 contiguous bytes
//                  (Sec. 4.2, coalesced continuous-size access; 2D column pass
//                  and the passes of long 1D transforms).  Optional extra
//                  inter-pass twiddle and transposed store for the four-step
//                  long transforms.
#pragma once
#include "common.h"
#include "kernels.h"

namespace tcfft {

// ---------------------------------------------------------------------------
// LDS addressing.  Position p (in complex words) -> word address.  Bits [2,6)
// (the 16-byte group inside a 256-byte bank row) are XORed with a fold of the
// bits above, so 16-byte groups stay aligned for ds_read/write_b128 while
// accesses whose positions differ only above bit 6 (long strides, the
// digit-reversed last stage, the transposed gather) spread over the banks.
__device__ __forceinline__ int lds_addr(int p) {
  return p ^ ((((p >> 6) ^ (p >> 10) ^ (p >> 14)) & 15) << 2);
}

__device__ __forceinline__ u4 lds_ld4(const uint32_t* lds, int p) {
  return *reinterpret_cast<const u4*>(lds + lds_addr(p));
}
__device__ __forceinline__ void lds_st4(uint32_t* lds, int p, u4 v) {
  *reinterpret_cast<u4*>(lds + lds_addr(p)) = v;
}
__device__ __forceinline__ uint32_t lds_ld1(const uint32_t* lds, int p) { return lds[lds_addr(p)]; }
__device__ __forceinline__ void lds_st1(uint32_t* lds, int p, uint32_t v) { lds[lds_addr(p)] = v; }

// Global-memory accesses through address-space-1 pointers: grouped launches
// read their buffer and table pointers from a descriptor in memory, where the
// compiler cannot infer the address space and would otherwise emit flat
// accesses (64-bit VGPR addresses, and LDS-counter waits at every barrier).
#define TCFFT_GLOBAL __attribute__((address_space(1)))
__device__ __forceinline__ u4 gld4(const uint32_t* ptr) {
  return *(const TCFFT_GLOBAL u4*)(ptr);
}
__device__ __forceinline__ void gst4(uint32_t* ptr, u4 v) { *(TCFFT_GLOBAL u4*)(ptr) = v; }
// Row passes stream their lines through once with non-temporal accesses
// (measured faster for contiguous 16-byte-per-lane lines; column passes, whose
// rows are 64-256-byte runs, keep the default cache policy, which measured
// faster for them, and so do the loads of a plane pass's row half).
__device__ __forceinline__ u4 rld4(const uint32_t* ptr) {
  return __builtin_nontemporal_load((const TCFFT_GLOBAL u4*)(ptr));
}
__device__ __forceinline__ void rst4(uint32_t* ptr, u4 v) {
  __builtin_nontemporal_store(v, (TCFFT_GLOBAL u4*)(ptr));
}
__device__ __forceinline__ uint32_t gld1(const uint32_t* ptr) {
  return *(const TCFFT_GLOBAL uint32_t*)(ptr);
}
__device__ __forceinline__ void gst1(uint32_t* ptr, uint32_t v) {
  *(TCFFT_GLOBAL uint32_t*)(ptr) = v;
}
// Table lookup: element i of a read-only FP32 complex table.
typedef float f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 tld(const float2* tab, int64_t i) {
  const f2v v = *(const TCFFT_GLOBAL f2v*)(tab + i);
  return make_float2(v.x, v.y);
}

// Position of the digit-reversed "high" index of the last stage: natural low
// output index klow = k0 + R0*(k1 + 16 k2 + ... + 16^(S-2) k_{S-1}) sits at
// hi = k0*16^(S-1) + k1*16^(S-2) + ... + k_{S-1} (position = hi*16 + row).
template <int R0, int S>
__device__ __forceinline__ int posrev_hi(int klow) {
  int k0 = klow % R0;
  int m = klow / R0;
  int hi = k0 << (4 * (S - 1));
#pragma unroll
  for (int s = 1; s < S; ++s) {
    hi += (m & 15) << (4 * (S - 1 - s));
    m >>= 4;
  }
  return hi;
}

// Loads the lane's A operands (see common.h).
struct FOps {
  h8 rh, ih, rl, il;
};
template <bool SPLIT>
__device__ __forceinline__ FOps load_fops(const void* fimg) {
  const TCFFT_GLOBAL h8* f = (const TCFFT_GLOBAL h8*)(fimg);
  const int lane = threadIdx.x & 63;
  FOps o;
  o.rh = f[lane];
  o.ih = f[64 + lane];
  if constexpr (SPLIT) {
    o.rl = f[128 + lane];
    o.il = f[192 + lane];
  } else {
    o.rl = o.rh;
    o.il = o.ih;
  }
  return o;
}

template <bool SPLIT>
__device__ __forceinline__ void dft_tile(u4 xh, u4 xl, const FOps& f, f4& yr, f4& yi) {
  if constexpr (SPLIT)
    mfma_dft16_split(xh, xl, f.rh, f.ih, f.rl, f.il, yr, yi);
  else
    mfma_dft16(xh, f.rh, f.ih, yr, yi);
}

template <bool SPLIT>
__device__ __forceinline__ void emit(float re, float im, uint32_t& h, uint32_t& l) {
  if constexpr (SPLIT)
    split2(re, im, h, l);
  else
    h = pack(re, im);
}

template <bool SPLIT>
__device__ __forceinline__ float2 value(uint32_t h, uint32_t l) {
  float2 v = unpack(h);
  if constexpr (SPLIT) {
    float2 w = unpack(l);
    v.x += w.x * (1.0f / 2048.0f);
    v.y += w.y * (1.0f / 2048.0f);
  }
  return v;
}

// ===========================================================================
// Row kernel: TPB contiguous lines per workgroup, LDS position p = tau*L + j.
// ===========================================================================
template <int L_, int R0_, int NT_, int WGP_ = 16384, bool NTL_ = true>
struct RowGeom {
  static constexpr int L = L_, R0 = R0_, NT = NT_;
  static constexpr bool NTL = NTL_;  // HBM loads non-temporal
  static constexpr int S = (ilog2c(L) - ilog2c(R0)) / 4;
  static_assert(pow16(S) * R0 == L, "L must be R0 * 16^S");
  // points per workgroup: 16384 = 4 quads per wave at 256 threads (64 KB of
  // FP16 LDS, two workgroups per CU); 8192 halves the LDS and the registers a
  // lane holds, for more resident waves
  static constexpr int WGPTS = WGP_;
  static constexpr int TPB = L >= WGPTS ? 1 : WGPTS / L;
  static constexpr int PTS = TPB * L;
  static constexpr int NW = NT / 64;
  static constexpr int NCOL = PTS / 16;
  static constexpr int NQ = NCOL / 64;
  static constexpr int QPW = NQ / NW;
  static_assert(QPW >= 1 && QPW * NW == NQ, "waves must split the quads evenly");
  static constexpr int P0 = L / R0;
  static constexpr int NCQ0 = PTS / R0 / 4;
};

// HBM load of a row pass (cache policy of the geometry).
template <class G>
__device__ __forceinline__ u4 row_ld4(const uint32_t* ptr) {
  if constexpr (G::NTL) return rld4(ptr);
  else return gld4(ptr);
}

// Position of element (row, col) of a radix-16 stage with digit stride P > 1.
template <int L, int P>
__device__ __forceinline__ int row_pos_t(int col, int row) {
  constexpr int NH = L / (16 * P);
  int lo = col % P;
  int rest = col / P;
  int hi = rest % NH;
  int tau = rest / NH;
  return tau * L + hi * 16 * P + row * P + lo;
}

// Twiddles of a stage whose 4 tiles sit at consecutive low indices r0 + t:
// W^{(4g+j)(r0+t)} = W^{(4g+j) r0} * W^{(4g+j) t}.  The second factor depends
// only on (g, j, t) and is loaded once per stage; the first is one lookup per
// row and quad.  `mul` maps the exponent onto the table W_L^m.
struct TwB {
  float2 b[4][3];  // [j][t-1] = W^{(4g+j) t}
};
__device__ __forceinline__ TwB load_twb(const float2* tw, int g, int mul) {
  TwB B;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int t = 1; t < 4; ++t) B.b[j][t - 1] = tld(tw, (4 * g + j) * t * mul);
  return B;
}

// Radix-R0 stage on the vector ALU, HBM -> LDS (always the first stage).
// SRCL: the input is already in LDS (natural order), read and rewritten in place.
template <class G, bool SPLIT, bool SRCL = false>
__device__ __forceinline__ void row_stage_r0(const KParams& kp, uint32_t* lds, int valid,
                                             int64_t g0) {
  constexpr int L = G::L, R0 = G::R0, P0 = G::P0;
  uint32_t* ldsl = lds + G::PTS;
  // W_L^{k t}, k < R0, t < 4: the same for every column quad
  float2 bt[R0][4];
#pragma unroll
  for (int k = 1; k < R0; ++k)
#pragma unroll
    for (int t = 1; t < 4; ++t) bt[k][t] = tld(kp.tw, k * t);
  constexpr int ITER = (G::NCQ0 + G::NT - 1) / G::NT;
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int cq = threadIdx.x + it * G::NT;
    if (G::NCQ0 % G::NT != 0 && cq >= G::NCQ0) break;
    const int col0 = 4 * cq;
    const int tau = col0 / P0;
    const int lo0 = col0 % P0;
    // lines past the end of the batch read line 0 of the tile (never stored)
    const int taul = (SRCL || tau < valid) ? tau : 0;
    u4 hh[R0], ll[R0];
#pragma unroll
    for (int d = 0; d < R0; ++d) {
      const int p = taul * L + d * P0 + lo0;
      if constexpr (SRCL) {
        hh[d] = lds_ld4(lds, p);
        if constexpr (SPLIT) ll[d] = lds_ld4(ldsl, p);
        else ll[d] = u4{0, 0, 0, 0};
      } else {
        hh[d] = row_ld4<G>(kp.in + g0 + p);
        if constexpr (SPLIT) ll[d] = row_ld4<G>(kp.in + kp.in_plane + g0 + p);
        else ll[d] = u4{0, 0, 0, 0};
      }
    }
    float2 a[R0];
#pragma unroll
    for (int k = 1; k < R0; ++k) {
      a[k] = tld(kp.tw, k * lo0);  // W_L^{k lo0}, k lo0 < L
      a[k].x *= kp.r0scale;
      a[k].y *= kp.r0scale;
    }
    float2 v[4][R0];
#pragma unroll
    for (int d = 0; d < R0; ++d)
#pragma unroll
      for (int t = 0; t < 4; ++t) v[t][d] = value<SPLIT>(hh[d][t], ll[d][t]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      small_dft<R0>(v[t], kp.sgn);
      v[t][0].x *= kp.r0scale;
      v[t][0].y *= kp.r0scale;
#pragma unroll
      for (int k = 1; k < R0; ++k) {
        const float2 w = t == 0 ? a[k] : cmul(a[k], bt[k][t]);  // W_L^{k (lo0 + t)}
        v[t][k] = cmul(v[t][k], w);
      }
    }
#pragma unroll
    for (int k = 0; k < R0; ++k) {
      u4 h, l;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        uint32_t eh = 0, el = 0;
        emit<SPLIT>(v[t][k].x, v[t][k].y, eh, el);
        h[t] = eh;
        l[t] = el;
      }
      const int p = tau * L + k * P0 + lo0;
      lds_st4(lds, p, h);
      if constexpr (SPLIT) lds_st4(ldsl, p, l);
    }
  }
}

// Radix-16 stage with digit stride P.  SRCG: read HBM (first stage), else LDS.
// P > 1: writes LDS (twiddled); P == 1: last stage, writes HBM in natural order.
// Loads of a stage (data, then twiddles) are all issued before the first use.
// HBM loads of a first radix-16 stage with P > 1 (rows 4g..4g+3 of each quad,
// 16 bytes along the low index), issued ahead of its compute by the pipelined
// row kernel.
template <class G>
struct Row16Regs {
  u4 h[G::QPW][4], l[G::QPW][4];
};
template <class G, int P, bool SPLIT>
__device__ __forceinline__ void row_stage16_load(const KParams& kp, int valid, int64_t g0,
                                                 Row16Regs<G>& r) {
  constexpr int L = G::L;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
#pragma unroll
  for (int qq = 0; qq < G::QPW; ++qq) {
    const int col0 = 4 * c16 + 64 * (wave * G::QPW + qq);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int p = row_pos_t<L, P>(col0, 4 * g + i);
      if (G::TPB > 1 && p / L >= valid) p -= (p / L) * L;  // clamp to line 0
      r.h[qq][i] = row_ld4<G>(kp.in + g0 + p);
      if constexpr (SPLIT) r.l[qq][i] = row_ld4<G>(kp.in + kp.in_plane + g0 + p);
      else r.l[qq][i] = u4{0, 0, 0, 0};
    }
  }
}

// TT (last stage only): transposed store for the second pass of a four-step
// transform.  The 4 tiles of a lane are 4 consecutive lines at one output
// index, so the lane writes output k of lines tau0..tau0+3 as one 16-byte
// group at b (q L) + k s_out + (line mod q) (line = global line index, q lines
// per transform): the pass writes X[k1 + q k2] with no gather.
//
// KEEP (last stage only): the results go to LDS in natural order instead of
// HBM, for an epilogue that reads whole lines.  The stage reads digit-reversed
// positions that other lanes overwrite, so the results wait in registers until
// every lane of the workgroup has read its inputs.
template <class G, int P, bool SRCG, bool SPLIT, bool PRE = false, bool TT = false,
          bool KEEP = false>
__device__ __forceinline__ void row_stage16(const KParams& kp, uint32_t* lds, int valid,
                                            int64_t g0, const FOps& f,
                                            const Row16Regs<G>* pre = nullptr) {
  constexpr int L = G::L, R0 = G::R0, S = G::S;
  constexpr int TM = P > 1 ? L / (16 * P) : 1;  // W_{16P}^e = W_L^{e TM}
  static_assert(!KEEP || (P == 1 && !SRCG && !TT && L / 16 >= 4), "natural-order LDS result");
  uint32_t* ldsl = lds + G::PTS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  u4 kh[KEEP ? G::QPW : 1][4], kl[KEEP && SPLIT ? G::QPW : 1][4];
  TwB B;
  if constexpr (P > 1) B = load_twb(kp.tw, g, TM);
#pragma unroll
  for (int qq = 0; qq < G::QPW; ++qq) {
    const int Q = wave * G::QPW + qq;
    const int col0 = 4 * c16 + 64 * Q;
    static_assert(!TT || (P == 1 && !SRCG && G::TPB >= 4 && G::TPB % 4 == 0), "transposed store");
    const int tau0 = TT ? 4 * ((col0 >> 2) % (G::TPB / 4)) : 0;
    const int klowT = TT ? (col0 >> 2) / (G::TPB / 4) : 0;
    u4 xh[4], xl[4];  // xh[t] = rows 4g..4g+3 of tile t
    if constexpr (P > 1) {
      // tiles along the contiguous low index: one 16-byte access per row
      u4 rh[4], rl[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int p = row_pos_t<L, P>(col0, 4 * g + i);
        if constexpr (PRE) {
          rh[i] = pre->h[qq][i];
          rl[i] = pre->l[qq][i];
        } else if constexpr (SRCG) {
          if (G::TPB > 1 && p / L >= valid) p -= (p / L) * L;  // clamp to line 0
          rh[i] = row_ld4<G>(kp.in + g0 + p);
          if constexpr (SPLIT) rl[i] = row_ld4<G>(kp.in + kp.in_plane + g0 + p);
        } else {
          rh[i] = lds_ld4(lds, p);
          if constexpr (SPLIT) rl[i] = lds_ld4(ldsl, p);
        }
        if constexpr (!SPLIT && !PRE) rl[i] = u4{0, 0, 0, 0};
      }
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          xh[t][i] = rh[i][t];
          xl[t][i] = rl[i][t];
        }
    } else {
      // last stage: rows are contiguous; columns enumerate natural order
      // (transposed store: lines tau0 + t at output column klowT)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = col0 + t;
        int tau = TT ? tau0 + t : col / (L / 16);
        if constexpr (SRCG && G::TPB > 1) tau = tau < valid ? tau : 0;
        const int p = tau * L + posrev_hi<R0, S>(TT ? klowT : col % (L / 16)) * 16 + 4 * g;
        if constexpr (SRCG) {
          xh[t] = row_ld4<G>(kp.in + g0 + p);
          if constexpr (SPLIT) xl[t] = row_ld4<G>(kp.in + kp.in_plane + g0 + p);
        } else {
          xh[t] = lds_ld4(lds, p);
          if constexpr (SPLIT) xl[t] = lds_ld4(ldsl, p);
        }
        if constexpr (!SPLIT) xl[t] = u4{0, 0, 0, 0};
      }
    }
    float2 a[4];  // W_{16P}^{(4g+j) r0}
    if constexpr (P > 1) {
      const int r0 = col0 % P;
#pragma unroll
      for (int j = 0; j < 4; ++j) a[j] = tld(kp.tw, (4 * g + j) * r0 * TM);
    }
    uint32_t oh[4][4], ol[4][4];  // [t][j]
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f4 yr, yi;
      dft_tile<SPLIT>(xh[t], xl[t], f, yr, yi);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float2 z = make_float2(yr[j], yi[j]);
        if constexpr (P > 1) z = cmul(z, t == 0 ? a[j] : cmul(a[j], B.b[j][t - 1]));
        uint32_t eh = 0, el = 0;
        emit<SPLIT>(z.x, z.y, eh, el);
        oh[t][j] = eh;
        ol[t][j] = el;
      }
    }
    if constexpr (P > 1) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = row_pos_t<L, P>(col0, 4 * g + j);
        lds_st4(lds, p, u4{oh[0][j], oh[1][j], oh[2][j], oh[3][j]});
        if constexpr (SPLIT) lds_st4(ldsl, p, u4{ol[0][j], ol[1][j], ol[2][j], ol[3][j]});
      }
    } else if constexpr (KEEP) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        kh[qq][j] = u4{oh[0][j], oh[1][j], oh[2][j], oh[3][j]};
        if constexpr (SPLIT) kl[qq][j] = u4{ol[0][j], ol[1][j], ol[2][j], ol[3][j]};
      }
    } else {
      // natural output index of (row, col): tau*L + klow + (L/16)*row
      if constexpr (TT) {
        const int64_t line0 = g0 / L + tau0;
        const int64_t b = line0 >> kp.q_log2;
        const int64_t base = b * kp.q * L + (line0 & (kp.q - 1));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t o = base + (int64_t)(klowT + (L / 16) * (4 * g + j)) * kp.s_out;
          if (tau0 + 3 < valid) {
            rst4(kp.out + o, u4{oh[0][j], oh[1][j], oh[2][j], oh[3][j]});
            if constexpr (SPLIT)
              rst4(kp.out + kp.out_plane + o, u4{ol[0][j], ol[1][j], ol[2][j], ol[3][j]});
          } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
              if (tau0 + t < valid) {
                gst1(kp.out + o + t, oh[t][j]);
                if constexpr (SPLIT) gst1(kp.out + kp.out_plane + o + t, ol[t][j]);
              }
          }
        }
      } else if constexpr (L / 16 >= 4) {
        const int tau = col0 / (L / 16);
        if (G::TPB == 1 || tau < valid) {
          const int klow0 = col0 % (L / 16);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int64_t o = g0 + (int64_t)tau * L + klow0 + (L / 16) * (4 * g + j);
            rst4(kp.out + o, u4{oh[0][j], oh[1][j], oh[2][j], oh[3][j]});
            if constexpr (SPLIT)
              rst4(kp.out + kp.out_plane + o, u4{ol[0][j], ol[1][j], ol[2][j], ol[3][j]});
          }
        }
      } else if constexpr (L == 16) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int tau = col0 + t;
          if (tau < valid) {
            const int64_t o = g0 + (int64_t)tau * 16 + 4 * g;
            rst4(kp.out + o, u4{oh[t][0], oh[t][1], oh[t][2], oh[t][3]});
            if constexpr (SPLIT)
              rst4(kp.out + kp.out_plane + o, u4{ol[t][0], ol[t][1], ol[t][2], ol[t][3]});
          }
        }
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int col = col0 + t;
          const int tau = col / (L / 16);
          if (tau < valid) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int64_t o = g0 + (int64_t)tau * L + col % (L / 16) + (L / 16) * (4 * g + j);
              gst1(kp.out + o, oh[t][j]);
              if constexpr (SPLIT) gst1(kp.out + kp.out_plane + o, ol[t][j]);
            }
          }
        }
      }
    }
  }
  if constexpr (KEEP) {
    __syncthreads();  // every lane has read its inputs
#pragma unroll
    for (int qq = 0; qq < G::QPW; ++qq) {
      const int col0 = 4 * c16 + 64 * (wave * G::QPW + qq);
      const int tau = col0 / (L / 16), klow0 = col0 % (L / 16);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = tau * L + klow0 + (L / 16) * (4 * g + j);
        lds_st4(lds, p, kh[qq][j]);
        if constexpr (SPLIT) lds_st4(ldsl, p, kl[qq][j]);
      }
    }
  }
}

// Whether the radix-R0 stage and the first radix-16 stage of a row pass run
// fused in registers (R0 in {2, 4}, at least two radix-16 stages, low-index
// quads, and whole super-quads per wave; see row_stage_fused).
template <class G>
struct RowFused {
  static constexpr int P = G::L / (16 * G::R0);  // digit stride of the first radix-16 stage
  static constexpr int NSQ = G::PTS / (64 * G::R0);
  static constexpr int ITF = NSQ / (16 * G::NW);
  static constexpr bool value = (G::R0 == 2 || G::R0 == 4) && G::S >= 2 && P >= 4 &&
                                ITF >= 1 && ITF * 16 * G::NW == NSQ;
};

// Radix-R0 stage fused with the first radix-16 stage (a radix-16*R0 block per
// column, Eq. 3 applied twice without an exchange in between).  A lane owns a
// super-quad: 4 adjacent low indices lo0..lo0+3 (16-byte accesses) of one line,
// rows m = 4g..4g+3 of the radix-16 digit and all R0 values of the radix-R0
// digit.  It runs the R0-point butterflies on the vector ALU, multiplies by
// W_L^{k (m P + lo)}, rounds once to FP16, and feeds the results as the B
// operands of R0 matrix-core DFTs (one per radix-R0 output k), whose results
// take the twiddle W_{16P}^{k1 lo} and go to LDS at the positions the unfused
// first radix-16 stage writes.
template <class G, bool SPLIT, bool SRCL = false>
__device__ __forceinline__ void row_stage_fused(const KParams& kp, uint32_t* lds, int valid,
                                                int64_t g0, const FOps& f) {
  constexpr int L = G::L, R0 = G::R0;
  using F = RowFused<G>;
  constexpr int P = F::P, P0 = 16 * P, ITF = F::ITF;
  uint32_t* ldsl = lds + G::PTS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  // W_L^{k (4g+i) P} (scaled by the radix-R0 stage scale) and W_L^{k t}
  float2 wm[R0][4], bt[R0][4];
#pragma unroll
  for (int k = 1; k < R0; ++k)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float2 w = tld(kp.tw, k * (4 * g + i) * P);
      w.x *= kp.r0scale;
      w.y *= kp.r0scale;
      wm[k][i] = w;
      bt[k][i] = tld(kp.tw, k * i);
    }
  const TwB B = load_twb(kp.tw, g, R0);  // W_{16P}^{(4g+j) t} = W_L^{(4g+j) t R0}
#pragma unroll
  for (int it = 0; it < ITF; ++it) {
    const int sq = (wave * ITF + it) * 16 + c16;
    const int tau = sq / (P / 4);
    const int lo0 = 4 * (sq % (P / 4));
    // past the batch: line 0 (LDS source: the lane's own positions, in place)
    const int taul = (!SRCL && G::TPB > 1 && tau >= valid) ? 0 : tau;
    u4 hh[R0][4], ll[R0][4];
#pragma unroll
    for (int d = 0; d < R0; ++d)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = taul * L + d * P0 + (4 * g + i) * P + lo0;
        if constexpr (SRCL) {
          hh[d][i] = lds_ld4(lds, p);
          if constexpr (SPLIT) ll[d][i] = lds_ld4(ldsl, p);
          else ll[d][i] = u4{0, 0, 0, 0};
        } else {
          hh[d][i] = row_ld4<G>(kp.in + g0 + p);
          if constexpr (SPLIT) ll[d][i] = row_ld4<G>(kp.in + kp.in_plane + g0 + p);
          else ll[d][i] = u4{0, 0, 0, 0};
        }
      }
    float2 at[R0][4];  // W_L^{k (lo0 + t)}
#pragma unroll
    for (int k = 1; k < R0; ++k) {
      const float2 a = tld(kp.tw, k * lo0);
      at[k][0] = a;
#pragma unroll
      for (int t = 1; t < 4; ++t) at[k][t] = cmul(a, bt[k][t]);
    }
    float2 a16[4];  // W_{16P}^{(4g+j) lo0}
#pragma unroll
    for (int j = 0; j < 4; ++j) a16[j] = tld(kp.tw, (4 * g + j) * lo0 * R0);
    uint32_t oh[R0][4][4], ol[R0][4][4];  // [k][t][j]
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      u4 xh[R0], xl[R0];  // B operands: rows i of the radix-16 digit, per k
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float2 v[R0];
#pragma unroll
        for (int d = 0; d < R0; ++d) v[d] = value<SPLIT>(hh[d][i][t], ll[d][i][t]);
        small_dft<R0>(v, kp.sgn);
        v[0].x *= kp.r0scale;
        v[0].y *= kp.r0scale;
#pragma unroll
        for (int k = 1; k < R0; ++k) v[k] = cmul(v[k], cmul(wm[k][i], at[k][t]));
#pragma unroll
        for (int k = 0; k < R0; ++k) {
          uint32_t eh = 0, el = 0;
          emit<SPLIT>(v[k].x, v[k].y, eh, el);
          xh[k][i] = eh;
          xl[k][i] = el;
        }
      }
#pragma unroll
      for (int k = 0; k < R0; ++k) {
        f4 yr, yi;
        dft_tile<SPLIT>(xh[k], xl[k], f, yr, yi);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          float2 z = make_float2(yr[j], yi[j]);
          z = cmul(z, t == 0 ? a16[j] : cmul(a16[j], B.b[j][t - 1]));
          uint32_t eh = 0, el = 0;
          emit<SPLIT>(z.x, z.y, eh, el);
          oh[k][t][j] = eh;
          ol[k][t][j] = el;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < R0; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = tau * L + k * P0 + (4 * g + j) * P + lo0;
        lds_st4(lds, p, u4{oh[k][0][j], oh[k][1][j], oh[k][2][j], oh[k][3][j]});
        if constexpr (SPLIT) lds_st4(ldsl, p, u4{ol[k][0][j], ol[k][1][j], ol[k][2][j], ol[k][3][j]});
      }
  }
}

// ---------------------------------------------------------------------------
// Radix-R0 x radix-16 block entirely on the matrix core (FP16 data; used by
// the column passes, see col_fused_mx).  With the
// digits n = d P0 + m P + lo of a line (P0 = 16 P) and the DIF order of the
// fused stage, radix-R0 output k and radix-16 output k1 are
//   Y[k][k1][lo] = W_L^{(k + R0 k1) lo} *
//                  sum_d W_R0^{k d} sum_m (F_16[k1][m] W_{16 R0}^{k m}) x[d][m][lo]
// (Eq. 3 applied twice: W_L^{k m P} = W_{16 R0}^{k m}).  The bracket is the
// A operand A_k of a radix-16 product, one image per k (plan table kp.fimg2,
// scaled by both stages' scales), and the radix-R0 sum over d accumulates R0
// such products in the MFMA accumulator.  W_R0^{k d} in {1, i, -1, -i} (R0 <= 4)
// multiplies A_k exactly: with the images (Yr, Yi) of A_k,
//   i A_k -> (-Yi, Yr),   -A_k -> (-Yr, -Yi),   -i A_k -> (Yi, -Yr),
// so the raw FP16 inputs are the B operands (no vector-ALU butterflies and no
// rounding before the product) and the only twiddle, W_L^{(k + R0 k1) lo},
// is applied once to the FP32 accumulator.  The code follows the forward
// sign: an inverse transform's W^{k d} is the forward W^{k' d} with
// k' = (R0 - k) mod R0, so slot k' of an inverse plan's table holds A_k and
// the block computed as k' is stored and twiddled as output k.
__device__ __forceinline__ h8 neg_h8(h8 a) {
  u4 v = __builtin_bit_cast(u4, a);
  v ^= u4{0x80008000u, 0x80008000u, 0x80008000u, 0x80008000u};
  return __builtin_bit_cast(h8, v);
}

// Images of one A_k and their negations.
struct FOpsMx {
  h8 r, i, nr, ni;
};

__device__ __forceinline__ FOpsMx load_fops_mx(const void* fimg2, int k) {
  const TCFFT_GLOBAL h8* f = (const TCFFT_GLOBAL h8*)(fimg2);
  const int lane = threadIdx.x & 63;
  FOpsMx o;
  o.r = f[256 * k + lane];
  o.i = f[256 * k + 64 + lane];
  o.nr = neg_h8(o.r);
  o.ni = neg_h8(o.i);
  return o;
}

// yr, yi += (W^{k d} A_k) . b, where the forward W^{k d} = e^{-2 pi i Q / 4}
// is Q quarter turns.
template <int Q>
__device__ __forceinline__ void mfma_rot(const FOpsMx& f, u4 b, f4& yr, f4& yi) {
  const h8 bh = __builtin_bit_cast(h8, b);
  h8 ar, ai;
  constexpr int qq = (4 - Q) & 3;  // in units of +i
  if constexpr (qq == 0) {
    ar = f.r;
    ai = f.i;
  } else if constexpr (qq == 1) {
    ar = f.ni;
    ai = f.r;
  } else if constexpr (qq == 2) {
    ar = f.nr;
    ai = f.ni;
  } else {
    ar = f.i;
    ai = f.nr;
  }
  yr = __builtin_amdgcn_mfma_f32_16x16x32_f16(ar, bh, yr, 0, 0, 0);
  yi = __builtin_amdgcn_mfma_f32_16x16x32_f16(ai, bh, yi, 0, 0, 0);
}

// Radix-R0 sum over d for output k of the fused block (compile-time k, d).
template <int R0, int K, int D = 0>
__device__ __forceinline__ void mfma_rsum(const FOpsMx& f, const u4 (&b)[R0], f4& yr, f4& yi) {
  mfma_rot<((K * D) % R0) * (4 / R0)>(f, b[D], yr, yi);
  if constexpr (D + 1 < R0) mfma_rsum<R0, K, D + 1>(f, b, yr, yi);
}

// ---------------------------------------------------------------------------
// Radix-16 LDS stage with digit stride 16 and its twiddle folded into the
// matrix-core operand (FP16 data).  Columns of the stage are (line, hi, lo),
// lo < 16; its DIF twiddle W_256^{k1 lo} depends on the output row k1 and on
// lo only, so an MFMA tile of 16 columns with one lo and 16 consecutive hi
// takes A_lo = diag(W_256^{k1 lo}) F_16 (16 images, plan table kp.fimg3) and
// needs no vector-ALU twiddle.  A lane's 4 tiles are lo0..lo0+3 (16-byte LDS
// accesses along lo), wave w takes lo0 = 4w and its quads run over the
// (line, hi-group) pairs, so it loads its 4 images once per stage.
template <class G>
struct RowFold {
  static constexpr int NH = G::L / 256;  // hi values per line at stride 16
  static constexpr bool value = G::L >= 4096 && G::NT == 256 && G::NW == 4 &&
                                G::TPB * NH / 16 == G::QPW;
};

template <class G>
__device__ __forceinline__ void row_stage16_fold(const KParams& kp, uint32_t* lds) {
  constexpr int L = G::L, P = 16, NH = RowFold<G>::NH, HG = NH / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  const int lo0 = 4 * wave;
  const TCFFT_GLOBAL h8* img = (const TCFFT_GLOBAL h8*)(kp.fimg3);
  h8 ar[4], ai[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    ar[t] = img[256 * (lo0 + t) + lane];
    ai[t] = img[256 * (lo0 + t) + 64 + lane];
  }
#pragma unroll
  for (int qq = 0; qq < G::QPW; ++qq) {
    const int tau = qq / HG, hi = (qq % HG) * 16 + c16;
    const int base = tau * L + hi * 16 * P + lo0;
    u4 rh[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) rh[i] = lds_ld4(lds, base + (4 * g + i) * P);
    uint32_t oh[4][4];  // [t][j]
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const h8 bh = __builtin_bit_cast(h8, u4{rh[0][t], rh[1][t], rh[2][t], rh[3][t]});
      const f4 z = {0.f, 0.f, 0.f, 0.f};
      const f4 yr = __builtin_amdgcn_mfma_f32_16x16x32_f16(ar[t], bh, z, 0, 0, 0);
      const f4 yi = __builtin_amdgcn_mfma_f32_16x16x32_f16(ai[t], bh, z, 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 4; ++j) oh[t][j] = pack(yr[j], yi[j]);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
      lds_st4(lds, base + (4 * g + j) * P, u4{oh[0][j], oh[1][j], oh[2][j], oh[3][j]});
  }
}

template <class G, int E, bool SPLIT, bool TT = false, bool KEEP = false>
__device__ __forceinline__ void row_stages_from(const KParams& kp, uint32_t* lds, int valid,
                                                int64_t g0, const FOps& f) {
  // radix-16 stages with stride 16^E, 16^(E-1), ..., 1, all reading LDS
  if constexpr (E == 1 && !SPLIT && RowFold<G>::value)
    row_stage16_fold<G>(kp, lds);
  else
    row_stage16<G, pow16(E), false, SPLIT, false, E == 0 && TT, E == 0 && KEEP>(kp, lds, valid,
                                                                                g0, f);
  if constexpr (E > 0) {
    __syncthreads();
    row_stages_from<G, E - 1, SPLIT, TT, KEEP>(kp, lds, valid, g0, f);
  }
}

// ---------------------------------------------------------------------------
// Real-input transforms fused into a row pass of M = L points.  An N = 2M
// point real sequence is read as M complex words z[m] = x[2m] + i x[2m+1];
// with Z its M-point DFT and W = W_N (the table kp.xtw_lo holds W^{dir k},
// k <= M), the even/odd split of Eq. 2 (N1 = 2) gives for the spectrum
//   X[k] = ((Z[k] + conj Z[M-k]) - i W^k (Z[k] - conj Z[M-k])) / 2,  k <= M,
// and for the inverse
//   Z'[k] = (X[k] + conj X[M-k]) + i W^-k (X[k] - conj X[M-k]),      k < M,
// whose inverse M-point DFT is N (x[2m] + i x[2m+1]).  Index k and M - k come
// from the same pair of inputs, and W^{M-k} = -conj(W^k), so one lane handles
// both.  Spectrum lines hold M + 1 words.

// Work split of the real epilogue / prologue: item (line, j), j < M/2, covers
// the index pair (j, M - j) (j = 0 pairs bin 0 with bin M); the self-paired
// middle index M/2 of each line is a separate short loop.  Thread t takes
// items it = 0 .. ITER-1 with, for M/2 >= NT, j = t + NT (it mod NQ) and
// line = it / NQ, else j = t mod M/2 and line = t / (M/2) + it NT / (M/2): the
// line and the high part of j are compile-time per item, and the twiddle
// W^j = W^t * W^{NT q} is one table load per thread times a uniform value.
// Items go in groups per thread with every load of a group issued before its
// first use: 32 items per group for the epilogue (LDS loads), 16 for the
// prologue (HBM loads; larger groups measured slower there).
template <class G>
struct RealLoop {
  static constexpr int M = G::L, HM = M / 2, NT = G::NT;
  static constexpr int ITER = G::TPB * HM / NT;
  static constexpr int UPOST = ITER < 32 ? ITER : 32, UPRE = ITER < 16 ? ITER : 16;
  static constexpr bool WIDE = HM >= NT;       // a line spans NQ items of a thread
  static constexpr int NQ = WIDE ? HM / NT : 1;
  static constexpr int LPI = WIDE ? 1 : NT / HM;  // lines per item step
  static_assert(ITER >= 1 && ITER * NT == G::TPB * HM && ITER % UPOST == 0 && ITER % UPRE == 0,
                "item split");
  __device__ static int line(int it) {
    return WIDE ? it / NQ : (int)threadIdx.x / HM + it * LPI;
  }
  __device__ static int j(int it) {
    return WIDE ? (int)threadIdx.x + NT * (it % NQ) : (int)threadIdx.x & (HM - 1);
  }
  // W^{NT (j div NT)}: uniform across the workgroup (1 when it does not vary)
  __device__ static float2 wq(const float2* tab, int it) {
    if constexpr (WIDE) return tld(tab, NT * (it % NQ));
    return make_float2(1.f, 0.f);
  }
  // W^j from the thread's W^{j mod NT} (wt) and the uniform factor
  __device__ static float2 w(float2 wt, float2 q, int it) {
    if constexpr (WIDE) return it % NQ == 0 ? wt : cmul(wt, q);
    return wt;
  }
  __device__ static float2 wthread(const float2* tab) {
    return tld(tab, WIDE ? (int)threadIdx.x : ((int)threadIdx.x & (HM - 1)));
  }
};

// Both members of an index pair from one twiddle product.  Forward, with
// a = Z[k], b = Z[M-k], e = a + conj b, d = a - conj b, v = -i W^k d:
//   X[k] = (e + v) / 2,   X[M-k] = conj(e - v) / 2
// (swapping a and b conjugates e, negates conj d, and W^{M-k} = -conj W^k).
// Inverse, with a = X[k], c = X[M-k], e = a + conj c, t = i W^-k (a - conj c):
//   Z'[k] = e + t,        Z'[M-k] = conj(e - t).
__device__ __forceinline__ void real_spec(float2 a, float2 b, float2 w, float2& xk, float2& xm) {
  const float2 h = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));  // e / 2
  const float2 d = make_float2(a.x - b.x, a.y + b.y);
  const float2 v = cmul(make_float2(0.5f * w.x, 0.5f * w.y), make_float2(d.y, -d.x));  // v / 2
  xk = make_float2(h.x + v.x, h.y + v.y);
  xm = make_float2(h.x - v.x, v.y - h.y);
}
__device__ __forceinline__ void real_zpre(float2 a, float2 c, float2 w, float2& zk, float2& zm) {
  const float2 e = make_float2(a.x + c.x, a.y - c.y);
  const float2 d = cmul(make_float2(a.x - c.x, a.y + c.y), w);
  const float2 t = make_float2(-d.y, d.x);  // i W^-k (a - conj c)
  zk = make_float2(e.x + t.x, e.y + t.y);
  zm = make_float2(e.x - t.x, t.y - e.y);
}

// R2C epilogue: Z of `valid` lines in LDS (natural order) -> X in HBM.
template <class G, bool SPLIT>
__device__ __forceinline__ void real_post(const KParams& kp, const uint32_t* lds, int valid,
                                          int64_t t0) {
  using R = RealLoop<G>;
  constexpr int M = R::M, HM = R::HM, U = R::UPOST;
  const uint32_t* ldsl = lds + G::PTS;
  uint32_t* const oh = kp.out + t0 * (int64_t)(M + 1);
  uint32_t* const ol = oh + kp.out_plane;
  auto rd = [&](int p) { return value<SPLIT>(lds_ld1(lds, p), SPLIT ? lds_ld1(ldsl, p) : 0u); };
  auto st = [&](uint32_t off, float2 v) {
    uint32_t h = 0, l = 0;
    emit<SPLIT>(v.x, v.y, h, l);
    gst1(oh + off, h);
    if constexpr (SPLIT) gst1(ol + off, l);
  };
  const float2 wt = R::wthread(kp.xtw_lo);
#pragma unroll
  for (int it0 = 0; it0 < R::ITER; it0 += U) {
    float2 a[U], b[U], q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int line = R::line(it0 + u), j = R::j(it0 + u);
      a[u] = rd(line * M + j);
      b[u] = rd(line * M + ((M - j) & (M - 1)));
      q[u] = R::wq(kp.xtw_lo, it0 + u);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int line = R::line(it0 + u), j = R::j(it0 + u);
      if (line < valid) {
        float2 xk, xm;
        real_spec(a[u], b[u], R::w(wt, q[u], it0 + u), xk, xm);
        const uint32_t off = (uint32_t)(line * (M + 1) + j);
        st(off, xk);
        st(off + (uint32_t)(M - 2 * j), xm);  // X[M-j]
      }
    }
  }
  const float2 wm = tld(kp.xtw_lo, HM);
  for (int line = threadIdx.x; line < valid; line += G::NT) {
    const float2 z = rd(line * M + HM);
    float2 xk, xm;
    real_spec(z, z, wm, xk, xm);
    st((uint32_t)(line * (M + 1) + HM), xk);
  }
}

// C2R prologue: X of `valid` lines in HBM -> Z' in LDS (natural order).  The
// imaginary parts of X[0] and X[M] are ignored (a real sequence has them 0).
template <class G, bool SPLIT>
__device__ __forceinline__ void real_pre(const KParams& kp, uint32_t* lds, int valid, int64_t t0) {
  using R = RealLoop<G>;
  constexpr int M = R::M, HM = R::HM, U = R::UPRE;
  uint32_t* ldsl = lds + G::PTS;
  const uint32_t* const xh = kp.in + t0 * (int64_t)(M + 1);
  const uint32_t* const xl = xh + kp.in_plane;
  auto rd = [&](uint32_t off) { return value<SPLIT>(gld1(xh + off), SPLIT ? gld1(xl + off) : 0u); };
  auto st = [&](int p, float2 v) {
    uint32_t h = 0, l = 0;
    emit<SPLIT>(v.x, v.y, h, l);
    lds_st1(lds, p, h);
    if constexpr (SPLIT) lds_st1(ldsl, p, l);
  };
  const float2 wt = R::wthread(kp.xtw_lo);
#pragma unroll
  for (int it0 = 0; it0 < R::ITER; it0 += U) {
    float2 a[U], c[U], q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int line = R::line(it0 + u);
      const int j = R::j(it0 + u);
      line = line < valid ? line : 0;  // past the batch: line 0, never stored
      const uint32_t off = (uint32_t)(line * (M + 1) + j);
      a[u] = rd(off);
      c[u] = rd(off + (uint32_t)(M - 2 * j));
      q[u] = R::wq(kp.xtw_lo, it0 + u);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int line = R::line(it0 + u), j = R::j(it0 + u);
      if (line < valid) {
        if (j == 0) {  // X[0] and X[M]: real parts only; Z'[M] does not exist
          a[u].y = 0.f;
          c[u].y = 0.f;
        }
        float2 zk, zm;
        real_zpre(a[u], c[u], R::w(wt, q[u], it0 + u), zk, zm);
        st(line * M + j, zk);
        if (j != 0) st(line * M + M - j, zm);
      }
    }
  }
  const float2 wm = tld(kp.xtw_lo, HM);
  for (int line = threadIdx.x; line < valid; line += G::NT) {
    const float2 x = rd((uint32_t)(line * (M + 1) + HM));
    float2 zk, zm;
    real_zpre(x, x, wm, zk, zm);
    st(line * M + HM, zk);
  }
}

// One workgroup's share of a row pass: workgroup index wg of the pass.
// RK: 0 complex; 1 real forward (spectrum epilogue); 2 real inverse (prologue);
// 3 results stay in LDS in natural order (the first half of a plane pass).
template <int L, int R0, int NT, bool SPLIT, bool TT = false, int RK = 0, int WGP = 16384>
__device__ __forceinline__ void row_body(const KParams& kp, int64_t wg, uint32_t* lds) {
  // a plane pass's row half (RK == 3) loads with the default cache policy
  using G = RowGeom<L, R0, NT, WGP, RK != 3>;
  static_assert(RK == 0 || (!TT && G::S >= 1 && L >= 64), "real / plane variants");
  constexpr bool KEEP = RK == 1 || RK == 3, SRCL = RK == 2;
  const int64_t t0 = wg * G::TPB;
  const int64_t rem = kp.ntrans - t0;
  const int valid = rem < G::TPB ? (int)rem : G::TPB;
  const int64_t g0 = t0 * L;
  const FOps f = load_fops<SPLIT>(kp.fimg);
  if constexpr (SRCL) {
    real_pre<G, SPLIT>(kp, lds, valid, t0);
    __syncthreads();
  }
  if constexpr (RowFused<G>::value) {
    row_stage_fused<G, SPLIT, SRCL>(kp, lds, valid, g0, f);
    __syncthreads();
    row_stages_from<G, G::S - 2, SPLIT, TT, KEEP>(kp, lds, valid, g0, f);
  } else if constexpr (R0 > 1) {
    row_stage_r0<G, SPLIT, SRCL>(kp, lds, valid, g0);
    __syncthreads();
    row_stages_from<G, G::S - 1, SPLIT, TT, KEEP>(kp, lds, valid, g0, f);
  } else {
    static_assert(!KEEP || G::S > 1, "the epilogue follows an LDS stage");
    row_stage16<G, pow16(G::S - 1), !SRCL, SPLIT>(kp, lds, valid, g0, f);
    if constexpr (G::S > 1) {
      __syncthreads();
      row_stages_from<G, G::S - 2, SPLIT, TT, KEEP>(kp, lds, valid, g0, f);
    }
  }
  if constexpr (RK == 1) {
    __syncthreads();
    real_post<G, SPLIT>(kp, lds, valid, t0);
  }
}

// Whether a row pass runs as a pipelined persistent kernel: passes whose first
// stage is radix-16 from HBM with P > 1, followed by at least one LDS stage,
// at 256 threads.  Workgroup b runs tiles b, b + grid, ... and overlaps its own
// next loads with its LDS stages: split data (two LDS planes, one workgroup
// per CU) and FP16 (4096: 221 -> 202 us for 2^27 points).  Passes with a fused
// radix-2/4 first stage keep one tile per workgroup: holding the next tile's
// inputs over the LDS stages leaves them one workgroup per CU (16384: 244 ->
// 259 us).
template <class G, bool SPLIT>
struct RowPipe {
  static constexpr bool value = G::NT == 256 && !RowFused<G>::value && G::R0 == 1 && G::S >= 2;
};

// Pipelined persistent row pass: workgroup b runs tiles b, b + grid, ...; the
// HBM loads of the next tile's first stage are issued right after the current
// tile's first stage has consumed its registers, so they are in flight while
// the current tile runs its LDS stages and stores.
template <int L, int R0, int NT, bool SPLIT>
__device__ __forceinline__ void row_pipe(const KParams& kp, uint32_t* lds) {
  using G = RowGeom<L, R0, NT>;
  constexpr int P1 = pow16(G::S - 1);
  const int64_t ntiles = (kp.ntrans + G::TPB - 1) / G::TPB;
  const FOps f = load_fops<SPLIT>(kp.fimg);
  auto valid_of = [&](int64_t w) {
    const int64_t rem = kp.ntrans - w * G::TPB;
    return rem < G::TPB ? (int)rem : G::TPB;
  };
  int64_t w = blockIdx.x;
  if (w >= ntiles) return;
  Row16Regs<G> r;
  row_stage16_load<G, P1, SPLIT>(kp, valid_of(w), w * G::TPB * L, r);
  for (; w < ntiles; w += gridDim.x) {
    const int valid = valid_of(w);
    const int64_t g0 = w * G::TPB * L;
    row_stage16<G, P1, true, SPLIT, true>(kp, lds, valid, g0, f, &r);
    const int64_t wn = w + gridDim.x;
    if (wn < ntiles) row_stage16_load<G, P1, SPLIT>(kp, valid_of(wn), wn * G::TPB * L, r);
    __syncthreads();
    row_stages_from<G, G::S - 2, SPLIT>(kp, lds, valid, g0, f);
    __syncthreads();  // the next tile's first stage rewrites LDS
  }
}

template <int L, int R0, int NT, bool SPLIT, bool TT = false, int RK = 0, int WGP = 16384>
__global__ __launch_bounds__(NT) void row_kernel(KParams kp) {
  extern __shared__ uint32_t lds[];
  if constexpr (!TT && RK == 0 && WGP == 16384 && RowPipe<RowGeom<L, R0, NT>, SPLIT>::value)
    row_pipe<L, R0, NT, SPLIT>(kp, lds);
  else
    row_body<L, R0, NT, SPLIT, TT, RK, WGP>(kp, blockIdx.x, lds);
}

// ===========================================================================
// Column kernel: C adjacent columns of an [L][inner] block per workgroup, LDS
// position p = j*C + c.  Tiles of 4 always run along c (contiguous in HBM and
// LDS), so every access is 16 bytes per lane and C*4 bytes per row.
// ===========================================================================
template <int L_, int R0_, int C_, int NT_>
struct ColGeom {
  static constexpr int L = L_, R0 = R0_, C = C_, NT = NT_;
  static constexpr int S = (ilog2c(L) - ilog2c(R0)) / 4;
  static_assert(pow16(S) * R0 == L, "L must be R0 * 16^S");
  static constexpr int PTS = L * C;
  static constexpr int NW = NT / 64;
  static constexpr int NCOL = PTS / 16;
  static constexpr int NQ = NCOL / 64 > 0 ? NCOL / 64 : 1;
  static constexpr int QPW = NQ / NW;
  static_assert(QPW >= 1 && QPW * NW == NQ, "waves must split the quads evenly");
  static constexpr int P0 = L / R0;
  static constexpr int NCQ0 = PTS / R0 / 4;
};

struct ColCtx {
  int64_t in_base, out_base;  // element offsets of tile column 0
  int lds_off = 0;            // LDS position of the block (several blocks per workgroup)
  int64_t i0;                 // first global column index of the tile
  int64_t outer;
};

// SRCL: the block is already in LDS (position j*C + c), read and rewritten in
// place by the same lane.
template <class G, bool SPLIT, bool SRCL = false>
__device__ __forceinline__ void col_stage_r0(const KParams& kp, uint32_t* lds, const ColCtx& cx) {
  constexpr int L = G::L, R0 = G::R0, C = G::C, P0 = G::P0;
  uint32_t* ldsl = lds + G::PTS;
  constexpr int ITER = (G::NCQ0 + G::NT - 1) / G::NT;
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int cq = threadIdx.x + it * G::NT;
    if (G::NCQ0 % G::NT != 0 && cq >= G::NCQ0) break;
    const int col0 = 4 * cq;
    const int c = col0 % C;
    const int lo = col0 / C;  // in [0, P0)
    u4 hh[R0], ll[R0];
#pragma unroll
    for (int d = 0; d < R0; ++d) {
      if constexpr (SRCL) {
        hh[d] = lds_ld4(lds, cx.lds_off + (d * P0 + lo) * C + c);
        if constexpr (SPLIT) ll[d] = lds_ld4(ldsl, cx.lds_off + (d * P0 + lo) * C + c);
        else ll[d] = u4{0, 0, 0, 0};
      } else {
        const int64_t a = cx.in_base + (int64_t)(d * P0 + lo) * kp.s_in + c;
        hh[d] = gld4(kp.in + a);
        if constexpr (SPLIT) ll[d] = gld4(kp.in + kp.in_plane + a);
        else ll[d] = u4{0, 0, 0, 0};
      }
    }
    float2 wt[R0];
#pragma unroll
    for (int k = 0; k < R0; ++k) wt[k] = tld(kp.tw, k * lo);
    float2 v[4][R0];
#pragma unroll
    for (int d = 0; d < R0; ++d)
#pragma unroll
      for (int t = 0; t < 4; ++t) v[t][d] = value<SPLIT>(hh[d][t], ll[d][t]);
#pragma unroll
    for (int t = 0; t < 4; ++t) small_dft<R0>(v[t], kp.sgn);
#pragma unroll
    for (int k = 0; k < R0; ++k) {
      float2 w = wt[k];
      w.x *= kp.r0scale;
      w.y *= kp.r0scale;
      u4 h, l;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float2 z = cmul(v[t][k], w);
        uint32_t eh = 0, el = 0;
        emit<SPLIT>(z.x, z.y, eh, el);
        h[t] = eh;
        l[t] = el;
      }
      const int p = cx.lds_off + (k * P0 + lo) * C + c;
      lds_st4(lds, p, h);
      if constexpr (SPLIT) lds_st4(ldsl, p, l);
    }
  }
}

// Extra inter-pass twiddle W_M^{ci * k} (two-level table, FP32).  M is a power
// of two below 2^32, so the exponent needs only the low 32 bits of ci * k.
__device__ __forceinline__ float2 xtwiddle(const KParams& kp, uint32_t ci, uint32_t k) {
  const uint32_t e = (ci * k) & kp.xmask;
  const float2 a = tld(kp.xtw_lo, e & ((1u << kp.xbits) - 1u));
  const float2 b = tld(kp.xtw_hi, e >> kp.xbits);
  return cmul(a, b);
}

// Where quad qq of the calling lane sits in a radix-16 column stage of digit
// stride P: its 4 adjacent columns c..c+3, its column block `rest` (restl: the
// block it reads, 0 for the idle lanes of tiles with fewer than 64 columns),
// the low index lo and the first row jb (row r of the digit is jb + r P).
template <class G, int P>
struct ColQuad {
  int c, rest, restl, lo, jb;
  bool active;
  __device__ __forceinline__ explicit ColQuad(int qq) {
    constexpr int L = G::L, R0 = G::R0, S = G::S, C = G::C;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c16 = lane & 15;
    const int col0 = 4 * c16 + 64 * (wave * G::QPW + qq);
    c = col0 % C;
    rest = col0 / C;
    constexpr bool kFull = G::NCOL >= 64 * G::NQ;
    active = kFull || rest < L / 16;
    restl = active ? rest : 0;
    lo = 0;
    if constexpr (P > 1) {
      lo = restl % P;
      jb = (restl / P) * 16 * P + lo;
    } else {
      jb = posrev_hi<R0, S>(restl) * 16;
    }
  }
};

// HBM loads of a first radix-16 column stage with P > 1 (rows 4g..4g+3 of each
// quad at its 4 adjacent columns), issued ahead of its compute by the pipelined
// column kernel.
template <class G>
struct Col16Regs {
  u4 h[G::QPW][4], l[G::QPW][4];
};
template <class G, int P, bool SPLIT>
__device__ __forceinline__ void col_stage16_load(const KParams& kp, const ColCtx& cx,
                                                 Col16Regs<G>& r) {
  const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int qq = 0; qq < G::QPW; ++qq) {
    const ColQuad<G, P> q(qq);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = q.jb + (4 * g + i) * P;
      const int64_t a = cx.in_base + (int64_t)j * kp.s_in + q.c;
      r.h[qq][i] = gld4(kp.in + a);
      if constexpr (SPLIT) r.l[qq][i] = gld4(kp.in + kp.in_plane + a);
      else r.l[qq][i] = u4{0, 0, 0, 0};
    }
  }
}

// Inter-pass twiddle factors of a last stage (P = 1): per quad and output row
// j, a = W_M^{(ci0 / xdiv) k} and the column step b = W_M^k (xdiv = 1; else
// unused).  Passes with a single radix-16 stage load them before their HBM
// reads, so the table lookups overlap those reads instead of waiting at the
// end of the pass.
template <class G>
struct XtwRegs {
  float2 a[G::QPW][4], b[G::QPW][4];
};
template <class G>
__device__ __forceinline__ void xtw_prefetch(const KParams& kp, const ColCtx& cx, XtwRegs<G>& x) {
  constexpr int L = G::L;
  const int g = (threadIdx.x & 63) >> 4;
  const uint32_t lo_mask = (1u << kp.xbits) - 1u;
#pragma unroll
  for (int qq = 0; qq < G::QPW; ++qq) {
    const ColQuad<G, 1> q(qq);
    const uint32_t ci = (uint32_t)(kp.xoff + cx.i0 + q.c);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t k = (uint32_t)(q.restl + (L / 16) * (4 * g + j));
      x.a[qq][j] = xtwiddle(kp, ci >> kp.xdiv_log2, k);
      x.b[qq][j] = tld(kp.xtw_lo, k & lo_mask);  // k < L <= 2^xbits where xdiv = 1
    }
  }
}

// PRE (first stage only): the stage's HBM inputs are already in `pre`.
// XPRE (last stage with XTW): the inter-pass twiddle factors are in `xp`.
template <class G, int P, bool SRCG, bool SPLIT, bool XTW, bool TSTORE, bool PRE = false,
          bool XPRE = false>
__device__ __forceinline__ void col_stage16(const KParams& kp, uint32_t* lds, const ColCtx& cx,
                                            const FOps& f, const Col16Regs<G>* pre = nullptr,
                                            const XtwRegs<G>* xp = nullptr) {
  constexpr int L = G::L, R0 = G::R0, S = G::S, C = G::C;
  static_assert(!PRE || (SRCG && P > 1), "prefetched inputs feed a first stage");
  uint32_t* ldsl = lds + G::PTS;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4;
#pragma unroll
  for (int qq = 0; qq < G::QPW; ++qq) {
    const ColQuad<G, P> q(qq);
    const int c = q.c, rest = q.rest, restl = q.restl, lo = q.lo, jb = q.jb;
    const bool active = q.active;
    u4 rh[4], rl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = jb + (4 * g + i) * P;
      if constexpr (PRE) {
        rh[i] = pre->h[qq][i];
        rl[i] = pre->l[qq][i];
      } else if constexpr (SRCG) {
        const int64_t a = cx.in_base + (int64_t)j * kp.s_in + c;
        rh[i] = gld4(kp.in + a);
        if constexpr (SPLIT) rl[i] = gld4(kp.in + kp.in_plane + a);
      } else {
        rh[i] = lds_ld4(lds, cx.lds_off + j * C + c);
        if constexpr (SPLIT) rl[i] = lds_ld4(ldsl, cx.lds_off + j * C + c);
      }
      if constexpr (!SPLIT) rl[i] = u4{0, 0, 0, 0};
    }
    // twiddles: the 4 tiles share (row, lo), hence one per row.  The extra
    // inter-pass twiddle W_M^{ci k} depends on the column ci too: with
    // ci = ci0 + t it is W_M^{ci0 k} * (W_M^k)^t (three lookups per row).
    // FOLD (FP16, stride 16, 64 columns per quad): every column of the quad
    // has the same lo, so the DIF twiddle W_256^{k1 lo} is folded into the
    // matrix-core operand, A_lo = diag(W_256^{k1 lo}) F_16 (table kp.fimg3).
    constexpr bool FOLD = !SPLIT && P == 16 && C >= 64;
    h8 far, fai;
    if constexpr (FOLD) {
      const TCFFT_GLOBAL h8* img = (const TCFFT_GLOBAL h8*)(kp.fimg3);
      far = img[256 * lo + lane];
      fai = img[256 * lo + 64 + lane];
    }
    float2 w[4][4];  // [t][j]
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (FOLD) {
      } else if constexpr (P > 1) {
        const float2 v = tld(kp.tw, (4 * g + j) * lo * (L / (16 * P)));  // W_{16P}^{row lo}
#pragma unroll
        for (int t = 0; t < 4; ++t) w[t][j] = v;
      } else if constexpr (XTW && XPRE) {
        const float2 a = xp->a[qq][j];
        w[0][j] = a;
        if (kp.xdiv == 1) {
#pragma unroll
          for (int t = 1; t < 4; ++t) w[t][j] = cmul(w[t - 1][j], xp->b[qq][j]);
        } else {
#pragma unroll
          for (int t = 1; t < 4; ++t) w[t][j] = a;
        }
      } else if constexpr (XTW) {
        const uint32_t k = (uint32_t)(restl + (L / 16) * (4 * g + j));  // natural output index
        const uint32_t ci = (uint32_t)(kp.xoff + cx.i0 + c);
        if (kp.xdiv == 1) {
          // W_M^{(ci + t) k} = W_M^{ci k} * (W_M^k)^t
          const float2 a = xtwiddle(kp, ci, k);
          const float2 b1 = tld(kp.xtw_lo, k);  // W_M^k (k < L <= 2^xbits)
          w[0][j] = a;
#pragma unroll
          for (int t = 1; t < 4; ++t) w[t][j] = cmul(w[t - 1][j], b1);
        } else {
          const float2 a = xtwiddle(kp, ci >> kp.xdiv_log2, k);  // same column group
#pragma unroll
          for (int t = 0; t < 4; ++t) w[t][j] = a;
        }
      }
    }
    u4 xh[4], xl[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        xh[t][i] = rh[i][t];
        xl[t][i] = rl[i][t];
      }
    uint32_t oh[4][4], ol[4][4];  // [t][j]
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f4 yr, yi;
      if constexpr (FOLD) {
        const h8 bh = __builtin_bit_cast(h8, xh[t]);
        const f4 z0 = {0.f, 0.f, 0.f, 0.f};
        yr = __builtin_amdgcn_mfma_f32_16x16x32_f16(far, bh, z0, 0, 0, 0);
        yi = __builtin_amdgcn_mfma_f32_16x16x32_f16(fai, bh, z0, 0, 0, 0);
      } else {
        dft_tile<SPLIT>(xh[t], xl[t], f, yr, yi);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float2 z = make_float2(yr[j], yi[j]);
        // the stage's own twiddle (P > 1, unless folded) or the inter-pass
        // twiddle of the last stage (P == 1)
        if constexpr ((P > 1 && !FOLD) || (P == 1 && XTW)) z = cmul(z, w[t][j]);
        uint32_t eh = 0, el = 0;
        emit<SPLIT>(z.x, z.y, eh, el);
        oh[t][j] = eh;
        ol[t][j] = el;
      }
    }
    if constexpr (P > 1 || TSTORE) {
      // in place in LDS (a transposed-store pass gathers natural order below)
      if (active) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int p = cx.lds_off + (jb + (4 * g + j) * P) * C + c;
          lds_st4(lds, p, u4{oh[0][j], oh[1][j], oh[2][j], oh[3][j]});
          if constexpr (SPLIT) lds_st4(ldsl, p, u4{ol[0][j], ol[1][j], ol[2][j], ol[3][j]});
        }
      }
    } else {
      if (active) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int64_t k = rest + (L / 16) * (4 * g + j);
          const int64_t a = cx.out_base + k * kp.s_out + c;
          gst4(kp.out + a, u4{oh[0][j], oh[1][j], oh[2][j], oh[3][j]});
          if constexpr (SPLIT) gst4(kp.out + kp.out_plane + a, u4{ol[0][j], ol[1][j], ol[2][j], ol[3][j]});
        }
      }
    }
  }
  if constexpr (P == 1 && TSTORE) {
    __syncthreads();
    // transposed store: column c of the tile becomes a row of L natural-order
    // outputs; output k sits at position posrev_hi(k mod L/16) * 16 + k / (L/16).
    // Each task gathers 4 consecutive outputs of one column from LDS and
    // writes them as one 16-byte store; adjacent lanes take adjacent k, so a
    // wave writes 1 KB of a row per instruction.
    constexpr int TASKS = C * (L / 4);
    constexpr int ITER = (TASKS + G::NT - 1) / G::NT;
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
      const int task = threadIdx.x + it * G::NT;
      if (TASKS % G::NT != 0 && task >= TASKS) break;
      const int c = task / (L / 4);
      const int k0 = 4 * (task % (L / 4));
      u4 h, l = {0, 0, 0, 0};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = k0 + i;
        const int j = posrev_hi<R0, S>(k % (L / 16)) * 16 + k / (L / 16);
        h[i] = lds_ld1(lds, j * C + c);
        if constexpr (SPLIT) l[i] = lds_ld1(ldsl, j * C + c);
      }
      const int tb = kp.tblk_log2;
      const int64_t a = cx.out_base + (int64_t)(k0 >> tb) * kp.tblk_stride +
                        ((int64_t)c << tb) + (k0 & ((1 << tb) - 1));
      gst4(kp.out + a, h);
      if constexpr (SPLIT) gst4(kp.out + kp.out_plane + a, l);
    }
  }
}

// Column-pass counterpart of row_stage_fused: a lane owns 4 adjacent columns
// c..c+3 (16-byte accesses) at one low index lo of the first radix-16 stage,
// rows m = 4g..4g+3 of that stage's digit and all R0 values of the radix-R0
// digit; both stages run in registers and the result goes to LDS.
template <class G>
struct ColFused {
  static constexpr int P = G::L / (16 * G::R0);
  static constexpr int NSQ = G::PTS / (64 * G::R0);
  static constexpr int ITF = NSQ / (16 * G::NW);
  static constexpr bool value = (G::R0 == 2 || G::R0 == 4) && G::S >= 2 && G::C >= 4 &&
                                ITF >= 1 && ITF * 16 * G::NW == NSQ;
};

template <class G, bool SPLIT>
__device__ __forceinline__ void col_stage_fused(const KParams& kp, uint32_t* lds, const ColCtx& cx,
                                                const FOps& f) {
  constexpr int L = G::L, R0 = G::R0, C = G::C;
  using F = ColFused<G>;
  constexpr int P = F::P, P0 = 16 * P, ITF = F::ITF;
  uint32_t* ldsl = lds + G::PTS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
  float2 wm[R0][4];  // W_L^{k (4g+i) P}, scaled by the radix-R0 stage scale
#pragma unroll
  for (int k = 1; k < R0; ++k)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float2 w = tld(kp.tw, k * (4 * g + i) * P);
      w.x *= kp.r0scale;
      w.y *= kp.r0scale;
      wm[k][i] = w;
    }
#pragma unroll
  for (int it = 0; it < ITF; ++it) {
    const int sq = (wave * ITF + it) * 16 + c16;
    const int c = 4 * (sq % (C / 4));
    const int lo = sq / (C / 4);  // in [0, P)
    u4 hh[R0][4], ll[R0][4];
#pragma unroll
    for (int d = 0; d < R0; ++d)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t a = cx.in_base + (int64_t)(d * P0 + (4 * g + i) * P + lo) * kp.s_in + c;
        hh[d][i] = gld4(kp.in + a);
        if constexpr (SPLIT) ll[d][i] = gld4(kp.in + kp.in_plane + a);
        else ll[d][i] = u4{0, 0, 0, 0};
      }
    // the 4 columns share (row, lo): one radix-R0 twiddle per (k, i), one
    // radix-16 twiddle per output row
    float2 w[R0][4];
#pragma unroll
    for (int k = 1; k < R0; ++k) {
      const float2 a = tld(kp.tw, k * lo);
#pragma unroll
      for (int i = 0; i < 4; ++i) w[k][i] = cmul(wm[k][i], a);
    }
    float2 a16[4];  // W_{16P}^{(4g+j) lo}
#pragma unroll
    for (int j = 0; j < 4; ++j) a16[j] = tld(kp.tw, (4 * g + j) * lo * R0);
    uint32_t oh[R0][4][4], ol[R0][4][4];  // [k][t][j]
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      u4 xh[R0], xl[R0];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float2 v[R0];
#pragma unroll
        for (int d = 0; d < R0; ++d) v[d] = value<SPLIT>(hh[d][i][t], ll[d][i][t]);
        small_dft<R0>(v, kp.sgn);
        v[0].x *= kp.r0scale;
        v[0].y *= kp.r0scale;
#pragma unroll
        for (int k = 1; k < R0; ++k) v[k] = cmul(v[k], w[k][i]);
#pragma unroll
        for (int k = 0; k < R0; ++k) {
          uint32_t eh = 0, el = 0;
          emit<SPLIT>(v[k].x, v[k].y, eh, el);
          xh[k][i] = eh;
          xl[k][i] = el;
        }
      }
#pragma unroll
      for (int k = 0; k < R0; ++k) {
        f4 yr, yi;
        dft_tile<SPLIT>(xh[k], xl[k], f, yr, yi);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float2 z = cmul(make_float2(yr[j], yi[j]), a16[j]);
          uint32_t eh = 0, el = 0;
          emit<SPLIT>(z.x, z.y, eh, el);
          oh[k][t][j] = eh;
          ol[k][t][j] = el;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < R0; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = (k * P0 + (4 * g + j) * P + lo) * C + c;
        lds_st4(lds, p, u4{oh[k][0][j], oh[k][1][j], oh[k][2][j], oh[k][3][j]});
        if constexpr (SPLIT) lds_st4(ldsl, p, u4{ol[k][0][j], ol[k][1][j], ol[k][2][j], ol[k][3][j]});
      }
  }
}

// The matrix-core radix-R0 x radix-16 block in a column pass: the 4 tiles of a
// lane are 4 adjacent columns at one low index lo, so the twiddle
// W_L^{(k + R0 k1) lo} is one lookup per output row.  (Row passes keep the
// vector-ALU radix-R0 stage: for the 16384-point pass the block's four-fold
// matrix-core work measured slower under sustained load, 239 against 230 us.)
template <class G>
struct ColFusedMx {
  static constexpr bool value = ColFused<G>::value && (G::R0 == 2 || G::R0 == 4);
};

template <class G, int K = 0>
__device__ __forceinline__ void col_fused_mx_k(const KParams& kp, uint32_t* lds,
                                               const u4 (&hh)[G::R0][4], int c, int lo) {
  constexpr int R0 = G::R0, C = G::C;
  constexpr int P = ColFused<G>::P, P0 = 16 * P;
  const int g = (threadIdx.x & 63) >> 4;
  const int k = kp.sgn < 0.f ? K : (R0 - K) % R0;  // the output this block is
  const FOpsMx fm = load_fops_mx(kp.fimg2, K);
  float2 w[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) w[j] = tld(kp.tw, (k + R0 * (4 * g + j)) * lo);
  uint32_t oh[4][4];  // [t][j]
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    u4 b[R0];
#pragma unroll
    for (int d = 0; d < R0; ++d) b[d] = u4{hh[d][0][t], hh[d][1][t], hh[d][2][t], hh[d][3][t]};
    f4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
    mfma_rsum<R0, K>(fm, b, yr, yi);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float2 z = cmul(make_float2(yr[j], yi[j]), w[j]);
      oh[t][j] = pack(z.x, z.y);
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int p = (k * P0 + (4 * g + j) * P + lo) * C + c;
    lds_st4(lds, p, u4{oh[0][j], oh[1][j], oh[2][j], oh[3][j]});
  }
  if constexpr (K + 1 < R0) col_fused_mx_k<G, K + 1>(kp, lds, hh, c, lo);
}

template <class G>
__device__ __forceinline__ void col_stage_fused_mx(const KParams& kp, uint32_t* lds,
                                                   const ColCtx& cx) {
  constexpr int R0 = G::R0, C = G::C;
  using F = ColFused<G>;
  constexpr int P = F::P, P0 = 16 * P, ITF = F::ITF;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
#pragma unroll
  for (int it = 0; it < ITF; ++it) {
    const int sq = (wave * ITF + it) * 16 + c16;
    const int c = 4 * (sq % (C / 4));
    const int lo = sq / (C / 4);  // in [0, P)
    u4 hh[R0][4];
#pragma unroll
    for (int d = 0; d < R0; ++d)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t a = cx.in_base + (int64_t)(d * P0 + (4 * g + i) * P + lo) * kp.s_in + c;
        hh[d][i] = gld4(kp.in + a);
      }
    col_fused_mx_k<G>(kp, lds, hh, c, lo);
  }
}

template <class G, int E, bool SPLIT, bool XTW, bool TSTORE, bool XPRE = false>
__device__ __forceinline__ void col_stages_from(const KParams& kp, uint32_t* lds, const ColCtx& cx,
                                                const FOps& f, const XtwRegs<G>* xp = nullptr) {
  col_stage16<G, pow16(E), false, SPLIT, XTW, TSTORE, false, XPRE && E == 0>(kp, lds, cx, f,
                                                                            nullptr, xp);
  if constexpr (E > 0) {
    __syncthreads();
    col_stages_from<G, E - 1, SPLIT, XTW, TSTORE, XPRE>(kp, lds, cx, f, xp);
  }
}

// Tile `wg` of a column pass: C adjacent columns of outer block wg / blocks.
template <bool TSTORE>
__device__ __forceinline__ ColCtx col_ctx(const KParams& kp, int64_t wg, int C) {
  ColCtx cx;
  cx.outer = wg >> kp.blocks_log2;
  cx.i0 = (wg & (kp.blocks - 1)) * C;
  cx.in_base = cx.outer * kp.in_outer + cx.i0;
  if constexpr (TSTORE)
    cx.out_base = cx.outer * kp.out_outer + (cx.i0 << kp.tblk_log2);
  else
    cx.out_base = cx.outer * kp.out_outer + (cx.i0 >> kp.q_log2) * kp.qstride + (cx.i0 & (kp.q - 1));
  return cx;
}

// One workgroup's share of a column pass: workgroup index wg of the pass.
template <int L, int R0, int C, int NT, bool SPLIT, bool XTW, bool TSTORE>
__device__ __forceinline__ void col_body(const KParams& kp, int64_t wg, uint32_t* lds) {
  using G = ColGeom<L, R0, C, NT>;
  const ColCtx cx = col_ctx<TSTORE>(kp, wg, C);
  const FOps f = load_fops<SPLIT>(kp.fimg);
  if constexpr (!SPLIT && ColFusedMx<G>::value) {
    col_stage_fused_mx<G>(kp, lds, cx);
    __syncthreads();
    col_stages_from<G, G::S - 2, SPLIT, XTW, TSTORE>(kp, lds, cx, f);
  } else if constexpr (ColFused<G>::value) {
    col_stage_fused<G, SPLIT>(kp, lds, cx, f);
    __syncthreads();
    col_stages_from<G, G::S - 2, SPLIT, XTW, TSTORE>(kp, lds, cx, f);
  } else if constexpr (R0 > 1) {
    // one radix-16 stage after the radix-R0 stage: its inter-pass twiddle
    // lookups go out before the pass's HBM reads (split: 1D 2^22 x 4 177 ->
    // 171 us, 65536 x 2048 998 -> 983 us; FP16 with the transposed store:
    // 2^15 x 4096 413 -> 397 us, 2^20 x 16 72.7 -> 70.4 us; the FP16 first
    // pass of the 65536-point plan measured slower, 220 -> 225 us, and keeps
    // its lookups in the last stage)
    constexpr bool XPRE = XTW && G::S == 1 && (SPLIT || TSTORE);
    XtwRegs<G> xr;
    if constexpr (XPRE) xtw_prefetch<G>(kp, cx, xr);
    col_stage_r0<G, SPLIT>(kp, lds, cx);
    __syncthreads();
    col_stages_from<G, G::S - 1, SPLIT, XTW, TSTORE, XPRE>(kp, lds, cx, f, &xr);
  } else {
    col_stage16<G, pow16(G::S - 1), true, SPLIT, XTW, TSTORE>(kp, lds, cx, f);
    if constexpr (G::S > 1) {
      __syncthreads();
      col_stages_from<G, G::S - 2, SPLIT, XTW, TSTORE>(kp, lds, cx, f);
    }
  }
}

// Whether a column pass runs as a pipelined persistent kernel: FP16 passes
// whose first stage is radix-16 from HBM with P > 1, at 256 threads (the
// 256-point columns).  Like the row pipeline, workgroup b runs tiles b, b +
// grid, ... and issues the next tile's HBM loads while the current one runs
// its LDS stages and stores; the register budget is capped at two waves per
// SIMD (two 64 KB workgroups per CU).  Split passes and transposed stores keep
// one tile per workgroup: with the held-over tile they do not fit that budget
// (split: hi and lo planes; the transposed store spills 240 bytes per lane).
template <class G, bool SPLIT, bool TSTORE>
struct ColPipe {
  static constexpr bool value = !SPLIT && !TSTORE && G::NT == 256 && G::R0 == 1 && G::S >= 2;
};

template <int L, int R0, int C, int NT, bool SPLIT, bool XTW, bool TSTORE>
__device__ __forceinline__ void col_pipe(const KParams& kp, uint32_t* lds) {
  using G = ColGeom<L, R0, C, NT>;
  constexpr int P1 = pow16(G::S - 1);
  const int64_t ntiles = kp.ntrans;  // column passes: the number of tiles
  const FOps f = load_fops<SPLIT>(kp.fimg);
  int64_t w = blockIdx.x;
  if (w >= ntiles) return;
  ColCtx cx = col_ctx<TSTORE>(kp, w, C);
  Col16Regs<G> r;
  col_stage16_load<G, P1, SPLIT>(kp, cx, r);
  for (; w < ntiles; w += gridDim.x) {
    col_stage16<G, P1, true, SPLIT, XTW, TSTORE, true>(kp, lds, cx, f, &r);
    const int64_t wn = w + gridDim.x;
    ColCtx cn = cx;
    if (wn < ntiles) {
      cn = col_ctx<TSTORE>(kp, wn, C);
      col_stage16_load<G, P1, SPLIT>(kp, cn, r);
    }
    __syncthreads();
    col_stages_from<G, G::S - 2, SPLIT, XTW, TSTORE>(kp, lds, cx, f);
    __syncthreads();  // the next tile's first stage rewrites LDS
    cx = cn;
  }
}

template <int L, int R0, int C, int NT, bool SPLIT, bool XTW, bool TSTORE>
__global__ __launch_bounds__(NT, (ColPipe<ColGeom<L, R0, C, NT>, SPLIT, TSTORE>::value ? 2 : 1))
void col_kernel(KParams kp) {
  extern __shared__ uint32_t lds[];
  if constexpr (ColPipe<ColGeom<L, R0, C, NT>, SPLIT, TSTORE>::value)
    col_pipe<L, R0, C, NT, SPLIT, XTW, TSTORE>(kp, lds);
  else
    col_body<L, R0, C, NT, SPLIT, XTW, TSTORE>(kp, blockIdx.x, lds);
}

// ===========================================================================
// Grouped mixed-size launch: one launch runs the same pass kernel for many
// jobs (different sizes of batch, buffers, tables).  Job j owns workgroup
// indices [prefix[j], prefix[j+1]).  The launch's only argument is a group
// header in device memory that points at the descriptor table and the prefix
// array, so a captured launch can be replayed for a new set of jobs by
// rewriting device memory.  The grid is persistent: each workgroup strides
// over the job tiles.
// ===========================================================================
// The group header, descriptor table and prefix array are written by the host
// before the launch and only read by it: read through the constant address
// space, they load into scalar registers (uniform per workgroup) instead of
// taking ~40 vector registers per lane for the descriptor.
#define TCFFT_CONST __attribute__((address_space(4)))
typedef const TCFFT_CONST GroupHdr CGroupHdr;
typedef const TCFFT_CONST KParams CKParams;
typedef const TCFFT_CONST int64_t CInt64;

// Copy of descriptor j (word by word: the struct has no constructor from the
// constant address space).
__device__ __forceinline__ KParams load_job(CKParams* jobs, int j) {
  KParams kp;
  const TCFFT_CONST uint32_t* src = (const TCFFT_CONST uint32_t*)(jobs + j);
  uint32_t* dst = reinterpret_cast<uint32_t*>(&kp);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(KParams) / 4); ++i) dst[i] = src[i];
  return kp;
}

__device__ __forceinline__ int find_job(CInt64* prefix, int njobs, int64_t w) {
  int lo = 0, hi = njobs - 1;  // largest j with prefix[j] <= w
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// FP16 row tiles use 64 KB of LDS, so two workgroups share a CU: the register
// budget is capped to match (the persistent loop otherwise keeps enough
// loop-invariant addresses live to drop to one workgroup per CU).
// (the real-input variants carry their epilogue / prologue through the
// persistent loop: one workgroup per CU keeps them out of scratch)
template <int L, int R0, int NT, bool SPLIT, bool TT = false, int RK = 0, int WGP = 16384>
__global__ __launch_bounds__(NT, (SPLIT || RK != 0) ? 1 : 2) void row_kernel_multi(
    const GroupHdr* __restrict__ hdr) {
  extern __shared__ uint32_t lds[];
  CGroupHdr* h = (CGroupHdr*)hdr;
  CKParams* jobs = (CKParams*)h->jobs;
  CInt64* prefix = (CInt64*)h->prefix;
  const int njobs = (int)h->njobs;
  const int64_t total = njobs > 0 ? prefix[njobs] : 0;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int j = find_job(prefix, njobs, w);
    const KParams kp = load_job(jobs, j);
    row_body<L, R0, NT, SPLIT, TT, RK, WGP>(kp, w - prefix[j], lds);
    __syncthreads();  // the next tile's first stage rewrites LDS
  }
}

template <int L, int R0, int C, int NT, bool SPLIT, bool XTW, bool TSTORE>
__global__ __launch_bounds__(NT) void col_kernel_multi(const GroupHdr* __restrict__ hdr) {
  extern __shared__ uint32_t lds[];
  CGroupHdr* h = (CGroupHdr*)hdr;
  CKParams* jobs = (CKParams*)h->jobs;
  CInt64* prefix = (CInt64*)h->prefix;
  const int njobs = (int)h->njobs;
  const int64_t total = njobs > 0 ? prefix[njobs] : 0;
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int j = find_job(prefix, njobs, w);
    const KParams kp = load_job(jobs, j);
    col_body<L, R0, C, NT, SPLIT, XTW, TSTORE>(kp, w - prefix[j], lds);
    __syncthreads();
  }
}

}  // namespace tcfft
