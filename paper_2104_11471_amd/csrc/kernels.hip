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
#include "common.h"
#include "kernels.h"

namespace tcfft {

// ---------------------------------------------------------------------------
// LDS addressing.  Position p (in complex words) -> word address.  The swizzle
// XORs address bits [4,6) with bits [8,10) so that groups of 4 consecutive
// words stay 16-byte aligned for ds_read/write_b128 while chunks that sit 1 KB
// apart move to different banks.
__device__ __forceinline__ int lds_addr(int p) { return p ^ (((p >> 8) & 3) << 4); }

__device__ __forceinline__ u4 lds_ld4(const uint32_t* lds, int p) {
  return *reinterpret_cast<const u4*>(lds + lds_addr(p));
}
__device__ __forceinline__ void lds_st4(uint32_t* lds, int p, u4 v) {
  *reinterpret_cast<u4*>(lds + lds_addr(p)) = v;
}
__device__ __forceinline__ uint32_t lds_ld1(const uint32_t* lds, int p) { return lds[lds_addr(p)]; }
__device__ __forceinline__ void lds_st1(uint32_t* lds, int p, uint32_t v) { lds[lds_addr(p)] = v; }

__device__ __forceinline__ u4 gld4(const uint32_t* ptr) { return *reinterpret_cast<const u4*>(ptr); }
__device__ __forceinline__ void gst4(uint32_t* ptr, u4 v) { *reinterpret_cast<u4*>(ptr) = v; }

// Position of the digit-reversed "high" index of the last stage: natural low
// output index klow = k0 + R0*(k1 + 16 k2 + ... + 16^(S-2) k_{S-1}) sits at
// hi = k0*16^(S-1) + k1*16^(S-2) + ... + k_{S-1} (position = hi*16 + row).
template <int R0, int S>
__device__ __forceinline__ int posrev_hi(int klow) {
  int k0 = klow % R0;
  int m = klow / R0;
  int hi = k0 * pow16(S - 1);
#pragma unroll
  for (int s = 1; s < S; ++s) {
    hi += (m & 15) * pow16(S - 1 - s);
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
  const h8* f = reinterpret_cast<const h8*>(fimg);
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
template <int L_, int R0_, int NT_>
struct RowGeom {
  static constexpr int L = L_, R0 = R0_, NT = NT_;
  static constexpr int S = (ilog2c(L) - ilog2c(R0)) / 4;
  static_assert(pow16(S) * R0 == L, "L must be R0 * 16^S");
  static constexpr int TPB = L >= 4096 ? 1 : 4096 / L;
  static constexpr int PTS = TPB * L;
  static constexpr int NW = NT / 64;
  static constexpr int NCOL = PTS / 16;
  static constexpr int NQ = NCOL / 64;
  static constexpr int QPW = NQ / NW;
  static_assert(QPW >= 1 && QPW * NW == NQ, "waves must split the quads evenly");
  static constexpr int P0 = L / R0;
  static constexpr int NCQ0 = PTS / R0 / 4;
};

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

// Radix-R0 stage on the vector ALU, HBM -> LDS (always the first stage).
template <class G, bool SPLIT>
__device__ __forceinline__ void row_stage_r0(const KParams& kp, uint32_t* lds, int valid,
                                             int64_t g0) {
  constexpr int L = G::L, R0 = G::R0, P0 = G::P0;
  uint32_t* ldsl = lds + G::PTS;
  for (int cq = threadIdx.x; cq < G::NCQ0; cq += G::NT) {
    const int col0 = 4 * cq;
    const int tau = col0 / P0;
    const int lo0 = col0 % P0;
    float2 v[4][R0];
#pragma unroll
    for (int d = 0; d < R0; ++d) {
      const int p = tau * L + d * P0 + lo0;
      u4 h = {0, 0, 0, 0}, l = {0, 0, 0, 0};
      if (tau < valid) {
        h = gld4(kp.in + g0 + p);
        if constexpr (SPLIT) l = gld4(kp.in + kp.in_plane + g0 + p);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) v[t][d] = value<SPLIT>(h[t], l[t]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      small_dft<R0>(v[t], kp.sgn);
      const int lo = lo0 + t;
#pragma unroll
      for (int k = 0; k < R0; ++k) {
        float2 w = kp.tw[k * lo];  // W_L^{k * lo}, k * lo < L
        w.x *= kp.r0scale;
        w.y *= kp.r0scale;
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
template <class G, int P, bool SRCG, bool SPLIT>
__device__ __forceinline__ void row_stage16(const KParams& kp, uint32_t* lds, int valid,
                                            int64_t g0, const FOps& f) {
  constexpr int L = G::L, R0 = G::R0, S = G::S;
  uint32_t* ldsl = lds + G::PTS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
#pragma unroll
  for (int qq = 0; qq < G::QPW; ++qq) {
    const int Q = wave * G::QPW + qq;
    const int col0 = 4 * c16 + 64 * Q;
    u4 xh[4], xl[4];  // xh[t] = rows 4g..4g+3 of tile t
    if constexpr (P > 1) {
      // tiles along the contiguous low index: one 16-byte access per row
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = row_pos_t<L, P>(col0, 4 * g + i);
        u4 h = {0, 0, 0, 0}, l = {0, 0, 0, 0};
        if constexpr (SRCG) {
          if (p / L < valid) {
            h = gld4(kp.in + g0 + p);
            if constexpr (SPLIT) l = gld4(kp.in + kp.in_plane + g0 + p);
          }
        } else {
          h = lds_ld4(lds, p);
          if constexpr (SPLIT) l = lds_ld4(ldsl, p);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          xh[t][i] = h[t];
          xl[t][i] = l[t];
        }
      }
    } else {
      // last stage: rows are contiguous; columns enumerate natural order
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = col0 + t;
        const int tau = col / (L / 16);
        const int p = tau * L + posrev_hi<R0, S>(col % (L / 16)) * 16 + 4 * g;
        u4 h = {0, 0, 0, 0}, l = {0, 0, 0, 0};
        if constexpr (SRCG) {
          if (tau < valid) {
            h = gld4(kp.in + g0 + p);
            if constexpr (SPLIT) l = gld4(kp.in + kp.in_plane + g0 + p);
          }
        } else {
          h = lds_ld4(lds, p);
          if constexpr (SPLIT) l = lds_ld4(ldsl, p);
        }
        xh[t] = h;
        xl[t] = l;
      }
    }
    uint32_t oh[4][4], ol[4][4];  // [t][j]
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f4 yr, yi;
      dft_tile<SPLIT>(xh[t], xl[t], f, yr, yi);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float re = yr[j], im = yi[j];
        if constexpr (P > 1) {
          const int lo = (col0 + t) % P;
          const int row = 4 * g + j;
          const float2 w = kp.tw[row * lo * (L / (16 * P))];  // W_{16P}^{row * lo}
          const float2 z = cmul(make_float2(re, im), w);
          re = z.x;
          im = z.y;
        }
        emit<SPLIT>(re, im, oh[t][j], ol[t][j]);
      }
    }
    if constexpr (P > 1) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int p = row_pos_t<L, P>(col0, 4 * g + j);
        u4 h = {oh[0][j], oh[1][j], oh[2][j], oh[3][j]};
        lds_st4(lds, p, h);
        if constexpr (SPLIT) {
          u4 l = {ol[0][j], ol[1][j], ol[2][j], ol[3][j]};
          lds_st4(ldsl, p, l);
        }
      }
    } else {
      // natural output index of (row, col): tau*L + klow + (L/16)*row
      if constexpr (L / 16 >= 4) {
        const int tau = col0 / (L / 16);
        if (tau < valid) {
          const int klow0 = col0 % (L / 16);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int64_t o = g0 + (int64_t)tau * L + klow0 + (L / 16) * (4 * g + j);
            gst4(kp.out + o, u4{oh[0][j], oh[1][j], oh[2][j], oh[3][j]});
            if constexpr (SPLIT)
              gst4(kp.out + kp.out_plane + o, u4{ol[0][j], ol[1][j], ol[2][j], ol[3][j]});
          }
        }
      } else if constexpr (L == 16) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int tau = col0 + t;
          if (tau < valid) {
            const int64_t o = g0 + (int64_t)tau * 16 + 4 * g;
            gst4(kp.out + o, u4{oh[t][0], oh[t][1], oh[t][2], oh[t][3]});
            if constexpr (SPLIT)
              gst4(kp.out + kp.out_plane + o, u4{ol[t][0], ol[t][1], ol[t][2], ol[t][3]});
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
              kp.out[o] = oh[t][j];
              if constexpr (SPLIT) kp.out[kp.out_plane + o] = ol[t][j];
            }
          }
        }
      }
    }
  }
}

template <class G, int E, bool SPLIT>
__device__ __forceinline__ void row_stages_from(const KParams& kp, uint32_t* lds, int valid,
                                                int64_t g0, const FOps& f) {
  // radix-16 stages with stride 16^E, 16^(E-1), ..., 1, all reading LDS
  row_stage16<G, pow16(E), false, SPLIT>(kp, lds, valid, g0, f);
  if constexpr (E > 0) {
    __syncthreads();
    row_stages_from<G, E - 1, SPLIT>(kp, lds, valid, g0, f);
  }
}

template <int L, int R0, int NT, bool SPLIT>
__global__ __launch_bounds__(NT) void row_kernel(KParams kp) {
  using G = RowGeom<L, R0, NT>;
  extern __shared__ uint32_t lds[];
  const int64_t t0 = (int64_t)blockIdx.x * G::TPB;
  const int64_t rem = kp.ntrans - t0;
  const int valid = rem < G::TPB ? (int)rem : G::TPB;
  const int64_t g0 = t0 * L;
  const FOps f = load_fops<SPLIT>(kp.fimg);
  if constexpr (R0 > 1) {
    row_stage_r0<G, SPLIT>(kp, lds, valid, g0);
    __syncthreads();
    row_stages_from<G, G::S - 1, SPLIT>(kp, lds, valid, g0, f);
  } else {
    row_stage16<G, pow16(G::S - 1), true, SPLIT>(kp, lds, valid, g0, f);
    if constexpr (G::S > 1) {
      __syncthreads();
      row_stages_from<G, G::S - 2, SPLIT>(kp, lds, valid, g0, f);
    }
  }
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
  int64_t i0;                 // first global column index of the tile
  int64_t outer;
};

template <class G, bool SPLIT>
__device__ __forceinline__ void col_stage_r0(const KParams& kp, uint32_t* lds, const ColCtx& cx) {
  constexpr int L = G::L, R0 = G::R0, C = G::C, P0 = G::P0;
  uint32_t* ldsl = lds + G::PTS;
  for (int cq = threadIdx.x; cq < G::NCQ0; cq += G::NT) {
    const int col0 = 4 * cq;
    const int c = col0 % C;
    const int lo = col0 / C;  // in [0, P0)
    float2 v[4][R0];
#pragma unroll
    for (int d = 0; d < R0; ++d) {
      const int64_t a = cx.in_base + (int64_t)(d * P0 + lo) * kp.s_in + c;
      u4 h = gld4(kp.in + a), l = {0, 0, 0, 0};
      if constexpr (SPLIT) l = gld4(kp.in + kp.in_plane + a);
#pragma unroll
      for (int t = 0; t < 4; ++t) v[t][d] = value<SPLIT>(h[t], l[t]);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) small_dft<R0>(v[t], kp.sgn);
#pragma unroll
    for (int k = 0; k < R0; ++k) {
      float2 w = kp.tw[k * lo];
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
      const int p = (k * P0 + lo) * C + c;
      lds_st4(lds, p, h);
      if constexpr (SPLIT) lds_st4(ldsl, p, l);
    }
  }
}

// Extra inter-pass twiddle W_M^{ci * k} (two-level table, FP32).
__device__ __forceinline__ float2 xtwiddle(const KParams& kp, int64_t ci, int64_t k) {
  const uint32_t e = (uint32_t)(((uint64_t)ci * (uint64_t)k) & kp.xmask);
  const float2 a = kp.xtw_lo[e & ((1u << kp.xbits) - 1u)];
  const float2 b = kp.xtw_hi[e >> kp.xbits];
  return cmul(a, b);
}

template <class G, int P, bool SRCG, bool SPLIT, bool XTW, bool TSTORE>
__device__ __forceinline__ void col_stage16(const KParams& kp, uint32_t* lds, const ColCtx& cx,
                                            const FOps& f) {
  constexpr int L = G::L, R0 = G::R0, S = G::S, C = G::C;
  uint32_t* ldsl = lds + G::PTS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c16 = lane & 15;
#pragma unroll
  for (int qq = 0; qq < G::QPW; ++qq) {
    const int Q = wave * G::QPW + qq;
    const int col0 = 4 * c16 + 64 * Q;
    const int c = col0 % C;
    const int rest = col0 / C;
    const bool active = rest < L / 16;  // masks idle lanes of tiny tiles
    int lo = 0, jb = 0;
    if constexpr (P > 1) {
      lo = rest % P;
      jb = (rest / P) * 16 * P + lo;  // j = jb + row * P
    } else {
      jb = posrev_hi<R0, S>(rest) * 16;  // j = jb + row
    }
    u4 xh[4], xl[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int j = jb + (4 * g + i) * P;
      u4 h = {0, 0, 0, 0}, l = {0, 0, 0, 0};
      if (active) {
        if constexpr (SRCG) {
          const int64_t a = cx.in_base + (int64_t)j * kp.s_in + c;
          h = gld4(kp.in + a);
          if constexpr (SPLIT) l = gld4(kp.in + kp.in_plane + a);
        } else {
          h = lds_ld4(lds, j * C + c);
          if constexpr (SPLIT) l = lds_ld4(ldsl, j * C + c);
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        xh[t][i] = h[t];
        xl[t][i] = l[t];
      }
    }
    uint32_t oh[4][4], ol[4][4];  // [t][j]
    // the 4 tiles share (row, lo), hence one twiddle per row
    float2 w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      w[j] = P > 1 ? kp.tw[(4 * g + j) * lo * (L / (16 * P))] : make_float2(1.f, 0.f);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f4 yr, yi;
      dft_tile<SPLIT>(xh[t], xl[t], f, yr, yi);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float2 z = make_float2(yr[j], yi[j]);
        const int row = 4 * g + j;
        if constexpr (P > 1) {
          z = cmul(z, w[j]);  // W_{16P}^{row * lo}
        } else if constexpr (XTW) {
          const int64_t k = rest + (L / 16) * row;  // natural output index
          z = cmul(z, xtwiddle(kp, (cx.i0 + c + t) / kp.xdiv, k));
        }
        emit<SPLIT>(z.x, z.y, oh[t][j], ol[t][j]);
      }
    }
    if constexpr (P > 1 || TSTORE) {
      // in place in LDS (a transposed-store pass gathers natural order below)
      if (active) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int p = (jb + (4 * g + j) * P) * C + c;
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
    // outputs; output k sits at position posrev_hi(k mod L/16) * 16 + k / (L/16)
    for (int task = threadIdx.x; task < C * (L / 4); task += G::NT) {
      const int c = task / (L / 4);
      const int k0 = 4 * (task % (L / 4));
      u4 h, l;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = k0 + i;
        const int j = posrev_hi<R0, S>(k % (L / 16)) * 16 + k / (L / 16);
        h[i] = lds_ld1(lds, j * C + c);
        l[i] = 0;
        if constexpr (SPLIT) l[i] = lds_ld1(ldsl, j * C + c);
      }
      const int64_t a = cx.out_base + (int64_t)c * L + k0;
      gst4(kp.out + a, h);
      if constexpr (SPLIT) gst4(kp.out + kp.out_plane + a, l);
    }
  }
}

template <class G, int E, bool SPLIT, bool XTW, bool TSTORE>
__device__ __forceinline__ void col_stages_from(const KParams& kp, uint32_t* lds, const ColCtx& cx,
                                                const FOps& f) {
  col_stage16<G, pow16(E), false, SPLIT, XTW, TSTORE>(kp, lds, cx, f);
  if constexpr (E > 0) {
    __syncthreads();
    col_stages_from<G, E - 1, SPLIT, XTW, TSTORE>(kp, lds, cx, f);
  }
}

template <int L, int R0, int C, int NT, bool SPLIT, bool XTW, bool TSTORE>
__global__ __launch_bounds__(NT) void col_kernel(KParams kp) {
  using G = ColGeom<L, R0, C, NT>;
  extern __shared__ uint32_t lds[];
  ColCtx cx;
  const int64_t w = blockIdx.x;
  cx.outer = w / kp.blocks;
  cx.i0 = (w % kp.blocks) * C;
  cx.in_base = cx.outer * kp.in_outer + cx.i0;
  if constexpr (TSTORE)
    cx.out_base = cx.outer * kp.out_outer + cx.i0 * L;
  else
    cx.out_base = cx.outer * kp.out_outer + (cx.i0 / kp.q) * kp.qstride + (cx.i0 % kp.q);
  const FOps f = load_fops<SPLIT>(kp.fimg);
  if constexpr (R0 > 1) {
    col_stage_r0<G, SPLIT>(kp, lds, cx);
    __syncthreads();
    col_stages_from<G, G::S - 1, SPLIT, XTW, TSTORE>(kp, lds, cx, f);
  } else {
    col_stage16<G, pow16(G::S - 1), true, SPLIT, XTW, TSTORE>(kp, lds, cx, f);
    if constexpr (G::S > 1) {
      __syncthreads();
      col_stages_from<G, G::S - 2, SPLIT, XTW, TSTORE>(kp, lds, cx, f);
    }
  }
}

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

__global__ void gen_fimg_kernel(h8* img, double sgn, double scale) {
  const int lane = threadIdx.x;  // 64 lanes
  const int g = lane >> 4, m = lane & 15;
  h8 rh, ih, rl, il;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = 4 * g + i;
    const int e = (m * r) & 15;
    double sn, cs;
    sincospi(2.0 * (double)e / 16.0, &sn, &cs);
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
                     scale);
}

// ===========================================================================
// Variant registry.
// ===========================================================================
#define ROWK(L_, R_, N_)                                                                \
  if (k.kind == K_ROW && k.L == L_ && k.R0 == R_ && k.NT == N_)                         \
    return k.split ? (KernelFn)row_kernel<L_, R_, N_, true> : (KernelFn)row_kernel<L_, R_, N_, false>;

#define COLK4(L_, R_, C_, N_, X_, T_)                                                   \
  if (k.kind == K_COL && k.L == L_ && k.R0 == R_ && k.C == C_ && k.NT == N_ &&          \
      k.xtw == X_ && k.tstore == T_)                                                    \
    return k.split ? (KernelFn)col_kernel<L_, R_, C_, N_, true, X_, T_>                 \
                   : (KernelFn)col_kernel<L_, R_, C_, N_, false, X_, T_>;
#define COLK(L_, R_, C_, N_)                                                            \
  COLK4(L_, R_, C_, N_, false, false) COLK4(L_, R_, C_, N_, true, false)                \
  COLK4(L_, R_, C_, N_, true, true)

KernelFn find_kernel(const KernelKey& k) {
  ROWK(16, 1, 256)
  ROWK(32, 2, 256)
  ROWK(64, 4, 256)
  ROWK(128, 8, 256)
  ROWK(256, 1, 256)
  ROWK(512, 2, 256)
  ROWK(1024, 4, 256)
  ROWK(2048, 8, 256)
  ROWK(4096, 1, 256)
  ROWK(8192, 2, 256)
  ROWK(16384, 4, 256)
  ROWK(8192, 2, 512)
  ROWK(16384, 4, 512)
  // column kernels: L * C <= 32768 points (128 KB FP16)
  COLK(16, 1, 64, 64)
  COLK(32, 2, 64, 128)
  COLK(64, 4, 64, 256)
  COLK(128, 8, 64, 256)
  COLK(256, 1, 64, 256)
  COLK(256, 1, 32, 256)
  COLK(512, 2, 32, 256)
  COLK(512, 2, 64, 256)
  COLK(1024, 4, 32, 256)
  COLK(1024, 4, 16, 256)
  COLK(2048, 8, 16, 256)
  COLK(512, 2, 16, 256)
  COLK(2048, 8, 8, 256)
  // narrow blocks for small inner sizes (2D with ny = 16 or 32)
  COLK(16, 1, 16, 64)
  COLK(32, 2, 16, 64)
  COLK(64, 4, 16, 64)
  COLK(128, 8, 16, 128)
  COLK(256, 1, 16, 256)
  COLK(16, 1, 32, 64)
  COLK(32, 2, 32, 64)
  COLK(64, 4, 32, 128)
  COLK(128, 8, 32, 256)
  return nullptr;
}

size_t kernel_lds_bytes(const KernelKey& k) {
  const int64_t pts = kernel_points_per_wg(k);
  return (size_t)pts * 4 * (k.split ? 2 : 1);
}

int64_t kernel_points_per_wg(const KernelKey& k) {
  if (k.kind == K_ROW) return k.L >= 4096 ? k.L : 4096;
  return (int64_t)k.L * k.C;
}

}  // namespace tcfft
