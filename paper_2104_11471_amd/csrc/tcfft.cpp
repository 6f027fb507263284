// Host runtime of libtcfft: planner, device tables, pass launcher and the C ABI
// declared in include/tcfft.h.
//
// Plan mechanism (paper Sec. 3.1, Fig. 1): a plan fixes, once, the sequence of
// merging kernels for a (rank, size, batch, precision, direction); the
// execution function then launches that sequence.  Here a "pass" is one kernel
// launch that does every merging process whose data fits in one workgroup's
// LDS; passes exchange data through HBM (Sec. 3.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tcfft.h"
#include "kernels.h"
#include "runtime.h"

using namespace tcfft;

namespace {

constexpr int64_t kMaxPointsPerPlan = (int64_t)1 << 31;
constexpr int kMaxRowL = 16384;  // largest single-pass contiguous length
constexpr int kMaxColL = 2048;   // largest strided length handled in one pass
constexpr size_t kMaxLds = 160 * 1024;  // LDS per workgroup on gfx950

bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

// TCFFT_LOG set (non-empty, not "0"): plan descriptions and failing statuses
// go to stderr.
bool log_on() {
  const char* v = std::getenv("TCFFT_LOG");
  return v && *v && std::strcmp(v, "0") != 0;
}
tcfft_status logged(tcfft_status st, const char* what) {
  if (st != TCFFT_OK && log_on()) std::fprintf(stderr, "tcfft: %s: status %d\n", what, (int)st);
  return st;
}
int ilog2(int64_t n) {
  int l = 0;
  while (((int64_t)1 << l) < n) ++l;
  return l;
}

// Radix split of a pass length L = R0 * 16^S (R0 in {1, 2, 4, 8}).
int r0_of(int L) { return 1 << (ilog2(L) % 4); }
int s16_of(int L) { return ilog2(L) / 4; }
// Output scale exponent of one pass (unitary-like: 2^-2 per radix-16 stage,
// 2^-1 for radix 2 or 4, 2^-2 for radix 8), so that FP16 never overflows.
int pass_scale(int L) {
  int r0 = r0_of(L);
  return 2 * s16_of(L) + (r0 == 1 ? 0 : (r0 == 8 ? 2 : 1));
}

struct PassSpec {
  KernelKey key;
  int64_t grid = 0;
  size_t lds = 0;
  // geometry
  int64_t ntrans = 0;  // row kernel: lines of the whole plan
  int64_t lines_per_batch = 0;  // row kernel: lines per transform of the batch
  int64_t tpb = 1;     // row kernel: lines per workgroup
  int64_t s_in = 0, s_out = 0, blocks = 0, in_outer = 0, out_outer = 0, q = 1, qstride = 0;
  // extra twiddle
  int64_t xmod = 0, xdiv = 1;
  int64_t outer_per_batch = 1;  // column kernel: [L][inner] blocks per transform
  // buffers: 0 = user in, 1 = user out, 2 = workspace
  int src = 0, dst = 1;
  int scale = 0;  // this pass's scale exponent
  // shard of a distributed transform: global index of column 0 for the extra
  // twiddle, and the blocked transposed store (0 = plain rows of L outputs)
  int64_t xoff = 0;
  int64_t tblk = 0, tblk_stride = 0;
};

struct Desc {
  int rank = 1;
  int64_t nx = 0, ny = 1, nz = 1;
  int64_t batch = 0;
  int dir = -1;
  int prec = 0;
  unsigned flags = 0;
  int nshards = 0;  // > 0: one shard of a distributed four-step 1D transform
  int shard = 0;
};

// Tunable planner knobs (the autotuner sweeps these).
struct Choice {
  int row_nt = 256;  // threads per workgroup of row passes (256, or 512 where compiled)
  int cmax = 64;     // widest column block a column pass may use
  int nf = 0;        // 0: default factorisation of long 1D lengths; else pass lengths f[]
  int f[3] = {0, 0, 0};
  int chunk = 0;     // multi-pass plans: transforms per chunk (0 = whole batch); all passes
                     // of a chunk run before the next chunk, reusing one workspace region
  int p2row = 0;     // two-pass 1D: pass 1 stores in natural order and pass 2 is a row
                     // pass over contiguous lines with a transposed store.  2D / 3D: 1
                     // keeps separate row and column passes where a plane pass exists
  int row_pts = 0;   // points per workgroup of plain row passes: 16384 or 8192; 0 = the
                     // measured default (8192 for split lines <= 8192 points, which
                     // then fit two workgroups per CU, and for FP16 1024-point lines)
};

struct PlanSpec {
  Desc d;
  Choice ch;
  bool tuned = false;
  double tuned_us = 0.0;
  int64_t npts = 0;  // points per transform
  std::vector<PassSpec> passes;
  int scale = 0;
  size_t ws_bytes = 0;
  size_t buf_bytes = 0;
  size_t in_bytes = 0, out_bytes = 0;
  // real plans: N of the real transform (0 for complex plans); npts and the
  // passes then describe the M = N/2 point complex transform inside
  int64_t real_n = 0;
  bool real_fused = false;  // the real step runs inside the (single) row pass
  size_t zbuf_bytes = 0;  // unfused: the complex transform's side of the elementwise pass
  // shard plans: passes[0] is step 1 (before the exchange), the rest step 2;
  // n1 = the step-1 length N1
  int64_t shard_n1 = 0;
};

tcfft_status col_choice(int L, int64_t inner, int cmax, bool split, bool xtw, bool tstore,
                        KernelKey* out) {
  for (int C : {64, 32, 16, 8}) {
    if (C > inner || C > cmax) continue;
    for (int NT : {256, 128, 64}) {
      KernelKey k{K_COL, L, r0_of(L), C, NT, split ? 1 : 0, xtw ? 1 : 0, tstore ? 1 : 0};
      if (find_kernel(k) && kernel_lds_bytes(k) <= kMaxLds) {
        *out = k;
        return TCFFT_OK;
      }
    }
  }
  return TCFFT_ERR_UNSUPPORTED;
}

tcfft_status row_choice(int L, int nt, bool split, KernelKey* out, int pts = 0) {
  if (pts == 0) pts = ((split && L <= 8192) || (!split && L == 1024)) && nt == 256 ? 8192 : 16384;
  if (pts == 8192 && L < 16384) {  // the smaller-workgroup variant (256 threads)
    KernelKey k{K_ROW, L, r0_of(L), pts, 256, split ? 1 : 0, 0, 0};
    if (find_kernel(k) && kernel_lds_bytes(k) <= kMaxLds) {
      *out = k;
      return TCFFT_OK;
    }
  }
  for (int NT : {nt, 256}) {
    KernelKey k{K_ROW, L, r0_of(L), 0, NT, split ? 1 : 0, 0, 0};
    if (find_kernel(k) && kernel_lds_bytes(k) <= kMaxLds) {
      *out = k;
      return TCFFT_OK;
    }
  }
  return TCFFT_ERR_UNSUPPORTED;
}

// Row pass over `lines` contiguous lines of L points.  q > 0: transposed store
// of lines in groups of q (line l of group b, output k at b q L + k q + l).
tcfft_status add_row_pass(PlanSpec& ps, int L, int64_t lines, int src, int dst, int64_t q = 0) {
  PassSpec p;
  tcfft_status st = row_choice(L, ps.ch.row_nt, ps.d.prec == TCFFT_PREC_SPLIT_FP16, &p.key,
                               q > 0 ? 16384 : ps.ch.row_pts);
  if (st) return st;
  if (q > 0) {
    p.key.tstore = 1;
    p.key.NT = 256;
    p.key.C = 0;
    if (!find_kernel(p.key) || q % 4 != 0 || !is_pow2(q)) return TCFFT_ERR_UNSUPPORTED;
    p.q = q;
    p.s_out = q;
  }
  const int64_t tpb = kernel_points_per_wg(p.key) / L;
  p.tpb = tpb;
  p.ntrans = lines;
  p.lines_per_batch = lines / ps.d.batch;
  p.grid = (lines + tpb - 1) / tpb;
  p.lds = kernel_lds_bytes(p.key);
  p.src = src;
  p.dst = dst;
  p.scale = pass_scale(L);
  ps.passes.push_back(p);
  return TCFFT_OK;
}

// Plane pass of a 3D transform: the 2D DFT of [ny][nz] planes in one
// workgroup, 16384 points per workgroup (one plane, or 2 or 4 planes of 8192 or
// 4096 points in FP16); `lines` = planes x ny.
tcfft_status add_plane_pass(PlanSpec& ps, int nz, int ny, int64_t lines) {
  PassSpec p;
  p.key = KernelKey{K_PLANE, nz, r0_of(nz), ny, 256, ps.d.prec == TCFFT_PREC_SPLIT_FP16 ? 1 : 0,
                    0, 0};
  const int64_t pl = (int64_t)nz * ny;
  if ((pl != 16384 && pl != 8192 && pl != 4096) || nz < 64 || !find_kernel(p.key))
    return TCFFT_ERR_UNSUPPORTED;
  p.tpb = 16384 / nz;  // lines per workgroup: whole planes
  p.ntrans = lines;
  p.lines_per_batch = lines / ps.d.batch;
  p.grid = (lines + p.tpb - 1) / p.tpb;
  p.s_out = nz;
  p.lds = kernel_lds_bytes(p.key);
  p.src = 0;
  p.dst = 1;
  p.scale = pass_scale(nz) + pass_scale(ny);
  ps.passes.push_back(p);
  return TCFFT_OK;
}

// Single-pass 65536-point transform (one workgroup per line, FP16 only).
tcfft_status add_big_pass(PlanSpec& ps, int64_t lines) {
  PassSpec p;
  p.key = KernelKey{K_BIG, 65536, 1, 0, 512, 0, 0, 0};
  if (!find_kernel(p.key)) return TCFFT_ERR_UNSUPPORTED;
  p.tpb = 1;
  p.ntrans = lines;
  p.lines_per_batch = lines / ps.d.batch;
  p.grid = lines;
  p.lds = kernel_lds_bytes(p.key);
  p.src = 0;
  p.dst = 1;
  p.scale = pass_scale(65536);
  ps.passes.push_back(p);
  return TCFFT_OK;
}

// Column pass: `outer` blocks of [L][inner]; input element (j, i) of block o at
// o*in_outer + j*inner + i.  Output per mode (see KParams).
tcfft_status add_col_pass(PlanSpec& ps, int L, int64_t inner, int64_t outer, int64_t in_outer,
                          int64_t out_outer, int64_t s_out, int64_t q, int64_t qstride,
                          bool tstore, int64_t xmod, int64_t xdiv, int src, int dst,
                          int64_t cgroup = 0) {
  PassSpec p;
  const bool xtw = xmod > 0;
  // a column block must not straddle a group of `cgroup` columns (3-pass pass 2)
  const int cmax = (int)std::min<int64_t>(ps.ch.cmax, cgroup > 0 ? cgroup : ps.ch.cmax);
  tcfft_status st =
      col_choice(L, inner, cmax, ps.d.prec == TCFFT_PREC_SPLIT_FP16, xtw, tstore, &p.key);
  if (st) return st;
  p.s_in = inner;
  p.s_out = s_out;
  p.blocks = inner / p.key.C;
  // the kernels divide by these with shifts
  if (!is_pow2(p.blocks) || !is_pow2(q) || !is_pow2(xdiv)) return TCFFT_ERR_INTERNAL;
  p.in_outer = in_outer;
  p.out_outer = out_outer;
  p.q = q;
  p.qstride = qstride;
  p.xmod = xmod;
  p.xdiv = xdiv;
  p.grid = outer * p.blocks;
  p.outer_per_batch = outer / ps.d.batch;
  p.lds = kernel_lds_bytes(p.key);
  p.src = src;
  p.dst = dst;
  p.scale = pass_scale(L);
  ps.passes.push_back(p);
  return TCFFT_OK;
}

// Splits a long 1D length into pass lengths (each <= kMaxColL), most balanced first.
std::vector<int> long_split(int64_t n) {
  const int lg = ilog2(n);
  const int lmax = ilog2(kMaxColL);
  const int np = (lg + lmax - 1) / lmax;
  std::vector<int> f;
  int rem = lg;
  for (int i = 0; i < np; ++i) {
    int e = rem / (np - i);
    f.push_back(1 << e);
    rem -= e;
  }
  // larger factors last: the last pass writes with the widest contiguous runs
  std::sort(f.begin(), f.end());
  return f;
}

tcfft_status validate(const Desc& d) {
  if (d.rank < 1 || d.rank > 3) return TCFFT_ERR_INVALID_ARG;
  if (d.batch <= 0) return TCFFT_ERR_INVALID_ARG;
  if (d.dir != TCFFT_FORWARD && d.dir != TCFFT_INVERSE) return TCFFT_ERR_INVALID_ARG;
  if (d.prec < 0 || d.prec > 3) return TCFFT_ERR_INVALID_ARG;
  if (d.flags & ~(unsigned)(TCFFT_FLAG_NO_SCALE | TCFFT_FLAG_TUNE |
                            TCFFT_FLAG_REAL))
    return TCFFT_ERR_INVALID_ARG;
  if (d.nx <= 0 || d.ny <= 0 || d.nz <= 0) return TCFFT_ERR_INVALID_ARG;
  if (!is_pow2(d.nx) || !is_pow2(d.ny) || !is_pow2(d.nz)) return TCFFT_ERR_UNSUPPORTED;
  if (d.prec == TCFFT_PREC_FP64 &&
      (d.rank != 1 || d.nx > 4096 || (d.flags & TCFFT_FLAG_REAL) || d.nshards != 0))
    return TCFFT_ERR_UNSUPPORTED;
  if (d.rank == 1) {
    if (d.nx < 16 || d.nx > ((int64_t)1 << 27)) return TCFFT_ERR_UNSUPPORTED;
  } else if (d.rank == 2) {
    if (d.nx < 16 || d.nx > kMaxColL || d.ny < 16 || d.ny > kMaxRowL) return TCFFT_ERR_UNSUPPORTED;
    if (d.prec == TCFFT_PREC_FP32_RADIX2) return TCFFT_ERR_UNSUPPORTED;
  } else {
    if (d.nx < 16 || d.nx > kMaxColL || d.ny < 16 || d.ny > kMaxColL || d.nz < 16 ||
        d.nz > kMaxRowL)
      return TCFFT_ERR_UNSUPPORTED;
    if (d.prec == TCFFT_PREC_FP32_RADIX2) return TCFFT_ERR_UNSUPPORTED;
  }
  if (d.flags & TCFFT_FLAG_REAL) {
    if (d.rank != 1 || d.prec == TCFFT_PREC_FP32_RADIX2 || d.nx < 32) return TCFFT_ERR_UNSUPPORTED;
  }
  if (d.nshards != 0) {
    if (d.nshards < 2 || !is_pow2(d.nshards) || d.shard < 0 || d.shard >= d.nshards)
      return TCFFT_ERR_INVALID_ARG;
    if (d.rank != 1 || (d.flags & TCFFT_FLAG_REAL) || d.prec == TCFFT_PREC_FP32_RADIX2 ||
        d.nx <= kMaxRowL)
      return TCFFT_ERR_UNSUPPORTED;
  }
  if (d.nx * d.ny > kMaxPointsPerPlan / d.nz) return TCFFT_ERR_UNSUPPORTED;
  const int64_t npts = d.nx * d.ny * d.nz;
  if (d.batch > kMaxPointsPerPlan / npts) return TCFFT_ERR_UNSUPPORTED;
  return TCFFT_OK;
}

// The complex transform inside a real plan: M = N/2 points, same batch,
// direction and precision.
Desc complex_desc(const Desc& d) {
  Desc c = d;
  if (d.flags & TCFFT_FLAG_REAL) {
    c.nx = d.nx / 2;
    c.flags &= ~(unsigned)TCFFT_FLAG_REAL;
  }
  return c;
}

tcfft_status build_spec(const Desc& d, const Choice& ch, PlanSpec* out) {
  tcfft_status st = validate(d);
  if (st) return st;
  if (d.flags & TCFFT_FLAG_REAL) {
    // N reals = M complex words: the M-point complex plan, then (forward) or
    // before it (inverse) one elementwise pass between it and the spectrum
    PlanSpec ps;
    Choice cc = ch;
    cc.row_pts = 16384;  // the real-input row kernels hold 16384 points per workgroup
    if ((st = build_spec(complex_desc(d), cc, &ps))) return st;
    const int64_t M = d.nx / 2;
    const size_t elt = d.prec == TCFFT_PREC_FP16 ? 4 : 8;
    const size_t zb = (size_t)(M * d.batch) * elt, xb = (size_t)((M + 1) * d.batch) * elt;
    ps.d = d;
    ps.real_n = d.nx;
    ps.zbuf_bytes = zb;
    // single-pass sizes: the spectrum step runs inside the row pass (an
    // epilogue forward, a prologue inverse), so the data crosses HBM once
    if (ps.passes.size() == 1 && ps.passes[0].key.kind == K_ROW) {
      KernelKey k = ps.passes[0].key;
      k.NT = 256;
      k.real = d.dir == TCFFT_FORWARD ? 1 : 2;
      if (find_kernel(k)) {
        ps.passes[0].key = k;
        ps.real_fused = true;
        ps.zbuf_bytes = 0;
      }
    }
    ps.in_bytes = d.dir == TCFFT_FORWARD ? zb : xb;
    ps.out_bytes = d.dir == TCFFT_FORWARD ? xb : zb;
    ps.buf_bytes = xb;
    *out = ps;
    return TCFFT_OK;
  }
  PlanSpec ps;
  ps.d = d;
  ps.ch = ch;
  ps.npts = d.nx * d.ny * d.nz;
  const int64_t B = d.batch;
  const size_t elt = d.prec == TCFFT_PREC_FP16 ? 4 : d.prec == TCFFT_PREC_FP64 ? 16 : 8;
  ps.buf_bytes = (size_t)(ps.npts * B) * elt;
  ps.in_bytes = ps.out_bytes = ps.buf_bytes;
  if (d.prec == TCFFT_PREC_FP64) {  // one matrix-core row pass, no workspace, no scaling
    ps.scale = 0;
    *out = ps;
    return TCFFT_OK;
  }
  if (d.prec == TCFFT_PREC_FP32_RADIX2) {
    ps.ws_bytes = ps.buf_bytes;
    ps.scale = 0;
    *out = ps;
    return TCFFT_OK;
  }
  if (d.nshards > 0) {
    // one shard of the four-step split N = N1 * M over G = nshards devices
    // (Sec. 2.1, Eq. 3, with the columns m dealt out in slabs of M / G):
    // step 1 runs the N1-point DFTs of the shard's columns m = g M/G + m_l
    // with the twiddle W_N^{m k1} at their global m, storing Z[h][m_l][k1_l]
    // (k1 = h N1/G + k1_l) so that block h is the contiguous chunk for device
    // h; after the exchange, device h holds [m][k1_l] and step 2 runs the
    // M-point DFTs over m (one column pass, or two when M > 2048), writing
    // X[k' N1 + h N1/G + k1_l] at [k'][k1_l].
    const int64_t N = d.nx, G = d.nshards;
    const std::vector<int> f = long_split(N);
    const int64_t N1 = f[0], M = N / N1, n1l = N1 / G, ml = M / G;
    if (n1l < 4 || ml < 8) return TCFFT_ERR_UNSUPPORTED;
    ps.shard_n1 = N1;
    // a shard buffer holds N/G points per transform: the kernels place the
    // lo plane of split data npts * batch words after the hi plane
    ps.npts = N / G;
    ps.buf_bytes = (size_t)(N / G * B) * elt;
    ps.in_bytes = ps.out_bytes = ps.buf_bytes;
    st = add_col_pass(ps, (int)N1, ml, B, N / G, N / G, 0, 1, 0, true, N, 1, 0, 1);
    if (!st) {
      PassSpec& p1 = ps.passes.back();
      p1.xoff = d.shard * ml;
      p1.tblk = n1l;
      p1.tblk_stride = ml * n1l;
    }
    if (!st && f.size() == 2) {
      st = add_col_pass(ps, (int)M, n1l, B, M * n1l, M * n1l, n1l, n1l, 0, false, 0, 1, 0, 1);
    } else if (!st && f.size() == 3) {
      const int64_t M2 = f[1], M3 = f[2];
      // over m2 (stride M3 n1l), twiddle W_M^{m3 k2}, store [m3][k2][k1_l]
      st = add_col_pass(ps, (int)M2, M3 * n1l, B, M * n1l, M * n1l, n1l, n1l, M2 * n1l, false, M,
                        n1l, 0, 1, n1l);
      // over m3 (stride M2 n1l), in place -> [k3 M2 + k2][k1_l]
      if (!st)
        st = add_col_pass(ps, (int)M3, M2 * n1l, B, M * n1l, M * n1l, M2 * n1l, M2 * n1l, 0, false,
                          0, 1, 1, 1);
    } else if (!st) {
      st = TCFFT_ERR_UNSUPPORTED;
    }
  } else if (d.rank == 1) {
    const int64_t N = d.nx;
    if (N <= kMaxRowL) {
      st = add_row_pass(ps, (int)N, B, 0, 1);
    } else if (ch.nf == 1) {
      // the single-pass kernel (65536 points, FP16)
      if (N != 65536 || ch.f[0] != 65536 || d.prec != TCFFT_PREC_FP16) return TCFFT_ERR_UNSUPPORTED;
      st = add_big_pass(ps, B);
    } else {
      std::vector<int> f = long_split(N);
      if (ch.nf > 0) {
        int64_t prod = 1;
        f.assign(ch.f, ch.f + ch.nf);
        for (int v : f) {
          if (v < 16 || v > kMaxColL || !is_pow2(v)) return TCFFT_ERR_UNSUPPORTED;
          prod *= v;
        }
        if (prod != N) return TCFFT_ERR_UNSUPPORTED;
      }
      if (f.size() == 2 && ch.p2row) {
        const int64_t N1 = f[0], N2 = f[1];
        // pass 1: N1-point DFTs over n1 (stride N2), twiddle W_N^{n2 k1}, natural
        // store Z[k1][n2]; pass 2: rows of N2 contiguous points, X[k1 + N1 k2]
        st = add_col_pass(ps, (int)N1, N2, B, N, N, N2, N2, 0, false, N, 1, 0, 2);
        if (!st) st = add_row_pass(ps, (int)N2, B * N1, 2, 1, N1);
      } else if (f.size() == 2) {
        const int64_t N1 = f[0], N2 = f[1];
        // pass 1: N1-point DFTs over n1 (stride N2), twiddle W_N^{n2 k1},
        // transposed store Z[n2][k1]
        st = add_col_pass(ps, (int)N1, N2, B, N, N, 0, 1, 0, true, N, 1, 0, 2);
        // pass 2: N2-point DFTs over n2 (stride N1) -> X[k2 N1 + k1]
        if (!st) st = add_col_pass(ps, (int)N2, N1, B, N, N, N1, N1, 0, false, 0, 1, 2, 1);
      } else if (f.size() == 3) {
        const int64_t N1 = f[0], N2 = f[1], N3 = f[2];
        // pass 1: over n1 (stride N2 N3), twiddle W_N^{(n2 N3 + n3) k1},
        // transposed store Z1[n2][n3][k1]
        st = add_col_pass(ps, (int)N1, N2 * N3, B, N, N, 0, 1, 0, true, N, 1, 0, 2);
        // pass 2: over n2 (stride N3 N1), twiddle W_{N2 N3}^{n3 k2}, store
        // Z2[n3][k2][k1] (into the output buffer)
        if (!st)
          st = add_col_pass(ps, (int)N2, N3 * N1, B, N, N, N1, N1, N2 * N1, false, N2 * N3, N1, 2, 1,
                            N1);
        // pass 3: over n3 (stride N2 N1) -> X[k3 N1 N2 + k2 N1 + k1], in place
        if (!st)
          st = add_col_pass(ps, (int)N3, N2 * N1, B, N, N, N2 * N1, N2 * N1, 0, false, 0, 1, 1, 1);
      } else {
        st = TCFFT_ERR_UNSUPPORTED;
      }
      ps.ws_bytes = ps.buf_bytes;
    }
  } else if (d.rank == 2) {
    const int64_t nx = d.nx, ny = d.ny;
    // a 16384-point array fits one workgroup: rows and columns in one pass
    const bool plane = !ch.p2row && add_plane_pass(ps, (int)ny, (int)nx, B * nx) == TCFFT_OK;
    // rows: B*nx contiguous ny-point transforms; then columns: B blocks of
    // [nx][ny], strided nx-point transforms, in place in the output
    if (!plane) st = add_row_pass(ps, (int)ny, B * nx, 0, 1);
    if (!plane && !st)
      st = add_col_pass(ps, (int)nx, ny, B, nx * ny, nx * ny, ny, ny, 0, false, 0, 1, 1, 1);
  } else {
    // the 3D DFT is separable: rows of nz (contiguous), then ny-point
    // transforms over the B*nx planes [ny][nz], then nx-point transforms over
    // the B blocks [nx][ny*nz]; the column passes run in place in the output
    const int64_t nx = d.nx, ny = d.ny, nz = d.nz;
    // a plane of 16384 points fits one workgroup: rows and columns of the
    // plane in one pass (the data cross HBM twice instead of three times)
    const bool plane = !ch.p2row && add_plane_pass(ps, (int)nz, (int)ny, B * nx * ny) == TCFFT_OK;
    if (!plane) {
      st = add_row_pass(ps, (int)nz, B * nx * ny, 0, 1);
      if (!st)
        st = add_col_pass(ps, (int)ny, nz, B * nx, ny * nz, ny * nz, nz, nz, 0, false, 0, 1, 1, 1);
    }
    if (!st)
      st = add_col_pass(ps, (int)nx, ny * nz, B, ps.npts, ps.npts, ny * nz, ny * nz, 0, false, 0, 1,
                        1, 1);
  }
  if (st) return st;
  if (d.prec == TCFFT_PREC_FP16 && ch.chunk > 0 && ch.chunk < B && ps.ws_bytes > 0)
    ps.ws_bytes = (size_t)((double)ps.ws_bytes * (double)ch.chunk / (double)B);
  if (d.flags & TCFFT_FLAG_NO_SCALE)
    for (auto& p : ps.passes) p.scale = 0;
  ps.scale = 0;
  for (auto& p : ps.passes) ps.scale += p.scale;
  *out = ps;
  return TCFFT_OK;
}

std::string describe(const PlanSpec& ps) {
  static const char* precs[] = {"fp16", "split_fp16", "fp32_radix2", "fp64"};
  char b[1024];
  std::string s;
  std::snprintf(b, sizeof b,
                "{\"rank\":%d,\"dims\":[%lld%s%s%s%s],\"batch\":%lld,\"dir\":%d,\"precision\":\"%s\","
                "\"scale_log2\":%d,\"buffer_bytes\":%zu,\"input_bytes\":%zu,\"output_bytes\":%zu,"
                "\"workspace_bytes\":%zu,\"real\":%lld,\"real_kernel\":\"%s\","
                "\"choice\":{\"row_nt\":%d,\"cmax\":%d,\"factors\":[%d,%d,%d],\"chunk\":%d,\"p2row\":%d,"
                "\"row_pts\":%d},\"tuned\":%s,"
                "\"tuned_us\":%.2f,\"nshards\":%d,\"shard\":%d,\"shard_n1\":%lld,\"points\":%lld,"
                "\"passes\":[",
                ps.d.rank, (long long)ps.d.nx, ps.d.rank >= 2 ? "," : "",
                ps.d.rank >= 2 ? std::to_string(ps.d.ny).c_str() : "", ps.d.rank == 3 ? "," : "",
                ps.d.rank == 3 ? std::to_string(ps.d.nz).c_str() : "", (long long)ps.d.batch, ps.d.dir,
                precs[ps.d.prec], ps.scale, ps.buf_bytes, ps.in_bytes, ps.out_bytes,
                ps.ws_bytes + ps.zbuf_bytes, (long long)ps.real_n,
                ps.real_n == 0 ? "" : ps.real_fused ? "fused" : (ps.d.dir == TCFFT_FORWARD ? "r2c_post" : "c2r_pre"),
                ps.ch.row_nt, ps.ch.cmax,
                ps.ch.nf > 0 ? ps.ch.f[0] : 0, ps.ch.nf > 1 ? ps.ch.f[1] : 0,
                ps.ch.nf > 2 ? ps.ch.f[2] : 0, ps.ch.chunk, ps.ch.p2row, ps.ch.row_pts,
                ps.tuned ? "true" : "false",
                ps.tuned_us, ps.d.nshards, ps.d.shard, (long long)ps.shard_n1, (long long)ps.npts);
  s += b;
  if (ps.d.prec == TCFFT_PREC_FP32_RADIX2) {
    std::snprintf(b, sizeof b, "{\"kernel\":\"radix2_fp32\",\"stages\":%d}", ilog2(ps.npts));
    s += b;
  }
  if (ps.d.prec == TCFFT_PREC_FP64) {
    const int l = ilog2(ps.npts);
    std::snprintf(b, sizeof b, "{\"kernel\":\"f64_row\",\"L\":%lld,\"R0\":%d,\"stages16\":%d}",
                  (long long)ps.npts, 1 << (l % 4), l / 4);
    s += b;
  }
  for (size_t i = 0; i < ps.passes.size(); ++i) {
    const PassSpec& p = ps.passes[i];
    std::string rad = "[";
    int r0 = p.key.R0, s16 = s16_of(p.key.L);
    bool first = true;
    if (r0 > 1) {
      rad += std::to_string(r0);
      first = false;
    }
    for (int k = 0; k < s16; ++k) {
      rad += first ? "16" : ",16";
      first = false;
    }
    rad += "]";
    std::snprintf(b, sizeof b,
                  "%s{\"kernel\":\"%s\",\"L\":%d,\"radices\":%s,\"C\":%d,\"NT\":%d,\"grid\":%lld,"
                  "\"lds\":%zu,\"xtw\":%d,\"tstore\":%d,\"scale\":%d,\"src\":%d,\"dst\":%d,"
                  "\"s_in\":%lld,\"s_out\":%lld,\"xmod\":%lld,\"real\":%d,\"blocks\":%lld,"
                  "\"in_outer\":%lld,\"out_outer\":%lld,\"q\":%lld,\"qstride\":%lld,"
                  "\"xdiv\":%lld,\"xoff\":%lld,\"tblk\":%lld,\"tblk_stride\":%lld,\"lines\":%lld,"
                  "\"tpb\":%lld,\"fused\":%d}",
                  i ? "," : "",
                  p.key.kind == K_ROW ? "row"
                  : p.key.kind == K_BIG ? "big"
                  : p.key.kind == K_PLANE ? "plane" : "col",
                  p.key.L, rad.c_str(), p.key.C,
                  p.key.NT, (long long)p.grid, p.lds, p.key.xtw, p.key.tstore, p.scale, p.src,
                  p.dst, (long long)p.s_in, (long long)p.s_out, (long long)p.xmod, p.key.real,
                  (long long)p.blocks, (long long)p.in_outer, (long long)p.out_outer, (long long)p.q,
                  (long long)p.qstride, (long long)p.xdiv, (long long)p.xoff,
                  (long long)(p.tblk > 0 ? p.tblk : p.key.L), (long long)p.tblk_stride,
                  (long long)p.ntrans, (long long)p.tpb, fused_variant(p.key) >= 0 ? 1 : 0);
    s += b;
  }
  s += "]}";
  return s;
}

int copy_out(const std::string& s, char* buf, size_t len) {
  if (buf && len) {
    size_t n = std::min(len - 1, s.size());
    std::memcpy(buf, s.data(), n);
    buf[n] = 0;
  }
  return (int)s.size();
}

// ---------------------------------------------------------------------------
// Device side of a plan.
struct DevPass {
  PassSpec spec;
  KernelFns fn;
  float2* tw = nullptr;      // W_L^m
  float2* xtw_lo = nullptr;  // two-level W_M tables
  float2* xtw_hi = nullptr;
  void* fimg2 = nullptr;     // A_k images of the matrix-core radix-R0 block (R0 = 2, 4)
  void* fimg3 = nullptr;     // A_lo images of a row pass's stride-16 stage (twiddle folded in)
  int xbits = 0;
  int persist_grid = 0;      // resident workgroups for the grouped (persistent) launch
  int single_grid = 0;       // resident workgroups of the single kernel (persistent variants)
};

}  // namespace

struct tcfft_plan_s {
  PlanSpec spec;
  int device = 0;
  std::vector<DevPass> dp;
  void* fimg = nullptr;     // radix-16 A operands (pass-independent: one scale variant)
  void* ws = nullptr;
  float2* r2tw = nullptr;   // FP32 radix-2 comparator: W_N^m
  double2* f64tw = nullptr; // FP64 matrix-core plans: W_N^m, m < N
  void* zbuf = nullptr;     // real plans: the complex transform's input or output
  float2* rtw = nullptr;    // real plans: W_N^{dir k}, k <= M
  std::vector<void*> allocs;
};

namespace {

tcfft_status dev_alloc(tcfft_plan_s* p, size_t bytes, void** out) {
  *out = nullptr;
  if (bytes == 0) return TCFFT_OK;
  if (std::getenv("TCFFT_TEST_FAIL_ALLOC")) return TCFFT_ERR_ALLOC;
  if (hipMalloc(out, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *out = nullptr;
    return TCFFT_ERR_ALLOC;
  }
  p->allocs.push_back(*out);
  return TCFFT_OK;
}

void free_plan(tcfft_plan_s* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  for (void* a : p->allocs) (void)hipFree(a);
  delete p;
}

tcfft_status check_device(int* dev, int* ncu) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return TCFFT_ERR_NO_DEVICE;
  }
  if (hipGetDevice(dev) != hipSuccess) return TCFFT_ERR_NO_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, *dev) != hipSuccess) return TCFFT_ERR_NO_DEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return TCFFT_ERR_NO_DEVICE;
  if (ncu) *ncu = prop.multiProcessorCount;
  return TCFFT_OK;
}

std::mutex g_attr_mu;

tcfft_status prepare_kernel(const void* fn, size_t lds) {
  if (lds <= 65536) return TCFFT_OK;
  std::lock_guard<std::mutex> lk(g_attr_mu);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
    (void)hipGetLastError();
    return TCFFT_ERR_LAUNCH;
  }
  return TCFFT_OK;
}

// Builds the device tables of a plan from its spec.  Table generation runs on
// a private stream so that plan creation never waits on other streams' work.
tcfft_status create_device_plan(const PlanSpec& ps, tcfft_plan_s** out) {
  int dev = 0, ncu = 256;
  tcfft_status st = check_device(&dev, &ncu);
  if (st) return st;
  tcfft_plan_s* p = new tcfft_plan_s();
  p->spec = ps;
  p->device = dev;
  const Desc& d = ps.d;
  const double sgn = (double)d.dir;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    delete p;
    return TCFFT_ERR_LAUNCH;
  }
  do {
    if (d.prec == TCFFT_PREC_FP64) {
      void* t = nullptr;
      if ((st = dev_alloc(p, (size_t)ps.npts * sizeof(double2), &t))) break;
      p->f64tw = (double2*)t;
      launch_gen_twiddles_f64(p->f64tw, ps.npts, ps.npts, sgn, s);
      break;
    }
    if (d.prec == TCFFT_PREC_FP32_RADIX2) {
      void* t = nullptr;
      if ((st = dev_alloc(p, (size_t)(ps.npts / 2) * sizeof(float2), &t))) break;
      p->r2tw = (float2*)t;
      launch_gen_twiddles(p->r2tw, ps.npts / 2, ps.npts, 1, sgn, s);
      if ((st = dev_alloc(p, ps.ws_bytes, &p->ws))) break;
      break;
    }
    if ((st = dev_alloc(p, 4 * 64 * 16, &p->fimg))) break;
    const bool noscale = (d.flags & TCFFT_FLAG_NO_SCALE) != 0;
    launch_gen_fimg(p->fimg, sgn, noscale ? 1.0 : 0.25, s);
    for (const PassSpec& sp : ps.passes) {
      DevPass dpp;
      dpp.spec = sp;
      if (!find_kernels(sp.key, &dpp.fn)) {
        st = TCFFT_ERR_INTERNAL;
        break;
      }
      if ((st = prepare_kernel((const void*)dpp.fn.single, sp.lds))) break;
      if ((st = prepare_kernel((const void*)dpp.fn.multi, sp.lds))) break;
      int per_cu = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)dpp.fn.multi,
                                                      sp.key.NT, sp.lds) != hipSuccess ||
          per_cu <= 0) {
        (void)hipGetLastError();
        per_cu = 1;
      }
      dpp.persist_grid = per_cu * ncu;
      if (dpp.fn.persistent) {
        per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)dpp.fn.single,
                                                        sp.key.NT, sp.lds) != hipSuccess ||
            per_cu <= 0) {
          (void)hipGetLastError();
          per_cu = 1;
        }
        dpp.single_grid = per_cu * ncu;
      }
      void* t = nullptr;
      const int r0 = r0_of(sp.key.L);
      if ((r0 == 2 || r0 == 4) && sp.key.kind == K_COL) {  // the column passes' matrix-core block
        if ((st = dev_alloc(p, (size_t)r0 * 256 * 16, &dpp.fimg2))) break;
        // both stages' scales: 2^-1 (radix 2 or 4) and 2^-2 (radix 16)
        launch_gen_fimg_r(dpp.fimg2, r0, sgn, noscale ? 1.0 : 0.125, s);
      }
      if (sp.key.kind != K_BIG) {  // read by FP16 stride-16 stages that fold their twiddle
        if ((st = dev_alloc(p, (size_t)16 * 256 * 16, &dpp.fimg3))) break;
        launch_gen_fimg_tw(dpp.fimg3, 16, sgn, noscale ? 1.0 : 0.25, s);
      }
      if ((st = dev_alloc(p, (size_t)sp.key.L * sizeof(float2), &t))) break;
      dpp.tw = (float2*)t;
      launch_gen_twiddles(dpp.tw, sp.key.L, sp.key.L, 1, sgn, s);
      if (sp.key.kind == K_PLANE) {  // W_ny for the plane's column half
        if ((st = dev_alloc(p, (size_t)sp.key.C * sizeof(float2), &t))) break;
        dpp.xtw_lo = (float2*)t;
        launch_gen_twiddles(dpp.xtw_lo, sp.key.C, sp.key.C, 1, sgn, s);
      }
      if (sp.key.kind == K_BIG) {  // W_4096 for the 4096-point sub-transforms
        if ((st = dev_alloc(p, 4096 * sizeof(float2), &t))) break;
        dpp.xtw_hi = (float2*)t;
        launch_gen_twiddles(dpp.xtw_hi, 4096, 4096, 1, sgn, s);
      }
      if (sp.xmod > 0) {
        const int lg = ilog2(sp.xmod);
        // the lo table also serves W_M^k for every output index k < L
        dpp.xbits = std::max((lg + 1) / 2, ilog2(sp.key.L));
        const int64_t nlo = (int64_t)1 << dpp.xbits, nhi = std::max<int64_t>(1, sp.xmod >> dpp.xbits);
        if ((st = dev_alloc(p, (size_t)nlo * sizeof(float2), &t))) break;
        dpp.xtw_lo = (float2*)t;
        if ((st = dev_alloc(p, (size_t)nhi * sizeof(float2), &t))) break;
        dpp.xtw_hi = (float2*)t;
        launch_gen_twiddles(dpp.xtw_lo, nlo, sp.xmod, 1, sgn, s);
        launch_gen_twiddles(dpp.xtw_hi, nhi, sp.xmod, nlo, sgn, s);
      }
      p->dp.push_back(dpp);
    }
    if (st) break;
    if ((st = dev_alloc(p, ps.ws_bytes, &p->ws))) break;
    if (ps.real_n > 0) {
      const int64_t M = ps.real_n / 2;
      if ((st = dev_alloc(p, ps.zbuf_bytes, &p->zbuf))) break;
      void* t = nullptr;
      if ((st = dev_alloc(p, (size_t)(M + 1) * sizeof(float2), &t))) break;
      p->rtw = (float2*)t;
      launch_gen_twiddles(p->rtw, M + 1, ps.real_n, 1, sgn, s);
    }
  } while (false);
  if (!st && hipGetLastError() != hipSuccess) st = TCFFT_ERR_LAUNCH;
  if (hipStreamSynchronize(s) != hipSuccess && !st) st = TCFFT_ERR_LAUNCH;
  (void)hipStreamDestroy(s);
  if (st) {
    free_plan(p);
    return st;
  }
  *out = p;
  return TCFFT_OK;
}

// Kernel parameters of one pass for a job of `batch` transforms (<= the plan's
// batch) with workspace `ws`; *grid receives the pass's workgroup count.
KParams make_kparams(const tcfft_plan_s* p, const DevPass& dpp, const void* in, void* out,
                     int64_t batch, void* ws, int64_t* grid) {
  const PlanSpec& ps = p->spec;
  const PassSpec& sp = dpp.spec;
  const bool split = ps.d.prec == TCFFT_PREC_SPLIT_FP16;
  const int64_t plane = ps.npts * batch;
  auto buf = [&](int which) -> uint32_t* {
    return which == 0 ? (uint32_t*)in : which == 1 ? (uint32_t*)out : (uint32_t*)ws;
  };
  KParams kp{};
  kp.in = buf(sp.src);
  kp.out = buf(sp.dst);
  kp.in_plane = split ? plane : 0;
  kp.out_plane = split ? plane : 0;
  if (sp.key.kind != K_COL) {
    kp.ntrans = sp.lines_per_batch * batch;
    *grid = (kp.ntrans + sp.tpb - 1) / sp.tpb;
  } else {  // column passes: ntrans is the number of tiles (read by the pipelined kernels)
    *grid = sp.blocks * batch * sp.outer_per_batch;
    kp.ntrans = *grid;
  }
  kp.tw = dpp.tw;
  kp.fimg = p->fimg;
  kp.fimg2 = dpp.fimg2;
  kp.fimg3 = dpp.fimg3;
  kp.r0scale = (float)std::ldexp(1.0, -(sp.scale - 2 * s16_of(sp.key.L)));
  kp.r0scale2 = 1.0f;
  if (sp.key.kind == K_PLANE) {  // rows of nz, then columns of ny, each with its own radix-R0 scale
    kp.r0scale = (float)std::ldexp(1.0, -(pass_scale(sp.key.L) - 2 * s16_of(sp.key.L)));
    kp.r0scale2 = (float)std::ldexp(1.0, -(pass_scale(sp.key.C) - 2 * s16_of(sp.key.C)));
  }
  if (ps.d.flags & TCFFT_FLAG_NO_SCALE) kp.r0scale = kp.r0scale2 = 1.0f;
  kp.sgn = (float)ps.d.dir;
  kp.s_in = sp.s_in;
  kp.s_out = sp.s_out;
  kp.blocks = sp.blocks;
  kp.in_outer = sp.in_outer;
  kp.out_outer = sp.out_outer;
  kp.q = sp.q;
  kp.qstride = sp.qstride;
  kp.xtw_lo = dpp.xtw_lo;
  kp.xtw_hi = dpp.xtw_hi;
  kp.xbits = dpp.xbits;
  kp.xmask = (uint32_t)(sp.xmod > 0 ? sp.xmod - 1 : 0);
  kp.xdiv = sp.xdiv;
  kp.blocks_log2 = sp.blocks > 0 ? ilog2(sp.blocks) : 0;
  kp.q_log2 = ilog2(sp.q);
  kp.xdiv_log2 = ilog2(sp.xdiv);
  kp.xoff = sp.xoff;
  kp.tblk_log2 = ilog2(sp.tblk > 0 ? sp.tblk : sp.key.L);
  kp.tblk_stride = sp.tblk_stride;
  if (sp.key.real) {  // spectrum lines hold M + 1 words; the row pass reads W_N from xtw_lo
    if (split && sp.key.real == 1) kp.out_plane = (ps.npts + 1) * batch;
    if (split && sp.key.real == 2) kp.in_plane = (ps.npts + 1) * batch;
    kp.xtw_lo = p->rtw;
  }
  return kp;
}

tcfft_status exec_r2(tcfft_plan_s* p, const void* in, void* out, hipStream_t s) {
  const PlanSpec& ps = p->spec;
  const int T = ilog2(ps.npts);
  const float2* src = (const float2*)in;
  float2* ws = (float2*)p->ws;
  float2* o = (float2*)out;
  for (int st = 0; st < T; ++st) {
    // the last stage lands in `out`; earlier ones alternate so that no stage
    // reads and writes the same buffer
    float2* dst = ((T - 1 - st) % 2 == 0) ? o : ws;
    if (st == 0 && dst == src) dst = ws;
    if (st > 0 && dst == src) dst = (dst == o) ? ws : o;
    launch_radix2_stage(src, dst, ps.npts, (int64_t)1 << st, ps.d.batch, p->r2tw, s);
    src = dst;
  }
  if (src != o)
    if (hipMemcpyAsync(o, src, ps.buf_bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return TCFFT_ERR_LAUNCH;
  return hipGetLastError() == hipSuccess ? TCFFT_OK : TCFFT_ERR_LAUNCH;
}

// Runs the plan's passes (the first `npasses` of them when npasses >= 0, the
// last of those writing to `out`).
tcfft_status exec_impl(tcfft_plan_s* p, const void* in, void* out, hipStream_t s,
                       int npasses = -1) {
  const PlanSpec& ps = p->spec;
  if (ps.d.prec == TCFFT_PREC_FP32_RADIX2) return exec_r2(p, in, out, s);
  if (ps.d.prec == TCFFT_PREC_FP64)
    return launch_f64_row((const double2*)in, (double2*)out, (int)ps.npts, ps.d.batch, p->f64tw,
                          s) == hipSuccess
               ? TCFFT_OK
               : TCFFT_ERR_LAUNCH;
  const int np = npasses < 0 ? (int)p->dp.size() : npasses;
  const int64_t B = ps.d.batch;
  // chunked execution of multi-pass plans: every pass of a chunk before the
  // next chunk, the workspace region reused, so the intermediate of a chunk
  // can stay in the memory-side cache.  Split planes move with the chunk.
  const bool split = ps.d.prec == TCFFT_PREC_SPLIT_FP16;
  const int64_t chunk =
      (!split && ps.ch.chunk > 0 && ps.ch.chunk < B && p->dp.size() > 1) ? ps.ch.chunk : B;
  for (int64_t b0 = 0; b0 < B; b0 += chunk) {
    const int64_t nb = std::min(chunk, B - b0);
    const void* cin = in;
    void* cout = out;
    if (chunk != B) {
      cin = (const uint32_t*)in + b0 * ps.npts;
      cout = (uint32_t*)out + b0 * ps.npts;
    }
    for (int i = 0; i < np; ++i) {
      DevPass dpp = p->dp[i];
      if (i == np - 1) dpp.spec.dst = 1;
      int64_t grid = 0;
      KParams kp = make_kparams(p, dpp, cin, cout, nb, p->ws, &grid);
      // persistent variants: one resident wave of workgroups strides over the tiles
      if (dpp.fn.persistent && dpp.single_grid > 0) grid = std::min<int64_t>(grid, dpp.single_grid);
      void* args[] = {&kp};
      if (hipLaunchKernel((const void*)dpp.fn.single, dim3((unsigned)grid),
                          dim3(dpp.spec.key.NT), args, dpp.spec.lds, s) != hipSuccess) {
        (void)hipGetLastError();
        return TCFFT_ERR_LAUNCH;
      }
    }
  }
  return TCFFT_OK;
}

// Real plans: the M-point complex transform from the input into zbuf, then the
// spectrum pass (forward); or the pass into zbuf, then the transform (inverse).
void launch_real_step(const tcfft_plan_s* p, const void* in, void* out, hipStream_t s) {
  const PlanSpec& ps = p->spec;
  const bool split = ps.d.prec == TCFFT_PREC_SPLIT_FP16;
  if (ps.d.dir == TCFFT_FORWARD)
    launch_r2c_post(p->zbuf, out, p->rtw, ps.npts, ps.d.batch, split, s);
  else
    launch_c2r_pre(in, p->zbuf, p->rtw, ps.npts, ps.d.batch, split, s);
}

tcfft_status exec_real(tcfft_plan_s* p, const void* in, void* out, hipStream_t s) {
  tcfft_status st;
  if (p->spec.real_fused) return exec_impl(p, in, out, s);
  if (p->spec.d.dir == TCFFT_FORWARD) {
    if ((st = exec_impl(p, in, p->zbuf, s))) return st;
    launch_real_step(p, nullptr, out, s);
  } else {
    launch_real_step(p, in, nullptr, s);
    if ((st = exec_impl(p, p->zbuf, out, s))) return st;
  }
  if (hipGetLastError() != hipSuccess) return TCFFT_ERR_LAUNCH;
  return TCFFT_OK;
}

tcfft_status exec_any(tcfft_plan_s* p, const void* in, void* out, hipStream_t s) {
  return p->spec.real_n > 0 ? exec_real(p, in, out, s) : exec_impl(p, in, out, s);
}

// One step of a shard plan: step 1 is pass 0, step 2 the remaining passes
// (the first reads `in`, every later one runs in place in `out`).
tcfft_status exec_shard_step(tcfft_plan_s* p, int step, const void* in, void* out, hipStream_t s) {
  const size_t first = step == 1 ? 0 : 1, last = step == 1 ? 1 : p->dp.size();
  for (size_t i = first; i < last; ++i) {
    const DevPass& dpp = p->dp[i];
    int64_t grid = 0;
    KParams kp = make_kparams(p, dpp, in, out, p->spec.d.batch, p->ws, &grid);
    void* args[] = {&kp};
    if (hipLaunchKernel((const void*)dpp.fn.single, dim3((unsigned)grid), dim3(dpp.spec.key.NT),
                        args, dpp.spec.lds, s) != hipSuccess) {
      (void)hipGetLastError();
      return TCFFT_ERR_LAUNCH;
    }
  }
  return TCFFT_OK;
}

// ---------------------------------------------------------------------------
// Grouped mixed-size execution.  Pass l of every job runs after pass l-1 of
// every job (stream order), so one launch per (pass level, kernel variant)
// serves all jobs of that variant: the descriptor table (one KParams per job)
// and the prefix sum of their workgroup counts go to device memory, and a
// persistent grid of resident workgroups strides over all their tiles.
struct KeyLess {
  bool operator()(const KernelKey& a, const KernelKey& b) const {
    return std::memcmp(&a, &b, sizeof(KernelKey)) < 0;
  }
};

// Pinned staging slots for descriptor uploads.  A slot is reused only after
// the copy that read it has completed (its event), so the host never rewrites
// memory an in-flight copy still reads.
struct StagingSlot {
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool pending = false;
};
std::mutex g_stage_mu;
StagingSlot g_stage[16];
unsigned g_stage_next = 0;

tcfft_status upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_stage_mu);
  StagingSlot& sl = g_stage[g_stage_next++ % 16];
  if (sl.pending) {
    if (hipEventSynchronize(sl.ev) != hipSuccess) return TCFFT_ERR_LAUNCH;
    sl.pending = false;
  }
  if (!sl.ev && hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return TCFFT_ERR_LAUNCH;
  }
  if (sl.cap < bytes) {
    if (sl.host) (void)hipHostFree(sl.host);
    sl.host = nullptr;
    sl.cap = 0;
    const size_t cap = std::max<size_t>(bytes, 64 * 1024);
    if (hipHostMalloc(&sl.host, cap, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      sl.host = nullptr;
      return TCFFT_ERR_ALLOC;
    }
    sl.cap = cap;
  }
  std::memcpy(sl.host, src, bytes);
  if (hipMemcpyAsync(dst, sl.host, bytes, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipEventRecord(sl.ev, s) != hipSuccess) {
    (void)hipGetLastError();
    return TCFFT_ERR_LAUNCH;
  }
  sl.pending = true;
  return TCFFT_OK;
}

struct Group {
  KernelFns fn;
  int nt = 0;
  size_t lds = 0;
  int persist = 0;
  std::vector<KParams> jobs;
  std::vector<int64_t> prefix{0};
};

// ---------------------------------------------------------------------------
// Fused launches (k_fused.hip): when every pass of every job has a fused
// variant, one kernel runs many variants.  TCFFT_FUSED in the environment:
//   unset or 1  one launch per (pass level, class): no waits inside a launch,
//               levels ordered by the stream (the default);
//   2           one launch per class for all levels, a job's pass waiting on
//               that job's previous pass through tile counters;
//   0           per-(level, variant) grouped launches.
// TCFFT_FUSED_WAIT_US bounds one dependency wait (default 1 s).
int fused_mode() {
  const char* e = std::getenv("TCFFT_FUSED");
  if (!e || !*e) return 1;
  return e[0] == '0' ? 0 : e[0] == '2' ? 2 : 1;
}

int64_t fused_wait_us() {
  const char* e = std::getenv("TCFFT_FUSED_WAIT_US");
  if (!e || !*e) return 1000000;
  const long long v = std::atoll(e);
  return v < 0 ? 0 : (int64_t)v;
}

constexpr size_t kFusedLdsMax = 163840;  // LDS of one CU

struct FusedDev {
  bool ready = false;
  int64_t clock_khz = 0;
};
std::mutex g_fused_mu;
std::map<int, FusedDev> g_fused_dev;

// One-time set-up of the fused kernels on the current device (their LDS
// limit); returns the device's wall-clock rate.
tcfft_status fused_prepare(int64_t* clock_khz) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return TCFFT_ERR_NO_DEVICE;
  std::lock_guard<std::mutex> lk(g_fused_mu);
  FusedDev& fd = g_fused_dev[dev];
  if (!fd.ready) {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
        khz <= 0) {
      (void)hipGetLastError();
      return TCFFT_ERR_NO_DEVICE;
    }
    for (bool sp : {false, true})
      if (hipFuncSetAttribute(fused_kernel(sp), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)kFusedLdsMax) != hipSuccess) {
        (void)hipGetLastError();
        return TCFFT_ERR_LAUNCH;
      }
    fd.clock_khz = khz;
    fd.ready = true;
  }
  *clock_khz = fd.clock_khz;
  return TCFFT_OK;
}

struct FusedClass {
  std::vector<KParams> kps;
  std::vector<FusedSeg> segs;
  std::vector<int32_t> starts;  // segs[s].start, compact for the device's binary search
  size_t lds = 0;
  int64_t total = 0;
  size_t off = 0;  // byte offset of the class's header in the upload
};

}  // namespace

size_t tcfft_internal_desc_bytes(int max_jobs) {
  // <= 3 pass levels: per level at most one group per job
  return (size_t)3 * (size_t)max_jobs * (sizeof(GroupHdr) + sizeof(KParams) + 2 * sizeof(int64_t)) + 4096;
}

tcfft::GraphCache::~GraphCache() {
  for (auto& kv : execs) (void)hipGraphExecDestroy((hipGraphExec_t)kv.second);
}

// The batch as fused launches (mode 1: one per pass level and class; mode 2:
// one per class, with dependency waits).  *applied is false (and nothing is
// enqueued) when some pass has no fused variant or the batch does not fit the
// fused kernel's limits; the caller then uses grouped launches.
static tcfft_status exec_fused(const tcfft::Job* jobs, int njobs, int levels, int mode,
                               hipStream_t s, void* desc_arena, size_t arena_cap,
                               tcfft::GraphCache* graphs, bool arg_upload, bool* applied) {
  *applied = false;
  // classes in launch order: FP16 with tiles of <= 64 KB of LDS (two
  // workgroups per CU), FP16 with larger tiles, then the same for split data
  // (mode 1: for each pass level in turn).  A launch's LDS is its largest
  // variant's, so small tiles do not share a launch with 128 KB ones.  In
  // mode 2 a job's passes must not go back to an earlier class, and a pass
  // whose previous pass is in an earlier launch needs no wait (stream order).
  const int NC = mode == 2 ? 4 : 4 * levels;
  std::vector<FusedClass> cls(NC);
  std::vector<int> last(njobs, -1), last_cls(njobs, -1);
  std::string sig = mode == 2 ? "fused2" : "fused1";
  for (int lv = 0; lv < levels; ++lv)
    for (int j = 0; j < njobs; ++j) {
      tcfft_plan_s* p = jobs[j].plan;
      if (p->spec.d.prec == TCFFT_PREC_FP32_RADIX2 || p->spec.d.prec == TCFFT_PREC_FP64 ||
          lv >= (int)p->dp.size())
        continue;
      const DevPass& dpp = p->dp[lv];
      const int var = fused_variant(dpp.spec.key);
      if (var < 0) return TCFFT_OK;
      const int k = (mode == 2 ? 0 : 4 * lv) + (dpp.spec.key.split ? 2 : 0) +
                    (dpp.spec.lds > 65536 ? 1 : 0);
      if (k < last_cls[j]) return TCFFT_OK;
      FusedClass& c = cls[k];
      int64_t tiles = 0;
      c.kps.push_back(make_kparams(p, dpp, jobs[j].in, jobs[j].out, jobs[j].batch, jobs[j].ws, &tiles));
      FusedSeg sg{};
      sg.start = c.total;
      sg.tiles = tiles;
      sg.var = var;
      sg.dep = mode == 2 && last_cls[j] == k ? last[j] : -1;
      if (sg.dep >= 0) c.segs[sg.dep].waited = 1;
      sg.kp = (int32_t)c.kps.size() - 1;
      last[j] = (int)c.segs.size();
      last_cls[j] = k;
      c.segs.push_back(sg);
      c.starts.push_back((int32_t)std::min<int64_t>(c.total, INT32_MAX));
      c.total += tiles;
      c.lds = std::max(c.lds, dpp.spec.lds);
      sig.append((const char*)&var, sizeof var);
      sig.append((const char*)&k, sizeof k);
    }
  // tables: per class the header, descriptors, segments and counters (8-byte aligned)
  size_t bytes = 0;
  int64_t clock_khz = 0;
  for (int k = 0; k < NC; ++k) {
    FusedClass& c = cls[k];
    if (c.segs.empty()) continue;
    c.lds = (c.lds + 15) / 16 * 16;
    if (c.lds + 16 > kFusedLdsMax || c.total >= ((int64_t)1 << 30)) return TCFFT_OK;
    tcfft_status st = fused_prepare(&clock_khz);
    if (st) return st;
    c.off = bytes;
    bytes += sizeof(FusedHdr) + c.kps.size() * sizeof(KParams) + c.segs.size() * sizeof(FusedSeg) +
             (c.segs.size() * sizeof(int32_t) + 7) / 8 * 8 +
             ((2 + c.segs.size()) * sizeof(int) + 7) / 8 * 8;
  }
  if (bytes == 0) return TCFFT_OK;
  uint8_t* dmem = (uint8_t*)desc_arena;
  if (dmem && bytes > arena_cap) return TCFFT_ERR_ALLOC;
  *applied = true;
  if (!dmem) {
    void* m = nullptr;
    if (hipMallocAsync(&m, bytes, s) != hipSuccess) {
      (void)hipGetLastError();
      return TCFFT_ERR_ALLOC;
    }
    dmem = (uint8_t*)m;
  }
  std::vector<uint8_t> host(bytes, 0);  // counters upload as zeros
  const int64_t ticks = fused_wait_us() * clock_khz / 1000;
  for (int k = 0; k < NC; ++k) {
    const FusedClass& c = cls[k];
    if (c.segs.empty()) continue;
    const size_t kb = c.kps.size() * sizeof(KParams), sb = c.segs.size() * sizeof(FusedSeg);
    const size_t tb = (c.segs.size() * sizeof(int32_t) + 7) / 8 * 8;
    FusedHdr h{};
    h.kps = (const KParams*)(dmem + c.off + sizeof(FusedHdr));
    h.segs = (const FusedSeg*)(dmem + c.off + sizeof(FusedHdr) + kb);
    h.starts = (const int32_t*)(dmem + c.off + sizeof(FusedHdr) + kb + sb);
    h.ctr = (int*)(dmem + c.off + sizeof(FusedHdr) + kb + sb + tb);
    h.nsegs = (int64_t)c.segs.size();
    h.total = c.total;
    h.lds_slot = (int64_t)(c.lds / 4);
    h.wait_ticks = ticks;
    h.ticketed = mode == 2 ? 1 : 0;
    std::memcpy(host.data() + c.off, &h, sizeof h);
    std::memcpy(host.data() + c.off + sizeof(FusedHdr), c.kps.data(), kb);
    std::memcpy(host.data() + c.off + sizeof(FusedHdr) + kb, c.segs.data(), sb);
    std::memcpy(host.data() + c.off + sizeof(FusedHdr) + kb + sb, c.starts.data(),
                c.starts.size() * sizeof(int32_t));
  }
  tcfft_status st = TCFFT_OK;
  if (arg_upload) {
    if (launch_write_words(dmem, host.data(), bytes, s) != hipSuccess) return TCFFT_ERR_LAUNCH;
  } else if ((st = upload(dmem, host.data(), bytes, s))) {
    return st;
  }
  // one workgroup per tile; a captured launch takes the next power of two
  // (workgroups past the total exit at once), so one graph serves every batch
  // of the same variant sequence and tile-count bucket
  auto grid_of = [](int64_t total, bool bucket) {
    int64_t g = std::max<int64_t>(1, total);
    if (bucket) g = (int64_t)1 << ilog2(2 * g - 1);
    return g;
  };
  auto launch_all = [&](bool bucket) -> tcfft_status {
    for (int k = 0; k < NC; ++k) {
      const FusedClass& c = cls[k];
      if (c.segs.empty()) continue;
      const FusedHdr* hdr = (const FusedHdr*)(dmem + c.off);
      const int64_t want = grid_of(c.total, bucket);
      void* args[] = {&hdr};
      if (hipLaunchKernel(fused_kernel((k & 2) != 0), dim3((unsigned)std::max<int64_t>(1, want)),
                          dim3(256), args, c.lds + 16, s) != hipSuccess) {
        (void)hipGetLastError();
        return TCFFT_ERR_LAUNCH;
      }
    }
    return TCFFT_OK;
  };
  bool use_graph = false;
  if (graphs && desc_arena) {
    for (int k = 0; k < NC; ++k) {
      const int64_t g = cls[k].segs.empty() ? 0 : grid_of(cls[k].total, true);
      sig.append((const char*)&g, sizeof g);
    }
    use_graph = graphs->execs.count(sig) > 0 || ++graphs->seen[sig] >= graphs->capture_after;
  }
  if (use_graph) {
    auto it = graphs->execs.find(sig);
    if (it == graphs->execs.end()) {
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return TCFFT_ERR_LAUNCH;
      }
      tcfft_status lst = launch_all(true);
      const hipError_t ce = hipStreamEndCapture(s, &graph);
      if (lst || ce != hipSuccess || hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        if (graph) (void)hipGraphDestroy(graph);
        return lst ? lst : TCFFT_ERR_LAUNCH;
      }
      (void)hipGraphDestroy(graph);
      it = graphs->execs.emplace(sig, (void*)exec).first;
    }
    if (hipGraphLaunch((hipGraphExec_t)it->second, s) != hipSuccess) {
      (void)hipGetLastError();
      return TCFFT_ERR_LAUNCH;
    }
  } else if ((st = launch_all(false))) {
    return st;
  }
  if (!desc_arena) (void)hipFreeAsync(dmem, s);  // stream-ordered: after the launch
  return hipGetLastError() == hipSuccess ? TCFFT_OK : TCFFT_ERR_LAUNCH;
}

tcfft_status tcfft_internal_exec_jobs(const tcfft::Job* jobs, int njobs, hipStream_t s,
                                      void* desc_arena, size_t arena_cap,
                                      tcfft::GraphCache* graphs, bool arg_upload) {
  int levels = 0;
  for (int j = 0; j < njobs; ++j) {
    tcfft_plan_s* p = jobs[j].plan;
    if (p->spec.d.prec == TCFFT_PREC_FP32_RADIX2 || p->spec.d.prec == TCFFT_PREC_FP64) {
      tcfft_status st = exec_impl(p, jobs[j].in, jobs[j].out, s);
      if (st) return st;
      continue;
    }
    levels = std::max(levels, (int)p->dp.size());
  }
  const int fmode = fused_mode();
  if (levels > 0 && fmode > 0) {
    bool applied = false;
    tcfft_status st = exec_fused(jobs, njobs, levels, fmode, s, desc_arena, arena_cap, graphs,
                                 arg_upload, &applied);
    if (st || applied) return st;
  }
  // every (pass level, variant) group of the batch, in launch order
  std::vector<Group> groups;
  std::vector<KernelKey> keys;
  for (int lv = 0; lv < levels; ++lv) {
    std::map<KernelKey, Group, KeyLess> lg;
    for (int j = 0; j < njobs; ++j) {
      tcfft_plan_s* p = jobs[j].plan;
      if (p->spec.d.prec == TCFFT_PREC_FP32_RADIX2 || p->spec.d.prec == TCFFT_PREC_FP64 ||
          lv >= (int)p->dp.size())
        continue;
      const DevPass& dpp = p->dp[lv];
      Group& g = lg[dpp.spec.key];
      g.fn = dpp.fn;
      g.nt = dpp.spec.key.NT;
      g.lds = dpp.spec.lds;
      g.persist = dpp.persist_grid;
      int64_t grid = 0;
      g.jobs.push_back(make_kparams(p, dpp, jobs[j].in, jobs[j].out, jobs[j].batch, jobs[j].ws, &grid));
      g.prefix.push_back(g.prefix.back() + grid);
    }
    for (auto& kv : lg) {
      keys.push_back(kv.first);
      groups.push_back(std::move(kv.second));
    }
  }
  if (groups.empty()) return hipGetLastError() == hipSuccess ? TCFFT_OK : TCFFT_ERR_LAUNCH;
  // one upload for the whole batch: the group headers, then per group its
  // KParams table and prefix array (all 8-byte aligned)
  const size_t G = groups.size();
  std::vector<size_t> off(G);
  size_t total_bytes = G * sizeof(GroupHdr);
  for (size_t i = 0; i < G; ++i) {
    off[i] = total_bytes;
    total_bytes += groups[i].jobs.size() * sizeof(KParams) + groups[i].prefix.size() * sizeof(int64_t);
  }
  uint8_t* dmem = (uint8_t*)desc_arena;
  if (dmem && total_bytes > arena_cap) return TCFFT_ERR_ALLOC;
  if (!dmem) {
    void* m = nullptr;
    if (hipMallocAsync(&m, total_bytes, s) != hipSuccess) {
      (void)hipGetLastError();
      return TCFFT_ERR_ALLOC;
    }
    dmem = (uint8_t*)m;
  }
  std::vector<uint8_t> host(total_bytes);
  for (size_t i = 0; i < G; ++i) {
    const size_t jb = groups[i].jobs.size() * sizeof(KParams);
    GroupHdr h{};
    h.jobs = (const KParams*)(dmem + off[i]);
    h.prefix = (const int64_t*)(dmem + off[i] + jb);
    h.njobs = (int64_t)groups[i].jobs.size();
    std::memcpy(host.data() + i * sizeof(GroupHdr), &h, sizeof h);
    std::memcpy(host.data() + off[i], groups[i].jobs.data(), jb);
    std::memcpy(host.data() + off[i] + jb, groups[i].prefix.data(),
                groups[i].prefix.size() * sizeof(int64_t));
  }
  tcfft_status st = TCFFT_OK;
  if (arg_upload) {
    if (launch_write_words(dmem, host.data(), total_bytes, s) != hipSuccess) return TCFFT_ERR_LAUNCH;
  } else if ((st = upload(dmem, host.data(), total_bytes, s))) {
    return st;
  }
  auto launch_all = [&](bool full_grid) -> tcfft_status {
    for (size_t i = 0; i < G; ++i) {
      const Group& g = groups[i];
      const GroupHdr* hdr = (const GroupHdr*)(dmem + i * sizeof(GroupHdr));
      const int64_t want = g.fn.multi_one ? g.prefix.back()  // one tile per workgroup
                           : full_grid    ? g.persist
                                          : std::min<int64_t>(g.prefix.back(), g.persist);
      const unsigned grid = (unsigned)std::max<int64_t>(1, want);
      void* args[] = {&hdr};
      if (hipLaunchKernel((const void*)g.fn.multi, dim3(grid), dim3(g.nt), args, g.lds, s) !=
          hipSuccess) {
        (void)hipGetLastError();
        return TCFFT_ERR_LAUNCH;
      }
    }
    return TCFFT_OK;
  };
  std::string sig;
  bool use_graph = false;
  if (graphs && desc_arena) {
    // the captured launches depend only on the variant sequence and on the
    // fixed header addresses, so one graph serves every batch of that shape;
    // a sequence is captured only once it recurs (capture costs far more
    // than a few launches)
    sig.assign((const char*)keys.data(), keys.size() * sizeof(KernelKey));
    // a one-tile-per-workgroup group's grid follows its tile count: such
    // batches are launched directly
    bool one = false;
    for (const Group& g : groups) one = one || g.fn.multi_one;
    use_graph = !one && (graphs->execs.count(sig) > 0 || ++graphs->seen[sig] >= graphs->capture_after);
  }
  if (use_graph) {
    auto it = graphs->execs.find(sig);
    if (it == graphs->execs.end()) {
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return TCFFT_ERR_LAUNCH;
      }
      tcfft_status lst = launch_all(true);
      const hipError_t ce = hipStreamEndCapture(s, &graph);
      if (lst || ce != hipSuccess || hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        if (graph) (void)hipGraphDestroy(graph);
        return lst ? lst : TCFFT_ERR_LAUNCH;
      }
      (void)hipGraphDestroy(graph);
      it = graphs->execs.emplace(sig, (void*)exec).first;
    }
    if (hipGraphLaunch((hipGraphExec_t)it->second, s) != hipSuccess) {
      (void)hipGetLastError();
      return TCFFT_ERR_LAUNCH;
    }
  } else {
    st = launch_all(false);
    if (st) return st;
  }
  if (!desc_arena) (void)hipFreeAsync(dmem, s);  // stream-ordered: after the launches
  return hipGetLastError() == hipSuccess ? TCFFT_OK : TCFFT_ERR_LAUNCH;
}

size_t tcfft_internal_plan_ws_bytes(const tcfft_plan_s* p, int64_t batch) {
  const PlanSpec& ps = p->spec;
  if (ps.ws_bytes == 0) return 0;
  return (size_t)((double)ps.ws_bytes * (double)batch / (double)ps.d.batch);
}

int64_t tcfft_internal_plan_batch(const tcfft_plan_s* p) { return p->spec.d.batch; }
int64_t tcfft_internal_plan_points(const tcfft_plan_s* p) { return p->spec.npts; }
int tcfft_internal_plan_prec(const tcfft_plan_s* p) { return p->spec.d.prec; }

namespace {

tcfft_status exec_many_impl(const tcfft_plan* plans, const void* const* in, void* const* out,
                            int njobs, hipStream_t s, bool use_static = false) {
  std::vector<Job> jobs;
  std::vector<int> post;  // real forward jobs: their spectrum pass runs after the group
  jobs.reserve(njobs);
  for (int j = 0; j < njobs; ++j) {
    tcfft_plan_s* p = plans[j];
    const PlanSpec& ps = p->spec;
    if (ps.d.prec == TCFFT_PREC_FP16 && ps.ch.chunk > 0 && ps.ch.chunk < ps.d.batch &&
        p->dp.size() > 1) {
      // a chunked plan's workspace holds one chunk: it runs on its own
      tcfft_status st = exec_any(p, in[j], out[j], s);
      if (st) return st;
      continue;
    }
    const void* ji = in[j];
    void* jo = out[j];
    const bool step = ps.real_n > 0 && !ps.real_fused;
    if (step && ps.d.dir == TCFFT_FORWARD) {
      jo = p->zbuf;
      post.push_back(j);
    } else if (step) {
      launch_real_step(p, in[j], nullptr, s);
      ji = p->zbuf;
    }
    jobs.push_back(Job{p, ji, jo, ps.d.batch, p->ws});
  }
  if (!jobs.empty()) {
    void* arena = nullptr;
    size_t cap = 0;
    if (use_static && static_scratch(&arena, &cap) != hipSuccess) {
      (void)hipGetLastError();
      return TCFFT_ERR_NO_DEVICE;
    }
    tcfft_status st = tcfft_internal_exec_jobs(jobs.data(), (int)jobs.size(), s, arena, cap,
                                               nullptr, use_static);
    if (st) return st;
  }
  for (int j : post) launch_real_step(plans[j], nullptr, out[j], s);
  return hipGetLastError() == hipSuccess ? TCFFT_OK : TCFFT_ERR_LAUNCH;
}

// ---------------------------------------------------------------------------
// Autotuner.  For a (rank, size, batch bucket, precision) it times every
// candidate Choice on scratch buffers (plan creation cost is excluded, as in
// the paper's measurement, Sec. 5.1) and keeps the fastest.  Results are
// cached in-process and can be saved/loaded as text ("wisdom").
std::mutex g_tune_mu;
std::map<std::string, std::pair<Choice, double>> g_tune;

std::string tune_key(const Desc& d) {
  char b[160];
  if (d.rank == 3)
    std::snprintf(b, sizeof b, "r3_%lldx%lldx%lld_b%d_p%d", (long long)d.nx, (long long)d.ny,
                  (long long)d.nz, ilog2(d.batch), d.prec);
  else
    std::snprintf(b, sizeof b, "r%d_%lldx%lld_b%d_p%d", d.rank, (long long)d.nx, (long long)d.ny,
                  ilog2(d.batch), d.prec);
  return b;
}

std::vector<Choice> candidates_base(const Desc& d);

// Adds chunked variants (64 MB and 128 MB of FP16 data per chunk) of every
// multi-pass FP16 candidate.
std::vector<Choice> candidates(const Desc& d) {
  std::vector<Choice> base = candidates_base(d);
  const bool multipass = d.rank >= 2 || d.nx > kMaxRowL;
  if (!multipass || d.prec != TCFFT_PREC_FP16) return base;
  std::vector<Choice> out = base;
  const int64_t per = d.nx * d.ny * d.nz * 4;  // bytes of one FP16 transform
  for (int64_t mb : {64, 128}) {
    const int64_t c = std::max<int64_t>(1, (mb << 20) / per);
    if (c >= d.batch) continue;
    for (Choice ch : base) {
      if (ch.nf == 1) continue;  // single pass: nothing to chunk
      ch.chunk = (int)c;
      out.push_back(ch);
    }
  }
  return out;
}

std::vector<Choice> candidates_base(const Desc& d) {
  std::vector<Choice> out;
  if (d.prec == TCFFT_PREC_FP32_RADIX2 || d.prec == TCFFT_PREC_FP64) return out;
  const bool longp = d.rank == 1 && d.nx > kMaxRowL;
  if (!longp) {
    for (int sep : {0, 1}) {
      // with a plane pass possible, also the separate row and column passes
      const int64_t plane_pts = d.rank == 2 ? d.nx * d.ny : d.ny * d.nz;
      if (sep && (d.rank == 1 || (plane_pts != 16384 && plane_pts != 8192 && plane_pts != 4096)))
        continue;
      for (int nt : {256, 512})
        for (int cmax : {64, 32, 16, 8})
          for (int pts : {16384, 8192}) {
            if (d.rank == 1 && cmax != 64) continue;
            if (pts == 8192 && nt != 256) continue;  // 8192-point row workgroups run 256 threads
            Choice c;
            c.row_nt = nt;
            c.cmax = cmax;
            c.p2row = sep;
            c.row_pts = pts;
            out.push_back(c);
          }
    }
    return out;
  }
  const int lg = ilog2(d.nx);
  if (d.nx == 65536 && d.prec == TCFFT_PREC_FP16) {  // the single-pass kernel
    Choice c;
    c.nf = 1;
    c.f[0] = 65536;
    out.push_back(c);
  }
  for (int e1 = 4; e1 <= 11; ++e1) {  // two passes
    const int e2 = lg - e1;
    if (e2 < 4 || e2 > 11) continue;
    for (int p2row : {0, 1}) {
      if (p2row && (e2 < 8 || e2 > 10)) continue;  // transposed-store row variants
      for (int cmax : {64, 32, 16, 8}) {
        Choice c;
        c.cmax = cmax;
        c.nf = 2;
        c.f[0] = 1 << e1;
        c.f[1] = 1 << e2;
        c.p2row = p2row;
        out.push_back(c);
      }
    }
  }
  if (lg >= 20) {  // three passes (above 2^22 the only split; from 2^20 an
                   // alternative whose short passes take wide column blocks)
    std::vector<int> base = long_split(d.nx);
    if (base.size() == 2) {  // a balanced three-way split as an extra candidate
      base = {1 << (lg / 3), 1 << ((lg - lg / 3) / 2), 1 << (lg - lg / 3 - (lg - lg / 3) / 2)};
    }
    std::sort(base.begin(), base.end());
    do {
      if (base.size() != 3 || base[0] < 16 || base[2] > kMaxColL) continue;
      // 32-column blocks: twice the tiles per pass (2^24 x 1: 84 -> 80 us)
      for (int cmax : {64, 32}) {
        Choice c;
        c.cmax = cmax;
        c.nf = 3;
        for (int i = 0; i < 3; ++i) c.f[i] = base[i];
        out.push_back(c);
      }
    } while (std::next_permutation(base.begin(), base.end()));
  }
  return out;
}

tcfft_status time_spec(const PlanSpec& ps, void* a, void* b, double* us) {
  tcfft_plan_s* p = nullptr;
  tcfft_status st = create_device_plan(ps, &p);
  if (st) return st;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    free_plan(p);
    return TCFFT_ERR_LAUNCH;
  }
  for (int i = 0; i < 2 && !st; ++i) st = exec_impl(p, a, b, s);
  const int reps = 5;
  (void)hipEventRecord(e0, s);
  for (int i = 0; i < reps && !st; ++i) st = exec_impl(p, a, b, s);
  (void)hipEventRecord(e1, s);
  float ms = 0.f;
  if (!st && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    st = TCFFT_ERR_LAUNCH;
  *us = ms * 1e3 / reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  free_plan(p);
  return st;
}

// Picks the Choice for `d`: the cached one, else (when tuning) the fastest
// candidate, else the defaults.
tcfft_status choose(const Desc& d, Choice* ch, bool* tuned, double* tuned_us) {
  const std::string key = tune_key(d);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      *ch = it->second.first;
      *tuned = true;
      *tuned_us = it->second.second;
      return TCFFT_OK;
    }
  }
  *ch = Choice{};
  *tuned = false;
  *tuned_us = 0.0;
  if (!(d.flags & TCFFT_FLAG_TUNE)) return TCFFT_OK;
  std::vector<Choice> cands = candidates(d);
  if (cands.size() <= 1) return TCFFT_OK;
  // tune on at most 2^27 points per buffer: the batch the plan will run, up
  // to 512 MiB of FP16 data (at half that batch the tuner's ranking of
  // multi-pass and chunked plans did not carry over)
  Desc dt = d;
  const int64_t npts = d.nx * d.ny * d.nz;
  dt.batch = std::max<int64_t>(1, std::min<int64_t>(d.batch, ((int64_t)1 << 27) / npts));
  size_t bytes = 0;
  std::vector<PlanSpec> specs;
  std::vector<std::string> seen;  // candidates that build the same kernels are timed once
  for (const Choice& c : cands) {
    PlanSpec ps;
    if (build_spec(dt, c, &ps) != TCFFT_OK) continue;
    std::string k = describe(ps);
    const size_t cut = k.find("\"choice\"");
    const size_t pas = k.find("\"passes\"");
    if (cut != std::string::npos && pas != std::string::npos) k.erase(cut, pas - cut);
    k += std::to_string(ps.ch.chunk);
    if (std::find(seen.begin(), seen.end(), k) != seen.end()) continue;
    seen.push_back(k);
    bytes = std::max(bytes, ps.buf_bytes);
    specs.push_back(ps);
  }
  if (specs.empty()) return TCFFT_OK;
  void *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
    (void)hipGetLastError();
    if (a) (void)hipFree(a);
    return TCFFT_ERR_ALLOC;
  }
  {  // on a private stream: tuning never waits on other streams' work
    hipStream_t fs = nullptr;
    if (hipStreamCreateWithFlags(&fs, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipFree(a);
      (void)hipFree(b);
      return TCFFT_ERR_LAUNCH;
    }
    launch_fill_pattern(a, (int64_t)(bytes / 4), fs);
    (void)hipStreamSynchronize(fs);
    (void)hipStreamDestroy(fs);
  }
  // round 1: every candidate once; round 2: the 4 fastest again, three times
  // each and interleaved (so clock drift under sustained load hits them
  // alike), keeping each one's best
  std::vector<std::pair<double, size_t>> r1;
  for (size_t i = 0; i < specs.size(); ++i) {
    double us = 0;
    if (time_spec(specs[i], a, b, &us) == TCFFT_OK) r1.push_back({us, i});
  }
  double best = 1e30;
  Choice bestc = specs[0].ch;
  if (!r1.empty()) {
    std::sort(r1.begin(), r1.end());
    const size_t K = std::min<size_t>(4, r1.size());
    std::vector<double> fin(K, 1e30);
    for (int rep = 0; rep < 3; ++rep)
      for (size_t k = 0; k < K; ++k) {
        double us = 0;
        if (time_spec(specs[r1[k].second], a, b, &us) == TCFFT_OK) fin[k] = std::min(fin[k], us);
      }
    for (size_t k = 0; k < K; ++k)
      if (fin[k] < best) {
        best = fin[k];
        bestc = specs[r1[k].second].ch;
      }
  }
  (void)hipFree(a);
  (void)hipFree(b);
  if (best >= 1e30) return TCFFT_OK;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = {bestc, best};
  }
  *ch = bestc;
  *tuned = true;
  *tuned_us = best;
  return TCFFT_OK;
}

tcfft_status create_impl(const Desc& d, tcfft_plan* out) {
  PlanSpec ps;
  tcfft_status st = build_spec(d, Choice{}, &ps);  // validates the arguments
  if (st) return st;
  int dev = 0;
  if ((st = check_device(&dev, nullptr))) return st;
  Choice ch;
  bool tuned = false;
  double tuned_us = 0.0;
  // a real plan shares the tuned choice of its complex transform; shard plans
  // keep the default factorisation (every device must split N alike)
  if (d.nshards == 0 && (st = choose(complex_desc(d), &ch, &tuned, &tuned_us))) return st;
  if ((st = build_spec(d, ch, &ps))) return st;
  ps.tuned = tuned;
  ps.tuned_us = tuned_us;
  st = create_device_plan(ps, out);
  if (!st && log_on()) std::fprintf(stderr, "tcfft: plan %s\n", describe(ps).c_str());
  return st;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// Whether exec writes plan-owned intermediate memory (workspace or spectrum buffer).
bool plan_has_scratch(const tcfft_plan_s* p) {
  return p->spec.ws_bytes > 0 || p->spec.zbuf_bytes > 0;
}

// Real plans read lines of M words and write lines of M + 1 (or the reverse):
// workgroups would overwrite input that others have not read yet, so their
// input and output must not overlap.
bool real_overlap(const tcfft_plan_s* p, const void* in, const void* out) {
  if (p->spec.real_n == 0) return false;
  const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
  return a < b + p->spec.out_bytes && b < a + p->spec.in_bytes;
}

}  // namespace

extern "C" {

tcfft_status tcfft_plan_create(tcfft_plan* out, int rank, const int64_t* dims, int64_t batch,
                               int dir, int precision, unsigned flags) {
  if (!out || !dims) return TCFFT_ERR_INVALID_ARG;
  *out = nullptr;
  Desc d;
  d.rank = rank;
  if (rank < 1 || rank > 3) return TCFFT_ERR_INVALID_ARG;
  d.nx = dims[0];
  d.ny = rank >= 2 ? dims[1] : 1;
  d.nz = rank == 3 ? dims[2] : 1;
  d.batch = batch;
  d.dir = dir;
  d.prec = precision;
  d.flags = flags;
  try {
    return logged(create_impl(d, out), "tcfft_plan_create");
  } catch (...) {
    return logged(TCFFT_ERR_INTERNAL, "tcfft_plan_create");
  }
}

tcfft_status tcfft_plan_1d(tcfft_plan* out, int64_t nx, int64_t batch) {
  int64_t dims[1] = {nx};
  return tcfft_plan_create(out, 1, dims, batch, TCFFT_FORWARD, TCFFT_PREC_FP16, 0);
}

tcfft_status tcfft_plan_2d(tcfft_plan* out, int64_t nx, int64_t ny, int64_t batch) {
  int64_t dims[2] = {nx, ny};
  return tcfft_plan_create(out, 2, dims, batch, TCFFT_FORWARD, TCFFT_PREC_FP16, 0);
}

tcfft_status tcfft_exec(tcfft_plan plan, const void* in, void* out, void* stream) {
  tcfft_status st = TCFFT_OK;
  if (!plan || !in || !out || !aligned16(in) || !aligned16(out) || real_overlap(plan, in, out))
    st = TCFFT_ERR_INVALID_ARG;
  else if (plan->spec.d.nshards > 0)
    st = TCFFT_ERR_UNSUPPORTED;  // two steps around an exchange
  else
    st = exec_any(plan, in, out, (hipStream_t)stream);
  return logged(st, "tcfft_exec");
}

tcfft_status tcfft_plan_create_shard(tcfft_plan* out, int64_t n, int64_t batch, int dir,
                                     int precision, int nshards, int shard, unsigned flags) {
  if (!out) return TCFFT_ERR_INVALID_ARG;
  *out = nullptr;
  if (nshards == 0) return TCFFT_ERR_INVALID_ARG;
  Desc d;
  d.nx = n;
  d.batch = batch;
  d.dir = dir;
  d.prec = precision;
  d.flags = flags & ~(unsigned)TCFFT_FLAG_TUNE;
  d.nshards = nshards;
  d.shard = shard;
  try {
    return logged(create_impl(d, out), "tcfft_plan_create_shard");
  } catch (...) {
    return TCFFT_ERR_INTERNAL;
  }
}

int tcfft_shard_dry_run(int64_t n, int64_t batch, int dir, int precision, int nshards, int shard,
                        unsigned flags, char* buf, size_t len) {
  if (nshards == 0) return -(int)TCFFT_ERR_INVALID_ARG;
  Desc d;
  d.nx = n;
  d.batch = batch;
  d.dir = dir;
  d.prec = precision;
  d.flags = flags & ~(unsigned)TCFFT_FLAG_TUNE;
  d.nshards = nshards;
  d.shard = shard;
  PlanSpec ps;
  tcfft_status st = build_spec(d, Choice{}, &ps);
  if (st) return -(int)st;
  return copy_out(describe(ps), buf, len);
}

tcfft_status tcfft_exec_shard(tcfft_plan plan, int step, const void* in, void* out, void* stream) {
  if (!plan || !in || !out || plan->spec.d.nshards == 0 || (step != 1 && step != 2))
    return TCFFT_ERR_INVALID_ARG;
  if (!aligned16(in) || !aligned16(out) || in == out) return TCFFT_ERR_INVALID_ARG;
  try {
    return exec_shard_step(plan, step, in, out, (hipStream_t)stream);
  } catch (...) {
    return TCFFT_ERR_INTERNAL;
  }
}

tcfft_status tcfft_exec_passes(tcfft_plan plan, const void* in, void* out, int npasses,
                               void* stream) {
  tcfft_status st = TCFFT_OK;
  if (!plan || !in || !out || in == out || !aligned16(in) || !aligned16(out))
    st = TCFFT_ERR_INVALID_ARG;
  else if (plan->spec.d.prec == TCFFT_PREC_FP32_RADIX2 || plan->spec.d.prec == TCFFT_PREC_FP64 ||
           plan->spec.real_n > 0 || plan->spec.d.nshards > 0)
    st = TCFFT_ERR_UNSUPPORTED;
  else if (npasses < 1 || npasses > (int)plan->dp.size())
    st = TCFFT_ERR_INVALID_ARG;
  else
    st = exec_impl(plan, in, out, (hipStream_t)stream, npasses);
  return logged(st, "tcfft_exec_passes");
}

}  // extern "C"

namespace {
tcfft_status check_many(const tcfft_plan* plans, const void* const* in, void* const* out,
                        int njobs) {
  if (njobs < 0 || (njobs > 0 && (!plans || !in || !out))) return TCFFT_ERR_INVALID_ARG;
  for (int j = 0; j < njobs; ++j)
    if (!plans[j] || !in[j] || !out[j] || !aligned16(in[j]) || !aligned16(out[j]) ||
        real_overlap(plans[j], in[j], out[j]) || plans[j]->spec.d.nshards > 0)
      return TCFFT_ERR_INVALID_ARG;
  // a plan with a workspace (multi-pass) or a spectrum buffer (real plans
  // with a separate spectrum pass) can serve only one job of a grouped launch:
  // two jobs would write the same intermediate inside one launch
  for (int j = 0; j < njobs; ++j) {
    if (!plan_has_scratch(plans[j])) continue;
    for (int i = 0; i < j; ++i)
      if (plans[i] == plans[j]) return TCFFT_ERR_INVALID_ARG;
  }
  return TCFFT_OK;
}
}  // namespace

extern "C" {

tcfft_status tcfft_exec_many(const tcfft_plan* plans, const void* const* in, void* const* out,
                             int njobs, void* stream) {
  tcfft_status st = check_many(plans, in, out, njobs);
  if (st || njobs == 0) return logged(st, "tcfft_exec_many");
  try {
    return logged(exec_many_impl(plans, in, out, njobs, (hipStream_t)stream), "tcfft_exec_many");
  } catch (...) {
    return TCFFT_ERR_INTERNAL;
  }
}

tcfft_status tcfft_fused_wait_failures(unsigned* count) {
  if (!count) return TCFFT_ERR_INVALID_ARG;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return TCFFT_ERR_NO_DEVICE;
  }
  unsigned v = 0;
  if (fused_wait_failures(&v) != hipSuccess) {
    (void)hipGetLastError();
    return TCFFT_ERR_NO_DEVICE;
  }
  *count = v;
  return TCFFT_OK;
}

tcfft_status tcfft_exec_many_static(const tcfft_plan* plans, const void* const* in,
                                    void* const* out, int njobs, void* stream) {
  if (njobs > TCFFT_STATIC_MAX_JOBS) return TCFFT_ERR_INVALID_ARG;
  tcfft_status st = check_many(plans, in, out, njobs);
  if (st || njobs == 0) return st;
  try {
    return logged(exec_many_impl(plans, in, out, njobs, (hipStream_t)stream, true),
                  "tcfft_exec_many_static");
  } catch (...) {
    return TCFFT_ERR_INTERNAL;
  }
}

tcfft_status tcfft_plan_destroy(tcfft_plan plan) {
  free_plan(plan);
  return TCFFT_OK;
}

int tcfft_plan_scale_log2(tcfft_plan plan) { return plan ? plan->spec.scale : -1; }

size_t tcfft_plan_buffer_bytes(tcfft_plan plan) { return plan ? plan->spec.buf_bytes : 0; }

size_t tcfft_plan_input_bytes(tcfft_plan plan) { return plan ? plan->spec.in_bytes : 0; }

size_t tcfft_plan_output_bytes(tcfft_plan plan) { return plan ? plan->spec.out_bytes : 0; }

size_t tcfft_plan_workspace_bytes(tcfft_plan plan) {
  return plan ? plan->spec.ws_bytes + plan->spec.zbuf_bytes : 0;
}

int tcfft_plan_num_launches(tcfft_plan plan) {
  if (!plan) return -1;
  if (plan->spec.d.prec == TCFFT_PREC_FP32_RADIX2) return ilog2(plan->spec.npts);
  if (plan->spec.d.prec == TCFFT_PREC_FP64) return 1;
  return (int)plan->spec.passes.size() + (plan->spec.real_n > 0 && !plan->spec.real_fused ? 1 : 0);
}

int tcfft_plan_describe(tcfft_plan plan, char* buf, size_t len) {
  if (!plan) return -1;
  return copy_out(describe(plan->spec), buf, len);
}

int tcfft_plan_dry_run(int rank, const int64_t* dims, int64_t batch, int dir, int precision,
                       unsigned flags, char* buf, size_t len) {
  if (!dims || rank < 1 || rank > 3) return -(int)TCFFT_ERR_INVALID_ARG;
  Desc d;
  d.rank = rank;
  d.nx = dims[0];
  d.ny = rank >= 2 ? dims[1] : 1;
  d.nz = rank == 3 ? dims[2] : 1;
  d.batch = batch;
  d.dir = dir;
  d.prec = precision;
  d.flags = flags;
  PlanSpec ps;
  tcfft_status st = build_spec(d, Choice{}, &ps);
  if (st) return -(int)st;
  return copy_out(describe(ps), buf, len);
}

int tcfft_tune_candidates(int rank, const int64_t* dims, int64_t batch, int precision, char* buf,
                          size_t len) {
  if (!dims || rank < 1 || rank > 3) return -(int)TCFFT_ERR_INVALID_ARG;
  Desc d;
  d.rank = rank;
  d.nx = dims[0];
  d.ny = rank >= 2 ? dims[1] : 1;
  d.nz = rank == 3 ? dims[2] : 1;
  d.batch = batch;
  d.prec = precision;
  tcfft_status st = validate(d);
  if (st) return -(int)st;
  std::string s = "[";
  bool first = true;
  for (const Choice& c : candidates(d)) {
    PlanSpec ps;
    if (build_spec(d, c, &ps) != TCFFT_OK) continue;
    s += first ? "" : ",";
    first = false;
    s += describe(ps);
  }
  s += "]";
  return copy_out(s, buf, len);
}

int tcfft_tune_cache_size(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return (int)g_tune.size();
}

tcfft_status tcfft_tune_cache_save(const char* path) {
  if (!path) return TCFFT_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return TCFFT_ERR_INVALID_ARG;
  std::fprintf(f, "tcfft-tune 4\n");
  for (const auto& kv : g_tune) {
    const Choice& c = kv.second.first;
    std::fprintf(f, "%s %d %d %d %d %d %d %d %d %d %.3f\n", kv.first.c_str(), c.row_nt, c.cmax,
                 c.nf, c.f[0], c.f[1], c.f[2], c.chunk, c.p2row, c.row_pts, kv.second.second);
  }
  std::fclose(f);
  return TCFFT_OK;
}

tcfft_status tcfft_tune_cache_load(const char* path) {
  if (!path) return TCFFT_ERR_INVALID_ARG;
  FILE* f = std::fopen(path, "r");
  if (!f) return TCFFT_ERR_INVALID_ARG;
  char key[160];
  int ver = 0;
  if (std::fscanf(f, "tcfft-tune %d\n", &ver) != 1 || (ver != 3 && ver != 4)) {
    std::fclose(f);
    return TCFFT_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  while (true) {
    // format 3 has no row_pts field
    Choice c;
    double us = 0;
    const int n = ver == 4 ? std::fscanf(f, "%159s %d %d %d %d %d %d %d %d %d %lf\n", key, &c.row_nt,
                                         &c.cmax, &c.nf, &c.f[0], &c.f[1], &c.f[2], &c.chunk,
                                         &c.p2row, &c.row_pts, &us)
                           : std::fscanf(f, "%159s %d %d %d %d %d %d %d %d %lf\n", key, &c.row_nt,
                                         &c.cmax, &c.nf, &c.f[0], &c.f[1], &c.f[2], &c.chunk,
                                         &c.p2row, &us);
    if (n != (ver == 4 ? 11 : 10)) break;
    if (c.nf < 0 || c.nf > 3 || (c.row_pts != 0 && c.row_pts != 8192 && c.row_pts != 16384))
      continue;
    g_tune[key] = {c, us};
  }
  std::fclose(f);
  return TCFFT_OK;
}

void tcfft_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

const char* tcfft_status_string(tcfft_status s) {
  // a C caller may pass any int: read the value without an enum-typed load
  int v = 0;
  std::memcpy(&v, &s, sizeof v);
  switch (v) {
    case TCFFT_OK: return "ok";
    case TCFFT_ERR_INVALID_ARG: return "invalid argument";
    case TCFFT_ERR_UNSUPPORTED: return "unsupported size or configuration";
    case TCFFT_ERR_NO_DEVICE: return "no gfx950 device";
    case TCFFT_ERR_ALLOC: return "device allocation failed";
    case TCFFT_ERR_LAUNCH: return "kernel launch failed";
    case TCFFT_ERR_INTERNAL: return "internal error";
    case TCFFT_ERR_TIMEOUT: return "timed out in the queue";
    case TCFFT_ERR_CANCELLED: return "cancelled";
  }
  return "unknown status";
}

const char* tcfft_version(void) { return "tcfft-mi355x 0.2"; }

}  // extern "C"
