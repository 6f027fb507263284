// Kernel parameter block and launch entry points shared by the device code
// (kernels.hip) and the host runtime (tcfft.cpp).  No torch types anywhere.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tcfft {

// Parameters of one pass.  All element counts/strides are in complex points.
struct KParams {
  const uint32_t* in;      // FP16 complex words (split: hi plane)
  uint32_t* out;
  int64_t in_plane;        // split: offset of the lo plane from `in` (else 0)
  int64_t out_plane;
  int64_t ntrans;          // row kernel: number of transforms; column kernel: number of tiles
  const float2* tw;        // W_L^m, m in [0, L)   (direction folded in)
  const void* fimg;        // radix-16 A-operand images (4 x 64 lanes x 8 halves)
  float r0scale;           // scale of the radix-2/4/8 stage (power of two)
  float sgn;               // -1 forward, +1 inverse
  // column kernel geometry: element (j, c) of a tile at in_base + j*s_in + c
  int64_t s_in, s_out;
  int64_t blocks;          // column blocks per outer block
  int64_t in_outer, out_outer;
  int64_t q, qstride;      // output column base: (i0 / q) * qstride + (i0 % q)
  // extra twiddle W_M^{ci * k} on the pass output, ci = (i0 + c) / xdiv
  const float2* xtw_lo;    // W_M^e, e in [0, 2^xbits)
  const float2* xtw_hi;    // W_M^{e * 2^xbits}, e in [0, M / 2^xbits)
  int32_t xbits;
  uint32_t xmask;          // M - 1
  int64_t xdiv;
  // log2 of blocks, q and xdiv (all powers of two)
  int32_t blocks_log2, q_log2, xdiv_log2;
  float r0scale2;          // plane kernel: scale of the column half's radix-R0 stage
  // column kernel, extra twiddle: global index of the pass's column 0 (a shard
  // of a distributed four-step transform holds columns xoff, xoff + 1, ...)
  int64_t xoff;
  // transposed store in blocks: output k of local column ci lands at
  // (k >> tblk_log2) * tblk_stride + (ci << tblk_log2) + (k & (2^tblk_log2 - 1));
  // tblk_log2 = log2(L) is the plain transposed store (row ci of L outputs)
  int64_t tblk_stride;
  int32_t tblk_log2;
  int32_t pad0;
  // A operands of the matrix-core radix-R0 x radix-16 block (R0 images A_k,
  // 256 h8 each: Yr-hi, Yi-hi, Yr-lo, Yi-lo), pass-specific
  const void* fimg2;
  // A operands of the radix-16 LDS stage of digit stride 16 with its twiddle
  // folded in (16 images A_lo, 256 h8 each), pass-specific
  const void* fimg3;
};

// The same struct is read by host code (x86-64) and, in grouped launches, by
// device code from a table in device memory: both ABIs lay it out alike
// (8-byte pointers and int64_t, 4-byte float/int32, natural alignment).
static_assert(sizeof(KParams) == 208, "KParams layout changed: host and device must agree");

// Kernel variants.  `kind` selects the family, the rest are the template
// parameters of that family (see kernels.hip).
enum KernelKind { K_ROW = 0, K_COL = 1, K_BIG = 2, K_PLANE = 3 };

struct KernelKey {
  int kind;    // KernelKind
  int L;       // transform length handled in LDS
  int R0;      // 1, 2, 4 or 8: radix of the vector-ALU stage
  int C;       // column kernel: adjacent columns per workgroup (0 for row); plane: ny
  int NT;      // threads per workgroup
  int split;   // 0 FP16, 1 split hi+lo
  int xtw;     // column kernel: apply the extra inter-pass twiddle
  int tstore;  // column kernel: transposed store (row of L contiguous outputs)
  int real = 0;  // row kernel: 1 real forward (spectrum epilogue), 2 real inverse (prologue)
};

// Header of one grouped launch, in device memory: job j of the group owns
// workgroups [prefix[j], prefix[j+1]) and is described by jobs[j].
struct GroupHdr {
  const KParams* jobs;
  const int64_t* prefix;  // njobs + 1 entries
  int64_t njobs;
  int64_t reserved;
};

// Fused launches of mixed batches (k_fused.hip).  A launch's passes form a run
// of segments, one per (job, pass), in the order (pass level, job); segment s
// owns tile indices [start, start + tiles) and runs fused variant `var` with
// descriptor kps[kp]; it may start a tile only once segment `dep` (the same
// job's previous pass, or -1) has finished all its tiles; only segments that
// are waited on publish and count their tiles.
struct FusedSeg {
  int64_t start;
  int64_t tiles;
  int32_t var;
  int32_t dep;
  int32_t kp;
  int32_t waited;  // 1: a later segment of the launch waits on this one
};
static_assert(sizeof(FusedSeg) == 32, "FusedSeg layout");

// Header of one fused launch, in device memory.  ctr[0] is the queue head,
// ctr[1] the wait-failure flag, ctr[2 + s] the finished tiles of segment s; the
// host uploads them as zeros with the tables.  lds_slot: LDS word index (past
// the largest variant's LDS) used to broadcast the dequeued tile.
struct FusedHdr {
  const KParams* kps;
  const FusedSeg* segs;
  const int32_t* starts;  // segs[s].start (compact copy for the search)
  int* ctr;
  int64_t nsegs;
  int64_t total;
  int64_t lds_slot;
  int64_t wait_ticks;  // bound of one dependency wait, wall-clock counter ticks
  int64_t ticketed;    // 1: tiles taken from the queue head (dependency waits); 0: tile = blockIdx.x
};

// Fused variant id of `key` in the fused kernels, or -1.
int fused_variant(const KernelKey& key);
// The fused kernel of one precision (FP16 or split).
const void* fused_kernel(bool split);
// Device-wide count of dependency waits that gave up (read with a copy).
hipError_t fused_wait_failures(unsigned* count);

typedef void (*KernelFn)(KParams);
typedef void (*MultiFn)(const GroupHdr*);

struct KernelFns {
  KernelFn single = nullptr;
  MultiFn multi = nullptr;
  bool persistent = false;  // `single` strides over tiles: any grid up to the tile count works
  bool multi_one = false;   // `multi` runs one tile per workgroup: its grid is the tile count
};

// Looks up the compiled variant for `key`; false when it is not compiled.
bool find_kernels(const KernelKey& key, KernelFns* out);
// Per translation unit lookups (row kernels, column kernels by length range).
bool find_row_kernels(const KernelKey& key, KernelFns* out);
bool find_col_kernels_small(const KernelKey& key, KernelFns* out);
bool find_col_kernels_256(const KernelKey& key, KernelFns* out);
bool find_col_kernels_large(const KernelKey& key, KernelFns* out);
bool find_big_kernels(const KernelKey& key, KernelFns* out);
bool find_real_row_kernels(const KernelKey& key, KernelFns* out);
bool find_plane_kernels(const KernelKey& key, KernelFns* out);
// Returns the single-launch kernel for `key`, or nullptr.
KernelFn find_kernel(const KernelKey& key);
// Dynamic LDS bytes the kernel needs.
size_t kernel_lds_bytes(const KernelKey& key);
// Points (complex elements) processed by one workgroup.
int64_t kernel_points_per_wg(const KernelKey& key);

// FP64 matrix-core row pass (k_f64.hip): `batch` transforms of L complex
// doubles (L = 16..4096, a power of two), in -> out (not in place), with the
// FP64 table tw[m] = W_L^m (direction folded in).
hipError_t launch_f64_row(const double2* in, double2* out, int L, int64_t batch,
                          const double2* tw, hipStream_t s);
// tw[m] = exp(sgn * 2 pi i m / modulus), m < count, in FP64.
void launch_gen_twiddles_f64(double2* tw, int64_t count, int64_t modulus, double sgn,
                             hipStream_t s);

// FP32 radix-2 Stockham comparator stage.
void launch_radix2_stage(const float2* in, float2* out, int64_t n, int64_t ns, int64_t batch,
                         const float2* tw, hipStream_t s);

// FP64 table generators (run once per plan on the device).
// tw[m] = exp(sgn * 2 pi i * ((m * mult) mod modulus) / modulus), rounded to FP32.
void launch_gen_twiddles(float2* tw, int64_t count, int64_t modulus, int64_t mult, double sgn,
                         hipStream_t s);
// Radix-16 A-operand images, F scaled by `scale` (a power of two):
// [0] Yr-hi, [1] Yi-hi, [2] Yr-lo, [3] Yi-lo; 64 lanes x 8 halves each.
void launch_gen_fimg(void* img, double sgn, double scale, hipStream_t s);
// A_k = F_16 . diag(W_{16 R}^{k m}) scaled by `scale`, for k = 0..R-1, at
// img + 256 k (h8 units; inverse sgn: slot k' holds k = (R - k') mod R), the
// same four images as launch_gen_fimg.
void launch_gen_fimg_r(void* img, int R, double sgn, double scale, hipStream_t s);
// A_lo = diag(W_{16 P}^{k1 lo}) . F_16 scaled by `scale`, for lo = 0..P-1, at
// img + 256 lo (h8 units), the same four images as launch_gen_fimg.
void launch_gen_fimg_tw(void* img, int P, double sgn, double scale, hipStream_t s);
void launch_fill_pattern(void* p, int64_t nwords, hipStream_t s);

// Real-input transforms around an M-point complex transform (N = 2M reals).
// r2c_post: Z (batch x M words) -> X (batch x (M+1) words), tw[k] = W_N^k, k <= M.
// c2r_pre:  X (batch x (M+1) words) -> Z' (batch x M words), tw[k] = W_N^-k.
// Split precision: hi plane then lo plane of each buffer.
void launch_r2c_post(const void* z, void* x, const float2* tw, int64_t M, int64_t batch,
                     bool split, hipStream_t s);
void launch_c2r_pre(const void* x, void* z, const float2* tw, int64_t M, int64_t batch,
                    bool split, hipStream_t s);

// Allocation-free execution (k_static.hip): the current device's copy of the
// static descriptor scratch array (address taken once per device) and its
// size; a device write of `bytes` (a multiple of 4) from host memory carried
// in kernel arguments, stream-ordered, with no staging allocation.
hipError_t static_scratch(void** out, size_t* bytes);
hipError_t launch_write_words(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace tcfft
