/*
 * tcfft.h -- C ABI of the MI355X (gfx950) matrix-core FP16 FFT library
 * (libtcfft.so).  Plain C: no HIP or torch types in any signature; streams are
 * passed as `void*` holding a hipStream_t (NULL = the default stream).
 *
 * Method: tcFFT (Li, Cheng, Lin, arXiv 2104.11471).  A transform is a chain of
 * merging processes X_out = F_N1 . (T (.) X_in) (Sec. 2.1, Eq. 3) with
 * radix-16 DFT-matrix products on the matrix cores and radix-2/4/8 on the
 * vector ALU (Sec. 3.1), grouped into passes that exchange data through LDS
 * inside a pass and through HBM between passes (Sec. 3.2), with coalesced
 * strided access (Sec. 4.2).
 *
 * What is computed (Sec. 2.1, Eq. 1): for every transform b of the batch,
 *     Y_b[k] = 2^-S * sum_n x_b[n] * exp(dir * 2*pi*i * n*k / N)
 * with dir = TCFFT_FORWARD (-1) or TCFFT_INVERSE (+1), unnormalised except for
 * the exact power-of-two output scale 2^-S reported by tcfft_plan_scale_log2().
 * 2D transforms (Sec. 3.1) use the separable sum over a row-major nx-by-ny
 * array whose second dimension (ny) is contiguous.
 *
 * Data layouts (all device memory, caller-owned, 16-byte aligned):
 *   TCFFT_PREC_FP16        interleaved complex FP16 (re, im), 4 B per point;
 *                          1D element (b, n) at b*N + n, 2D (b, x, y) at
 *                          (b*nx + x)*ny + y.
 *   TCFFT_PREC_SPLIT_FP16  two such planes in one buffer: hi plane of B*N
 *                          points, then lo plane of B*N points; the value is
 *                          hi + 2^-11 * lo.
 *   TCFFT_PREC_FP32_RADIX2 interleaved complex FP32 (the plain radix-2
 *                          comparator path), 8 B per point.
 * Output is in natural order, in the same layout as the input.  in == out is
 * allowed (in-place).
 *
 * Errors: every entry point returns a status code; nothing aborts or prints.
 * Kernel faults surface asynchronously at the caller's next synchronisation.
 */
#ifndef TCFFT_H_
#define TCFFT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tcfft_plan_s* tcfft_plan; /* opaque, owned by the library */

typedef enum {
  TCFFT_OK = 0,
  TCFFT_ERR_INVALID_ARG = 1, /* null/misaligned pointer, batch <= 0, bad dir/precision */
  TCFFT_ERR_UNSUPPORTED = 2, /* size outside the supported set (see tcfft_plan_create) */
  TCFFT_ERR_NO_DEVICE = 3,   /* no gfx950 device visible */
  TCFFT_ERR_ALLOC = 4,       /* device allocation failed */
  TCFFT_ERR_LAUNCH = 5,      /* a kernel launch was rejected by the runtime */
  TCFFT_ERR_INTERNAL = 6
} tcfft_status;

#define TCFFT_FORWARD (-1)
#define TCFFT_INVERSE (+1)

enum {
  TCFFT_PREC_FP16 = 0,        /* FP16 storage, FP16 matrix-core products, FP32 accumulation */
  TCFFT_PREC_SPLIT_FP16 = 1,  /* hi+lo FP16 pairs, compensated products (precision recovery) */
  TCFFT_PREC_FP32_RADIX2 = 2  /* plain FP32 radix-2 Stockham, one launch per stage (comparator) */
};

enum {
  TCFFT_FLAG_NO_SCALE = 1u, /* S = 0: literally unnormalised (may overflow FP16 for large N) */
  TCFFT_FLAG_NO_GRAPH = 2u  /* reserved: never capture the pass sequence in a HIP graph */
};

/*
 * Creates a plan (Sec. 3.1 and Fig. 1: the plan picks the merging kernels once,
 * the execution function runs them many times).
 *   out        receives the plan handle (set to NULL on failure)
 *   rank       1 or 2
 *   dims       rank values: {N} or {nx, ny}; powers of two.  1D: 16 <= N <= 2^27.
 *              2D: 16 <= nx <= 2048, 16 <= ny <= 16384.
 *   batch      number of transforms, >= 1 (batch * points <= 2^31 per plan)
 *   dir        TCFFT_FORWARD or TCFFT_INVERSE
 *   precision  TCFFT_PREC_*
 *   flags      TCFFT_FLAG_* bit set
 * Allocates the plan's device tables (DFT-matrix operands, twiddles generated
 * in FP64 on the device) and its workspace on the current device; the call
 * synchronises the current device before returning.
 * Errors: INVALID_ARG, UNSUPPORTED, NO_DEVICE, ALLOC, LAUNCH.
 */
tcfft_status tcfft_plan_create(tcfft_plan* out, int rank, const int64_t* dims, int64_t batch,
                               int dir, int precision, unsigned flags);

/* The paper's plan functions (Sec. 3.1): forward FP16 plans of nx points
 * (1D) or nx-by-ny arrays (2D, ny contiguous). */
tcfft_status tcfft_plan_1d(tcfft_plan* out, int64_t nx, int64_t batch);
tcfft_status tcfft_plan_2d(tcfft_plan* out, int64_t nx, int64_t ny, int64_t batch);

/*
 * Executes a plan (the "execution function" of Fig. 1): reads `in`, writes
 * `out` (device pointers, each tcfft_plan_buffer_bytes() long, 16-byte
 * aligned; in == out allowed), enqueued asynchronously on `stream` (a
 * hipStream_t or NULL).  One exec per plan may be in flight at a time (the
 * plan's workspace is shared).
 * Errors: INVALID_ARG (null plan/pointer, misalignment), LAUNCH.
 */
tcfft_status tcfft_exec(tcfft_plan plan, const void* in, void* out, void* stream);

/*
 * Executes several plans in order on one stream: job j runs plans[j] on
 * (in[j], out[j]).  Each job's result equals tcfft_exec of that job alone.
 * Errors: as tcfft_exec; INVALID_ARG for njobs < 0 or null arrays.
 */
tcfft_status tcfft_exec_many(const tcfft_plan* plans, const void* const* in, void* const* out,
                             int njobs, void* stream);

/* Releases the plan and its device memory (synchronises the device first).
 * NULL is accepted.  Errors: none besides INTERNAL. */
tcfft_status tcfft_plan_destroy(tcfft_plan plan);

/* S such that out = DFT(in) * 2^-S (0 for NO_SCALE and the FP32 path); -1 for NULL. */
int tcfft_plan_scale_log2(tcfft_plan plan);

/* Bytes of one input (= output) buffer of the plan; 0 for NULL. */
size_t tcfft_plan_buffer_bytes(tcfft_plan plan);

/* Device workspace bytes held by the plan; 0 for NULL. */
size_t tcfft_plan_workspace_bytes(tcfft_plan plan);

/* Number of kernel launches of one exec; -1 for NULL. */
int tcfft_plan_num_launches(tcfft_plan plan);

/*
 * Writes a JSON description of the plan (passes, radices, kernels, scale) into
 * buf (NUL-terminated, truncated to len).  Returns the length the full text
 * needs (excluding the NUL), or -1 for NULL.
 */
int tcfft_plan_describe(tcfft_plan plan, char* buf, size_t len);

/*
 * Runs only the planner (no device needed) and writes the JSON description
 * the same arguments would produce.  Returns the needed length, or -(status)
 * when the arguments are rejected.
 */
int tcfft_plan_dry_run(int rank, const int64_t* dims, int64_t batch, int dir, int precision,
                       unsigned flags, char* buf, size_t len);

/* Static text for a status code. */
const char* tcfft_status_string(tcfft_status s);

/* Library version string. */
const char* tcfft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TCFFT_H_ */
