/*
 * FP64 CPU oracle for the batched complex FFT — TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load this library.  The product path (paper_2104_11471_amd/) never links,
 * imports or calls it, and it shares no code, header or table with that path.
 *
 * What it computes (tcFFT paper, Sec. 2.1):
 *   - Eq. (1), the DFT itself:  X[k] = sum_n x[n] * exp(sign * 2*pi*i * n*k / N),
 *     unnormalised, sign = -1 forward and +1 inverse (the inverse is not stated in
 *     the paper; it is read as the same sum with the opposite sign, so that
 *     inverse(forward(x)) = N * x).
 *   - Eq. (2) applied recursively with N1 = 2: the radix-2 Cooley-Tukey FFT,
 *     X[k] = X_0[k mod N/2] + W_N^k * X_1[k mod N/2], where X_m is the DFT of the
 *     subsequence x_m[n] = x[2n + m].
 *   - Sec. 3.1 (batched and 2D): a 2D transform of a row-major nx-by-ny array is
 *     ny-point transforms of the nx rows followed by nx-point transforms of the ny
 *     (strided) columns.
 *
 * Data: interleaved complex doubles (re, im), transform b of a batch starts at
 * element b*N.  All functions return 0 on success, -1 on a bad argument.
 *
 * Plain C, no intrinsics; OpenMP only distributes independent transforms (or
 * independent butterflies of one stage when the batch is smaller than the
 * thread count).  Twiddles come from libm cos/sin of 2*pi*j/len for every j
 * (never a recurrence), so the error stays O(u log N).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double TWO_PI = 6.283185307179586476925286766559;

static int is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

static int ilog2(int64_t n) {
  int l = 0;
  while (((int64_t)1 << l) < n) ++l;
  return l;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/*
 * Eq. (1) written out, O(N^2).  The exponent n*k is reduced modulo N in
 * integers before it is turned into an angle, so the angle is exact up to the
 * final FP64 multiply and the cos/sin evaluation.
 */
int oracle_dft_direct(const double* x, double* X, int64_t n, int sign) {
  if (n <= 0 || (sign != 1 && sign != -1) || !x || !X) return -1;
  for (int64_t k = 0; k < n; ++k) {
    double sr = 0.0, si = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      int64_t m = (j * k) % n;
      double ang = (double)sign * TWO_PI * (double)m / (double)n;
      double c = cos(ang), s = sin(ang);
      double xr = x[2 * j], xi = x[2 * j + 1];
      sr += xr * c - xi * s;
      si += xr * s + xi * c;
    }
    X[2 * k] = sr;
    X[2 * k + 1] = si;
  }
  return 0;
}

/* Bit-reversal permutation: after it, slot i holds x[bitrev(i)]. */
static void bit_reverse(double* a, int64_t n) {
  int lg = ilog2(n);
  for (int64_t i = 0; i < n; ++i) {
    int64_t r = 0;
    for (int b = 0; b < lg; ++b)
      if (i & ((int64_t)1 << b)) r |= (int64_t)1 << (lg - 1 - b);
    if (r > i) {
      double tr = a[2 * i], ti = a[2 * i + 1];
      a[2 * i] = a[2 * r];
      a[2 * i + 1] = a[2 * r + 1];
      a[2 * r] = tr;
      a[2 * r + 1] = ti;
    }
  }
}

/*
 * One stage of Eq. (2) with N1 = 2 on every block of length len:
 * for j < len/2, with w = W_len^j = exp(sign*2*pi*i*j/len),
 *   a[s+j]         <- a[s+j] + w * a[s+j+len/2]
 *   a[s+j+len/2]   <- a[s+j] - w * a[s+j+len/2]
 * The first half of a block holds X_0 (even samples), the second X_1 (odd
 * samples) thanks to the bit-reversed ordering.
 */
static void radix2_stage(double* a, int64_t n, int64_t len, const double* w,
                         int parallel) {
  int64_t half = len / 2;
  int64_t nbf = n / 2;
#pragma omp parallel for schedule(static) if (parallel)
  for (int64_t b = 0; b < nbf; ++b) {
    int64_t j = b % half;
    int64_t s = (b / half) * len;
    double ur = a[2 * (s + j)], ui = a[2 * (s + j) + 1];
    double vr0 = a[2 * (s + j + half)], vi0 = a[2 * (s + j + half) + 1];
    double wr = w[2 * j], wi = w[2 * j + 1];
    double vr = vr0 * wr - vi0 * wi;
    double vi = vr0 * wi + vi0 * wr;
    a[2 * (s + j)] = ur + vr;
    a[2 * (s + j) + 1] = ui + vi;
    a[2 * (s + j + half)] = ur - vr;
    a[2 * (s + j + half) + 1] = ui - vi;
  }
}

static void stage_twiddles(double* w, int64_t len, int sign, int parallel) {
  int64_t half = len / 2;
#pragma omp parallel for schedule(static) if (parallel)
  for (int64_t j = 0; j < half; ++j) {
    double ang = (double)sign * TWO_PI * (double)j / (double)len;
    w[2 * j] = cos(ang);
    w[2 * j + 1] = sin(ang);
  }
}

/* In-place radix-2 DIT FFT of one length-n sequence. */
static void fft_one(double* a, int64_t n, int sign, double* w, int parallel) {
  if (n == 1) return;
  bit_reverse(a, n);
  for (int64_t len = 2; len <= n; len <<= 1) {
    stage_twiddles(w, len, sign, parallel && len >= 4096);
    radix2_stage(a, n, len, w, parallel);
  }
}

/*
 * Batched 1D transform: batch sequences of n points, out-of-place (x may equal
 * X).  nthreads <= 0 means the OpenMP default.
 */
int oracle_fft(const double* x, double* X, int64_t n, int64_t batch, int sign,
               int nthreads) {
  if (!is_pow2(n) || batch <= 0 || (sign != 1 && sign != -1) || !x || !X)
    return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  int nt = omp_get_max_threads();
#else
  int nt = 1;
#endif
  if (x != X) memcpy(X, x, (size_t)(2 * n * batch) * sizeof(double));
  if (batch >= nt) {
#pragma omp parallel
    {
      double* w = (double*)malloc((size_t)n * sizeof(double));
#pragma omp for schedule(dynamic, 1)
      for (int64_t b = 0; b < batch; ++b) fft_one(X + 2 * n * b, n, sign, w, 0);
      free(w);
    }
  } else {
    double* w = (double*)malloc((size_t)n * sizeof(double));
    for (int64_t b = 0; b < batch; ++b) fft_one(X + 2 * n * b, n, sign, w, 1);
    free(w);
  }
  return 0;
}

/*
 * Batched 2D transform of row-major nx-by-ny arrays (ny contiguous): the ny-point
 * transform of each row, then the nx-point transform of each column.
 */
int oracle_fft2(const double* x, double* X, int64_t nx, int64_t ny, int64_t batch,
                int sign, int nthreads) {
  if (!is_pow2(nx) || !is_pow2(ny) || batch <= 0 || (sign != 1 && sign != -1) ||
      !x || !X)
    return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  int rc = oracle_fft(x, X, ny, nx * batch, sign, nthreads);
  if (rc) return rc;
  int64_t ncols = ny * batch;
#pragma omp parallel
  {
    double* col = (double*)malloc((size_t)(2 * nx) * sizeof(double));
    double* w = (double*)malloc((size_t)nx * sizeof(double));
#pragma omp for schedule(dynamic, 4)
    for (int64_t c = 0; c < ncols; ++c) {
      int64_t b = c / ny, y = c % ny;
      double* base = X + 2 * (b * nx * ny + y);
      for (int64_t i = 0; i < nx; ++i) {
        col[2 * i] = base[2 * i * ny];
        col[2 * i + 1] = base[2 * i * ny + 1];
      }
      fft_one(col, nx, sign, w, 0);
      for (int64_t i = 0; i < nx; ++i) {
        base[2 * i * ny] = col[2 * i];
        base[2 * i * ny + 1] = col[2 * i + 1];
      }
    }
    free(col);
    free(w);
  }
  return 0;
}

/*
 * One merging process, Eq. (3):  X_out = F_{N1} . (T_{N1 N2} (.) X_in).
 * X_in is N1-by-N2 (row m holds X_m, the DFT of x_m[n] = x[n*N1 + m]);
 * (T)_{m,k} = W_N^{m k}; (F)_{l,m} = W_{N1}^{l m}; X_out[l][k] = X[l*N2 + k].
 * Written as the two products literally, to pin the matrix form against Eq. (2).
 */
int oracle_merge(const double* Xin, double* Xout, int64_t n1, int64_t n2, int sign) {
  if (n1 <= 0 || n2 <= 0 || (sign != 1 && sign != -1) || !Xin || !Xout) return -1;
  int64_t n = n1 * n2;
  double* t = (double*)malloc((size_t)(2 * n) * sizeof(double));
  for (int64_t m = 0; m < n1; ++m)
    for (int64_t k = 0; k < n2; ++k) {
      int64_t e = (m * k) % n;
      double ang = (double)sign * TWO_PI * (double)e / (double)n;
      double c = cos(ang), s = sin(ang);
      double xr = Xin[2 * (m * n2 + k)], xi = Xin[2 * (m * n2 + k) + 1];
      t[2 * (m * n2 + k)] = xr * c - xi * s;
      t[2 * (m * n2 + k) + 1] = xr * s + xi * c;
    }
  for (int64_t l = 0; l < n1; ++l)
    for (int64_t k = 0; k < n2; ++k) {
      double sr = 0.0, si = 0.0;
      for (int64_t m = 0; m < n1; ++m) {
        int64_t e = (l * m) % n1;
        double ang = (double)sign * TWO_PI * (double)e / (double)n1;
        double c = cos(ang), s = sin(ang);
        double vr = t[2 * (m * n2 + k)], vi = t[2 * (m * n2 + k) + 1];
        sr += c * vr - s * vi;
        si += c * vi + s * vr;
      }
      Xout[2 * (l * n2 + k)] = sr;
      Xout[2 * (l * n2 + k) + 1] = si;
    }
  free(t);
  return 0;
}
