/*
 * FP64 CPU oracle for the complex discrete Fourier transform.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library or its Python
 * binding may include, link, load or call this file; it is used by the test
 * suite, by the smoke check and by the benchmark's CPU-baseline leg.  It shares
 * no source with the GPU path (no headers, tables or helpers in common).
 *
 * What it computes (Zhang, Hu, Yin, Hu, "A GPU Based Memory Optimized Parallel
 * Method For FFT Implementation", Sec. 2.1):
 *   forward (eq. 1):  X(k) = sum_n x(n) W_N^{nk},            k = 0..N-1
 *   inverse (eq. 2):  x(n) = (1/N) sum_k X(k) W_N^{-nk},     n = 0..N-1
 * with W_N = exp(-2*pi*i/N).  The paper never writes W_N out; the forward
 * sign follows the FFTW/CUFFT convention of the libraries it compares
 * against (Sec. 3).  Forward is unscaled; the inverse carries 1/N.
 *
 * How it computes it:
 *   oracle_fft1d   - the serial, one-butterfly-at-a-time Cooley-Tukey method
 *                    the paper calls the previous CPU method (Sec. 2.2):
 *                    iterative radix-2 decimation in time, bit-reversed input
 *                    order, natural output order.  Twiddles come straight
 *                    from cos/sin of the exact integer ratio j/len at every
 *                    stage (no recurrence), so each one carries ~1 ulp of
 *                    FP64 error.
 *   oracle_dft_direct - eq. 1 / eq. 2 evaluated term by term in long double,
 *                    with the exponent n*k reduced mod N first (periodicity,
 *                    eq. 3); used to check oracle_fft1d on small N.
 *   oracle_dft_at  - the same sum for a few selected outputs k of a long
 *                    transform (O(N) each), for checking results the full
 *                    oracle is too slow or too large for.
 *   oracle_fft2d   - 1-D transforms of every row, then of every column
 *                    (rows first, then columns: Sec. 2.3.2).
 *   oracle_fft_many - independent 1-D transforms packed back to back.
 *
 * Data are interleaved complex doubles (re, im), row-major, batch outermost.
 * A transform is applied in place.  OpenMP is used only across independent
 * transforms (or rows/columns); every transform itself is sequential, so the
 * results do not depend on the thread count.
 *
 * Error behaviour: every entry point returns 0 on success, -1 for a null
 * pointer or a non-positive size, -2 for a size that is not a power of two
 * (oracle_dft_direct accepts any N >= 1), -6 if scratch memory cannot be had.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double ORACLE_TWO_PI = 6.283185307179586476925286766559;

static int is_pow2(int64_t n) { return n >= 1 && (n & (n - 1)) == 0; }

static int log2_exact(int64_t n) {
  int m = 0;
  while (((int64_t)1 << m) < n) ++m;
  return m;
}

/* Reverse the low m bits of i. */
static int64_t bit_reverse(int64_t i, int m) {
  int64_t r = 0;
  for (int b = 0; b < m; ++b) {
    r = (r << 1) | (i & 1);
    i >>= 1;
  }
  return r;
}

/*
 * One in-place 1-D transform of x[0..n) (interleaved, element stride
 * `stride` complex values), direction `sign` (-1 forward, +1 inverse), then
 * every element times `scale`.  `w` is scratch for n/2 complex values.
 */
static void fft1d_strided(double *x, int64_t n, int64_t stride, int sign,
                          double scale, double *w) {
  const int m = log2_exact(n);
#define RE(i) x[2 * (i) * stride]
#define IM(i) x[2 * (i) * stride + 1]
  /* Decimation in time needs the input in bit-reversed order. */
  for (int64_t i = 0; i < n; ++i) {
    int64_t r = bit_reverse(i, m);
    if (i < r) {
      double tr = RE(i), ti = IM(i);
      RE(i) = RE(r);
      IM(i) = IM(r);
      RE(r) = tr;
      IM(r) = ti;
    }
  }
  /* Stage s merges pairs of length-len/2 transforms into length-len ones:
   * with u = first half, t = W_len^j * second half, the outputs are u + t
   * and u - t (the radix-2 butterfly). */
  for (int s = 1; s <= m; ++s) {
    const int64_t len = (int64_t)1 << s;
    const int64_t half = len >> 1;
    for (int64_t j = 0; j < half; ++j) {
      const double ang = ORACLE_TWO_PI * (double)j / (double)len;
      w[2 * j] = cos(ang);
      w[2 * j + 1] = (double)sign * sin(ang);
    }
    for (int64_t b = 0; b < n; b += len) {
      for (int64_t j = 0; j < half; ++j) {
        const double wr = w[2 * j], wi = w[2 * j + 1];
        const int64_t p = b + j, q = b + j + half;
        const double tr = wr * RE(q) - wi * IM(q);
        const double ti = wr * IM(q) + wi * RE(q);
        const double ur = RE(p), ui = IM(p);
        RE(p) = ur + tr;
        IM(p) = ui + ti;
        RE(q) = ur - tr;
        IM(q) = ui - ti;
      }
    }
  }
  if (scale != 1.0) {
    for (int64_t i = 0; i < n; ++i) {
      RE(i) *= scale;
      IM(i) *= scale;
    }
  }
#undef RE
#undef IM
}

static int check_dir(int sign) { return sign == -1 || sign == 1; }

/* Default scale of eq. 1 / eq. 2 for the given direction. */
static double default_scale(int64_t n, int sign) {
  return sign > 0 ? 1.0 / (double)n : 1.0;
}

/*
 * batch independent length-n transforms, contiguous, back to back.
 * scale < 0 selects the default of eq. 1 / eq. 2 (1 forward, 1/n inverse);
 * any scale >= 0 is applied as given (scale 1 with sign +1 is the adjoint of
 * the forward transform).
 */
int oracle_fft1d(double *x, int64_t n, int64_t batch, int sign, double scale) {
  if (!x || n < 1 || batch < 1 || !check_dir(sign)) return -1;
  if (!is_pow2(n)) return -2;
  const double sc = scale < 0 ? default_scale(n, sign) : scale;
  int fail = 0;
#pragma omp parallel
  {
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 1 ? n : 2));
    if (!w) {
#pragma omp atomic write
      fail = 1;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t b = 0; b < batch; ++b)
        fft1d_strided(x + 2 * b * n, n, 1, sign, sc, w);
    }
    free(w);
  }
  return fail ? -6 : 0;
}

/*
 * batch independent rows x cols 2-D transforms: every row (length cols),
 * then every column (length rows).  scale as for oracle_fft1d, with the
 * default 1/(rows*cols) for the inverse.
 */
int oracle_fft2d(double *x, int64_t rows, int64_t cols, int64_t batch,
                 int sign, double scale) {
  if (!x || rows < 1 || cols < 1 || batch < 1 || !check_dir(sign)) return -1;
  if (!is_pow2(rows) || !is_pow2(cols)) return -2;
  const double sc = scale < 0 ? default_scale(rows * cols, sign) : scale;
  const int64_t big = rows > cols ? rows : cols;
  int fail = 0;
  for (int64_t b = 0; b < batch; ++b) {
    double *img = x + 2 * b * rows * cols;
#pragma omp parallel
    {
      double *w = (double *)malloc(sizeof(double) * (size_t)(big > 1 ? big : 2));
      if (!w) {
#pragma omp atomic write
        fail = 1;
      } else {
#pragma omp for schedule(static)
        for (int64_t r = 0; r < rows; ++r)
          fft1d_strided(img + 2 * r * cols, cols, 1, sign, 1.0, w);
#pragma omp for schedule(static)
        for (int64_t c = 0; c < cols; ++c)
          fft1d_strided(img + 2 * c, rows, cols, sign, sc, w);
      }
      free(w);
    }
  }
  return fail ? -6 : 0;
}

/*
 * count independent 1-D transforms of lengths sizes[0..count) packed back to
 * back in that order.  scale < 0: the default per transform (1/sizes[i] for
 * the inverse); otherwise the given scale for every transform.
 */
int oracle_fft_many(double *x, const int64_t *sizes, int64_t count, int sign,
                    double scale) {
  if (!x || !sizes || count < 1 || !check_dir(sign)) return -1;
  int64_t big = 1;
  for (int64_t i = 0; i < count; ++i) {
    if (sizes[i] < 1) return -1;
    if (!is_pow2(sizes[i])) return -2;
    if (sizes[i] > big) big = sizes[i];
  }
  int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)count);
  if (!off) return -6;
  int64_t acc = 0;
  for (int64_t i = 0; i < count; ++i) {
    off[i] = acc;
    acc += sizes[i];
  }
  int fail = 0;
#pragma omp parallel
  {
    double *w = (double *)malloc(sizeof(double) * (size_t)(big > 1 ? big : 2));
    if (!w) {
#pragma omp atomic write
      fail = 1;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t i = 0; i < count; ++i) {
        const double sc = scale < 0 ? default_scale(sizes[i], sign) : scale;
        fft1d_strided(x + 2 * off[i], sizes[i], 1, sign, sc, w);
      }
    }
    free(w);
  }
  free(off);
  return fail ? -6 : 0;
}

/*
 * Eq. 1 (sign -1) or eq. 2 (sign +1, with 1/N) term by term, out of place,
 * in long double.  W_N^{nk} is formed from (n*k) mod N (eq. 3), so the angle
 * never grows past 2*pi.  O(N^2); meant for N up to a few thousand.
 */
int oracle_dft_direct(const double *in, double *out, int64_t n, int sign) {
  if (!in || !out || n < 1 || !check_dir(sign)) return -1;
  const long double two_pi = 6.283185307179586476925286766559005768L;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    long double sr = 0.0L, si = 0.0L;
    for (int64_t t = 0; t < n; ++t) {
      const int64_t e = (int64_t)(((unsigned __int128)t * (unsigned __int128)k) %
                                  (unsigned __int128)n);
      const long double ang = two_pi * (long double)e / (long double)n;
      const long double c = cosl(ang), s = (long double)sign * sinl(ang);
      const long double xr = in[2 * t], xi = in[2 * t + 1];
      sr += xr * c - xi * s;
      si += xr * s + xi * c;
    }
    if (sign > 0) {
      sr /= (long double)n;
      si /= (long double)n;
    }
    out[2 * k] = (double)sr;
    out[2 * k + 1] = (double)si;
  }
  return 0;
}

/*
 * Outputs X[ks[i]] of eq. 1 (sign -1) or eq. 2 (sign +1), each
 * sum_t x[t] W_N^{sign * t k}, times `scale` (negative: 1 forward, 1/N
 * inverse), in long double.  The exponent t*k is reduced mod N exactly; with
 * t = a*S + b (S = 2^ceil(log2(N)/2)) the factor W_N^{tk} is the product of
 * W_N^{(a S k) mod N} and W_N^{(b k) mod N}, each from cosl/sinl of an
 * exact ratio, so the sum costs one complex multiply-add per term.  N must
 * be a power of two.
 */
int oracle_dft_at(const double *in, int64_t n, const int64_t *ks, int64_t nk, int sign,
                  double scale, double *out) {
  if (!in || !ks || !out || n < 1 || nk < 0 || !check_dir(sign)) return -1;
  if (!is_pow2(n)) return -2;
  const int m = log2_exact(n);
  const int64_t S = (int64_t)1 << ((m + 1) / 2);
  const int64_t A = n / S < 1 ? 1 : n / S;
  const int64_t Sb = n < S ? n : S;
  const long double two_pi = 6.283185307179586476925286766559005768L;
  const long double sc = scale < 0.0 ? (long double)default_scale(n, sign) : (long double)scale;
  int fail = 0;
#pragma omp parallel
  {
    long double *ta = (long double *)malloc((size_t)A * 2 * sizeof(long double));
    long double *tb = (long double *)malloc((size_t)Sb * 2 * sizeof(long double));
    if (!ta || !tb) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = 0; i < nk; ++i) {
      if (!ta || !tb) continue;
      const int64_t k = ((ks[i] % n) + n) % n;
      for (int64_t a = 0; a < A; ++a) {
        const int64_t e = (int64_t)(((unsigned __int128)(a * Sb) * (unsigned __int128)k) %
                                    (unsigned __int128)n);
        const long double ang = two_pi * (long double)e / (long double)n;
        ta[2 * a] = cosl(ang);
        ta[2 * a + 1] = (long double)sign * sinl(ang);
      }
      for (int64_t b = 0; b < Sb; ++b) {
        const int64_t e = (int64_t)(((unsigned __int128)b * (unsigned __int128)k) % (unsigned __int128)n);
        const long double ang = two_pi * (long double)e / (long double)n;
        tb[2 * b] = cosl(ang);
        tb[2 * b + 1] = (long double)sign * sinl(ang);
      }
      long double sr = 0.0L, si = 0.0L;
      for (int64_t a = 0; a < A; ++a) {
        long double pr = 0.0L, pi = 0.0L;
        const double *xa = in + 2 * a * Sb;
        for (int64_t b = 0; b < Sb; ++b) {
          const long double xr = xa[2 * b], xi = xa[2 * b + 1];
          pr += xr * tb[2 * b] - xi * tb[2 * b + 1];
          pi += xr * tb[2 * b + 1] + xi * tb[2 * b];
        }
        sr += pr * ta[2 * a] - pi * ta[2 * a + 1];
        si += pr * ta[2 * a + 1] + pi * ta[2 * a];
      }
      out[2 * i] = (double)(sr * sc);
      out[2 * i + 1] = (double)(si * sc);
    }
    free(ta);
    free(tb);
  }
  return fail ? -6 : 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Set the OpenMP thread count used by the calls above (n >= 1). */
void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
