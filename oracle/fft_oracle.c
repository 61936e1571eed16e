/*
 * FP64 reference ("oracle") for the complex 2D discrete Fourier transform.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links or calls this
 * file; it exists so that tests and benchmarks can check the GPU kernels against
 * a plain, slow and obviously correct CPU computation. It shares no code,
 * header, table or constant with the HIP implementation.
 *
 * Conventions (the paper never writes the DFT out; these readings are fixed
 * here and pinned by the tests, see the oracle tests):
 *   forward  X[k,l] = sum_{m,n} x[m,n] exp(-2 pi i (k m / M + l n / N))  (unscaled)
 *   inverse  x[m,n] = 1/(M N) sum_{k,l} X[k,l] exp(+2 pi i (k m / M + l n / N))
 * The sign argument below is the sign of the exponent (-1 forward, +1 inverse);
 * scaling is a separate argument so that unscaled adjoints can be formed.
 *
 * Data are interleaved complex (re, im) pairs, row-major [batch][M][N] with the
 * N index contiguous. Inputs are complex64 (promoted exactly to complex128),
 * outputs complex128.
 *
 * Functions:
 *   oracle_fft1d_recursive  radix-2 Cooley-Tukey in its recursive divide-and-
 *                           conquer form (Section 2.2 of the paper).
 *   oracle_fft1d_listing    the iterative radix-2 form of Listing 1 (Section
 *                           2.2): bit-reversal permutation, then log2(n) steps
 *                           whose butterfly span doubles each step (1, 2, 4...),
 *                           twiddles read from a table of n/2 entries.
 *   oracle_dft1d_direct / oracle_dft2d_direct
 *                           the definition itself, O(n^2) / O((MN)^2), with the
 *                           phase reduced exactly in integers.
 *   oracle_fft2d            FFT along every row, then along every column
 *                           (the row/column scheme of Section 5, Fig. 6), using
 *                           the recursive 1D form, OpenMP over rows/columns.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double TWO_PI = 6.283185307179586476925286766559;

static int is_pow2(int64_t n) { return n >= 1 && (n & (n - 1)) == 0; }

static int ilog2(int64_t n) {
  int k = 0;
  while (((int64_t)1 << k) < n) ++k;
  return k;
}

/* w[j] = exp(sign * 2 pi i j / n) for j < n/2, each entry from cos/sin of its
 * own angle (no recurrences, so every entry is correctly rounded-ish in FP64). */
static void fill_twiddles(cplx* w, int64_t n, int sign) {
  for (int64_t j = 0; j < n / 2; ++j) {
    double a = TWO_PI * (double)j / (double)n;
    w[j] = cos(a) + I * ((double)sign * sin(a));
  }
}

/*
 * Recursive radix-2 decimation in time. The length-n transform of the samples
 * x[0], x[s], x[2s], ... is written to out[0..n). The even-indexed samples and
 * the odd-indexed samples are transformed separately (the two halves of out),
 * then combined: X[k] = E[k] + w^k O[k], X[k + n/2] = E[k] - w^k O[k], where
 * w = exp(sign 2 pi i / n). The table w_top holds the twiddles of the top
 * length top_n, so w_n^k = w_top[k * (top_n / n)].
 */
static void rec(const cplx* x, int64_t s, cplx* out, int64_t n, const cplx* w_top, int64_t top_n) {
  if (n == 1) {
    out[0] = x[0];
    return;
  }
  int64_t h = n / 2;
  rec(x, 2 * s, out, h, w_top, top_n);
  rec(x + s, 2 * s, out + h, h, w_top, top_n);
  int64_t step = top_n / n;
  for (int64_t k = 0; k < h; ++k) {
    cplx e = out[k];
    cplx t = w_top[k * step] * out[k + h];
    out[k] = e + t;
    out[k + h] = e - t;
  }
}

/* In-place recursive FFT of n contiguous complex128 values (re, im pairs). */
int oracle_fft1d_recursive(double* data, int64_t n, int sign) {
  if (!data || !is_pow2(n) || (sign != 1 && sign != -1)) return -1;
  if (n == 1) return 0;
  cplx* x = (cplx*)data;
  cplx* w = (cplx*)malloc(sizeof(cplx) * (size_t)(n / 2));
  cplx* tmp = (cplx*)malloc(sizeof(cplx) * (size_t)n);
  if (!w || !tmp) { free(w); free(tmp); return -2; }
  fill_twiddles(w, n, sign);
  rec(x, 1, tmp, n, w, n);
  memcpy(x, tmp, sizeof(cplx) * (size_t)n);
  free(w);
  free(tmp);
  return 0;
}

/* Reverse the lowest `bits` bits of v. */
static int64_t bit_reverse(int64_t v, int bits) {
  int64_t r = 0;
  for (int b = 0; b < bits; ++b) {
    r = (r << 1) | (v & 1);
    v >>= 1;
  }
  return r;
}

/*
 * Iterative radix-2 form of Listing 1, on separate real and imaginary arrays.
 * Reading of the elided values (the listing leaves them as "..."):
 *   number of steps log2(n), the loop counter running 0 .. last = log2(n) - 1;
 *   at step s the second point of a pair sits `span` = 2^s after the first
 *   (1, 2, 4 for the three steps of the 8-point example);
 *   there are 2^s distinct twiddles (the listing's spectra) in step s, and pairs with the
 *   same spectrum repeat every 2^(s+1) points;
 *   the spectrum j uses table entry j << (last - s) of w[q] = W_n^q, q < n/2.
 * Because the butterflies apply the twiddle before the add/subtract with a
 * growing span (decimation in time), natural-order output needs bit-reversed
 * input, so the data are permuted first.
 *
 * oracle_fft1d_listing_steps runs only the steps step_lo .. step_hi and
 * permutes first only if `permute` is nonzero (used to pin the schedule);
 * oracle_fft1d_listing is the whole transform.
 */
int oracle_fft1d_listing_steps(double* re, double* im, int64_t n, int sign, int permute, int step_lo, int step_hi) {
  if (!re || !im || !is_pow2(n) || (sign != 1 && sign != -1)) return -1;
  int bits = ilog2(n);
  if (permute) {
    for (int64_t j = 0; j < n; ++j) {
      int64_t r = bit_reverse(j, bits);
      if (r > j) {
        double t = re[j]; re[j] = re[r]; re[r] = t;
        t = im[j]; im[j] = im[r]; im[r] = t;
      }
    }
  }
  if (n == 1) return 0;
  double* wr = (double*)malloc(sizeof(double) * (size_t)(n / 2));
  double* wi = (double*)malloc(sizeof(double) * (size_t)(n / 2));
  if (!wr || !wi) { free(wr); free(wi); return -2; }
  for (int64_t q = 0; q < n / 2; ++q) {
    double a = TWO_PI * (double)q / (double)n;
    wr[q] = cos(a);
    wi[q] = (double)sign * sin(a);
  }
  int last = bits - 1;
  if (step_lo < 0) step_lo = 0;
  if (step_hi > last) step_hi = last;
  for (int s = step_lo; s <= step_hi; ++s) {
    int64_t span = (int64_t)1 << s;
    int64_t group = span << 1;
    for (int64_t spec = 0; spec < span; ++spec) {
      int64_t q = spec << (last - s);
      double tr = wr[q], ti = wi[q];
      for (int64_t base = 0; base < n; base += group) {
        int64_t a = base + spec, b = a + span;
        double fr = re[b] * tr - im[b] * ti;
        double fi = re[b] * ti + im[b] * tr;
        re[b] = re[a] - fr;
        im[b] = im[a] - fi;
        re[a] = re[a] + fr;
        im[a] = im[a] + fi;
      }
    }
  }
  free(wr);
  free(wi);
  return 0;
}

int oracle_fft1d_listing(double* re, double* im, int64_t n, int sign) {
  return oracle_fft1d_listing_steps(re, im, n, sign, 1, 0, 62);
}

/* Direct evaluation of the 1D definition: out[k] = sum_m x[m] exp(sign 2 pi i k m / n).
 * The phase k*m is reduced modulo n in integers before it becomes an angle. */
int oracle_dft1d_direct(const double* in, double* out, int64_t n, int sign) {
  if (!in || !out || n < 1 || (sign != 1 && sign != -1)) return -1;
  const cplx* x = (const cplx*)in;
  cplx* y = (cplx*)out;
  for (int64_t k = 0; k < n; ++k) {
    cplx acc = 0;
    for (int64_t m = 0; m < n; ++m) {
      int64_t p = (k * m) % n;
      double a = TWO_PI * (double)p / (double)n;
      acc += x[m] * (cos(a) + I * ((double)sign * sin(a)));
    }
    y[k] = acc;
  }
  return 0;
}

/* Direct evaluation of the 2D definition for one M x N grid. The phase
 * k m / M + l n / N is the integer ((k m mod M) N + (l n mod N) M) mod (M N)
 * over M N, so the angle is formed from an exact integer ratio. */
int oracle_dft2d_direct(const double* in, double* out, int64_t M, int64_t N, int sign) {
  if (!in || !out || M < 1 || N < 1 || (sign != 1 && sign != -1)) return -1;
  const cplx* x = (const cplx*)in;
  cplx* y = (cplx*)out;
  int64_t MN = M * N;
  for (int64_t k = 0; k < M; ++k) {
    for (int64_t l = 0; l < N; ++l) {
      cplx acc = 0;
      for (int64_t m = 0; m < M; ++m) {
        for (int64_t n = 0; n < N; ++n) {
          int64_t p = (((k * m) % M) * N + ((l * n) % N) * M) % MN;
          double a = TWO_PI * (double)p / (double)MN;
          acc += x[m * N + n] * (cos(a) + I * ((double)sign * sin(a)));
        }
      }
      y[k * N + l] = acc;
    }
  }
  return 0;
}

#ifdef _OPENMP
/* The process's OpenMP thread count before any call of this file changed it. */
static int default_threads(void) {
  static int n = 0;
  if (n == 0) n = omp_get_max_threads();
  return n;
}
#endif

/*
 * 2D transform of `batch` grids of M x N. complex64 input `in` (may be NULL if
 * `in64` is given instead), complex128 output `out`. Every row gets a length-N
 * transform, then every column a length-M transform; the result is multiplied
 * by `scale` (1 for the forward transform, 1/(M N) for the inverse).
 * `threads` <= 0 uses the OpenMP default of the process (every call sets the
 * count, so an earlier call with a small count does not stick).
 */
int oracle_fft2d(const float* in, const double* in64, double* out, int64_t batch, int64_t M, int64_t N,
                 int sign, double scale, int threads) {
  if ((!in && !in64) || !out || batch < 0 || !is_pow2(M) || !is_pow2(N) || (sign != 1 && sign != -1)) return -1;
#ifdef _OPENMP
  const int all = default_threads();  /* captured before the first change */
  omp_set_num_threads(threads > 0 ? threads : all);
#else
  (void)threads;
#endif
  int64_t P = M * N;
  cplx* y = (cplx*)out;
  for (int64_t i = 0; i < 2 * batch * P; ++i) out[i] = in ? (double)in[i] : in64[i];
  cplx* wN = (cplx*)malloc(sizeof(cplx) * (size_t)(N / 2 + 1));
  cplx* wM = (cplx*)malloc(sizeof(cplx) * (size_t)(M / 2 + 1));
  if (!wN || !wM) { free(wN); free(wM); return -2; }
  fill_twiddles(wN, N, sign);
  fill_twiddles(wM, M, sign);
  int status = 0;
  for (int64_t b = 0; b < batch; ++b) {
    cplx* g = y + b * P;
    /* rows */
#pragma omp parallel
    {
      cplx* tmp = (cplx*)malloc(sizeof(cplx) * (size_t)N);
      if (!tmp) {
#pragma omp atomic write
        status = -2;
      } else {
#pragma omp for schedule(static)
        for (int64_t r = 0; r < M; ++r) {
          if (N > 1) {
            rec(g + r * N, 1, tmp, N, wN, N);
            memcpy(g + r * N, tmp, sizeof(cplx) * (size_t)N);
          }
        }
        free(tmp);
      }
    }
    /* columns: gather each column, transform it, scatter it back */
#pragma omp parallel
    {
      cplx* col = (cplx*)malloc(sizeof(cplx) * (size_t)M);
      cplx* tmp = (cplx*)malloc(sizeof(cplx) * (size_t)M);
      if (!col || !tmp) {
#pragma omp atomic write
        status = -2;
      } else {
#pragma omp for schedule(static)
        for (int64_t c = 0; c < N; ++c) {
          if (M > 1) {
            for (int64_t r = 0; r < M; ++r) col[r] = g[r * N + c];
            rec(col, 1, tmp, M, wM, M);
            for (int64_t r = 0; r < M; ++r) g[r * N + c] = tmp[r];
          }
        }
      }
      free(col);
      free(tmp);
    }
    if (scale != 1.0)
      for (int64_t i = 0; i < P; ++i) g[i] *= scale;
  }
  free(wN);
  free(wM);
  return status;
}

/* Number of OpenMP threads a parallel region uses by default (1 without OpenMP). */
int oracle_max_threads(void) {
#ifdef _OPENMP
  return default_threads();
#else
  return 1;
#endif
}
