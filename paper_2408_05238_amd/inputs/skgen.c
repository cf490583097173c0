/*
 * Seeded synthetic inputs for the skew-symmetric LTL^T / Pfaffian library.
 *
 * This module only draws random numbers.  It holds none of the factorization's
 * arithmetic and is shared by the GPU path's benchmarks/tests and by the CPU
 * oracle's tests, which is the one thing the two sides are allowed to share.
 *
 * Determinism: every value is a pure function of (seed, stream, counter) and is
 * computed with IEEE-754 +,-,*,/ and sqrt only (no libm transcendental calls,
 * whose last bits differ between C libraries and CPU dispatch paths).  The file
 * must be compiled with -ffp-contract=off and without -ffast-math; the result is
 * then bit-identical on every x86-64 host.
 *
 *   uniform bits : SplitMix64 in counter mode, out(key, i) = mix64(key + (i+1)*G)
 *                  with G = 0x9E3779B97F4A7C15 and mix64 the SplitMix64 finalizer.
 *   N(0,1) draw  : Marsaglia's polar method, one normal per accepted pair; the
 *                  attempt t of counter c uses uniforms out(key, 2(64c+t)) and
 *                  out(key, 2(64c+t)+1); at most 64 attempts (failure probability
 *                  0.2146^64 ~ 1e-43, then 0.0 is returned).
 *   log          : ln x = e ln2 + 2 atanh((m-1)/(m+1)), m in [sqrt(1/2), sqrt(2)),
 *                  atanh by its Taylor series to 13 terms (|f| <= 0.1716).
 */
#include <stdint.h>
#include <math.h>

#define SK_GAMMA 0x9E3779B97F4A7C15ULL

uint64_t skgen_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Key of an independent stream: stream ids are documented with the workloads. */
uint64_t skgen_key(uint64_t seed, uint64_t stream) {
  return skgen_mix64(seed * SK_GAMMA + skgen_mix64(stream + 0x632BE59BD9B4E019ULL));
}

static inline uint64_t sk_out(uint64_t key, uint64_t i) {
  return skgen_mix64(key + (i + 1) * SK_GAMMA);
}

/* Uniform on the open interval (-1, 1), symmetric, never 0: (2s+1-2^52)/2^52. */
static inline double sk_sym_uniform(uint64_t x) {
  int64_t s = (int64_t)(x >> 12);
  int64_t k = 2 * s + 1 - ((int64_t)1 << 52);
  return (double)k * 0x1p-52;
}

/* Uniform on [0, 1) with 53 random bits. */
double skgen_uniform(uint64_t key, uint64_t ctr) {
  return (double)(sk_out(key, ctr) >> 11) * 0x1p-53;
}

static double sk_log(double x) {
  int e;
  double m = frexp(x, &e);                 /* exact: x = m 2^e, m in [0.5, 1) */
  if (m < 0.70710678118654752440) {
    m = m * 2.0;
    e = e - 1;
  }
  double f = (m - 1.0) / (m + 1.0);
  double t = f * f;
  double p = 0.0;
  for (int k = 12; k >= 0; --k) p = p * t + 1.0 / (double)(2 * k + 1);
  const double ln2_hi = 6.93147180369123816490e-01; /* 0x3FE62E42FEE00000 */
  const double ln2_lo = 1.90821492927058770002e-10;
  double de = (double)e;
  return de * ln2_hi + (de * ln2_lo + 2.0 * f * p);
}

double skgen_log(double x) { return sk_log(x); }

double skgen_gauss(uint64_t key, uint64_t ctr) {
  for (uint64_t t = 0; t < 64; ++t) {
    uint64_t base = 2 * (64 * ctr + t);
    double v1 = sk_sym_uniform(sk_out(key, base));
    double v2 = sk_sym_uniform(sk_out(key, base + 1));
    double s = v1 * v1 + v2 * v2;
    if (s < 1.0 && s > 0.0) return v1 * sqrt(-2.0 * sk_log(s) / s);
  }
  return 0.0;
}

/* Dense skew-symmetric Gaussian matrix, column-major, both triangles written:
 * for i < j, A[i,j] = z(i,j) ~ N(0,1) with counter c = i*n - i(i+1)/2 + (j-i-1)
 * (row-major order over the strict upper triangle), A[j,i] = -A[i,j], A[i,i] = 0. */
void skgen_skew_gaussian(int64_t n, double* A, int64_t lda, uint64_t seed, uint64_t stream) {
  uint64_t key = skgen_key(seed, stream);
  for (int64_t j = 0; j < n; ++j) {
    for (int64_t i = 0; i < j; ++i) {
      uint64_t c = (uint64_t)(i * n - i * (i + 1) / 2 + (j - i - 1));
      double z = skgen_gauss(key, c);
      A[i + j * lda] = z;
      A[j + i * lda] = -z;
    }
    A[j + j * lda] = 0.0;
  }
}

/* Same draws, only the columns [j0, j1) written (for threaded fills). */
void skgen_skew_gaussian_cols(int64_t n, double* A, int64_t lda, uint64_t seed, uint64_t stream,
                              int64_t j0, int64_t j1) {
  uint64_t key = skgen_key(seed, stream);
  for (int64_t j = j0; j < j1; ++j) {
    for (int64_t i = 0; i < n; ++i) {
      double v;
      if (i < j) {
        uint64_t c = (uint64_t)(i * n - i * (i + 1) / 2 + (j - i - 1));
        v = skgen_gauss(key, c);
      } else if (i > j) {
        uint64_t c = (uint64_t)(j * n - j * (j + 1) / 2 + (i - j - 1));
        v = -skgen_gauss(key, c);
      } else {
        v = 0.0;
      }
      A[i + j * lda] = v;
    }
  }
}

/* Dense Gaussian rows x cols block (right-hand sides), counter c = i + j*rows. */
void skgen_gaussian(int64_t rows, int64_t cols, double* B, int64_t ldb, uint64_t seed, uint64_t stream) {
  uint64_t key = skgen_key(seed, stream);
  for (int64_t j = 0; j < cols; ++j)
    for (int64_t i = 0; i < rows; ++i) B[i + j * ldb] = skgen_gauss(key, (uint64_t)(i + j * rows));
}

/* Even sizes uniform on {nmin, nmin+2, ..., nmax} (nmin, nmax even). */
void skgen_even_sizes(int64_t count, int64_t nmin, int64_t nmax, int64_t* out, uint64_t seed, uint64_t stream) {
  uint64_t key = skgen_key(seed, stream);
  uint64_t nvals = (uint64_t)((nmax - nmin) / 2 + 1);
  for (int64_t b = 0; b < count; ++b) {
    uint64_t x = sk_out(key, (uint64_t)b);
    /* multiply-high maps 64 random bits to [0, nvals) without modulo bias beyond 2^-64 */
    uint64_t idx = (uint64_t)(((unsigned __int128)x * nvals) >> 64);
    out[b] = nmin + 2 * (int64_t)idx;
  }
}
