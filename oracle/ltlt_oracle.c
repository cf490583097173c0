/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct FP64 reference for the skew-symmetric
 * LTL^T factorization with partial pivoting (Gaussian congruence elimination in
 * the manner of Parlett and Reid, 1970, specialised to skew-symmetric A), the
 * Pfaffian that follows from it, and the solve with the factors.  Only tests,
 * the smoke check and the benchmark's CPU-baseline leg may load this library;
 * the GPU product path never does.  It shares no code with the GPU path.
 *
 * Storage (column-major, lda >= n, only the strict lower triangle is read):
 *   P A P^T = L T L^T, L unit lower triangular with L[:,0] = e_0,
 *   T skew tridiagonal with T(k+1,k) = T[k] and T(k,k+1) = -T[k].
 *   On exit L[i,j] (i > j >= 1) sits at A[i, j-1]; A[k+1,k] = T[k];
 *   ipiv[0] = 0 and ipiv[j] = p >= j records the interchange of rows/columns
 *   j and p made at elimination step j-1.
 *
 * Elimination step k (k = 0 .. n-3), exactly as the definition reads:
 *   1. p = first index i >= k+1 maximising |A[i,k]| (ties -> lowest index);
 *   2. symmetric interchange of rows/columns k+1 and p;
 *   3. alpha = A[k+1,k] = T[k]; l_i = A[i,k]/alpha (l = 0 if alpha == 0);
 *   4. congruence with I - l e_{k+1}^T, i.e. for i > j >= k+2
 *        A[i,j] := (A[i,j] + l_i v_j) - v_i l_j,   v = A[k+2:, k+1].
 * then T[n-2] = A[n-1,n-2].  One full rank-2 update per column: 2n^3/3 flops.
 * Compile with -ffp-contract=off so every product and sum is rounded as written.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ENONFINITE (-103)
#define ORC_EARG (-1)

#define AT(i, j) A[(i) + (int64_t)(j) * lda]

typedef struct {
  double* A;
  int64_t lda, n;
  int nthreads;
  int64_t nsteps;
  int32_t* ipiv;
  double* T;
  double* gap;
  double* M;      /* optional: running sums of |terms| per entry (same layout, ldm) */
  int64_t ldm;
  int status;
  pthread_barrier_t bar;
  int64_t k;      /* current step, published by thread 0 */
  int64_t kstep;  /* 1: every step; 2: even steps only (Pfaffian-only reduction) */
  int stop;       /* set by thread 0 to end the loop */
} orc_ctx;

typedef struct {
  orc_ctx* c;
  int tid;
} orc_arg;

#define MT(i, j) M[(i) + (int64_t)(j) * ldm]

/* The symmetric interchange of rows/columns r < p applied to the magnitude
 * sums: the same moves as the entries, without the sign changes. */
static void orc_swap_mag(orc_ctx* c, int64_t r, int64_t p) {
  double* M = c->M;
  int64_t ldm = c->ldm, n = c->n;
  for (int64_t j = 0; j < r; ++j) {
    double t = MT(r, j);
    MT(r, j) = MT(p, j);
    MT(p, j) = t;
  }
  for (int64_t j = r + 1; j < p; ++j) {
    double t = MT(j, r);
    MT(j, r) = MT(p, j);
    MT(p, j) = t;
  }
  for (int64_t j = p + 1; j < n; ++j) {
    double t = MT(j, r);
    MT(j, r) = MT(j, p);
    MT(j, p) = t;
  }
}

/* Steps 1-3 for column k; returns 0, or ORC_ENONFINITE. */
static int orc_pivot_swap_scale(orc_ctx* c, int64_t k) {
  double* A = c->A;
  int64_t lda = c->lda, n = c->n;
  int64_t p = k + 1;
  double best = -1.0, second = -1.0;
  for (int64_t i = k + 1; i < n; ++i) {
    double x = AT(i, k);
    if (!isfinite(x)) return ORC_ENONFINITE;
    double ax = fabs(x);
    if (ax > best) {
      second = best;
      best = ax;
      p = i;
    } else if (ax > second) {
      second = ax;
    }
  }
  if (c->gap) c->gap[k] = (best > 0.0 && second >= 0.0) ? (best - second) / best : 1.0;
  int64_t r = k + 1;
  if (p != r && c->M) orc_swap_mag(c, r, p);
  if (p != r) {
    for (int64_t j = 0; j < r; ++j) {          /* row segments left of r */
      double t = AT(r, j);
      AT(r, j) = AT(p, j);
      AT(p, j) = t;
    }
    for (int64_t j = r + 1; j < p; ++j) {      /* column r against row p, both negated */
      double t = AT(j, r);
      AT(j, r) = -AT(p, j);
      AT(p, j) = -t;
    }
    AT(p, r) = -AT(p, r);
    for (int64_t j = p + 1; j < n; ++j) {      /* column segments below p */
      double t = AT(j, r);
      AT(j, r) = AT(j, p);
      AT(j, p) = t;
    }
  }
  c->ipiv[r] = (int32_t)p;
  double alpha = AT(r, k);
  c->T[k] = alpha;
  for (int64_t i = k + 2; i < n; ++i) AT(i, k) = (alpha != 0.0) ? AT(i, k) / alpha : 0.0;
  return 0;
}

/* Step 4 for the columns j = k+2+tid, k+2+tid+nthreads, ... */
static void orc_update(orc_ctx* c, int64_t k, int tid) {
  double* A = c->A;
  int64_t lda = c->lda, n = c->n;
  const double* l = &AT(0, k);
  const double* v = &AT(0, k + 1);
  for (int64_t j = k + 2 + tid; j < n; j += c->nthreads) {
    double lj = l[j], vj = v[j];
    double* col = &AT(0, j);
    for (int64_t i = j + 1; i < n; ++i) col[i] = (col[i] + l[i] * vj) - v[i] * lj;
  }
  if (c->M) {
    /* each entry's sum of the magnitudes of the terms it has accumulated */
    double* M = c->M;
    int64_t ldm = c->ldm;
    for (int64_t j = k + 2 + tid; j < n; j += c->nthreads) {
      double lj = fabs(l[j]), vj = fabs(v[j]);
      double* mc = &MT(0, j);
      for (int64_t i = j + 1; i < n; ++i) mc[i] = mc[i] + (fabs(l[i]) * vj + fabs(v[i]) * lj);
    }
  }
}

/* M[i,j] := |A[i,j]| on the strict lower triangle (the input's own term). */
static void orc_init_mag(orc_ctx* c) {
  double* A = c->A;
  double* M = c->M;
  int64_t lda = c->lda, ldm = c->ldm, n = c->n;
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = j + 1; i < n; ++i) MT(i, j) = fabs(AT(i, j));
}

static void* orc_worker(void* p) {
  orc_arg* a = (orc_arg*)p;
  orc_ctx* c = a->c;
  for (;;) {
    if (a->tid == 0) {
      int64_t k = c->k;
      if (k >= c->n - 2 || k >= c->nsteps || c->status != 0) {
        c->stop = 1;
      } else {
        int st = orc_pivot_swap_scale(c, k);
        if (st != 0) {
          c->status = st;
          c->stop = 1;
        }
      }
    }
    pthread_barrier_wait(&c->bar);
    if (c->stop) break;
    orc_update(c, c->k, a->tid);
    pthread_barrier_wait(&c->bar);
    if (a->tid == 0) c->k += c->kstep;
  }
  return NULL;
}

/*
 * Factor n x n skew A (strict lower triangle) in place.  nsteps < 0 runs the
 * whole factorization; otherwise only the first nsteps elimination steps are
 * done (a bounded sample for timing; T[nsteps..] and the tail are then not set).
 * gap (optional, length n) receives per step (|c|_(1) - |c|_(2)) / |c|_(1).
 * M (optional, n x n, ldm): on exit M[i,j] (i > j) is the sum of the magnitudes
 * of every term the entry A[i,j] accumulated before it was last used: |input|
 * plus |l_i v_j| + |v_i l_j| per update, moved with the entry by the
 * interchanges.  So M[k+1,k] belongs to T[k], and M[i,j-1] (i > j) to the
 * numerator of L[i,j] (its pivot's sum is M[j,j-1]).  A recursive sum of m
 * rounded products carries an error of at most gamma_m times this sum.
 * Returns 0, 1+k for the first even k with T[k] == 0 (exactly singular),
 * or ORC_ENONFINITE if a pivot column held a NaN or an infinity.
 */
int oracle_ltlt_mag(int64_t n, double* A, int64_t lda, int32_t* ipiv, double* T, double* gap,
                    double* M, int64_t ldm, int64_t nsteps, int nthreads) {
  if (n < 0 || lda < (n > 1 ? n : 1) || (n > 0 && (!A || !ipiv)) || (n > 1 && !T)) return ORC_EARG;
  if (M && ldm < (n > 1 ? n : 1)) return ORC_EARG;
  if (n == 0) return 0;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  orc_ctx c;
  memset(&c, 0, sizeof c);
  c.A = A;
  c.lda = lda;
  c.n = n;
  c.nthreads = nthreads;
  c.nsteps = nsteps < 0 ? n : nsteps;
  c.kstep = 1;
  c.ipiv = ipiv;
  c.T = T;
  c.gap = gap;
  c.M = M;
  c.ldm = ldm;
  if (M) orc_init_mag(&c);
  ipiv[0] = 0;
  pthread_barrier_init(&c.bar, NULL, (unsigned)nthreads);
  pthread_t th[64];
  orc_arg args[64];
  for (int t = 0; t < nthreads; ++t) {
    args[t].c = &c;
    args[t].tid = t;
    if (t > 0) pthread_create(&th[t], NULL, orc_worker, &args[t]);
  }
  orc_worker(&args[0]);
  for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
  pthread_barrier_destroy(&c.bar);
  if (c.status != 0) return c.status;
  if (nsteps >= 0 && nsteps < n - 2) return 0;
  if (n >= 2) {
    T[n - 2] = AT(n - 1, n - 2);
    if (!isfinite(T[n - 2])) return ORC_ENONFINITE;
    ipiv[n - 1] = (int32_t)(n - 1);
  }
  for (int64_t k = 0; k + 1 < n; k += 2)
    if (T[k] == 0.0) return (int)(k + 1);
  return 0;
}

int oracle_ltlt(int64_t n, double* A, int64_t lda, int32_t* ipiv, double* T, double* gap,
                int64_t nsteps, int nthreads) {
  return oracle_ltlt_mag(n, A, lda, ipiv, T, gap, NULL, 0, nsteps, nthreads);
}

/*
 * Pfaffian-only reduction: the same elimination step (pivot search, symmetric
 * interchange, multipliers, rank-2 congruence update) taken at the even steps
 * k = 0, 2, ..., n-4 only.  Step k leaves rows/columns k and k+1 as the 2 x 2
 * block [[0, -T[k]], [T[k], 0]] decoupled from the rest (the update is a
 * congruence with a unit lower triangular matrix, which keeps the Pfaffian),
 * so the next step may start directly at column k+2: half the pivot steps of
 * the full factorization, the same n^3/3 flops, and
 *   Pf(A) = (-1)^{s + n/2} prod_{k even} T[k],  s = #{j : ipiv[j] != j},
 * exactly as from the full factors (oracle_logpf applies unchanged).
 * On exit ipiv[k+1] (k even) holds the interchange of step k and every other
 * ipiv[j] = j; T[k] (k even) holds the pivots and T[k] (k odd) = 0; A is left
 * as scratch (no L).  n odd: Pf = 0, returns n without touching A.
 * M (optional) as for oracle_ltlt_mag: M[k+1,k] is the magnitude sum of T[k].
 * Returns as oracle_ltlt.
 */
int oracle_pfonly_mag(int64_t n, double* A, int64_t lda, int32_t* ipiv, double* T, double* M,
                      int64_t ldm, int nthreads) {
  if (n < 0 || lda < (n > 1 ? n : 1) || (n > 0 && (!A || !ipiv)) || (n > 1 && !T)) return ORC_EARG;
  if (M && ldm < (n > 1 ? n : 1)) return ORC_EARG;
  if (n == 0) return 0;
  for (int64_t j = 0; j < n; ++j) ipiv[j] = (int32_t)j;
  for (int64_t k = 0; k + 1 < n; ++k) T[k] = 0.0;
  if (n % 2 == 1) return (int)n;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  orc_ctx c;
  memset(&c, 0, sizeof c);
  c.A = A;
  c.lda = lda;
  c.n = n;
  c.nthreads = nthreads;
  c.nsteps = n;
  c.kstep = 2;
  c.ipiv = ipiv;
  c.T = T;
  c.gap = NULL;
  c.M = M;
  c.ldm = ldm;
  if (M) orc_init_mag(&c);
  pthread_barrier_init(&c.bar, NULL, (unsigned)nthreads);
  pthread_t th[64];
  orc_arg args[64];
  for (int t = 0; t < nthreads; ++t) {
    args[t].c = &c;
    args[t].tid = t;
    if (t > 0) pthread_create(&th[t], NULL, orc_worker, &args[t]);
  }
  orc_worker(&args[0]);
  for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
  pthread_barrier_destroy(&c.bar);
  if (c.status != 0) return c.status;
  T[n - 2] = AT(n - 1, n - 2);
  if (!isfinite(T[n - 2])) return ORC_ENONFINITE;
  for (int64_t k = 0; k + 1 < n; k += 2)
    if (T[k] == 0.0) return (int)(k + 1);
  return 0;
}

int oracle_pfonly(int64_t n, double* A, int64_t lda, int32_t* ipiv, double* T, int nthreads) {
  return oracle_pfonly_mag(n, A, lda, ipiv, T, NULL, 0, nthreads);
}

/*
 * Pfaffian from the factors: Pf(A) = det(P) Pf(T), det(P) = (-1)^s with s the
 * number of j with ipiv[j] != j, and Pf(T) = prod_{k even} T(k,k+1)
 * = (-1)^{n/2} prod_{k even} T[k].  Odd n: Pf = 0 (sign 0, logabs -inf);
 * n = 0: Pf = 1.  The sum of logarithms runs in index order.
 */
void oracle_logpf(int64_t n, const int32_t* ipiv, const double* T, double* logabs, int* sign) {
  if (n == 0) {
    *logabs = 0.0;
    *sign = 1;
    return;
  }
  if (n % 2 == 1) {
    *logabs = -INFINITY;
    *sign = 0;
    return;
  }
  int64_t s = 0;
  for (int64_t j = 0; j < n; ++j)
    if (ipiv[j] != j) ++s;
  int neg = (int)((s + n / 2) & 1);
  double la = 0.0;
  for (int64_t k = 0; k < n - 1; k += 2) {
    double t = T[k];
    if (t == 0.0) {
      *logabs = -INFINITY;
      *sign = 0;
      return;
    }
    if (t < 0.0) neg ^= 1;
    la += log(fabs(t));
  }
  *logabs = la;
  *sign = neg ? -1 : 1;
}

/*
 * Solve A X = B with the factors, nrhs columns of B (ldb >= n), in place:
 *   X = P^T L^{-T} T^{-1} L^{-1} P B.
 * P is applied as the recorded interchanges in order; L is unit lower with
 * L[i,j] (i > j >= 1) at LT[i, j-1]; the tridiagonal T is solved by Gaussian
 * elimination with partial pivoting (the textbook tridiagonal GEPP).
 * Returns 0, or 1+k for the first even k with T[k] == 0 (T singular), or
 * ORC_EARG; odd n is singular and returns n.
 */
int oracle_solve(int64_t n, int64_t nrhs, const double* LT, int64_t lda, const int32_t* ipiv,
                 const double* T, double* B, int64_t ldb) {
  if (n < 0 || nrhs < 0 || lda < (n > 1 ? n : 1) || ldb < (n > 1 ? n : 1)) return ORC_EARG;
  if (n == 0 || nrhs == 0) return 0;
  if (n % 2 == 1) return (int)n;
  for (int64_t k = 0; k + 1 < n; k += 2)
    if (T[k] == 0.0) return (int)(k + 1);
  /* tridiagonal of T: sub dl[i] = T(i+1,i) = T[i], super du[i] = T(i,i+1) = -T[i], diag 0 */
  double* dl = (double*)malloc(sizeof(double) * (size_t)n);
  double* dd = (double*)malloc(sizeof(double) * (size_t)n);
  double* du = (double*)malloc(sizeof(double) * (size_t)n);
  double* du2 = (double*)malloc(sizeof(double) * (size_t)n);
  int64_t* piv = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int info = 0;
  for (int64_t c = 0; c < nrhs; ++c) {
    double* b = B + c * ldb;
    /* b := P b, interchanges in order */
    for (int64_t j = 1; j < n; ++j) {
      int64_t p = ipiv[j];
      if (p != j) {
        double t = b[j];
        b[j] = b[p];
        b[p] = t;
      }
    }
    /* b := L^{-1} b (unit lower, column 0 of L is e_0) */
    for (int64_t j = 1; j < n; ++j) {
      double bj = b[j];
      for (int64_t i = j + 1; i < n; ++i) b[i] = b[i] - LT[i + (j - 1) * lda] * bj;
    }
    /* b := T^{-1} b by tridiagonal Gaussian elimination with partial pivoting */
    for (int64_t i = 0; i < n; ++i) {
      dd[i] = 0.0;
      dl[i] = (i + 1 < n) ? T[i] : 0.0;
      du[i] = (i + 1 < n) ? -T[i] : 0.0;
      du2[i] = 0.0;
    }
    for (int64_t i = 0; i + 1 < n; ++i) {
      /* rows i and i+1; column i entries dd[i] (row i) and dl[i] (row i+1) */
      if (fabs(dd[i]) >= fabs(dl[i])) {
        piv[i] = i;
        if (dd[i] == 0.0) {
          info = (int)(i + 1);
          goto done;
        }
        double f = dl[i] / dd[i];
        dd[i + 1] = dd[i + 1] - f * du[i];
        b[i + 1] = b[i + 1] - f * b[i];
        dl[i] = 0.0;  /* eliminated */
      } else {
        piv[i] = i + 1;
        double f = dd[i] / dl[i];
        /* swap rows i and i+1 */
        dd[i] = dl[i];
        double t = dd[i + 1];
        dd[i + 1] = du[i] - f * t;
        du[i] = t;
        if (i + 2 < n) {
          du2[i] = du[i + 1];
          du[i + 1] = -f * du2[i];
        }
        double tb = b[i];
        b[i] = b[i + 1];
        b[i + 1] = tb - f * b[i];
      }
    }
    if (dd[n - 1] == 0.0) {
      info = (int)n;
      goto done;
    }
    /* back substitution with upper bands dd, du, du2 */
    b[n - 1] = b[n - 1] / dd[n - 1];
    if (n >= 2) b[n - 2] = (b[n - 2] - du[n - 2] * b[n - 1]) / dd[n - 2];
    for (int64_t i = n - 3; i >= 0; --i)
      b[i] = (b[i] - du[i] * b[i + 1] - du2[i] * b[i + 2]) / dd[i];
    /* b := L^{-T} b */
    for (int64_t j = n - 1; j >= 1; --j) {
      double s = b[j];
      for (int64_t i = j + 1; i < n; ++i) s = s - LT[i + (j - 1) * lda] * b[i];
      b[j] = s;
    }
    /* b := P^T b, interchanges in reverse order */
    for (int64_t j = n - 1; j >= 1; --j) {
      int64_t p = ipiv[j];
      if (p != j) {
        double t = b[j];
        b[j] = b[p];
        b[p] = t;
      }
    }
  }
done:
  free(dl);
  free(dd);
  free(du);
  free(du2);
  free(piv);
  return info;
}
