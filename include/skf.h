/*
 * skf -- skew-symmetric LTL^T factorization and Pfaffians on AMD MI355X (gfx950).
 *
 * Plain C ABI.  Every array argument is a DEVICE pointer owned by the caller
 * unless the comment says "host".  Streams are passed as `void*` holding a
 * hipStream_t (NULL = the default stream).  The library never frees caller
 * memory and allocates no device memory on these paths: scratch space is the
 * caller's `work` buffer, whose size the matching *_workspace query returns.
 *
 * Mathematics (standard, no particular paper passage: the method is Gaussian
 * congruence elimination with partial pivoting in the manner of Parlett and
 * Reid, 1970, specialised to skew-symmetric matrices):
 *   P A P^T = L T L^T, L unit lower triangular with L[:,0] = e_0, T skew
 *   tridiagonal (T(k+1,k) = T[k], T(k,k+1) = -T[k]); Pf(A) = det(P) Pf(T),
 *   Pf(T) = (-1)^{n/2} prod_{k even} T[k]; 2*log|Pf(A)| = log|det(A)|.
 *
 * Storage conventions shared by all entry points (column-major, 0-based):
 *   - A is n x n with leading dimension lda >= max(1,n); ONLY the strict lower
 *     triangle is read.  The diagonal and the strict upper triangle are never
 *     written and their values never used (the residual and solve kernels may
 *     issue a discarded load of A[0,0] as a clamped address; NaN or Inf there
 *     changes nothing).
 *   - On exit from a factorization, L[i,j] (i > j >= 1) is stored at A[i, j-1],
 *     the subdiagonal A[k+1,k] holds T[k], and T[k] is also written to T[].
 *   - ipiv[0] = 0; ipiv[j] = p >= j means rows/columns j and p were interchanged
 *     at elimination step j-1 (P is the product of these interchanges, in order).
 *   - Pivoting chooses the largest |entry| of the current column below the
 *     subdiagonal; ties go to the lowest row index; an all-zero column gives no
 *     interchange and a zero multiplier column.
 *
 * Status codes: entry points return 0 once the work is enqueued, or a negative
 * code for an argument / device error detected on the host before any launch
 * (-i = the i-th argument, 1-based, is invalid; SKF_E* below).  Numerical
 * outcomes are reported through `dinfo` (a device int) when it is non-NULL, in
 * which case the call is asynchronous on `stream`.  When `dinfo` is NULL the
 * call synchronizes `stream` and returns the numerical outcome instead:
 *   0            success
 *   k+1 > 0      the first even step k with T[k] == 0: A is exactly singular
 *                (Pf = 0); the factorization itself is complete
 *   SKF_ENONFINITE  a pivot column held a NaN or an infinity; the outputs are
 *                partial and must not be used
 *   SKF_ETIMEOUT the persistent kernel's co-residency wait gave up (the device
 *                could not run all of its workgroups at once); outputs invalid
 */
#ifndef SKF_H
#define SKF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int64_t skf_int;

#define SKF_PREC_F64 0          /* FP64 everywhere */
#define SKF_PREC_F32_TRAILING 1 /* FP32-MFMA trailing skr2k; FP64 panel, pivots, T and storage */

#define SKF_OK 0
#define SKF_ENOMEM (-100)
#define SKF_EDEVICE (-101)
#define SKF_ENOTIMPL (-102)
#define SKF_ENONFINITE (-103)
#define SKF_EWORK (-104)
#define SKF_ETIMEOUT (-105)
#define SKF_ESCRATCH (-106)    /* size beyond an allocation-free entry point's fixed scratch */

/*
 * Tuning table: parameters chosen by measurement on the device.  The package's
 * tuner (paper_2408_05238_amd/tune.py) times the candidates, stores its choices
 * as JSON and the Python binding loads them here when the library is first
 * used.  Each entry covers the orders n_lo <= n <= n_hi; a later entry covering
 * the same order wins over an earlier one.  Without an entry the built-in rule
 * applies (the widest panel of 128, 64, 32, 16 whose workgroups fit on the
 * device; band of 8 block rows; width 256, one panel workgroup per CU, only
 * from a table entry or the override).  The environment variable
 * SKF_NB=16|32|64|128|256 overrides both panel widths.  A table value that is infeasible for a given n
 * (too many panel workgroups to be resident) is ignored for that n.  Host-only;
 * thread-safe; takes effect for calls made afterwards (workspace sizes cover
 * every feasible width).
 */
#define SKF_TUNE_LTLT_NB 0    /* panel width of skf_ltlt and skf_ltlt-based calls: 16, 32, 64, 128 or 256 */
#define SKF_TUNE_PFONLY_NB 1  /* panel width (twice the steps per panel) of skf_pfonly / skf_logpf: 16, 32, 64, 128 or 256 */
#define SKF_TUNE_SKR2K_BAND 2 /* block rows per band of the trailing update's tile walk, by trailing order: 1..64 */
#define SKF_TUNE_NPARAMS 3
/* Add an entry; returns 0, or -1 (param), -2 (n_lo < 0), -3 (n_hi < n_lo), -4 (value not allowed). */
int skf_tune_set(int param, skf_int n_lo, skf_int n_hi, int value);
/* The value in effect for order n (entry, environment override or built-in rule); -1 for a bad param,
 * 0 when no panel width is feasible for n. */
int skf_tune_get(int param, skf_int n);
/* Remove every entry (the built-in rules apply again). */
int skf_tune_clear(void);

/* Library version string (static storage). */
const char* skf_version(void);

/* Last HIP error text seen by the library on this thread (static storage). */
const char* skf_last_error(void);

/*
 * Device workspace (bytes) needed by skf_ltlt / skf_logpf / skf_pfaffian for an
 * n x n matrix in precision `prec`.  The buffer must be 256-byte aligned and is
 * not preserved between calls.  Blocked path: one n x n FP64 ping-pong copy of
 * the trailing matrix plus O(n * nb) panel buffers.
 */
size_t skf_ltlt_workspace(skf_int n, int prec);

/*
 * Blocked, partially pivoted LTL^T of the skew matrix held in the strict lower
 * triangle of A (right-looking; panels of nb paired elimination steps with the
 * pivot search on the device, trailing skew rank-2k updates on the matrix cores).
 *   n      order (>= 0)
 *   A      device, lda x n, overwritten by L and T as described above
 *   ipiv   device int32[n] (n >= 1), output
 *   T      device double[max(n-1,1)], output
 *   prec   SKF_PREC_F64 or SKF_PREC_F32_TRAILING
 *   work   device workspace of at least skf_ltlt_workspace(n, prec) bytes
 *   dinfo  device int or NULL (see status codes)
 * Orders: a panel runs one workgroup per 64 rows, all resident at once (at most
 * six per CU), so the panel width is the widest that fits (on 256 CUs: 256 up
 * to n = 16385 when chosen, 128 up to 32769, 64 up to 65537, 32 or 16 up to
 * 98305); beyond, SKF_ENOTIMPL.  skf_pfonly: the same.
 */
int skf_ltlt(skf_int n, double* A, skf_int lda, int32_t* ipiv, double* T, int prec,
             void* work, size_t lwork, int* dinfo, void* stream);

/*
 * Pfaffian-only reduction of one matrix (the blocked form of the reduction
 * described at skf_pfonly_batched: Parlett-Reid elimination steps at even k
 * only, pivot on column k, interchange of rows/columns k+1 and p, skew rank-2
 * term l v^T - v l^T on A[k+2:, k+2:]).  Panels of nb/2 such steps run on the
 * device with the pivot search as in skf_ltlt; their nb/2 (l, v) pairs form one
 * skew rank-nb trailing update on the matrix cores.  Half as many pivot
 * searches as skf_ltlt for the same flops; no L is formed.
 *   n, lda, prec, work, lwork, dinfo, stream  as skf_ltlt (same workspace size)
 *   A      device, lda x n: used as scratch, contents unspecified on return
 *   ipiv   device int32[n], output: ipiv[k+1] (k even) = step k's interchange,
 *          the other entries j
 *   T      device double[max(n-1,1)], output: T[k] (k even) = pivot of step k,
 *          the odd entries 0
 * Pf(A) = (-1)^{s + n/2} prod_{k even} T[k] (s = #{j : ipiv[j] != j}), so
 * skf_logpf_from_factors applies.  Odd n: ipiv = identity, T = 0, info = n.
 * Otherwise info as skf_ltlt (1 + the first even k with T[k] = 0, or a
 * negative status).  Returns 0, the info (dinfo NULL) or an argument error.
 */
int skf_pfonly(skf_int n, double* A, skf_int lda, int32_t* ipiv, double* T, int prec, void* work,
               size_t lwork, int* dinfo, void* stream);

/*
 * log|Pf(A)| and sign(Pf(A)) from factors produced by skf_ltlt:
 * log|Pf| = sum_{k even} log|T[k]| (fixed summation order), sign =
 * (-1)^{s + n/2} prod_{k even} sgn T[k], s = #{j : ipiv[j] != j}.
 * Odd n or a zero even T[k]: *sign = 0 and *logabs = -inf.  n = 0: Pf = 1.
 * logabs, sign: device scalars.  Asynchronous; never fails numerically.
 */
int skf_logpf_from_factors(skf_int n, const int32_t* ipiv, const double* T, double* logabs,
                           int* sign, void* stream);

/* Device workspace (bytes) for skf_logpf / skf_pfaffian (the factorization's
 * workspace plus room for ipiv and T). */
size_t skf_logpf_workspace(skf_int n, int prec);

/* Reduce A by skf_pfonly (destroying A), then to log|Pf| and sign; outputs are
 * device scalars. */
int skf_logpf(skf_int n, double* A, skf_int lda, double* logabs, int* sign, int prec, void* work,
              size_t lwork, int* dinfo, void* stream);

/* As skf_logpf but returns Pf itself (device double; may overflow to +-inf or underflow to 0). */
int skf_pfaffian(skf_int n, double* A, skf_int lda, double* pf, int prec, void* work, size_t lwork,
                 int* dinfo, void* stream);

/*
 * Skew-symmetric rank-2k update of the strict lower triangle of C (n x n):
 *   C := beta C + alpha (A B^T - B A^T),  A, B: n x k (lda, ldb >= n).
 * The diagonal and upper triangle of C are not referenced.  beta == 0 does not
 * read C.  FP64 matrix-core (MFMA) tiles.
 */
int skf_skr2k(skf_int n, skf_int k, double alpha, const double* A, skf_int lda, const double* B,
              skf_int ldb, double beta, double* C, skf_int ldc, void* stream);

/* The same update with A and B rounded to FP32, FP32 MFMA products and FP32
 * accumulation over k, added to the FP64 C in FP64. */
int skf_skr2k_f32(skf_int n, skf_int k, double alpha, const double* A, skf_int lda, const double* B,
                  skf_int ldb, double beta, double* C, skf_int ldc, void* stream);

/* Device workspace (bytes) for skf_solve with nrhs right-hand sides. */
size_t skf_solve_workspace(skf_int n, skf_int nrhs);

/*
 * Solve A X = B with the factors of skf_ltlt: X = P^T L^{-T} T^{-1} L^{-1} P B,
 * in place over B (n x nrhs, ldb >= n).  T is solved by Gaussian elimination
 * with partial pivoting on the tridiagonal.
 * Numerical outcome (dinfo / return): 0, or k+1 for the first even k with
 * T[k] == 0, or n for odd n (T, hence A, is singular; B is then unspecified).
 */
int skf_solve(skf_int n, skf_int nrhs, const double* LT, skf_int lda, const int32_t* ipiv,
              const double* T, double* B, skf_int ldb, void* work, size_t lwork, int* dinfo,
              void* stream);

/*
 * skf_solve without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Same operation, kernels and results as skf_solve
 * (bitwise, for the same inputs); its workspace is a fixed device array of the
 * library (8 405 504 bytes, the skf_solve workspace of order 4096, per device,
 * held until the process ends), so the call allocates nothing.
 *   n       order, 0 <= n <= SKF_SOLVE_NOALLOC_MAX_N, else SKF_ESCRATCH before
 *           any launch (skf_last_error names the limit)
 *   other arguments as skf_solve
 * Every call on one device shares that device's array and leaves its contents
 * behind: calls that overlap on one device (on different streams or host
 * threads) race and must be ordered by the caller.
 */
#define SKF_SOLVE_NOALLOC_MAX_N 4096
int skf_solve_noalloc(skf_int n, skf_int nrhs, const double* LT, skf_int lda, const int32_t* ipiv,
                      const double* T, double* B, skf_int ldb, int* dinfo, void* stream);

/* Device workspace (bytes) for skf_pfonly_c128: four n x n FP64 planes and the
 * panel buffers (blocked form), at least a full n x n complex128 copy. */
size_t skf_pfonly_c128_workspace(skf_int n);

/*
 * Pfaffian-only reduction of a complex (complex128) skew-symmetric matrix: the
 * elimination of skf_pfonly at even steps k, with the pivot the largest
 * |z|^2 = re^2 + im^2 below the diagonal of column k (lowest index on ties).
 * Pf(A) = (-1)^{s + n/2} prod_{k even} T[k], s = #{j : ipiv[j] != j}.
 * Blocked (n up to 64 x 256 panel workgroups of the device, i.e. 16385 with the
 * wide panel and 32769 with the narrow one on 256 CUs): the input is split into
 * real and imaginary planes in the workspace, each panel of nb/2 even steps runs
 * as one persistent kernel and the complex rank-nb trailing update as two real
 * skew rank-2nb updates on the matrix cores (one per plane).  Beyond that, or
 * with SKF_C128_UNBLOCKED set, the unblocked form: a full copy and a few
 * launches per step (n <= 65535).  Both give the same interchanges on generic
 * input; T agrees to rounding.
 *   A      device, lda x n complex128 (interleaved re, im), strict lower triangle
 *          read, not modified
 *   ipiv   device int32[n]: ipiv[k+1] (k even) = step k's interchange, else j
 *   T      device complex128[max(n-1,1)]: T[k] (k even) pivots, odd entries 0
 *   work   device workspace of skf_pfonly_c128_workspace(n) bytes (256-aligned)
 *   dinfo  device int or NULL: 0; n for odd n; 1 + the first even k with
 *          T[k] = 0; SKF_ENONFINITE for a non-finite pivot column
 * Returns 0, the outcome (dinfo NULL: synchronous) or an argument error.
 */
int skf_pfonly_c128(skf_int n, const double* A, skf_int lda, int32_t* ipiv, double* T, void* work,
                    size_t lwork, int* dinfo, void* stream);

/* Device workspace (bytes) for skf_ltlt_c128: four n x n FP64 planes and the
 * panel buffers; 0 when no panel width fits the order on this device. */
size_t skf_ltlt_c128_workspace(skf_int n);

/*
 * Partially pivoted LTL^T of a complex (complex128) skew-symmetric matrix:
 * P A P^T = L T L^T with L unit lower triangular (L[:,0] = e_0) and T complex
 * skew tridiagonal (T(k+1,k) = T[k], T(k,k+1) = -T[k]); plain transposes.
 * The elimination step of skf_ltlt at every k with the pivot the largest
 * |z|^2 = re^2 + im^2 below the diagonal of column k (lowest index on ties).
 * Blocked: panels of 64 steps (n up to 64 x 256 panel workgroups on 256 CUs,
 * i.e. 16385), 32 steps (up to 32769) or 16 steps (up to 65537), each a
 * persistent kernel on the real and imaginary planes, its pairs (l, v) applied
 * as one real skew rank-2k update per plane on the matrix cores; beyond,
 * SKF_ENOTIMPL.
 *   A      device, lda x n complex128 (interleaved re, im), strict lower triangle
 *          read; on exit as skf_ltlt's A: L[i,j] (i > j >= 1) at A[i, j-1], the
 *          subdiagonal A[k+1,k] = T[k]
 *   ipiv   device int32[n] (n >= 1), output, as skf_ltlt
 *   T      device complex128[max(n-1,1)], output
 *   work   device workspace of skf_ltlt_c128_workspace(n) bytes (256-aligned)
 *   dinfo  device int or NULL: 0; 1 + the first even k with T[k] = 0 (then
 *          Pf = 0; the factorization is complete); SKF_ENONFINITE for a
 *          non-finite pivot column
 * Pf(A) follows from (ipiv, T) by skf_logpf_c128_from_factors.
 * Returns 0, the outcome (dinfo NULL: synchronous) or an argument error.
 */
int skf_ltlt_c128(skf_int n, double* A, skf_int lda, int32_t* ipiv, double* T, void* work, size_t lwork, int* dinfo,
                  void* stream);

/* Device workspace (bytes) for skf_solve_c128 with nrhs right-hand sides. */
size_t skf_solve_c128_workspace(skf_int n, skf_int nrhs);

/*
 * Solve A X = B with the factors of skf_ltlt_c128 (complex128, interleaved):
 * X = P^T L^{-T} T^{-1} L^{-1} P B in place over B (n x nrhs, ldb >= n), as
 * skf_solve: triangular solves by 64-row blocks, T by Gaussian elimination with
 * partial pivoting on the tridiagonal (row i+1 becomes the pivot row when
 * |T(i+1,i)|^2 exceeds the running diagonal's |.|^2).
 * Numerical outcome (dinfo / return): 0; n for odd n; 1 + the first even k with
 * T[k] = 0 (B is then left as it is); the elimination's own zero pivot.
 */
int skf_solve_c128(skf_int n, skf_int nrhs, const double* LT, skf_int lda, const int32_t* ipiv, const double* T,
                   double* B, skf_int ldb, void* work, size_t lwork, int* dinfo, void* stream);

/* log|Pf| and phase = Pf/|Pf| (device double[2], re and im; 0 when Pf = 0)
 * from the factors of skf_pfonly_c128, in index order.  n = 0: Pf = 1. */
int skf_logpf_c128_from_factors(skf_int n, const int32_t* ipiv, const double* T, double* logabs,
                                double* phase, void* stream);

/* Device workspace (bytes) for skf_pf_ratio (0 if r is out of range). */
size_t skf_pf_ratio_workspace(skf_int n, skf_int r);

/*
 * Pfaffian ratio of a low-rank skew update, from the resident factors of A:
 *   Pf(A + U V^T - V U^T) / Pf(A),  U, V: n x r (device, column-major), 0 <= r <= 32.
 * With W = [U V] and J = [[0, I_r], [-I_r, 0]] the ratio equals
 * Pf(W^T A^-1 W - J) / Pf(-J) (the Schur-complement identity of the Pfaffian
 * for the bordered matrix [[A, W], [-W^T, -J]]), so the call costs one solve
 * with 2r right-hand sides through the factors (as skf_solve), a 2r x 2r Gram
 * product and a 2r x 2r Pfaffian, instead of a factorization of the updated
 * matrix.  The factors (LT, ipiv, T) come from skf_ltlt of A.
 *   logabs, sign  device scalars: log|ratio| and its sign (0 when the updated
 *                 matrix is singular: logabs = -inf)
 *   work          device workspace of skf_pf_ratio_workspace(n, r) bytes (256-aligned)
 *   dinfo         device int or NULL: 0; the solve's outcome when A is singular
 *                 (odd n, or a zero even pivot: the ratio is undefined, logabs = NaN,
 *                 sign = 0); SKF_ENONFINITE for non-finite U, V or factors.
 * r = 0 (and n = 0) give the ratio 1 without examining the factors.
 * Returns 0, the outcome (dinfo NULL: the call then synchronizes) or an
 * argument error (-2: r out of range).
 */
int skf_pf_ratio(skf_int n, skf_int r, const double* LT, skf_int lda, const int32_t* ipiv,
                 const double* T, const double* U, skf_int ldu, const double* V, skf_int ldv,
                 double* logabs, int* sign, void* work, size_t lwork, int* dinfo, void* stream);

/* Device workspace (bytes) for skf_solve_refine. */
size_t skf_refine_workspace(skf_int n, skf_int nrhs);

/*
 * Iterative refinement (synchronous): X_0 = solve(B); repeat R = B - A0 X in
 * FP64 (A0 = the ORIGINAL matrix, strict lower triangle read), D = solve(R),
 * X += D, until the componentwise-normwise backward error
 *   eta = max_j ||b_j - A0 x_j||_inf / (||A0||_inf ||x_j||_inf + ||b_j||_inf)
 * is <= tol or maxit corrections were applied.  Factors may come from either
 * precision.  iters, berr: host outputs (iters = corrections applied).
 * Returns the numerical outcome as skf_solve does; 1 if tol was not reached.
 */
int skf_solve_refine(skf_int n, skf_int nrhs, const double* A0, skf_int lda0, const double* LT,
                     skf_int lda, const int32_t* ipiv, const double* T, const double* B,
                     skf_int ldb, double* X, skf_int ldx, double tol, int maxit, int* iters,
                     double* berr, void* work, size_t lwork, void* stream);

/* Device workspace (bytes) for the batched calls over `batch` matrices of
 * orders n_host[0..batch) (host array; includes room for skf_solve_batched
 * with up to 16 right-hand sides). */
size_t skf_batched_workspace(skf_int batch, const skf_int* n_host);

/*
 * Batched LTL^T + Pfaffian: `batch` independent skew matrices, each of order
 * n <= 512, factored by ONE persistent launch: every workgroup takes matrices
 * from a device work queue (largest first) and factors one at a time in its
 * storage (paired elimination steps, eager interchanges, delayed rank-16
 * updates).  A matrix's results do not depend on the rest of the batch.
 *   n_host, lda_host  host arrays [batch]: orders and leading dimensions
 *   A                 device array [batch] of device pointers (overwritten by L, T)
 *   ipiv, T           device arrays [batch] of device pointers, or NULL to skip
 *                     (T[b] needs max(n-1,1) doubles, ipiv[b] n ints)
 *   logabs, sign, info  device arrays [batch]: log|Pf|, sign, per-matrix outcome
 * Asynchronous on `stream`.
 */
int skf_ltlt_batched(skf_int batch, const skf_int* n_host, double* const* A, const skf_int* lda_host,
                     int32_t* const* ipiv, double* const* T, double* logabs, int* sign, int* info,
                     void* work, size_t lwork, void* stream);

/*
 * Batched Pfaffian-only reduction: the elimination step of skf_ltlt taken at
 * the even steps only.  Step k pivots on column k (largest |A[i,k]|, i > k,
 * lowest index on ties), interchanges rows/columns k+1 and p, and adds the
 * skew rank-2 term l v^T - v l^T to A[k+2:, k+2:]; rows/columns k and k+1 are
 * then decoupled (a congruence with a unit lower triangular matrix keeps the
 * Pfaffian), so the next step is k+2: n/2 pivot steps instead of n, the same
 * n^3/3 flops, and Pf(A) = (-1)^{s + n/2} prod_{k even} T[k] with s the number
 * of interchanges.  Its pivots differ from skf_ltlt's (the odd steps are
 * skipped); the Pfaffian is the same.  One persistent launch as
 * skf_ltlt_batched; A is scratch (no factor is left in it).
 *   ipiv, T   device arrays [batch] of device pointers, or NULL to skip:
 *             ipiv[b][k+1] (k even) receives step k's interchange, the other
 *             entries j; T[b][k] (k even) the pivots, the odd entries 0
 *   logabs, sign, info  as skf_ltlt_batched (info = n for odd n)
 * Returns 0 or a negative argument / launch error (-7: logabs or sign NULL).
 */
int skf_pfonly_batched(skf_int batch, const skf_int* n_host, double* const* A, const skf_int* lda_host,
                       int32_t* const* ipiv, double* const* T, double* logabs, int* sign, int* info,
                       void* work, size_t lwork, void* stream);

/* log|Pf| and sign of every matrix of the batch by the Pfaffian-only reduction
 * (skf_pfonly_batched without ipiv / T).  A is used as scratch. */
int skf_logpf_batched(skf_int batch, const skf_int* n_host, double* const* A, const skf_int* lda_host,
                      double* logabs, int* sign, int* info, void* work, size_t lwork, void* stream);

/* Device workspace (bytes) for skf_solve_batched (host arrays n_host, nrhs_host). */
size_t skf_solve_batched_workspace(skf_int batch, const skf_int* n_host, const skf_int* nrhs_host);

/*
 * Batched solves with factors from skf_ltlt_batched (or skf_ltlt): B[b]
 * (n_b x nrhs_host[b], ldb_host[b]) overwritten by X[b] = A_b^{-1} B[b], the
 * same steps as skf_solve.  One launch for every matrix of order <= 1024, one
 * wave per (matrix, right-hand side); asynchronous on `stream` (the host size
 * arrays are staged into the workspace).  Matrices of larger order are solved
 * one after the other by the skf_solve path after a synchronous read-back of
 * the pointer arrays.  LT, ipiv, T, B: device arrays of device pointers.
 * info[b] (device) as for skf_solve.  work: skf_solve_batched_workspace bytes
 * (256-aligned; skf_batched_workspace covers up to 16 right-hand sides).
 * Returns 0, or an argument error (-1: batch, -2: a pointer or size array).
 */
int skf_solve_batched(skf_int batch, const skf_int* n_host, double* const* LT, const skf_int* lda_host,
                      int32_t* const* ipiv, double* const* T, const skf_int* nrhs_host,
                      double* const* B, const skf_int* ldb_host, int* info, void* work, size_t lwork,
                      void* stream);

/*
 * Kernel timing for benchmarks.  While enabled, every launch of the blocked
 * factorization's panel kernel (class 0) and trailing skew rank-2k update
 * (class 1) is bracketed by HIP events recorded on the launch's own stream,
 * together with the launch's algorithmic flop count (class 1: 2 * K * m(m-1)/2
 * with K = 2 * pairs, m the trailing order).  skf_profile_read synchronizes the
 * recorded events and returns, per class, total milliseconds, total flops and
 * the number of launches (arrays of length 2, host memory); reset != 0 clears
 * the record.  Not thread-safe against concurrent factorizations.
 */
int skf_profile_enable(int on);
int skf_profile_read(double* ms, double* flops, int64_t* launches, int reset);

#ifdef __cplusplus
}
#endif

#endif /* SKF_H */
