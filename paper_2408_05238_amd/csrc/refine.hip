// Residual, norms and the iterative-refinement loop for A X = B.
//
// A0 is the ORIGINAL skew matrix (strict lower triangle read), S = tril(A0,-1)
// - tril(A0,-1)^T.  R = B - S X is computed in FP64 by 64-row blocks: block I
// reads the blocks left of its diagonal block (row panel, used as stored) and
// the blocks below it (column panel, used transposed and negated), so every
// stored block is read once as a row block and once as a column block and no
// floating-point atomics are needed (the result does not depend on timing).
// The refinement loop itself runs on the host: each iteration launches the
// residual, reads three per-column maxima, and, if the backward error
//   eta = max_j ||r_j||_inf / (||A0||_inf ||x_j||_inf + ||b_j||_inf)
// is above the tolerance, solves for the correction with the resident factors.
// When a correction step shrinks eta by less than half (factors computed with
// FP32 trailing products can be too inexact for plain refinement to contract),
// later corrections are computed by GMRES on the left-preconditioned system
// M^{-1} A d = M^{-1} r with M = P^T L T L^T P from the same factors, in FP64
// (GMRES-based iterative refinement, Carson and Higham 2017): restarted Arnoldi
// with classical Gram-Schmidt applied twice, all right-hand sides side by side,
// the small Hessenberg least-squares problems (Givens rotations) on the host.
#include <algorithm>
#include <vector>

#include "skf_internal.h"

namespace skf {


namespace {

constexpr int BS = 64;
constexpr int RC = 16;
constexpr int NT = 256;

// R[:, c0:c0+nr] = B - S X (rows of block I = blockIdx.x); optionally also the
// absolute row sums of S (||A0||_inf = max of them).  The next block of S and
// of X are fetched into registers (clamped addresses, masks and signs applied
// afterwards) while the current one is multiplied, into the other half of a
// double-buffered LDS tile; the 64 x 16 product keeps four sums per thread.
constexpr int kPer = BS * BS / NT;  // S elements per thread and block (16)
constexpr int kPerX = BS * RC / NT;  // X elements per thread and block (4)

__global__ void __launch_bounds__(NT) residual_kernel(int64_t n, int nr, const double* __restrict__ A0, int64_t lda,
                                                      const double* __restrict__ X, int64_t ldx,
                                                      const double* __restrict__ B, int64_t ldb,
                                                      double* __restrict__ R, int64_t ldr,
                                                      double* __restrict__ rowabs) {
  static_assert(NT == BS * (RC / 4), "one thread per row and group of four columns");
  __shared__ double Ab[2][BS][BS + 1];
  __shared__ double xs[2][BS][RC + 1];
  const int64_t nb = (n + BS - 1) / BS;
  const int64_t I = blockIdx.x;
  const int64_t r0 = I * BS;
  const int bs = (int)min((int64_t)BS, n - r0);
  const int tid = threadIdx.x;
  const int mi = tid % BS, g = tid / BS;  // product: row mi, columns 4g .. 4g+3
  double acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = 4 * g + q;
    acc[q] = (mi < bs && c < nr && B) ? B[r0 + mi + (int64_t)c * ldb] : 0.0;
  }
  double ra = 0.0;  // |S| row sum of row mi (threads of column group 0)
  // element e = tid + NT q: (i, j) = (e % BS, e / BS) for blocks on or left of the
  // diagonal (stored rows i, consecutive threads down a column), (e / BS, e % BS)
  // right of it (stored block (J, I) read down its columns)
  auto fetch = [&](int64_t J, double (&v)[kPer], double (&xv)[kPerX]) {
    const int64_t c0 = J * BS;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + NT * q;
      const int i = (J <= I) ? e % BS : e / BS, j = (J <= I) ? e / BS : e % BS;
      const int64_t gi = r0 + i, gj = c0 + j;
      const bool ok = gi < n && gj < n && gi != gj;
      const int64_t a = gi > gj ? gi + gj * lda : gj + gi * lda;
      v[q] = A0[ok ? a : 0];
    }
#pragma unroll
    for (int q = 0; q < kPerX; ++q) {
      const int e = tid + NT * q;
      const int j = e % BS, c = e / BS;
      const bool ok = c0 + j < n && c < nr;
      xv[q] = X[ok ? c0 + j + (int64_t)c * ldx : 0];
    }
  };
  auto put = [&](int buf, int64_t J, const double (&v)[kPer], const double (&xv)[kPerX]) {
    const int64_t c0 = J * BS;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + NT * q;
      const int i = (J <= I) ? e % BS : e / BS, j = (J <= I) ? e / BS : e % BS;
      const int64_t gi = r0 + i, gj = c0 + j;
      const bool ok = gi < n && gj < n && gi != gj;
      Ab[buf][i][j] = ok ? (gi > gj ? v[q] : -v[q]) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kPerX; ++q) {
      const int e = tid + NT * q;
      const int j = e % BS, c = e / BS;
      xs[buf][j][c] = (c0 + j < n && c < nr) ? xv[q] : 0.0;
    }
  };
  double v[kPer], xv[kPerX];
  fetch(0, v, xv);
  put(0, 0, v, xv);
  __syncthreads();
  for (int64_t J = 0; J < nb; ++J) {
    const int buf = (int)(J & 1);
    const bool more = J + 1 < nb;
    if (more) fetch(J + 1, v, xv);
#pragma unroll 8
    for (int j = 0; j < BS; ++j) {
      const double a = Ab[buf][mi][j];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] -= a * xs[buf][j][4 * g + q];
    }
    if (rowabs && g == 0) {
      double sa = 0.0;
      for (int j = 0; j < BS; ++j) sa += fabs(Ab[buf][mi][j]);
      ra += sa;
    }
    if (more) put(buf ^ 1, J + 1, v, xv);  // the other half was last read before the previous barrier
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = 4 * g + q;
    if (mi < bs && c < nr) R[r0 + mi + (int64_t)c * ldr] = acc[q];
  }
  if (rowabs && g == 0 && mi < bs) rowabs[r0 + mi] = ra;
}

// out[3c + {0,1,2}] = max_i |R[i,c]|, max_i |X[i,c]|, max_i |B[i,c]|; out[3 nrhs] = max rowabs.
__global__ void colmax_kernel(int64_t n, int64_t nrhs, const double* __restrict__ R, int64_t ldr,
                              const double* __restrict__ X, int64_t ldx, const double* __restrict__ B, int64_t ldb,
                              const double* __restrict__ rowabs, double* __restrict__ out) {
  __shared__ double red[256];
  const int64_t c = blockIdx.x;
  for (int which = 0; which < 4; ++which) {
    if (which == 3 && c != 0) break;
    double m = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
      double v;
      if (which == 0) v = R[i + c * ldr];
      else if (which == 1) v = X[i + c * ldx];
      else if (which == 2) v = B[i + c * ldb];
      else v = rowabs ? rowabs[i] : 0.0;
      v = fabs(v);
      m = (v > m || v != v) ? v : m;  // NaN propagates
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (threadIdx.x < s) {
        const double o = red[threadIdx.x + s];
        if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) out[which < 3 ? 3 * c + which : 3 * nrhs] = red[0];
    __syncthreads();
  }
}

// X += D (n x nrhs)
__global__ void axpy_kernel(int64_t n, int64_t nrhs, const double* __restrict__ D, int64_t ldd,
                            double* __restrict__ X, int64_t ldx) {
  const int64_t c = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    X[i + c * ldx] += D[i + c * ldd];
}

// Y = B (n x nrhs)
__global__ void copy_cols_kernel(int64_t n, const double* __restrict__ B, int64_t ldb, double* __restrict__ Y,
                                 int64_t ldy) {
  const int64_t c = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Y[i + c * ldy] = B[i + c * ldb];
}

// ---- GMRES building blocks (n x nrhs blocks, leading dimension n) ----

// Y = alpha X
__global__ void scale_copy_kernel(int64_t n, double alpha, const double* X, double* Y) {  // X may be Y
  const int64_t c = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Y[i + c * n] = alpha * X[i + c * n];
}

// h[i * nrhs + c] = V_i[:, c] . w[:, c] for i < nvec (fixed-order reduction)
__global__ void __launch_bounds__(256) dots_kernel(int64_t n, int64_t nrhs, const double* __restrict__ V,
                                                   const double* __restrict__ w, double* __restrict__ h) {
  __shared__ double red[256];
  const int64_t i = blockIdx.x, c = blockIdx.y;
  const double* v = V + (i * nrhs + c) * n;
  const double* x = w + c * n;
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += 256) acc += v[r] * x[r];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) h[i * nrhs + c] = red[0];
}

// w[:, c] -= sum_{i < nvec} h[i * nrhs + c] V_i[:, c];  acc[i * nrhs + c] += h (if acc)
__global__ void gs_update_kernel(int64_t n, int64_t nrhs, int nvec, const double* __restrict__ V,
                                 const double* __restrict__ h, double* __restrict__ w) {
  const int64_t c = blockIdx.y;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    double s = w[r + c * n];
    for (int i = 0; i < nvec; ++i) s -= h[i * nrhs + c] * V[(i * nrhs + c) * n + r];
    w[r + c * n] = s;
  }
}

// v[:, c] = w[:, c] / nrm[c] (0 if nrm[c] == 0)
__global__ void normalize_kernel(int64_t n, const double* __restrict__ nrm, const double* __restrict__ w,
                                 double* __restrict__ v) {
  const int64_t c = blockIdx.y;
  const double d = nrm[c];
  const double inv = d > 0.0 ? 1.0 / d : 0.0;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    v[r + c * n] = w[r + c * n] * inv;
}

// ||w[:, c]||_2
__global__ void __launch_bounds__(256) norm2_kernel(int64_t n, const double* __restrict__ w, double* __restrict__ out) {
  __shared__ double red[256];
  const int64_t c = blockIdx.y;
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += 256) acc += w[r + c * n] * w[r + c * n];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = sqrt(red[0]);
}

// X[:, c] += sum_{i < nvec} y[i * nrhs + c] V_i[:, c]
__global__ void combine_kernel(int64_t n, int64_t nrhs, int nvec, const double* __restrict__ V,
                               const double* __restrict__ y, double* __restrict__ X, int64_t ldx) {
  const int64_t c = blockIdx.y;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < nvec; ++i) s += y[i * nrhs + c] * V[(i * nrhs + c) * n + r];
    X[r + c * ldx] += s;
  }
}

constexpr int kGmresM = 30;  // Krylov dimension per restart

}  // namespace

// workspace: solve ws | R (n*nrhs) | rowabs (n) | colmax (3 nrhs + 1) | info (int)
//            | GMRES: V ((M+1) n nrhs) | W (n nrhs) | h ((M+1) nrhs) | nrm (nrhs) | y (M nrhs)
static size_t gmres_bytes(int64_t n, int64_t nrhs) {
  const size_t nn = (size_t)std::max<int64_t>(n, 1) * std::max<int64_t>(nrhs, 1);
  const size_t r = (size_t)std::max<int64_t>(nrhs, 1);
  return align_up(sizeof(double) * nn * (kGmresM + 1), 256) + align_up(sizeof(double) * nn, 256) +
         align_up(sizeof(double) * r * (kGmresM + 1), 256) + align_up(sizeof(double) * r, 256) +
         align_up(sizeof(double) * r * kGmresM, 256);
}

size_t refine_workspace_bytes(int64_t n, int64_t nrhs) {
  return align_up(solve_workspace_bytes(n, nrhs), 256) + align_up(sizeof(double) * (size_t)std::max<int64_t>(n, 1) * std::max<int64_t>(nrhs, 1), 256) +
         align_up(sizeof(double) * (size_t)std::max<int64_t>(n, 1), 256) + align_up(sizeof(double) * (size_t)(3 * nrhs + 1), 256) + 256 +
         gmres_bytes(n, nrhs);
}

int launch_residual(int64_t n, int64_t nrhs, const double* A0, int64_t lda0, const double* X, int64_t ldx,
                    const double* B, int64_t ldb, double* R, int64_t ldr, double* rowabs, hipStream_t s) {
  const int64_t nb = (n + BS - 1) / BS;
  for (int64_t c0 = 0; c0 < nrhs; c0 += RC) {
    const int nr = (int)std::min<int64_t>(RC, nrhs - c0);
    hipLaunchKernelGGL(residual_kernel, dim3((unsigned)nb), dim3(NT), 0, s, n, nr, A0, lda0, X + c0 * ldx, ldx,
                       B ? B + c0 * ldb : nullptr, ldb, R + c0 * ldr, ldr, (c0 == 0) ? rowabs : nullptr);
    SKF_CHECK_LAUNCH("residual");
  }
  return 0;
}

// X += d with d an approximate solution of A d = R (R = B - A X on entry), by
// left-preconditioned GMRES with the factors (one cycle of at most kGmresM
// steps, stopping once every column's preconditioned residual estimate has
// dropped by rtol).  g points at the GMRES part of the refinement workspace.
static int gmres_correct(int64_t n, int64_t nrhs, const double* A0, int64_t lda0, const double* LT, int64_t lda,
                         const int32_t* ipiv, const double* T, const double* R, double* X, int64_t ldx, void* swork,
                         size_t sw, int* dinfo, char* g, double rtol, hipStream_t s) {
  constexpr int M = kGmresM;
  const size_t nn = (size_t)n * nrhs;
  double* V = (double*)g;
  double* W = (double*)(g + align_up(sizeof(double) * nn * (M + 1), 256));
  double* hd = (double*)((char*)W + align_up(sizeof(double) * nn, 256));
  double* nrm = (double*)((char*)hd + align_up(sizeof(double) * nrhs * (M + 1), 256));
  double* yd = (double*)((char*)nrm + align_up(sizeof(double) * nrhs, 256));
  const unsigned gx = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
  const dim3 grid2(gx, (unsigned)nrhs);
  int rc;
  // z = M^{-1} r, beta = ||z||, v_0 = z / beta
  hipLaunchKernelGGL(scale_copy_kernel, grid2, dim3(256), 0, s, n, 1.0, R, W);
  SKF_CHECK_LAUNCH("gmres copy");
  if ((rc = run_solve(n, nrhs, LT, lda, ipiv, T, W, n, swork, sw, dinfo, s))) return rc;
  hipLaunchKernelGGL(norm2_kernel, dim3(1, (unsigned)nrhs), dim3(256), 0, s, n, W, nrm);
  hipLaunchKernelGGL(normalize_kernel, grid2, dim3(256), 0, s, n, nrm, W, V);
  SKF_CHECK_LAUNCH("gmres start");
  std::vector<double> beta0((size_t)nrhs), hn((size_t)nrhs), h1((size_t)nrhs * M), h2((size_t)nrhs * M);
  SKF_CHECK(hipMemcpyAsync(beta0.data(), nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s), "gmres beta");
  SKF_CHECK(hipStreamSynchronize(s), "sync");
  // per column c: R factor of the Hessenberg matrix (column-major, (M+1) x M),
  // Givens rotations, and the rotated right-hand side beta e_1
  std::vector<double> H((size_t)nrhs * (M + 1) * M, 0.0), cs((size_t)nrhs * M), sn((size_t)nrhs * M),
      gv((size_t)nrhs * (M + 1), 0.0);
  for (int64_t c = 0; c < nrhs; ++c) gv[(size_t)c * (M + 1)] = beta0[c];
  int k = 0;
  for (int j = 0; j < M; ++j) {
    const double* vj = V + (size_t)j * nn;
    // w = M^{-1} A v_j   (the residual kernel gives -A v_j for a zero right-hand side)
    if ((rc = launch_residual(n, nrhs, A0, lda0, vj, n, nullptr, n, W, n, nullptr, s))) return rc;
    hipLaunchKernelGGL(scale_copy_kernel, grid2, dim3(256), 0, s, n, -1.0, W, W);
    SKF_CHECK_LAUNCH("gmres negate");
    if ((rc = run_solve(n, nrhs, LT, lda, ipiv, T, W, n, swork, sw, dinfo, s))) return rc;
    // classical Gram-Schmidt, twice
    hipLaunchKernelGGL(dots_kernel, dim3((unsigned)(j + 1), (unsigned)nrhs), dim3(256), 0, s, n, nrhs, V, W, hd);
    hipLaunchKernelGGL(gs_update_kernel, grid2, dim3(256), 0, s, n, nrhs, j + 1, V, hd, W);
    hipLaunchKernelGGL(dots_kernel, dim3((unsigned)(j + 1), (unsigned)nrhs), dim3(256), 0, s, n, nrhs, V, W, yd);
    hipLaunchKernelGGL(gs_update_kernel, grid2, dim3(256), 0, s, n, nrhs, j + 1, V, yd, W);
    hipLaunchKernelGGL(norm2_kernel, dim3(1, (unsigned)nrhs), dim3(256), 0, s, n, W, nrm);
    hipLaunchKernelGGL(normalize_kernel, grid2, dim3(256), 0, s, n, nrm, W, V + (size_t)(j + 1) * nn);
    SKF_CHECK_LAUNCH("gmres arnoldi");
    SKF_CHECK(hipMemcpyAsync(h1.data(), hd, sizeof(double) * nrhs * (j + 1), hipMemcpyDeviceToHost, s), "h1");
    SKF_CHECK(hipMemcpyAsync(h2.data(), yd, sizeof(double) * nrhs * (j + 1), hipMemcpyDeviceToHost, s), "h2");
    SKF_CHECK(hipMemcpyAsync(hn.data(), nrm, sizeof(double) * nrhs, hipMemcpyDeviceToHost, s), "hn");
    SKF_CHECK(hipStreamSynchronize(s), "sync");
    k = j + 1;
    bool done = true;
    for (int64_t c = 0; c < nrhs; ++c) {
      double* Hc = H.data() + (size_t)c * (M + 1) * M + (size_t)j * (M + 1);
      for (int i = 0; i <= j; ++i) Hc[i] = h1[(size_t)i * nrhs + c] + h2[(size_t)i * nrhs + c];
      Hc[j + 1] = hn[c];
      double* csc = cs.data() + (size_t)c * M;
      double* snc = sn.data() + (size_t)c * M;
      for (int i = 0; i < j; ++i) {  // earlier rotations
        const double a = Hc[i], b = Hc[i + 1];
        Hc[i] = csc[i] * a + snc[i] * b;
        Hc[i + 1] = -snc[i] * a + csc[i] * b;
      }
      const double a = Hc[j], b = Hc[j + 1];
      const double r = std::hypot(a, b);
      csc[j] = r > 0.0 ? a / r : 1.0;
      snc[j] = r > 0.0 ? b / r : 0.0;
      Hc[j] = r;
      Hc[j + 1] = 0.0;
      double* gc = gv.data() + (size_t)c * (M + 1);
      gc[j + 1] = -snc[j] * gc[j];
      gc[j] = csc[j] * gc[j];
      if (!(std::fabs(gc[j + 1]) <= rtol * beta0[c])) done = false;
    }
    if (done) break;
  }
  // y = R^{-1} g per column (back substitution), X += V y
  std::vector<double> y((size_t)nrhs * M, 0.0);
  for (int64_t c = 0; c < nrhs; ++c) {
    const double* Hc = H.data() + (size_t)c * (M + 1) * M;
    const double* gc = gv.data() + (size_t)c * (M + 1);
    for (int i = k - 1; i >= 0; --i) {
      double t = gc[i];
      for (int l = i + 1; l < k; ++l) t -= Hc[(size_t)l * (M + 1) + i] * y[(size_t)l * nrhs + c];
      const double d = Hc[(size_t)i * (M + 1) + i];
      y[(size_t)i * nrhs + c] = d != 0.0 ? t / d : 0.0;
    }
  }
  SKF_CHECK(hipMemcpyAsync(yd, y.data(), sizeof(double) * nrhs * k, hipMemcpyHostToDevice, s), "y");
  hipLaunchKernelGGL(combine_kernel, grid2, dim3(256), 0, s, n, nrhs, k, V, yd, X, ldx);
  SKF_CHECK_LAUNCH("gmres update");
  SKF_CHECK(hipStreamSynchronize(s), "sync");  // y lives on this host stack frame
  return 0;
}

int run_refine(int64_t n, int64_t nrhs, const double* A0, int64_t lda0, const double* LT, int64_t lda,
               const int32_t* ipiv, const double* T, const double* B, int64_t ldb, double* X, int64_t ldx,
               double tol, int maxit, int* iters, double* berr, void* work, size_t lwork, hipStream_t s) {
  const size_t sw = align_up(solve_workspace_bytes(n, nrhs), 256);
  if (lwork < refine_workspace_bytes(n, nrhs)) return SKF_EWORK;
  char* base = (char*)work;
  double* R = (double*)(base + sw);
  double* rowabs = (double*)((char*)R + align_up(sizeof(double) * (size_t)std::max<int64_t>(n, 1) * std::max<int64_t>(nrhs, 1), 256));
  double* cm = (double*)((char*)rowabs + align_up(sizeof(double) * (size_t)std::max<int64_t>(n, 1), 256));
  int* dinfo = (int*)((char*)cm + align_up(sizeof(double) * (size_t)(3 * nrhs + 1), 256));
  if (iters) *iters = 0;
  if (berr) *berr = 0.0;
  if (n == 0 || nrhs == 0) return 0;
  const unsigned gx = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
  int rc;
  // X_0 = solve(B)
  hipLaunchKernelGGL(copy_cols_kernel, dim3(gx, (unsigned)nrhs), dim3(256), 0, s, n, B, ldb, X, ldx);
  SKF_CHECK_LAUNCH("copy");
  if ((rc = run_solve(n, nrhs, LT, lda, ipiv, T, X, ldx, work, sw, dinfo, s))) return rc;
  int hinfo = 0;
  SKF_CHECK(hipMemcpyAsync(&hinfo, dinfo, sizeof(int), hipMemcpyDeviceToHost, s), "info");
  SKF_CHECK(hipStreamSynchronize(s), "sync");
  if (hinfo != 0) return hinfo;
  std::vector<double> h((size_t)(3 * nrhs + 1));
  double eta = 0.0, eta_prev = INFINITY;
  bool gmres = false;
  char* gbase = (char*)dinfo + 256;
  int it = 0;
  for (;; ++it) {
    if ((rc = launch_residual(n, nrhs, A0, lda0, X, ldx, B, ldb, R, n, (it == 0) ? rowabs : nullptr, s))) return rc;
    hipLaunchKernelGGL(colmax_kernel, dim3((unsigned)nrhs), dim3(256), 0, s, n, nrhs, R, n, X, ldx, B, ldb, rowabs,
                       cm);
    SKF_CHECK_LAUNCH("colmax");
    SKF_CHECK(hipMemcpyAsync(h.data(), cm, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s), "colmax copy");
    SKF_CHECK(hipStreamSynchronize(s), "sync");
    const double anorm = h[3 * nrhs];
    eta = 0.0;
    for (int64_t c = 0; c < nrhs; ++c) {
      const double den = anorm * h[3 * c + 1] + h[3 * c + 2];
      const double e = (den > 0.0) ? h[3 * c] / den : (h[3 * c] > 0.0 ? INFINITY : 0.0);
      if (!(e <= eta)) eta = e;  // NaN-safe max
    }
    if (eta <= tol || it >= maxit) break;
    if (it >= 1 && !(eta <= 0.5 * eta_prev)) gmres = true;  // plain refinement does not contract
    eta_prev = eta;
    if (gmres) {
      if ((rc = gmres_correct(n, nrhs, A0, lda0, LT, lda, ipiv, T, R, X, ldx, work, sw, dinfo, gbase, 1e-10, s)))
        return rc;
    } else {
      if ((rc = run_solve(n, nrhs, LT, lda, ipiv, T, R, n, work, sw, dinfo, s))) return rc;
      hipLaunchKernelGGL(axpy_kernel, dim3(gx, (unsigned)nrhs), dim3(256), 0, s, n, nrhs, R, n, X, ldx);
      SKF_CHECK_LAUNCH("axpy");
    }
  }
  if (iters) *iters = it;
  if (berr) *berr = eta;
  return (eta <= tol) ? 0 : 1;
}

}  // namespace skf
