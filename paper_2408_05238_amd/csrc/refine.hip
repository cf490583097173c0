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
#include <algorithm>
#include <vector>

#include "skf_internal.h"

namespace skf {

int run_solve(int64_t n, int64_t nrhs, const double* LT, int64_t lda, const int32_t* ipiv, const double* T,
              double* B, int64_t ldb, void* work, size_t lwork, int* dinfo, hipStream_t s);
size_t solve_workspace_bytes(int64_t n, int64_t nrhs);

namespace {

constexpr int BS = 64;
constexpr int RC = 16;
constexpr int NT = 256;

// R[:, c0:c0+nr] = B - S X (rows of block I = blockIdx.x); optionally also the
// absolute row sums of S (||A0||_inf = max of them).
__global__ void __launch_bounds__(NT) residual_kernel(int64_t n, int nr, const double* __restrict__ A0, int64_t lda,
                                                      const double* __restrict__ X, int64_t ldx,
                                                      const double* __restrict__ B, int64_t ldb,
                                                      double* __restrict__ R, int64_t ldr,
                                                      double* __restrict__ rowabs) {
  __shared__ double Ab[BS][BS + 1];
  __shared__ double xs[BS][RC + 1];
  __shared__ double acc[BS][RC + 1];
  __shared__ double ra[BS];
  const int64_t nb = (n + BS - 1) / BS;
  const int64_t I = blockIdx.x;
  const int64_t r0 = I * BS;
  const int bs = (int)min((int64_t)BS, n - r0);
  const int tid = threadIdx.x;
  for (int t = tid; t < BS * RC; t += NT) {
    const int i = t % BS, c = t / BS;
    acc[i][c] = (i < bs && c < nr) ? B[r0 + i + (int64_t)c * ldb] : 0.0;
  }
  if (tid < BS) ra[tid] = 0.0;
  for (int64_t J = 0; J < nb; ++J) {
    const int64_t c0 = J * BS;
    const int cs = (int)min((int64_t)BS, n - c0);
    __syncthreads();
    // S_IJ: J < I stored block (I, J); J > I -(stored block (J, I))^T; J == I skew diagonal block
    for (int t = tid; t < BS * BS; t += NT) {
      // consecutive threads walk down a stored column in both orientations
      const int i = (J <= I) ? t % BS : t / BS, j = (J <= I) ? t / BS : t % BS;
      double v = 0.0;
      if (i < bs && j < cs) {
        const int64_t gi = r0 + i, gj = c0 + j;
        if (gi > gj) v = A0[gi + gj * lda];
        else if (gi < gj) v = -A0[gj + gi * lda];
      }
      Ab[i][j] = v;
    }
    for (int t = tid; t < BS * RC; t += NT) {
      const int j = t % BS, c = t / BS;
      xs[j][c] = (j < cs && c < nr) ? X[c0 + j + (int64_t)c * ldx] : 0.0;
    }
    __syncthreads();
    for (int t = tid; t < BS * RC; t += NT) {
      const int i = t % BS, c = t / BS;
      double sum = 0.0;
#pragma unroll 8
      for (int j = 0; j < BS; ++j) sum += Ab[i][j] * xs[j][c];
      acc[i][c] -= sum;
    }
    if (rowabs && tid < BS) {
      double sa = 0.0;
      for (int j = 0; j < BS; ++j) sa += fabs(Ab[tid][j]);
      ra[tid] += sa;
    }
  }
  __syncthreads();
  for (int t = tid; t < BS * RC; t += NT) {
    const int i = t % BS, c = t / BS;
    if (i < bs && c < nr) R[r0 + i + (int64_t)c * ldr] = acc[i][c];
  }
  if (rowabs && tid < bs) rowabs[r0 + tid] = ra[tid];
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

}  // namespace

// workspace: solve ws | R (n*nrhs) | rowabs (n) | colmax (3 nrhs + 1) | info (int)
size_t refine_workspace_bytes(int64_t n, int64_t nrhs) {
  return align_up(solve_workspace_bytes(n, nrhs), 256) + align_up(sizeof(double) * (size_t)std::max<int64_t>(n, 1) * std::max<int64_t>(nrhs, 1), 256) +
         align_up(sizeof(double) * (size_t)std::max<int64_t>(n, 1), 256) + align_up(sizeof(double) * (size_t)(3 * nrhs + 1), 256) + 256;
}

int launch_residual(int64_t n, int64_t nrhs, const double* A0, int64_t lda0, const double* X, int64_t ldx,
                    const double* B, int64_t ldb, double* R, int64_t ldr, double* rowabs, hipStream_t s) {
  const int64_t nb = (n + BS - 1) / BS;
  for (int64_t c0 = 0; c0 < nrhs; c0 += RC) {
    const int nr = (int)std::min<int64_t>(RC, nrhs - c0);
    hipLaunchKernelGGL(residual_kernel, dim3((unsigned)nb), dim3(NT), 0, s, n, nr, A0, lda0, X + c0 * ldx, ldx,
                       B + c0 * ldb, ldb, R + c0 * ldr, ldr, (c0 == 0) ? rowabs : nullptr);
    SKF_CHECK_LAUNCH("residual");
  }
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
  double eta = 0.0;
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
    if ((rc = run_solve(n, nrhs, LT, lda, ipiv, T, R, n, work, sw, dinfo, s))) return rc;
    hipLaunchKernelGGL(axpy_kernel, dim3(gx, (unsigned)nrhs), dim3(256), 0, s, n, nrhs, R, n, X, ldx);
    SKF_CHECK_LAUNCH("axpy");
  }
  if (iters) *iters = it;
  if (berr) *berr = eta;
  return (eta <= tol) ? 0 : 1;
}

}  // namespace skf
