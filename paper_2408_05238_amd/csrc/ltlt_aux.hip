// Data-movement and reduction kernels around the blocked skew LTL^T:
// scratch fills, panel L write-back, composition of the panels' permutations,
// the final row-permuted copy of L, the status/info word and the Pfaffian
// reduction from (ipiv, T).  All are HBM-bound O(n^2) or smaller.
#include "skf_internal.h"

namespace skf {
namespace {

__global__ void fill_u64_kernel(uint64_t* p, size_t count, uint64_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_i32_kernel(int32_t* p, size_t count, int32_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void iota_i32_kernel(int32_t* p, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = (int32_t)i;
}

// W[i, k0+c] = Lbuf[i, c] for rows below the subdiagonal of column k0+c.
__global__ void copy_panel_L_kernel(int64_t n, int64_t k0, int nsteps, const double* __restrict__ Lbuf,
                                    double* __restrict__ W, int64_t ldw) {
  const int c = blockIdx.y;
  const int64_t col = k0 + c;
  for (int64_t i = col + 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    W[i + col * ldw] = Lbuf[i + (int64_t)c * n];
}

// sigma[P][i] = pi_{P+1}(pi_{P+2}(... pi_{last}(i))): the row of panel P's
// output order that ends up at final row i.
__global__ void compose_sigma_kernel(int64_t n, int npanels, const int32_t* __restrict__ pis,
                                     int32_t* __restrict__ sigma) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t x = i;
    for (int P = npanels - 1; P >= 0; --P) {
      sigma[(int64_t)P * n + i] = (int32_t)x;
      x = pis[(int64_t)P * n + x];
    }
  }
}

// A[i, c] = W[sigma_P(i), c] for i > c, P = panel of column c.  The reads of a
// column are scattered by the permutation, so all kFinalSubs workgroups of one
// column run on one XCD (workgroups are dealt to the eight XCDs round-robin by
// linear index): index g 8 kFinalSubs + s 8 + cc -> column 8 g + cc, part s; the
// column's cache lines are then fetched into one L2 only.
constexpr int kFinalSubs = 32;
__global__ void final_L_kernel(int64_t n, int nb, const double* __restrict__ W, int64_t ldw,
                               const int32_t* __restrict__ sigma, double* __restrict__ A, int64_t lda) {
  const int64_t id = blockIdx.x;
  const int64_t g = id / (8 * kFinalSubs), rem = id % (8 * kFinalSubs);
  const int sub = (int)(rem / 8);
  const int64_t c = 8 * g + rem % 8;
  if (c >= n - 1) return;
  const int64_t P = c / nb;
  const int32_t* sg = sigma + P * n;
  for (int64_t i = c + 1 + (int64_t)sub * blockDim.x + threadIdx.x; i < n; i += (int64_t)kFinalSubs * blockDim.x)
    A[i + c * lda] = W[(int64_t)sg[i] + c * ldw];
}

// dinfo = status if nonzero, else 1 + (first even k with T[k] == 0), else 0.
__global__ void ltlt_info_kernel(int64_t n, const double* __restrict__ T, const int* __restrict__ status,
                                 int* __restrict__ dinfo) {
  __shared__ int64_t best[256];
  int64_t b = INT64_MAX;
  for (int64_t k = 2 * threadIdx.x; k + 1 < n; k += 2 * blockDim.x)
    if (T[k] == 0.0) {
      b = k;
      break;
    }
  best[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) best[threadIdx.x] = min(best[threadIdx.x], best[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int st = status ? *status : 0;
    *dinfo = st != 0 ? st : (best[0] == INT64_MAX ? 0 : (int)(best[0] + 1));
  }
}

// log|Pf| = sum_{k even} log|T[k]| in a fixed order (contiguous chunks per
// thread, then a fixed tree), sign = (-1)^{s + n/2} prod sgn(T[k even]).
__global__ void logpf_kernel(int64_t n, const int32_t* __restrict__ ipiv, const double* __restrict__ T,
                             double* logabs, int* sign, double* pf) {
  __shared__ double ssum[256];
  __shared__ int sneg[256];
  __shared__ int szero[256];
  const int t = threadIdx.x;
  const int64_t npairs = n / 2;
  const int64_t chunk = (npairs + 255) / 256;
  double acc = 0.0;
  int neg = 0, zero = 0;
  if (n % 2 == 0) {
    for (int64_t q = t * chunk; q < min(npairs, (t + 1) * chunk); ++q) {
      const double v = T[2 * q];
      if (v == 0.0) zero = 1;
      if (v < 0.0) neg ^= 1;
      acc += log(fabs(v));
    }
  }
  int swaps = 0;
  for (int64_t j = t; j < n; j += 256) swaps ^= (ipiv[j] != (int32_t)j) ? 1 : 0;
  ssum[t] = acc;
  sneg[t] = neg ^ swaps;
  szero[t] = zero;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      ssum[t] = ssum[t] + ssum[t + s];
      sneg[t] ^= sneg[t + s];
      szero[t] |= szero[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    double la;
    int sg;
    if (n == 0) {
      la = 0.0;
      sg = 1;
    } else if (n % 2 == 1 || szero[0]) {
      la = -INFINITY;
      sg = 0;
    } else {
      la = ssum[0];
      sg = ((sneg[0] ^ (int)(npairs & 1)) & 1) ? -1 : 1;
    }
    if (logabs) *logabs = la;
    if (sign) *sign = sg;
    if (pf) *pf = (sg == 0) ? 0.0 : (double)sg * exp(la);
  }
}

}  // namespace

static unsigned grid_for(size_t count, unsigned block) {
  size_t g = (count + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g == 0) g = 1;
  return (unsigned)g;
}

int launch_fill_u64(uint64_t* p, size_t count, uint64_t v, hipStream_t s) {
  if (!count) return 0;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count, v);
  SKF_CHECK_LAUNCH("fill_u64");
  return 0;
}

int launch_iota_i32(int32_t* p, size_t count, hipStream_t s) {
  if (count == 0) return 0;
  hipLaunchKernelGGL(iota_i32_kernel, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count);
  SKF_CHECK_LAUNCH("iota_i32");
  return 0;
}

int launch_fill_i32(int32_t* p, size_t count, int32_t v, hipStream_t s) {
  if (!count) return 0;
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(count, 256)), dim3(256), 0, s, p, count, v);
  SKF_CHECK_LAUNCH("fill_i32");
  return 0;
}

int launch_copy_panel_L(int64_t n, int64_t k0, int nsteps, const double* Lbuf, double* W, int64_t ldw,
                        hipStream_t s) {
  if (nsteps <= 0) return 0;
  const int64_t rows = n - k0;
  dim3 grid(grid_for((size_t)rows, 256) > 64 ? 64 : grid_for((size_t)rows, 256), nsteps);
  hipLaunchKernelGGL(copy_panel_L_kernel, grid, dim3(256), 0, s, n, k0, nsteps, Lbuf, W, ldw);
  SKF_CHECK_LAUNCH("copy_panel_L");
  return 0;
}

int launch_compose_sigma(int64_t n, int npanels, const int32_t* pis, int32_t* sigma, hipStream_t s) {
  if (n <= 0 || npanels <= 0) return 0;
  hipLaunchKernelGGL(compose_sigma_kernel, dim3(grid_for((size_t)n, 256)), dim3(256), 0, s, n, npanels,
                     pis, sigma);
  SKF_CHECK_LAUNCH("compose_sigma");
  return 0;
}

int launch_final_L(int64_t n, int nb, int npanels, const double* W, int64_t ldw, const int32_t* sigma,
                   double* A, int64_t lda, hipStream_t s) {
  (void)npanels;
  if (n < 2) return 0;
  const int64_t groups = (n - 1 + 7) / 8;
  hipLaunchKernelGGL(final_L_kernel, dim3((unsigned)(groups * 8 * kFinalSubs)), dim3(256), 0, s, n, nb, W, ldw,
                     sigma, A, lda);
  SKF_CHECK_LAUNCH("final_L");
  return 0;
}

int launch_ltlt_info(int64_t n, const double* T, const int* status, int* dinfo, hipStream_t s) {
  hipLaunchKernelGGL(ltlt_info_kernel, dim3(1), dim3(256), 0, s, n, T, status, dinfo);
  SKF_CHECK_LAUNCH("ltlt_info");
  return 0;
}

int launch_logpf(int64_t n, const int32_t* ipiv, const double* T, double* logabs, int* sign, double* pf,
                 hipStream_t s) {
  hipLaunchKernelGGL(logpf_kernel, dim3(1), dim3(256), 0, s, n, ipiv, T, logabs, sign, pf);
  SKF_CHECK_LAUNCH("logpf");
  return 0;
}

}  // namespace skf
