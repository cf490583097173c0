// Pfaffian ratio of a low-rank skew update with resident factors.
//
// For B = A + U V^T - V U^T (U, V: n x r) write B = A + W J W^T with W = [U V]
// (n x 2r) and J = [[0, I_r], [-I_r, 0]].  The Pfaffian of a bordered skew
// matrix [[A, W], [-W^T, D]] with A and D invertible expands by either Schur
// complement:  Pf(A) Pf(D + W^T A^-1 W) = Pf(D) Pf(A + W D^-1 W^T).
// With D = J^-1 = -J the right-hand matrix is B, so
//     Pf(B) / Pf(A) = Pf(K) / Pf(-J),   K = W^T A^-1 W - J,   Pf(-J) = (-1)^{r(r+1)/2}.
// One solve with the 2r columns of W through the factors of A, a 2r x 2r Gram
// product and a 2r x 2r Pfaffian replace the factorization of B.
//
// Kernels: pack W into the solve's right-hand sides; one workgroup per entry of
// the strict lower triangle of W^T X (X = A^-1 W), a dot product of two columns
// with a fixed-order tree reduction; one wave forms K in LDS and reduces it by
// pivoted elimination at even steps (the Pfaffian-only reduction).
#include <math.h>

#include "skf_internal.h"

namespace skf {


namespace {

constexpr int kMaxM = 2 * 32;  // 2r for the largest supported r

__host__ __device__ inline int npairs_of(int m) { return m * (m - 1) / 2; }

// X[:, c] = U[:, c] for c < r, V[:, c - r] otherwise (X: n x 2r, ld n).
__global__ void pack_kernel(int64_t n, int r, const double* __restrict__ U, int64_t ldu,
                            const double* __restrict__ V, int64_t ldv, double* __restrict__ X) {
  const int c = blockIdx.y;
  const double* src = (c < r) ? U + (int64_t)c * ldu : V + (int64_t)(c - r) * ldv;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    X[i + (int64_t)c * n] = src[i];
}

// Pair p of the strict lower triangle of an m x m matrix, row-major over rows:
// p = a (a - 1) / 2 + b with 0 <= b < a.
__device__ inline void pair_ab(int p, int* a, int* b) {
  int x = (int)((1.0 + sqrt(1.0 + 8.0 * (double)p)) * 0.5);
  while (x * (x - 1) / 2 > p) --x;
  while ((x + 1) * x / 2 <= p) ++x;
  *a = x;
  *b = p - x * (x - 1) / 2;
}

// G[p] = W[:, a] . X[:, b] for pair p = (a, b), a > b: one workgroup per pair.
__global__ void __launch_bounds__(256) gram_kernel(int64_t n, int r, const double* __restrict__ U, int64_t ldu,
                                                   const double* __restrict__ V, int64_t ldv,
                                                   const double* __restrict__ X, double* __restrict__ G) {
  __shared__ double red[256];
  int a, b;
  pair_ab((int)blockIdx.x, &a, &b);
  const double* __restrict__ w = (a < r) ? U + (int64_t)a * ldu : V + (int64_t)(a - r) * ldv;
  const double* __restrict__ x = X + (int64_t)b * n;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t i = threadIdx.x;
  for (; i + 768 < n; i += 1024) {
    s0 += w[i] * x[i];
    s1 += w[i + 256] * x[i + 256];
    s2 += w[i + 512] * x[i + 512];
    s3 += w[i + 768] * x[i + 768];
  }
  for (; i < n; i += 256) s0 += w[i] * x[i];
  red[threadIdx.x] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) G[blockIdx.x] = red[0];
}

// One wave: K = W^T X - J in LDS, then its Pfaffian by pivoted
// elimination at even steps; out: log|ratio|, sign.  solve_info != 0 (A singular)
// or a non-finite K leave logabs = NaN, sign = 0 and the outcome in *dinfo.
__global__ void __launch_bounds__(64) ratio_final_kernel(int r, const double* __restrict__ G,
                                                         const int* __restrict__ solve_info, double* logabs,
                                                         int* sign, int* dinfo) {
  __shared__ double K[kMaxM][kMaxM + 1];
  __shared__ double lv[2][kMaxM];
  __shared__ int bad;
  const int t = threadIdx.x;
  const int m = 2 * r;
  const int np = npairs_of(m);
  if (t == 0) bad = 0;
  __syncthreads();
  for (int p = t; p < np; p += blockDim.x) {
    int a, b;
    pair_ab(p, &a, &b);
    // J[a][b] (a > b) is -1 at a = b + r, else 0
    const double k = G[p] + ((a == b + r) ? 1.0 : 0.0);
    if (!isfinite(k)) atomicOr(&bad, 1);
    K[a][b] = k;
    K[b][a] = -k;
  }
  if (t < m) K[t][t] = 0.0;
  __syncthreads();
  const int st = *solve_info;
  if (st != 0 || bad) {
    if (t == 0) {
      *logabs = NAN;
      *sign = 0;
      *dinfo = (st != 0) ? st : SKF_ENONFINITE;
    }
    return;
  }
  double la = 0.0;
  int sg = 1, swaps = 0;
  for (int k = 0; k + 1 < m; k += 2) {
    // pivot: largest |K[i][k]|, i > k, lowest index on ties (one lane; m <= 64)
    int p = k + 1;
    if (t == 0) {
      double best = fabs(K[k + 1][k]);
      for (int i = k + 2; i < m; ++i)
        if (fabs(K[i][k]) > best) {
          best = fabs(K[i][k]);
          p = i;
        }
      lv[0][0] = (double)p;
    }
    __syncthreads();
    p = (int)lv[0][0];
    __syncthreads();
    if (p != k + 1) {
      ++swaps;
      if (t < m) {  // columns, then rows
        const double x = K[t][k + 1];
        K[t][k + 1] = K[t][p];
        K[t][p] = x;
      }
      __syncthreads();
      if (t < m) {
        const double x = K[k + 1][t];
        K[k + 1][t] = K[p][t];
        K[p][t] = x;
      }
      __syncthreads();
    }
    const double alpha = K[k + 1][k];
    if (alpha == 0.0) {
      sg = 0;
      la = -INFINITY;
      break;
    }
    la += log(fabs(alpha));
    if (alpha < 0.0) sg = -sg;
    if (t >= k + 2 && t < m) {
      lv[0][t] = K[t][k] / alpha;
      lv[1][t] = K[t][k + 1];
    }
    __syncthreads();
    if (t >= k + 2 && t < m)
      for (int j = k + 2; j < m; ++j) K[t][j] += lv[0][t] * lv[1][j] - lv[1][t] * lv[0][j];
    __syncthreads();
  }
  if (t == 0) {
    // Pf(K) = (-1)^{swaps + m/2} prod alpha; the ratio divides by Pf(-J) = (-1)^{r(r+1)/2}
    const int par = (swaps + r + r * (r + 1) / 2) & 1;
    *logabs = la;
    *sign = (sg == 0) ? 0 : (par ? -sg : sg);
    *dinfo = 0;
  }
}

struct RatioWork {
  double* X;
  double* G;
  int* solve_info;
  void* solve_work;
  size_t solve_bytes;
  size_t bytes;
};

RatioWork ratio_carve(void* base, int64_t n, int r) {
  RatioWork w{};
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = align_up(off + b, 256);
    return base ? (void*)((char*)base + o) : nullptr;
  };
  const int m = 2 * r;
  w.X = (double*)take(sizeof(double) * (size_t)std::max<int64_t>(n * m, 1));
  w.G = (double*)take(sizeof(double) * (size_t)std::max(npairs_of(m), 1));
  w.solve_info = (int*)take(256);
  w.solve_bytes = solve_workspace_bytes(n, m);
  w.solve_work = take(w.solve_bytes);
  w.bytes = off;
  return w;
}

}  // namespace

int pf_ratio_max_rank() { return kMaxM / 2; }

size_t pf_ratio_workspace_bytes(int64_t n, int r) { return ratio_carve(nullptr, n, r).bytes; }

int run_pf_ratio(int64_t n, int r, const double* LT, int64_t lda, const int32_t* ipiv, const double* T,
                 const double* U, int64_t ldu, const double* V, int64_t ldv, double* logabs, int* sign,
                 void* work, size_t lwork, int* dinfo, hipStream_t s) {
  RatioWork w = ratio_carve(work, n, r);
  if (lwork < w.bytes) return SKF_EWORK;
  const int m = 2 * r;
  int rc;
  if (n > 0 && m > 0) {
    const unsigned gx = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(pack_kernel, dim3(gx, (unsigned)m), dim3(256), 0, s, n, r, U, ldu, V, ldv, w.X);
    SKF_CHECK_LAUNCH("ratio pack");
  }
  // X = A^-1 W (and the singularity outcome of A's factors)
  if (n > 0) {
    if ((rc = run_solve(n, m, LT, lda, ipiv, T, w.X, n, w.solve_work, w.solve_bytes, w.solve_info, s)))
      return rc;
  } else if ((rc = launch_fill_i32(w.solve_info, 1, 0, s))) {
    return rc;
  }
  const int np = npairs_of(m);
  if (np > 0) {
    if (n > 0) {
      hipLaunchKernelGGL(gram_kernel, dim3((unsigned)np), dim3(256), 0, s, n, r, U, ldu, V, ldv, w.X, w.G);
      SKF_CHECK_LAUNCH("ratio gram");
    } else if ((rc = launch_fill_u64((uint64_t*)w.G, (size_t)np, 0, s))) {
      return rc;
    }
  }
  hipLaunchKernelGGL(ratio_final_kernel, dim3(1), dim3(64), 0, s, r, w.G, w.solve_info, logabs, sign, dinfo);
  SKF_CHECK_LAUNCH("ratio final");
  return 0;
}

}  // namespace skf
