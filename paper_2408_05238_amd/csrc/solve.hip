// Solve A X = B with the factors P A P^T = L T L^T:
//   X = P^T L^{-T} T^{-1} L^{-1} P B.
//
// Steps (all on the device, one stream):
//   perm   final row permutation from the interchanges: perm[j] = original row
//          at position j (each j traced back independently through the earlier
//          interchanges, so all j run in parallel);
//   gather Y = P B (workspace);
//   L^{-1} blocked forward substitution over 64-row blocks: the unit-lower
//          64 x 64 diagonal blocks are inverted first (all in parallel), then
//          block I accumulates -L_IJ Y_J as each Y_J is published (a tagged
//          per-block flag) and finishes with Y_I = inv(L_II) acc;
//   T^{-1} Gaussian elimination with partial pivoting on the tridiagonal
//          (sequential over rows, one lane per right-hand side);
//   L^{-T} the same blocked scheme from the last block upwards with the
//          transposed blocks;
//   scatter B[perm[i], :] = Z[i, :].
// L[i,j] (i > j >= 1) is read from LT[i, j-1]; L[:,0] = e_0.
#include <algorithm>

#include "skf_internal.h"

namespace skf {
namespace {

constexpr int BS = 64;        // row block of the triangular solves
constexpr int RC = 16;        // right-hand sides per pass
constexpr int NT = 256;

__device__ inline uint64_t ld_flag(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_flag(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
// Values published by other workgroups are read and written at agent scope.
__device__ inline double ld_agent(const double* p) {
  return __longlong_as_double((long long)__hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT));
}
__device__ inline void st_agent(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), (uint64_t)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
constexpr uint64_t kWaitTicks = 200000000ull;  // 2 s of the 100 MHz counter

// L element (i, j), i > j, from the factored array.
__device__ inline double Lij(const double* __restrict__ LT, int64_t lda, int64_t i, int64_t j) {
  return (j == 0) ? 0.0 : LT[i + (j - 1) * lda];
}

// perm[j]: start at ipiv[j] and walk back through the earlier interchanges
// (position q before step s held what position s held before step s' when
// ipiv[s'] == q for the last such s' < s).  The interchanges stream through LDS.
__global__ void __launch_bounds__(256) perm_kernel(int64_t n, const int32_t* __restrict__ ipiv,
                                                   int32_t* __restrict__ perm) {
  constexpr int CH = 4096;
  __shared__ int32_t sp[CH];
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t jmax = min(n - 1, (int64_t)(blockIdx.x + 1) * blockDim.x - 1);
  int64_t pos = (j < n) ? ipiv[j] : 0;
  for (int64_t hi = jmax; hi > 1; hi -= CH) {  // chunk covers s in [max(1, hi-CH), hi)
    const int64_t lo = max((int64_t)1, hi - CH);
    __syncthreads();
    for (int64_t s = lo + threadIdx.x; s < hi; s += blockDim.x) sp[s - lo] = ipiv[s];
    __syncthreads();
    for (int64_t s = hi - 1; s >= lo; --s)
      if (s < j && sp[s - lo] == pos) pos = s;
  }
  if (j < n) perm[j] = (int32_t)pos;
}

// Y[i, c] = B[perm[i], c0 + c]
__global__ void gather_kernel(int64_t n, int nr, const int32_t* __restrict__ perm, const double* __restrict__ B,
                              int64_t ldb, double* __restrict__ Y) {
  const int c = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    Y[i + (int64_t)c * n] = (c < nr) ? B[perm[i] + (int64_t)c * ldb] : 0.0;
}

// B[perm[i], c0 + c] = Z[i, c]
__global__ void scatter_kernel(int64_t n, int nr, const int32_t* __restrict__ perm, const double* __restrict__ Z,
                               double* __restrict__ B, int64_t ldb) {
  const int c = blockIdx.y;
  if (c >= nr) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    B[perm[i] + (int64_t)c * ldb] = Z[i + (int64_t)c * n];
}

// Inverse of the unit-lower diagonal block I of L (BS x BS, column-major in Dinv).
// Column c of the inverse solves L_II x = e_c by forward substitution; thread c owns it.
__global__ void inv_diag_kernel(int64_t n, const double* __restrict__ LT, int64_t lda, double* __restrict__ Dinv) {
  __shared__ double Ls[BS][BS + 1];
  const int64_t I = blockIdx.x;
  const int64_t r0 = I * BS;
  const int bs = (int)min((int64_t)BS, n - r0);
  for (int t = threadIdx.x; t < BS * BS; t += blockDim.x) {
    const int i = t % BS, j = t / BS;
    Ls[i][j] = (i > j && i < bs) ? Lij(LT, lda, r0 + i, r0 + j) : 0.0;
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < BS) {
    double x[BS];
#pragma unroll
    for (int i = 0; i < BS; ++i) x[i] = (i == c) ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < BS; ++j)
#pragma unroll
      for (int i = j + 1; i < BS; ++i) x[i] -= Ls[i][j] * x[j];
    double* D = Dinv + I * BS * BS;
#pragma unroll
    for (int i = 0; i < BS; ++i) D[i + c * BS] = (i < bs && c < bs) ? x[i] : 0.0;
  }
}

// Blocked substitution with L (forward, kTrans = false) or L^T (backward, kTrans = true)
// on Y (n x RC, in place).  Workgroup b handles row block I = b (forward) or
// I = nb-1-b (backward); flags[I] carries `tag` once Y_I is final.
template <bool kTrans>
__global__ void __launch_bounds__(NT) trsv_kernel(int64_t n, const double* __restrict__ LT, int64_t lda,
                                                  const double* __restrict__ Dinv, double* __restrict__ Y,
                                                  uint64_t* __restrict__ flags, uint64_t tag, int* status) {
  __shared__ double Lb[BS][BS + 1];
  __shared__ double yJ[BS][RC + 1];
  __shared__ double acc[BS][RC + 1];
  __shared__ int stop;
  const int64_t nb = (n + BS - 1) / BS;
  const int64_t I = kTrans ? nb - 1 - blockIdx.x : blockIdx.x;
  const int64_t r0 = I * BS;
  const int bs = (int)min((int64_t)BS, n - r0);
  const int tid = threadIdx.x;
  for (int t = tid; t < BS * RC; t += NT) {
    const int i = t % BS, c = t / BS;
    acc[i][c] = (i < bs) ? Y[r0 + i + (int64_t)c * n] : 0.0;
  }
  if (tid == 0) stop = 0;
  __syncthreads();
  // contributions of the other blocks J (J < I forward, J > I backward), in order of readiness
  const int64_t jfirst = kTrans ? nb - 1 : 0;
  const int64_t jstep = kTrans ? -1 : 1;
  for (int64_t J = jfirst; kTrans ? (J > I) : (J < I); J += jstep) {
    const int64_t c0 = J * BS;
    const int cs = (int)min((int64_t)BS, n - c0);
    // block of L (rows I, cols J) forward, or of L^T = (L rows J, cols I)^T backward
    for (int t = tid; t < BS * BS; t += NT) {
      // consecutive threads walk down a stored column of L in both orientations
      const int i = kTrans ? t / BS : t % BS, j = kTrans ? t % BS : t / BS;
      double v = 0.0;
      if (!kTrans) {
        if (i < bs && j < cs) v = Lij(LT, lda, r0 + i, c0 + j);
      } else {
        if (i < bs && j < cs) v = Lij(LT, lda, c0 + j, r0 + i);
      }
      Lb[i][j] = v;
    }
    if (tid == 0) {
      const uint64_t t0 = wall_clock64();
      while (ld_flag(flags + J) != tag) {
        if (wall_clock64() - t0 > kWaitTicks) {
          stop = 1;
          break;
        }
      }
    }
    __syncthreads();
    if (stop) break;
    for (int t = tid; t < BS * RC; t += NT) {
      const int j = t % BS, c = t / BS;
      yJ[j][c] = (j < cs) ? ld_agent(Y + c0 + j + (int64_t)c * n) : 0.0;
    }
    __syncthreads();
    for (int t = tid; t < BS * RC; t += NT) {
      const int i = t % BS, c = t / BS;
      double s = 0.0;
#pragma unroll 8
      for (int j = 0; j < BS; ++j) s += Lb[i][j] * yJ[j][c];
      acc[i][c] -= s;
    }
    __syncthreads();
  }
  if (stop) {
    if (tid == 0) atomicMin(status, SKF_ETIMEOUT);
    if (tid == 0) st_flag(flags + I, tag);  // let dependants finish (their result is void)
    return;
  }
  // Y_I = inv(L_II) acc  (forward)  or  inv(L_II)^T acc  (backward)
  const double* D = Dinv + I * BS * BS;
  for (int t = tid; t < BS * BS; t += NT) {
    const int i = t % BS, j = t / BS;
    Lb[i][j] = kTrans ? D[j + i * BS] : D[i + j * BS];
  }
  __syncthreads();
  for (int t = tid; t < BS * RC; t += NT) {
    const int i = t % BS, c = t / BS;
    double s = 0.0;
#pragma unroll 8
    for (int j = 0; j < BS; ++j) s += Lb[i][j] * acc[j][c];
    if (i < bs) st_agent(Y + r0 + i + (int64_t)c * n, s);
  }
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    st_flag(flags + I, tag);
  }
}

// T^{-1} on Y (n x RC) by Gaussian elimination with partial pivoting on the
// tridiagonal (sub T[i], super -T[i], zero diagonal); lane c owns column c.
// Rows are streamed; the working bands live in a per-column scratch.
__global__ void tridiag_kernel(int64_t n, int nr, const double* __restrict__ T, double* __restrict__ Y,
                               double* __restrict__ scratch, int* status) {
  const int c = threadIdx.x;
  if (c >= RC) return;
  double* y = Y + (int64_t)c * n;
  double* dd = scratch + (int64_t)c * 3 * n;  // diagonal, super, second super of U
  double* du = dd + n;
  double* du2 = du + n;
  // elimination
  double d_i = 0.0;                 // current diagonal entry of row i
  double u_i = (n > 1) ? -T[0] : 0.0;  // current super entry of row i
  double y_i = y[0];
  int sing = 0;
  for (int64_t i = 0; i + 1 < n; ++i) {
    const double l = T[i];                      // sub entry: row i+1, column i
    const double d_next = 0.0;                  // row i+1 diagonal
    const double u_next = (i + 2 < n) ? -T[i + 1] : 0.0;  // row i+1 super
    const double y_next = y[i + 1];
    if (fabs(d_i) >= fabs(l)) {
      if (d_i == 0.0) {
        sing = (int)(i + 1);
        break;
      }
      const double f = l / d_i;
      dd[i] = d_i;
      du[i] = u_i;
      du2[i] = 0.0;
      y[i] = y_i;
      d_i = d_next - f * u_i;
      u_i = u_next;
      y_i = y_next - f * y_i;
    } else {
      const double f = d_i / l;
      dd[i] = l;
      du[i] = d_next;
      du2[i] = u_next;
      y[i] = y_next;
      d_i = u_i - f * d_next;
      u_i = -f * u_next;
      y_i = y_i - f * y_next;
    }
  }
  if (!sing) {
    if (d_i == 0.0) sing = (int)n;
    dd[n - 1] = d_i;
    y[n - 1] = y_i;
  }
  if (sing) return;  // singular T: the info word reports it from T
  // back substitution
  y[n - 1] = y[n - 1] / dd[n - 1];
  if (n >= 2) y[n - 2] = (y[n - 2] - du[n - 2] * y[n - 1]) / dd[n - 2];
  for (int64_t i = n - 3; i >= 0; --i) y[i] = (y[i] - du[i] * y[i + 1] - du2[i] * y[i + 2]) / dd[i];
  (void)nr;
}

// info = 1 + first even k with T[k] == 0, or n for odd n, or 0.
__global__ void solve_info_kernel(int64_t n, const double* __restrict__ T, const int* status, int* dinfo) {
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
    int v = 0;
    if (status && *status != 0) v = *status;
    else if (n % 2 == 1) v = (int)n;
    else if (best[0] != INT64_MAX) v = (int)(best[0] + 1);
    *dinfo = v;
  }
}

}  // namespace

// Workspace: perm (n int32) | Dinv (nb*BS*BS) | Y (n*RC) | tri scratch (3*n*RC) | flags (2*nb) | status
struct SolveWork {
  int32_t* perm;
  double* Dinv;
  double* Y;
  double* tri;
  uint64_t* flags;
  int* status;
  size_t bytes;
};

static SolveWork solve_carve(void* base, int64_t n) {
  SolveWork w{};
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = align_up(off + b, 256);
    return base ? (void*)((char*)base + o) : nullptr;
  };
  const int64_t nb = (n + BS - 1) / BS;
  w.perm = (int32_t*)take(sizeof(int32_t) * (size_t)std::max<int64_t>(n, 1));
  w.Dinv = (double*)take(sizeof(double) * (size_t)std::max<int64_t>(nb, 1) * BS * BS);
  w.Y = (double*)take(sizeof(double) * (size_t)std::max<int64_t>(n, 1) * RC);
  w.tri = (double*)take(sizeof(double) * (size_t)std::max<int64_t>(n, 1) * 3 * RC);
  w.flags = (uint64_t*)take(sizeof(uint64_t) * (size_t)std::max<int64_t>(nb, 1) * 2);
  w.status = (int*)take(256);
  w.bytes = off;
  return w;
}

size_t solve_workspace_bytes(int64_t n, int64_t nrhs) {
  (void)nrhs;
  return solve_carve(nullptr, n).bytes + 256;
}

// Solve in place over B; dinfo (device) receives the numerical outcome.
int run_solve(int64_t n, int64_t nrhs, const double* LT, int64_t lda, const int32_t* ipiv, const double* T,
              double* B, int64_t ldb, void* work, size_t lwork, int* dinfo, hipStream_t s) {
  SolveWork w = solve_carve(work, n);
  if (lwork < w.bytes) return SKF_EWORK;
  int rc;
  if ((rc = launch_fill_i32(w.status, 1, 0, s))) return rc;
  if (n == 0 || nrhs == 0) return launch_fill_i32(dinfo, 1, 0, s);
  const int64_t nb = (n + BS - 1) / BS;
  const bool singular = (n % 2 == 1);
  if (!singular) {
    hipLaunchKernelGGL(perm_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, ipiv, w.perm);
    SKF_CHECK_LAUNCH("perm");
    hipLaunchKernelGGL(inv_diag_kernel, dim3((unsigned)nb), dim3(BS), 0, s, n, LT, lda, w.Dinv);
    SKF_CHECK_LAUNCH("inv_diag");
    if ((rc = launch_fill_u64(w.flags, (size_t)nb * 2, 0, s))) return rc;
    unsigned gx = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    uint64_t tag = 0;
    for (int64_t c0 = 0; c0 < nrhs; c0 += RC) {
      const int nr = (int)std::min<int64_t>(RC, nrhs - c0);
      hipLaunchKernelGGL(gather_kernel, dim3(gx, RC), dim3(256), 0, s, n, nr, w.perm, B + c0 * ldb, ldb, w.Y);
      SKF_CHECK_LAUNCH("gather");
      ++tag;
      hipLaunchKernelGGL(trsv_kernel<false>, dim3((unsigned)nb), dim3(NT), 0, s, n, LT, lda, w.Dinv, w.Y,
                         w.flags, tag, w.status);
      SKF_CHECK_LAUNCH("trsv fwd");
      hipLaunchKernelGGL(tridiag_kernel, dim3(1), dim3(64), 0, s, n, nr, T, w.Y, w.tri, w.status);
      SKF_CHECK_LAUNCH("tridiag");
      ++tag;
      hipLaunchKernelGGL(trsv_kernel<true>, dim3((unsigned)nb), dim3(NT), 0, s, n, LT, lda, w.Dinv, w.Y,
                         w.flags + nb, tag, w.status);
      SKF_CHECK_LAUNCH("trsv bwd");
      hipLaunchKernelGGL(scatter_kernel, dim3(gx, RC), dim3(256), 0, s, n, nr, w.perm, w.Y, B + c0 * ldb, ldb);
      SKF_CHECK_LAUNCH("scatter");
    }
  }
  hipLaunchKernelGGL(solve_info_kernel, dim3(1), dim3(256), 0, s, n, T, w.status, dinfo);
  SKF_CHECK_LAUNCH("solve info");
  return 0;
}

}  // namespace skf
