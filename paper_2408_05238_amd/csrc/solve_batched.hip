// Batched solves A_b X_b = B_b with the factors P A Pᵀ = L T Lᵀ of each
// matrix, all in one launch: one wave per (matrix, right-hand side) column,
//   x = Pᵀ L⁻ᵀ T⁻¹ L⁻¹ P b.
// The column lives in registers (lane l holds rows l, l + 64, ...) for the two
// triangular solves and in LDS for the interchanges and the tridiagonal solve:
//   P b     the recorded interchanges applied in order (lane 0, LDS);
//   L⁻¹     for j = 1 .. n-1: b_j is final, broadcast from its lane, and
//           b_i -= L[i, j] b_j for i > j (column j of L: coalesced loads, issued
//           D steps ahead into a ring of registers);
//   T⁻¹     Gaussian elimination with partial pivoting on the tridiagonal,
//           T(k+1, k) = T[k], T(k, k+1) = -T[k] (lane 0, the running rows in
//           registers, the U bands in LDS), then back substitution;
//   L⁻ᵀ     for j = n-1 .. 2: x_j is final and x_i -= L[j, i] x_j for
//           1 <= i < j (row j of L, read across columns; each line is reused by
//           the rows that follow);
//   Pᵀ x    the interchanges in reverse order.
// L[i, j] (i > j >= 1) is read from LT[i, j-1]; L[:, 0] = e_0.
#include <algorithm>
#include <vector>

#include "skf_internal.h"

namespace skf {
namespace {

constexpr int64_t kBsMaxN = 1024;  // rows per lane up to 16 (beyond, the registers spill)

struct BsArgs {
  const int64_t* n;
  const int64_t* lda;
  const int64_t* nrhs;
  const int64_t* ldb;
  const double* const* LT;
  const int32_t* const* ipiv;
  const double* const* T;
  double* const* B;
  int* info;
  int64_t ncol;  // columns per matrix in the grid (the largest nrhs, at least 1)
  int64_t nmax;  // LDS rows
};

// LDS per wave: b, T, and the three U bands (doubles), interchanges (int32).
__host__ __device__ constexpr int64_t bs_lds_bytes(int64_t nmax) { return nmax * (5 * 8 + 4); }

__device__ inline double bcast(double v, int lane) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t h = (uint32_t)__builtin_amdgcn_readlane((int)(u >> 32), lane);
  const uint32_t l = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
  return __longlong_as_double((long long)(((uint64_t)h << 32) | l));
}

template <int Q, int D>
__global__ void __launch_bounds__(64) solve_batched_kernel(BsArgs a) {
  extern __shared__ double sh[];
  const int64_t id = blockIdx.x;
  const int64_t b = id / a.ncol, c = id % a.ncol;
  const int lane = threadIdx.x;
  const int64_t n = a.n[b];
  const int64_t nr = a.nrhs[b];
  if (n > 64 * Q) return;  // solved on the host path
  if (c > 0 && c >= nr) return;
  const double* __restrict__ T = a.T[b];
  // outcome as for a single solve: n for odd n, else 1 + the first even k with
  // T[k] == 0, else what the tridiagonal elimination meets (below)
  int inf = (n % 2 == 1) ? (int)n : 0;
  if (inf == 0) {
    int64_t first = INT64_MAX;
    for (int64_t k = 2 * lane; k + 1 < n; k += 128)
      if (T[k] == 0.0) {
        first = k;
        break;
      }
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) {
      const int64_t o = __shfl_xor(first, s);
      first = min(first, o);
    }
    if (first != INT64_MAX) inf = (int)(first + 1);
  }
  if (inf != 0 || n == 0 || c >= nr) {
    if (c == 0 && lane == 0) a.info[b] = inf;
    return;
  }
  const int64_t lda = a.lda[b];
  const double* __restrict__ LT = a.LT[b];
  double* __restrict__ Bc = a.B[b] + c * a.ldb[b];
  const int32_t* __restrict__ ipv = a.ipiv[b];
  const int64_t nm = a.nmax;
  double* ys = sh;
  double* tl = sh + nm;
  double* dd = sh + 2 * nm;
  double* du = sh + 3 * nm;
  double* du2 = sh + 4 * nm;
  int32_t* ip = reinterpret_cast<int32_t*>(sh + 5 * nm);

  for (int64_t i = lane; i < n; i += 64) {
    ys[i] = Bc[i];
    ip[i] = ipv[i];
    tl[i] = (i + 1 < n) ? T[i] : 0.0;
  }
  __syncthreads();
  if (lane == 0)
    for (int64_t j = 1; j < n; ++j) {
      const int64_t p = min(max((int64_t)ip[j], (int64_t)0), n - 1);
      if (p != j) {
        const double t = ys[j];
        ys[j] = ys[p];
        ys[p] = t;
      }
    }
  __syncthreads();
  double y[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t i = lane + 64 * q;
    y[q] = (i < n) ? ys[i] : 0.0;
  }

  // The steps run block by block (qb: 64 rows held as y[qb] across the wave), so
  // every register index is fixed at compile time; ring[d] holds the operand
  // loads of the step j with j % D == d, issued D steps ahead.
  const int qtop = (int)((n - 1) >> 6);  // last block holding a row

  // ---- y := L^{-1} y: step j (1 <= j < n) subtracts column j of L
  // (= column j-1 of LT) times the final y_j from the rows below j ----
  {
    double ring[D][Q];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const double* col = LT + (max(min((int64_t)d, n - 1), (int64_t)1) - 1) * lda;
#pragma unroll
      for (int q = 0; q < Q; ++q) ring[d][q] = col[min((int64_t)lane + 64 * q, n - 1)];
    }
#pragma unroll
    for (int qb = 0; qb < Q; ++qb) {
      if (qb > qtop) break;
      for (int jj0 = 0; jj0 < 64; jj0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const int64_t j = 64 * qb + jj0 + d;
          const double bj = bcast(y[qb], jj0 + d);
          const bool live = j >= 1 && j < n;
#pragma unroll
          for (int q = qb; q < Q; ++q) {
            const int64_t i = lane + 64 * q;
            if (live && i > j && i < n) y[q] = fma(-ring[d][q], bj, y[q]);
          }
          const int64_t jn = j + D;  // next step of this slot
          if (jn < n) {
            const double* col = LT + (jn - 1) * lda;
#pragma unroll
            for (int q = qb; q < Q; ++q) ring[d][q] = col[min((int64_t)lane + 64 * q, n - 1)];
          }
        }
      }
    }
  }

  // ---- y := T^{-1} y (lane 0; U bands in LDS) ----
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t i = lane + 64 * q;
    if (i < n) ys[i] = y[q];
  }
  __syncthreads();
  int sing = 0;
  if (lane == 0) {
    double cd = 0.0, cu = -tl[0], cb = ys[0];  // row i: diagonal, super, right-hand side
    for (int64_t i = 0; i + 1 < n; ++i) {
      const double dl = tl[i];                          // T(i+1, i)
      double nd = 0.0;                                  // row i+1: diagonal
      double nu = (i + 2 < n) ? -tl[i + 1] : 0.0;       // row i+1: super
      double nb = ys[i + 1];
      if (fabs(cd) >= fabs(dl)) {
        if (cd == 0.0) {
          sing = (int)(i + 1);
          break;
        }
        const double f = dl / cd;
        nd = nd - f * cu;
        nb = nb - f * cb;
        dd[i] = cd;
        du[i] = cu;
        du2[i] = 0.0;
        ys[i] = cb;
      } else {
        const double f = cd / dl;
        const double t = nd;
        dd[i] = dl;
        du[i] = t;
        const double nd2 = cu - f * t;
        double u2 = 0.0;
        if (i + 2 < n) {
          u2 = nu;
          nu = -f * u2;
        }
        du2[i] = u2;
        ys[i] = nb;
        nb = cb - f * nb;
        nd = nd2;
      }
      cd = nd;
      cu = nu;
      cb = nb;
    }
    if (sing == 0) {
      if (cd == 0.0) {
        sing = (int)n;
      } else {
        dd[n - 1] = cd;
        double x1 = cb / cd;  // row n-1
        ys[n - 1] = x1;
        if (n >= 2) {
          const double x0 = (ys[n - 2] - du[n - 2] * x1) / dd[n - 2];
          ys[n - 2] = x0;
          double xa = x0, xb = x1;  // x[i+1], x[i+2]
          for (int64_t i = n - 3; i >= 0; --i) {
            const double xi = (ys[i] - du[i] * xa - du2[i] * xb) / dd[i];
            ys[i] = xi;
            xb = xa;
            xa = xi;
          }
        }
      }
    }
  }
  sing = __builtin_amdgcn_readfirstlane(sing);
  if (sing != 0) {
    if (c == 0 && lane == 0) a.info[b] = sing;
    return;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t i = lane + 64 * q;
    y[q] = (i < n) ? ys[i] : 0.0;
  }

  // ---- y := L^{-T} y: step j (n-1 >= j >= 2) subtracts row j of L
  // (L[j, i] = LT[j, i-1], 1 <= i < j) times the final x_j; x_1 and x_0 receive
  // nothing (L[1, 0] = 0).  The steps run from the top of block qtop, the
  // first few (j >= n) doing nothing ----
  {
    double ring[D][Q];
    const int64_t jtop = 64 * (int64_t)qtop + 63;
#pragma unroll
    for (int d = 0; d < D; ++d) {  // slot (jtop - d) % D = D - 1 - d
      const int64_t j = jtop - d;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int64_t jr = min(max(j, (int64_t)2), n - 1);
        const int64_t i = min(max((int64_t)lane + 64 * q, (int64_t)1), jr - 1);
        ring[D - 1 - d][q] = (n >= 3) ? LT[jr + (i - 1) * lda] : 0.0;
      }
    }
#pragma unroll
    for (int qb = Q - 1; qb >= 0; --qb) {
      if (qb > qtop) continue;
      for (int jj0 = 63; jj0 >= 0; jj0 -= D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const int64_t j = 64 * qb + jj0 - d;
          const int sl = D - 1 - d;  // j % D
          const double xj = bcast(y[qb], jj0 - d);
          const bool live = j >= 2 && j < n;
#pragma unroll
          for (int q = 0; q <= qb; ++q) {
            const int64_t i = lane + 64 * q;
            if (live && i >= 1 && i < j) y[q] = fma(-ring[sl][q], xj, y[q]);
          }
          const int64_t jn = j - D;
          if (jn >= 2 && jn < n) {
#pragma unroll
            for (int q = 0; q <= qb; ++q) {
              const int64_t i = min(max((int64_t)lane + 64 * q, (int64_t)1), jn - 1);
              ring[sl][q] = LT[jn + (i - 1) * lda];
            }
          }
        }
      }
    }
  }

  // ---- x := P^T y, written back ----
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t i = lane + 64 * q;
    if (i < n) ys[i] = y[q];
  }
  __syncthreads();
  if (lane == 0)
    for (int64_t j = n - 1; j >= 1; --j) {
      const int64_t p = min(max((int64_t)ip[j], (int64_t)0), n - 1);
      if (p != j) {
        const double t = ys[j];
        ys[j] = ys[p];
        ys[p] = t;
      }
    }
  __syncthreads();
  for (int64_t i = lane; i < n; i += 64) Bc[i] = ys[i];
  if (c == 0 && lane == 0) a.info[b] = 0;
}

template <int Q, int D>
int launch_bs(const BsArgs& a, int64_t batch, hipStream_t s) {
  const size_t lds = (size_t)bs_lds_bytes(a.nmax);
  if (lds > 64 * 1024) {
    SKF_CHECK(hipFuncSetAttribute((const void*)solve_batched_kernel<Q, D>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
              "solve_batched lds");
  }
  hipLaunchKernelGGL((solve_batched_kernel<Q, D>), dim3((unsigned)(batch * a.ncol)), dim3(64), lds, s, a);
  SKF_CHECK_LAUNCH("solve_batched");
  return 0;
}

}  // namespace

size_t solve_batched_workspace_bytes(int64_t batch, const int64_t* n_host, const int64_t* nrhs_host) {
  size_t b = align_up(sizeof(int64_t) * 4 * (size_t)std::max<int64_t>(batch, 1), 256);
  size_t big = 0;
  for (int64_t i = 0; i < batch; ++i)
    if (n_host[i] > kBsMaxN) big = std::max(big, solve_workspace_bytes(n_host[i], nrhs_host[i]));
  return b + big;
}

int run_solve_batched(int64_t batch, const int64_t* n_host, const double* const* LT, const int64_t* lda_host,
                      const int32_t* const* ipiv, const double* const* T, const int64_t* nrhs_host,
                      double* const* B, const int64_t* ldb_host, int* info, void* work, size_t lwork,
                      hipStream_t s) {
  if (batch == 0) return 0;
  if (lwork < solve_batched_workspace_bytes(batch, n_host, nrhs_host)) return SKF_EWORK;
  int64_t* stage = (int64_t*)work;
  const size_t nb = sizeof(int64_t) * (size_t)batch;
  SKF_CHECK(hipMemcpyAsync(stage, n_host, nb, hipMemcpyHostToDevice, s), "n");
  SKF_CHECK(hipMemcpyAsync(stage + batch, lda_host, nb, hipMemcpyHostToDevice, s), "lda");
  SKF_CHECK(hipMemcpyAsync(stage + 2 * batch, nrhs_host, nb, hipMemcpyHostToDevice, s), "nrhs");
  SKF_CHECK(hipMemcpyAsync(stage + 3 * batch, ldb_host, nb, hipMemcpyHostToDevice, s), "ldb");
  int64_t nmax = 1, ncol = 1;
  bool big = false;
  for (int64_t i = 0; i < batch; ++i) {
    if (n_host[i] > kBsMaxN) {
      big = true;
      continue;
    }
    nmax = std::max(nmax, n_host[i]);
    ncol = std::max(ncol, nrhs_host[i]);
  }
  BsArgs a{stage, stage + batch, stage + 2 * batch, stage + 3 * batch, LT, ipiv, T, B, info, ncol, nmax};
  if (batch * ncol > (int64_t)INT32_MAX) return SKF_ENOTIMPL;
  int rc;
  const int64_t q = (nmax + 63) / 64;
  // ring depth: as deep as the registers allow without spilling
  if (q <= 1) rc = launch_bs<1, 8>(a, batch, s);
  else if (q <= 2) rc = launch_bs<2, 8>(a, batch, s);
  else if (q <= 4) rc = launch_bs<4, 8>(a, batch, s);
  else if (q <= 8) rc = launch_bs<8, 4>(a, batch, s);
  else rc = launch_bs<16, 1>(a, batch, s);
  if (rc || !big) return rc;
  // orders beyond one wave's reach: the blocked single-matrix solve, after
  // reading their pointers back (the only synchronous step, taken only then)
  std::vector<const double*> hLT((size_t)batch), hT((size_t)batch);
  std::vector<double*> hB((size_t)batch);
  std::vector<const int32_t*> hP((size_t)batch);
  SKF_CHECK(hipMemcpyAsync(hLT.data(), LT, sizeof(double*) * batch, hipMemcpyDeviceToHost, s), "ptrs");
  SKF_CHECK(hipMemcpyAsync(hT.data(), T, sizeof(double*) * batch, hipMemcpyDeviceToHost, s), "ptrs");
  SKF_CHECK(hipMemcpyAsync(hB.data(), B, sizeof(double*) * batch, hipMemcpyDeviceToHost, s), "ptrs");
  SKF_CHECK(hipMemcpyAsync(hP.data(), ipiv, sizeof(int32_t*) * batch, hipMemcpyDeviceToHost, s), "ptrs");
  SKF_CHECK(hipStreamSynchronize(s), "ptrs");
  char* big_work = (char*)work + align_up(sizeof(int64_t) * 4 * (size_t)batch, 256);
  const size_t big_bytes = lwork - align_up(sizeof(int64_t) * 4 * (size_t)batch, 256);
  for (int64_t i = 0; i < batch; ++i) {
    if (n_host[i] <= kBsMaxN) continue;
    if ((rc = run_solve(n_host[i], nrhs_host[i], hLT[i], lda_host[i], hP[i], hT[i], hB[i], ldb_host[i], big_work,
                        big_bytes, info + i, s)))
      return rc;
  }
  return 0;
}

}  // namespace skf
