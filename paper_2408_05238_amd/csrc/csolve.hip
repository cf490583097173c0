// Solve A X = B with the complex factors P A Pᵀ = L T Lᵀ (plain transposes: A
// is complex skew, Aᵀ = -A):  X = Pᵀ L⁻ᵀ T⁻¹ L⁻¹ P B.
//
// Steps (one stream; every array complex128 interleaved unless noted):
//   perm    the original row at each position (the real solve's kernel);
//   gather  Y = P B (workspace, n x nrhs);
//   L⁻¹     by 64-row blocks J = 0, 1, ...: the unit lower diagonal block is
//           solved by one workgroup (column sweep in LDS), then every block
//           below subtracts L[I, J] Y_J (one workgroup per block row and group
//           of four right-hand sides, the 64 x 64 block of L read once);
//   T⁻¹     the tridiagonal T(k+1, k) = T[k], T(k, k+1) = -T[k] (zero
//           diagonal) split into its even rows (odd unknowns) and odd rows
//           (even unknowns): two bidiagonal substitutions, run together by two
//           waves, into Z;
//   L⁻ᵀ     by blocks from the last on Z: the transposed diagonal block by one
//           workgroup, then every block above subtracts L[I, J]ᵀ Z_I;
//   scatter B[perm[i], :] = Z[i, :].
// L[i, j] (i > j >= 1) is read from LT[i, j-1]; L[:, 0] = e_0.
// Each step is a launch; a block's launches wait for the previous block's
// through the stream, so no workgroup waits on another.
#include <algorithm>

#include "skf_internal.h"

// products rounded as written (the pivot comparisons use |z|^2 of rounded
// products, as the definition of the elimination does)
#pragma clang fp contract(off)

namespace skf {
namespace {

constexpr int kBs = 64;  // row block
constexpr int kRc = 4;   // right-hand sides per workgroup pass

struct z2 {
  double re, im;
};
__device__ inline z2 zmul(z2 a, z2 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline z2 zsub(z2 a, z2 b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline double zn2(z2 a) { return a.re * a.re + a.im * a.im; }
// a / b by Smith's method with true divisions
__device__ inline z2 zdiv(z2 a, z2 b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  const double r = b.re / b.im, d = b.re * r + b.im;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
__device__ inline z2 ld2(const double* p, int64_t e) { return {p[2 * e], p[2 * e + 1]}; }
__device__ inline void st2(double* p, int64_t e, z2 v) {
  p[2 * e] = v.re;
  p[2 * e + 1] = v.im;
}
// L[i, j] for i > j from the packed factor: 0 in column 0 (L[:, 0] = e_0)
__device__ inline z2 lij(const double* LT, int64_t lda, int64_t i, int64_t j) {
  return (j >= 1) ? ld2(LT, i + (j - 1) * lda) : z2{0.0, 0.0};
}

__global__ void cgather_kernel(int64_t n, int64_t nr, const int32_t* __restrict__ perm, const double* __restrict__ B,
                               int64_t ldb, double* __restrict__ Y) {
  const int64_t c = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    st2(Y, i + c * n, ld2(B, perm[i] + c * ldb));
}

__global__ void cscatter_kernel(int64_t n, int64_t nr, const int32_t* __restrict__ perm, const double* __restrict__ Y,
                                double* __restrict__ B, int64_t ldb, const int* __restrict__ status) {
  const int64_t c = blockIdx.y;
  if (*status != 0) return;  // singular T: B is left as it is
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    st2(B, perm[i] + c * ldb, ld2(Y, i + c * n));
}

// The 64 x 64 block L[I0 .. I0+63, J0 .. J0+63] (zero outside the strict lower
// part of L, rows past n zero) into LDS, by the whole workgroup in one round
// trip: lb[j][r] = L[I0 + r, J0 + j].
__device__ inline void stage_block(z2 (*lb)[kBs + 1], const double* __restrict__ LT, int64_t lda, int64_t n, int64_t I0,
                                   int64_t J0) {
  for (int e = threadIdx.x; e < kBs * kBs; e += blockDim.x) {
    const int r = e % kBs, j = e / kBs;
    const int64_t i = I0 + r, jj = J0 + j;
    lb[j][r] = (i < n && jj < n && i > jj) ? lij(LT, lda, i, jj) : z2{0.0, 0.0};
  }
}

// Diagonal block J, forward: Y_J := L_JJ^{-1} Y_J.  Wave c takes right-hand side
// c0 + c, lane r row j0 + r; the final y_j is broadcast by readlane (no barrier).
__global__ void __launch_bounds__(kBs* kRc) cdiag_fwd_kernel(int64_t n, int64_t nr, const double* __restrict__ LT,
                                                             int64_t lda, double* __restrict__ Y, int64_t j0) {
  __shared__ z2 lb[kBs][kBs + 1];  // padded: column reads (lb[r][t]) stay conflict-free
  stage_block(lb, LT, lda, n, j0, j0);
  __syncthreads();
  const int r = threadIdx.x % kBs, c = threadIdx.x / kBs;
  const int64_t i = j0 + r, col = (int64_t)blockIdx.x * kRc + c;
  if (col >= nr) return;  // a whole wave
  const int m = (int)min((int64_t)kBs, n - j0);
  z2 y = (r < m) ? ld2(Y, i + col * n) : z2{0.0, 0.0};
  for (int j = 0; j < m - 1; ++j) {
    const z2 yj = {__shfl(y.re, j), __shfl(y.im, j)};
    if (r > j) y = zsub(y, zmul(lb[j][r], yj));
  }
  if (r < m) st2(Y, i + col * n, y);
}

// Blocks below J: Y_I -= L[I, J] Y_J, one workgroup per block row I and group of
// kRc right-hand sides; the block of L and Y_J staged in LDS.
__global__ void __launch_bounds__(kBs* kRc) cupdate_fwd_kernel(int64_t n, int64_t nr, const double* __restrict__ LT,
                                                               int64_t lda, double* __restrict__ Y, int64_t j0) {
  __shared__ z2 lb[kBs][kBs + 1];  // padded: column reads (lb[r][t]) stay conflict-free
  __shared__ z2 ys[kRc][kBs];
  const int r = threadIdx.x % kBs, c = threadIdx.x / kBs;
  const int64_t i0 = j0 + kBs * (1 + (int64_t)blockIdx.x), i = i0 + r;
  const int64_t col = (int64_t)blockIdx.y * kRc + c;
  const int m = (int)min((int64_t)kBs, n - j0);
  stage_block(lb, LT, lda, n, i0, j0);
  ys[c][r] = (r < m && col < nr) ? ld2(Y, j0 + r + col * n) : z2{0.0, 0.0};
  __syncthreads();
  if (i >= n || col >= nr) return;
  z2 acc = ld2(Y, i + col * n);
  for (int j = 0; j < m; ++j) acc = zsub(acc, zmul(lb[j][r], ys[c][j]));
  st2(Y, i + col * n, acc);
}

// Diagonal block J, backward: Y_J := L_JJ^{-T} Y_J (x_j final from the last row
// up; x_i -= L[j, i] x_j for i < j inside the block), one wave per right-hand side.
__global__ void __launch_bounds__(kBs* kRc) cdiag_bwd_kernel(int64_t n, int64_t nr, const double* __restrict__ LT,
                                                             int64_t lda, double* __restrict__ Y, int64_t j0) {
  __shared__ z2 lb[kBs][kBs + 1];  // padded: column reads (lb[r][t]) stay conflict-free
  stage_block(lb, LT, lda, n, j0, j0);
  __syncthreads();
  const int r = threadIdx.x % kBs, c = threadIdx.x / kBs;
  const int64_t i = j0 + r, col = (int64_t)blockIdx.x * kRc + c;
  if (col >= nr) return;  // a whole wave
  const int m = (int)min((int64_t)kBs, n - j0);
  z2 y = (r < m) ? ld2(Y, i + col * n) : z2{0.0, 0.0};
  for (int j = m - 1; j >= 1; --j) {
    const z2 xj = {__shfl(y.re, j), __shfl(y.im, j)};
    if (r < j) y = zsub(y, zmul(lb[r][j], xj));  // L[j0 + j, j0 + r] = lb[r][j]
  }
  if (r < m) st2(Y, i + col * n, y);
}

// Blocks above I: Y_J -= L[I, J]^T Y_I for every block J < I: thread (r, c)
// forms column j0+r's sum over the rows of block I, in row order; the block of
// L and Y_I staged in LDS.
__global__ void __launch_bounds__(kBs* kRc) cupdate_bwd_kernel(int64_t n, int64_t nr, const double* __restrict__ LT,
                                                               int64_t lda, double* __restrict__ Y, int64_t i0) {
  __shared__ z2 lb[kBs][kBs + 1];  // padded: column reads (lb[r][t]) stay conflict-free
  __shared__ z2 ys[kRc][kBs];
  const int r = threadIdx.x % kBs, c = threadIdx.x / kBs;
  const int64_t j0 = kBs * (int64_t)blockIdx.x, j = j0 + r;
  const int64_t col = (int64_t)blockIdx.y * kRc + c;
  const int m = (int)min((int64_t)kBs, n - i0);
  stage_block(lb, LT, lda, n, i0, j0);
  ys[c][r] = (r < m && col < nr) ? ld2(Y, i0 + r + col * n) : z2{0.0, 0.0};
  __syncthreads();
  if (col >= nr) return;
  z2 acc = ld2(Y, j + col * n);
  for (int t = 0; t < m; ++t) acc = zsub(acc, zmul(lb[r][t], ys[c][t]));  // L[i0 + t, j0 + r]
  st2(Y, j + col * n, acc);
}

// T^{-1} on Y (n x nrhs, n even).  The complex skew tridiagonal T has a zero
// diagonal, so its even rows hold only the odd unknowns and its odd rows only
// the even ones: two bidiagonal triangular systems whose diagonals are the
// even entries T[2i] (all nonzero here: a zero one stops the solve first),
// each solved by substitution (componentwise backward stable):
//   x_{2i+1} = a_i x_{2i-1} + b_i,  a_i = T[2i-1] r_i,  b_i = -y_{2i} r_i
//   x_{2i}   = c_i x_{2i+2} + d_i,  c_i = T[2i+1] r_i,  d_i = y_{2i+1} r_i
// with r_i = 1/T[2i] (Smith's division).  Per chunk of kTc pairs, threads
// 0..kTc-1 form the forward chain's coefficients and the others the backward
// chain's; then wave 0 runs the forward chain and wave 1 the backward one
// (lane = right-hand side, kCc per workgroup), one complex multiply-add per
// step; chunks are padded with identity steps so the loop has no guard.  The
// solution goes to Z, so neither chain overwrites a right-hand side the other
// still reads.
constexpr int kTc = 128;                   // pairs per chunk
constexpr int kCc = 16;                    // right-hand sides per workgroup
constexpr int kTpad = 8;                   // guard entries on each side of a row
constexpr int kTs = kTc + 2 * kTpad + 1;   // row stride: the lanes' rows in distinct LDS banks

__device__ inline z2 zfma(z2 a, z2 x, z2 b) {  // a x + b
  return {fma(a.re, x.re, fma(-a.im, x.im, b.re)), fma(a.re, x.im, fma(a.im, x.re, b.im))};
}

template <int DIR>
__device__ inline void cchain(const z2* __restrict__ aa, z2* __restrict__ bb, z2& x) {
  // step j takes entry j (DIR = +1, from the chunk's start) or kTc-1-j (DIR = -1);
  // eight steps per block, the next block's coefficients read while it runs
  constexpr int G8 = 8;
  const int base = (DIR > 0) ? 0 : kTc - 1;
  z2 ca[G8], cb[G8];
#pragma unroll
  for (int u = 0; u < G8; ++u) {
    ca[u] = aa[base + DIR * u];
    cb[u] = bb[base + DIR * u];
  }
  for (int j0 = 0; j0 < kTc; j0 += G8) {
    z2 na[G8], nb[G8];
#pragma unroll
    for (int u = 0; u < G8; ++u) {
      na[u] = aa[base + DIR * (j0 + G8 + u)];
      nb[u] = bb[base + DIR * (j0 + G8 + u)];
    }
#pragma unroll
    for (int u = 0; u < G8; ++u) {
      x = zfma(ca[u], x, cb[u]);
      bb[base + DIR * (j0 + u)] = x;
    }
#pragma unroll
    for (int u = 0; u < G8; ++u) {
      ca[u] = na[u];
      cb[u] = nb[u];
    }
  }
}

__global__ void __launch_bounds__(256) ctri_kernel(int64_t n, int64_t nr, const double* __restrict__ T,
                                                   const int* __restrict__ status, const double* __restrict__ Y,
                                                   double* __restrict__ Z) {
  __shared__ z2 sa[2][kTs];
  __shared__ z2 sb[2][kCc][kTs];
  if (*status != 0) return;  // singular T: B is left as it is
  const int tid = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * kCc;
  const int ncol = (int)min((int64_t)kCc, nr - c0);
  const int64_t np = n / 2, nch = (np + kTc - 1) / kTc;
  const int d = tid / kTc, q = tid % kTc;  // coefficient phase: direction and pair of the chunk
  const int w = tid >> 6, lane = tid & 63;
  z2 x = {0.0, 0.0};  // x_{2i-1} (wave 0) or x_{2i+2} (wave 1) carried across chunks
  for (int64_t ch = 0; ch < nch; ++ch) {
    const int64_t p = (d == 0 ? ch : nch - 1 - ch) * kTc + q;
    {
      z2 av = {1.0, 0.0}, bv[kCc];
#pragma unroll
      for (int k = 0; k < kCc; ++k) bv[k] = z2{0.0, 0.0};
      if (p < np) {
        const z2 r = zdiv(z2{1.0, 0.0}, ld2(T, 2 * p));
        const z2 t = (d == 0) ? (p > 0 ? ld2(T, 2 * p - 1) : z2{0.0, 0.0})
                              : (2 * p + 2 < n ? ld2(T, 2 * p + 1) : z2{0.0, 0.0});
#pragma unroll
        for (int k = 0; k < kCc; ++k) bv[k] = (k < ncol) ? ld2(Y, 2 * p + d + (c0 + k) * n) : z2{0.0, 0.0};
        av = zmul(t, r);
#pragma unroll
        for (int k = 0; k < kCc; ++k) {
          const z2 v = zmul(bv[k], r);
          bv[k] = (d == 0) ? z2{-v.re, -v.im} : v;
        }
      }
      sa[d][kTpad + q] = av;
#pragma unroll
      for (int k = 0; k < kCc; ++k) sb[d][k][kTpad + q] = bv[k];
    }
    __syncthreads();
    if (w == 0 && lane < ncol) cchain<1>(sa[0] + kTpad, sb[0][lane] + kTpad, x);
    else if (w == 1 && lane < ncol) cchain<-1>(sa[1] + kTpad, sb[1][lane] + kTpad, x);
    __syncthreads();
    // x_{2p+1} (forward chain) and x_{2p} (backward chain) to their rows of Z
    if (p < np) {
#pragma unroll
      for (int k = 0; k < kCc; ++k)
        if (k < ncol) st2(Z, 2 * p + 1 - d + (c0 + k) * n, sb[d][k][kTpad + q]);
    }
    __syncthreads();  // the chunk buffers are refilled next
  }
}

// info: n for odd n; else 1 + the first even k with T[k] = 0; else 0.
__global__ void __launch_bounds__(256) csolve_info_kernel(int64_t n, const double* __restrict__ T,
                                                          const int* __restrict__ status, int* __restrict__ dinfo) {
  const int64_t z = first_zero_even_pivot(n, T, true);
  if (threadIdx.x != 0) return;
  int v = 0;
  if (n % 2 == 1) v = (int)n;
  if (v == 0 && z != INT64_MAX) v = (int)(z + 1);
  if (v == 0 && status) v = *status;
  *dinfo = v;
}

// Odd n or a zero even pivot into status before anything else runs, so the
// tridiagonal steps and the scatter are skipped for a singular T.
__global__ void __launch_bounds__(256) csolve_precheck_kernel(int64_t n, const double* __restrict__ T,
                                                              int* __restrict__ status) {
  const int64_t z = first_zero_even_pivot(n, T, true);
  if (threadIdx.x != 0) return;
  int v = (n % 2 == 1) ? (int)n : 0;
  if (v == 0 && z != INT64_MAX) v = (int)(z + 1);
  *status = v;
}

struct CSolveWork {
  int32_t* perm;
  double *Y, *Z;  // P B, then L^{-1} P B; T^{-1} of it, then the solution before P^T
  int* status;
  size_t bytes;
};

CSolveWork cs_carve(void* base, int64_t n, int64_t nrhs) {
  CSolveWork w{};
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = align_up(off + b, 256);
    return base ? (void*)((char*)base + o) : nullptr;
  };
  const size_t m = (size_t)std::max<int64_t>(n, 1), r = (size_t)std::max<int64_t>(nrhs, 1);
  w.perm = (int32_t*)take(sizeof(int32_t) * m);
  w.Y = (double*)take(2 * sizeof(double) * m * r);
  w.Z = (double*)take(2 * sizeof(double) * m * r);
  w.status = (int*)take(256);
  w.bytes = off;
  return w;
}

}  // namespace

size_t solve_c128_workspace_bytes(int64_t n, int64_t nrhs) { return cs_carve(nullptr, n, nrhs).bytes; }

int run_solve_c128(int64_t n, int64_t nrhs, const double* LT, int64_t lda, const int32_t* ipiv, const double* T,
                   double* B, int64_t ldb, void* work, size_t lwork, int* dinfo, hipStream_t s) {
  CSolveWork w = cs_carve(work, n, nrhs);
  if (lwork < w.bytes) return SKF_EWORK;
  if (n == 0) return dinfo ? launch_fill_i32(dinfo, 1, 0, s) : 0;
  if (nrhs > 65535 * (int64_t)kRc) return SKF_ENOTIMPL;
  int rc;
  hipLaunchKernelGGL(csolve_precheck_kernel, dim3(1), dim3(256), 0, s, n, T, w.status);
  SKF_CHECK_LAUNCH("csolve precheck");
  if (n % 2 == 0 && nrhs > 0) {
    // a singular T (found on the device) leaves B as it is: the tridiagonal
    // steps and the scatter read the status; the triangular steps before and
    // after them work on the workspace copy only
    if ((rc = launch_solve_perm(n, ipiv, w.perm, s))) return rc;
    const unsigned gx = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(cgather_kernel, dim3(gx, (unsigned)nrhs), dim3(256), 0, s, n, nrhs, w.perm, B, ldb, w.Y);
    SKF_CHECK_LAUNCH("csolve gather");
    const int64_t nbk = (n + kBs - 1) / kBs;
    const unsigned gr = (unsigned)((nrhs + kRc - 1) / kRc);
    for (int64_t J = 0; J < nbk; ++J) {
      const int64_t j0 = J * kBs;
      hipLaunchKernelGGL(cdiag_fwd_kernel, dim3(gr), dim3(kBs * kRc), 0, s, n, nrhs, LT, lda, w.Y, j0);
      SKF_CHECK_LAUNCH("csolve diag fwd");
      if (J + 1 < nbk) {
        hipLaunchKernelGGL(cupdate_fwd_kernel, dim3((unsigned)(nbk - J - 1), gr), dim3(kBs * kRc), 0, s, n, nrhs, LT,
                           lda, w.Y, j0);
        SKF_CHECK_LAUNCH("csolve update fwd");
      }
    }
    hipLaunchKernelGGL(ctri_kernel, dim3((unsigned)((nrhs + kCc - 1) / kCc)), dim3(256), 0, s, n, nrhs, T, w.status,
                       w.Y, w.Z);
    SKF_CHECK_LAUNCH("csolve tri");
    for (int64_t I = nbk - 1; I >= 0; --I) {
      const int64_t i0 = I * kBs;
      hipLaunchKernelGGL(cdiag_bwd_kernel, dim3(gr), dim3(kBs * kRc), 0, s, n, nrhs, LT, lda, w.Z, i0);
      SKF_CHECK_LAUNCH("csolve diag bwd");
      if (I > 0) {
        hipLaunchKernelGGL(cupdate_bwd_kernel, dim3((unsigned)I, gr), dim3(kBs * kRc), 0, s, n, nrhs, LT, lda, w.Z,
                           i0);
        SKF_CHECK_LAUNCH("csolve update bwd");
      }
    }
    hipLaunchKernelGGL(cscatter_kernel, dim3(gx, (unsigned)nrhs), dim3(256), 0, s, n, nrhs, w.perm, w.Z, B, ldb,
                       w.status);
    SKF_CHECK_LAUNCH("csolve scatter");
  }
  if (dinfo) {
    hipLaunchKernelGGL(csolve_info_kernel, dim3(1), dim3(256), 0, s, n, T, w.status, dinfo);
    SKF_CHECK_LAUNCH("csolve info");
  }
  return 0;
}

}  // namespace skf
