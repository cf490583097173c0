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
//   T⁻¹     Gaussian elimination with partial pivoting on the tridiagonal
//           T(k+1, k) = T[k], T(k, k+1) = -T[k]: the pivot choices depend on T
//           only, so they are recorded once (multipliers and the U bands), then
//           one workgroup per right-hand side applies them and back-substitutes
//           (each chain on one thread over chunks staged in LDS);
//   L⁻ᵀ     by blocks from the last: the transposed diagonal block by one
//           workgroup, then every block above subtracts L[I, J]ᵀ Y_I;
//   scatter B[perm[i], :] = Y[i, :].
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

// The tridiagonal's elimination with partial pivoting: per row i the choice
// sw[i] (row i+1 taken as pivot row), the multiplier f[i] and the U bands dd,
// du, du2; status = the first zero pivot (1-based) if it meets one.  The chain
// runs on thread 0 over chunks of kCh rows staged in LDS by the whole
// workgroup (one load round trip and one store round trip per chunk).
constexpr int kCh = 512;

__global__ void __launch_bounds__(256) ctri_factor_kernel(int64_t n, const double* __restrict__ T,
                                                          double* __restrict__ dd, double* __restrict__ du,
                                                          double* __restrict__ du2, double* __restrict__ f,
                                                          int32_t* __restrict__ sw, int* __restrict__ status) {
  __shared__ z2 tch[kCh + 1];
  __shared__ z2 o_dd[kCh], o_du[kCh], o_du2[kCh], o_f[kCh];
  __shared__ int o_sw[kCh];
  __shared__ int stop;
  const int t = threadIdx.x;
  if (*status != 0) return;  // singular T found before (uniform)
  if (t == 0) stop = 0;
  z2 cd = {0.0, 0.0};                                 // running diagonal of row i (thread 0)
  z2 cu = (n > 1) ? ld2(T, 0) : z2{0.0, 0.0};         // running super entry of row i
  cu = zsub(z2{0.0, 0.0}, cu);
  for (int64_t c0 = 0; c0 < n - 1; c0 += kCh) {
    const int cnt = (int)min((int64_t)kCh, n - 1 - c0);
    const int nld = (int)min((int64_t)cnt + 1, n - 1 - c0);  // T[c0 .. c0 + cnt] where it exists
    for (int e = t; e < nld; e += blockDim.x) tch[e] = ld2(T, c0 + e);
    __syncthreads();
    if (t == 0) {
      for (int e = 0; e < cnt; ++e) {
        const int64_t i = c0 + e;
        const z2 dl = tch[e];
        z2 nd = {0.0, 0.0};
        z2 nu = (i + 2 < n) ? zsub(z2{0.0, 0.0}, tch[e + 1]) : z2{0.0, 0.0};
        if (zn2(cd) >= zn2(dl)) {
          if (cd.re == 0.0 && cd.im == 0.0) {
            *status = (int)(i + 1);
            stop = 1;
            break;
          }
          const z2 fm = zdiv(dl, cd);
          nd = zsub(nd, zmul(fm, cu));
          o_dd[e] = cd;
          o_du[e] = cu;
          o_du2[e] = z2{0.0, 0.0};
          o_f[e] = fm;
          o_sw[e] = 0;
        } else {
          const z2 fm = zdiv(cd, dl);
          const z2 tt = nd;
          o_dd[e] = dl;
          o_du[e] = tt;
          const z2 nd2 = zsub(cu, zmul(fm, tt));
          z2 u2 = {0.0, 0.0};
          if (i + 2 < n) {
            u2 = nu;
            nu = zsub(z2{0.0, 0.0}, zmul(fm, u2));
          }
          o_du2[e] = u2;
          o_f[e] = fm;
          o_sw[e] = 1;
          nd = nd2;
        }
        cd = nd;
        cu = nu;
      }
    }
    __syncthreads();
    if (stop) return;
    for (int e = t; e < cnt; e += blockDim.x) {
      st2(dd, c0 + e, o_dd[e]);
      st2(du, c0 + e, o_du[e]);
      st2(du2, c0 + e, o_du2[e]);
      st2(f, c0 + e, o_f[e]);
      sw[c0 + e] = o_sw[e];
    }
    __syncthreads();
  }
  if (t == 0) {
    if (cd.re == 0.0 && cd.im == 0.0) *status = (int)n;
    else st2(dd, n - 1, cd);
  }
}

// One workgroup per right-hand side: the recorded elimination, then back
// substitution, each chained on thread 0 over chunks staged in LDS.
__global__ void __launch_bounds__(256) ctri_apply_kernel(int64_t n, const double* __restrict__ dd,
                                                         const double* __restrict__ du,
                                                         const double* __restrict__ du2,
                                                         const double* __restrict__ f,
                                                         const int32_t* __restrict__ sw,
                                                         const int* __restrict__ status, double* __restrict__ Y) {
  __shared__ z2 a[kCh + 1], b[kCh], c[kCh], d[kCh];
  __shared__ int w[kCh];
  const int t = threadIdx.x;
  if (*status != 0) return;
  double* __restrict__ y = Y + 2 * (int64_t)blockIdx.x * n;
  // forward: rows c0 .. c0 + cnt - 1; a = y[c0 + 1 ..] (as yet untouched), b = f, w = choices, c = output
  z2 cb = ld2(y, 0);
  for (int64_t c0 = 0; c0 < n - 1; c0 += kCh) {
    const int cnt = (int)min((int64_t)kCh, n - 1 - c0);
    for (int e = t; e < cnt; e += blockDim.x) {
      a[e] = ld2(y, c0 + 1 + e);
      b[e] = ld2(f, c0 + e);
      w[e] = sw[c0 + e];
    }
    __syncthreads();
    if (t == 0)
      for (int e = 0; e < cnt; ++e) {
        const z2 nb = a[e];
        if (w[e] == 0) {
          c[e] = cb;
          cb = zsub(nb, zmul(b[e], cb));
        } else {
          c[e] = nb;
          cb = zsub(cb, zmul(b[e], nb));
        }
      }
    __syncthreads();
    for (int e = t; e < cnt; e += blockDim.x) st2(y, c0 + e, c[e]);
    __syncthreads();
  }
  // back substitution from the last row: x[i] = (y[i] - du[i] x[i+1] - du2[i] x[i+2]) / dd[i]
  z2 xa = {0.0, 0.0}, xb = {0.0, 0.0};  // x[i+1], x[i+2] (thread 0)
  if (t == 0) {
    xa = zdiv(cb, ld2(dd, n - 1));
    st2(y, n - 1, xa);
  }
  for (int64_t c1 = n - 1; c1 > 0; c1 -= kCh) {  // rows c1 - cnt .. c1 - 1
    const int cnt = (int)min((int64_t)kCh, c1);
    const int64_t r0 = c1 - cnt;
    for (int e = t; e < cnt; e += blockDim.x) {
      a[e] = ld2(y, r0 + e);
      b[e] = ld2(dd, r0 + e);
      c[e] = ld2(du, r0 + e);
      d[e] = ld2(du2, r0 + e);
    }
    __syncthreads();
    if (t == 0)
      for (int e = cnt - 1; e >= 0; --e) {
        const int64_t i = r0 + e;
        const z2 num = (i == n - 2) ? zsub(a[e], zmul(c[e], xa)) : zsub(zsub(a[e], zmul(c[e], xa)), zmul(d[e], xb));
        const z2 xi = zdiv(num, b[e]);
        a[e] = xi;
        xb = xa;
        xa = xi;
      }
    __syncthreads();
    for (int e = t; e < cnt; e += blockDim.x) st2(y, r0 + e, a[e]);
    __syncthreads();
  }
}

// info: n for odd n; else 1 + the first even k with T[k] = 0; else the
// elimination's own zero pivot; else 0.
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
  double *Y, *dd, *du, *du2, *f;
  int32_t* sw;
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
  w.dd = (double*)take(2 * sizeof(double) * m);
  w.du = (double*)take(2 * sizeof(double) * m);
  w.du2 = (double*)take(2 * sizeof(double) * m);
  w.f = (double*)take(2 * sizeof(double) * m);
  w.sw = (int32_t*)take(sizeof(int32_t) * m);
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
    hipLaunchKernelGGL(ctri_factor_kernel, dim3(1), dim3(256), 0, s, n, T, w.dd, w.du, w.du2, w.f, w.sw, w.status);
    SKF_CHECK_LAUNCH("csolve tri factor");
    hipLaunchKernelGGL(ctri_apply_kernel, dim3((unsigned)nrhs), dim3(256), 0, s, n, w.dd, w.du, w.du2, w.f, w.sw,
                       w.status, w.Y);
    SKF_CHECK_LAUNCH("csolve tri apply");
    for (int64_t I = nbk - 1; I >= 0; --I) {
      const int64_t i0 = I * kBs;
      hipLaunchKernelGGL(cdiag_bwd_kernel, dim3(gr), dim3(kBs * kRc), 0, s, n, nrhs, LT, lda, w.Y, i0);
      SKF_CHECK_LAUNCH("csolve diag bwd");
      if (I > 0) {
        hipLaunchKernelGGL(cupdate_bwd_kernel, dim3((unsigned)I, gr), dim3(kBs * kRc), 0, s, n, nrhs, LT, lda, w.Y,
                           i0);
        SKF_CHECK_LAUNCH("csolve update bwd");
      }
    }
    hipLaunchKernelGGL(cscatter_kernel, dim3(gx, (unsigned)nrhs), dim3(256), 0, s, n, nrhs, w.perm, w.Y, B, ldb,
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
