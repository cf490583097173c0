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
//           only, so one thread records them (multipliers and the U bands),
//           then one lane per right-hand side applies them and back-substitutes;
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

// Diagonal block J, forward: Y_J := L_JJ^{-1} Y_J.  Thread (r, c): row j0+r of
// right-hand side c0+c; column sweep, the final y_j published through LDS.
__global__ void __launch_bounds__(kBs* kRc) cdiag_fwd_kernel(int64_t n, int64_t nr, const double* __restrict__ LT,
                                                             int64_t lda, double* __restrict__ Y, int64_t j0) {
  __shared__ z2 yj[kRc];
  const int r = threadIdx.x % kBs, c = threadIdx.x / kBs;
  const int64_t i = j0 + r, col = (int64_t)blockIdx.x * kRc + c;
  const int m = (int)min((int64_t)kBs, n - j0);
  const bool act = r < m && col < nr;
  z2 y = act ? ld2(Y, i + col * n) : z2{0.0, 0.0};
  for (int j = 0; j < m - 1; ++j) {
    if (r == j) yj[c] = y;
    __syncthreads();
    if (act && r > j) y = zsub(y, zmul(lij(LT, lda, i, j0 + j), yj[c]));
    __syncthreads();
  }
  if (act) st2(Y, i + col * n, y);
}

// Blocks below J: Y_I -= L[I, J] Y_J, one workgroup per block row I and group of
// kRc right-hand sides; Y_J staged in LDS, L read column by column (coalesced).
__global__ void __launch_bounds__(kBs* kRc) cupdate_fwd_kernel(int64_t n, int64_t nr, const double* __restrict__ LT,
                                                               int64_t lda, double* __restrict__ Y, int64_t j0) {
  __shared__ z2 ys[kRc][kBs];
  const int r = threadIdx.x % kBs, c = threadIdx.x / kBs;
  const int64_t i0 = j0 + kBs * (1 + (int64_t)blockIdx.x), i = i0 + r;
  const int64_t col = (int64_t)blockIdx.y * kRc + c;
  const int m = (int)min((int64_t)kBs, n - j0);
  ys[c][r] = (r < m && col < nr) ? ld2(Y, j0 + r + col * n) : z2{0.0, 0.0};
  __syncthreads();
  if (i >= n || col >= nr) return;
  z2 acc = ld2(Y, i + col * n);
  for (int j = 0; j < m; ++j) acc = zsub(acc, zmul(lij(LT, lda, i, j0 + j), ys[c][j]));
  st2(Y, i + col * n, acc);
}

// Diagonal block J, backward: Y_J := L_JJ^{-T} Y_J (x_j final from the last row
// up; x_i -= L[j, i] x_j for i < j inside the block).
__global__ void __launch_bounds__(kBs* kRc) cdiag_bwd_kernel(int64_t n, int64_t nr, const double* __restrict__ LT,
                                                             int64_t lda, double* __restrict__ Y, int64_t j0) {
  __shared__ z2 xj[kRc];
  const int r = threadIdx.x % kBs, c = threadIdx.x / kBs;
  const int64_t i = j0 + r, col = (int64_t)blockIdx.x * kRc + c;
  const int m = (int)min((int64_t)kBs, n - j0);
  const bool act = r < m && col < nr;
  z2 y = act ? ld2(Y, i + col * n) : z2{0.0, 0.0};
  for (int j = m - 1; j >= 1; --j) {
    if (r == j) xj[c] = y;
    __syncthreads();
    if (act && r < j) y = zsub(y, zmul(lij(LT, lda, j0 + j, i), xj[c]));
    __syncthreads();
  }
  if (act) st2(Y, i + col * n, y);
}

// Blocks above I: Y_J -= L[I, J]^T Y_I for every block J < I: thread (r, c)
// forms column j0+r's sum over the rows of block I, in row order.
__global__ void __launch_bounds__(kBs* kRc) cupdate_bwd_kernel(int64_t n, int64_t nr, const double* __restrict__ LT,
                                                               int64_t lda, double* __restrict__ Y, int64_t i0) {
  __shared__ z2 ys[kRc][kBs];
  const int r = threadIdx.x % kBs, c = threadIdx.x / kBs;
  const int64_t j0 = kBs * (int64_t)blockIdx.x, j = j0 + r;
  const int64_t col = (int64_t)blockIdx.y * kRc + c;
  const int m = (int)min((int64_t)kBs, n - i0);
  ys[c][r] = (r < m && col < nr) ? ld2(Y, i0 + r + col * n) : z2{0.0, 0.0};
  __syncthreads();
  if (col >= nr) return;
  z2 acc = ld2(Y, j + col * n);
  for (int t = 0; t < m; ++t) acc = zsub(acc, zmul(lij(LT, lda, i0 + t, j), ys[c][t]));
  st2(Y, j + col * n, acc);
}

// The tridiagonal's elimination with partial pivoting (one thread): per row i
// the choice sw[i] (row i+1 taken as pivot row), the multiplier f[i], and the U
// bands dd, du, du2; status = the first zero pivot (1-based) or 0.
__global__ void ctri_factor_kernel(int64_t n, const double* __restrict__ T, double* __restrict__ dd,
                                   double* __restrict__ du, double* __restrict__ du2, double* __restrict__ f,
                                   int32_t* __restrict__ sw, int* __restrict__ status) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || *status != 0) return;
  z2 cd = {0.0, 0.0};                                   // running diagonal of row i
  z2 cu = (n > 1) ? z2{-T[0], -T[1]} : z2{0.0, 0.0};    // running super entry of row i
  for (int64_t i = 0; i + 1 < n; ++i) {
    const z2 dl = ld2(T, i);
    z2 nd = {0.0, 0.0};
    z2 nu = (i + 2 < n) ? z2{-T[2 * (i + 1)], -T[2 * (i + 1) + 1]} : z2{0.0, 0.0};
    if (zn2(cd) >= zn2(dl)) {
      if (cd.re == 0.0 && cd.im == 0.0) {
        *status = (int)(i + 1);
        return;
      }
      const z2 fm = zdiv(dl, cd);
      nd = zsub(nd, zmul(fm, cu));
      st2(dd, i, cd);
      st2(du, i, cu);
      st2(du2, i, z2{0.0, 0.0});
      st2(f, i, fm);
      sw[i] = 0;
    } else {
      const z2 fm = zdiv(cd, dl);
      const z2 t = nd;
      st2(dd, i, dl);
      st2(du, i, t);
      const z2 nd2 = zsub(cu, zmul(fm, t));
      z2 u2 = {0.0, 0.0};
      if (i + 2 < n) {
        u2 = nu;
        nu = zsub(z2{0.0, 0.0}, zmul(fm, u2));
      }
      st2(du2, i, u2);
      st2(f, i, fm);
      sw[i] = 1;
      nd = nd2;
    }
    cd = nd;
    cu = nu;
  }
  if (cd.re == 0.0 && cd.im == 0.0) {
    *status = (int)n;
    return;
  }
  st2(dd, n - 1, cd);
}

// One lane per right-hand side: the recorded elimination, then back substitution.
__global__ void ctri_apply_kernel(int64_t n, int64_t nr, const double* __restrict__ dd, const double* __restrict__ du,
                                  const double* __restrict__ du2, const double* __restrict__ f,
                                  const int32_t* __restrict__ sw, const int* __restrict__ status,
                                  double* __restrict__ Y) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= nr || *status != 0) return;
  double* y = Y + 2 * col * n;
  z2 cb = ld2(y, 0);
  for (int64_t i = 0; i + 1 < n; ++i) {
    const z2 nb = ld2(y, i + 1);
    const z2 fm = ld2(f, i);
    if (sw[i] == 0) {
      st2(y, i, cb);
      cb = zsub(nb, zmul(fm, cb));
    } else {
      st2(y, i, nb);
      cb = zsub(cb, zmul(fm, nb));
    }
  }
  // back substitution with the bands dd, du, du2
  z2 xb = zdiv(cb, ld2(dd, n - 1));
  st2(y, n - 1, xb);
  if (n >= 2) {
    z2 xa = zdiv(zsub(ld2(y, n - 2), zmul(ld2(du, n - 2), xb)), ld2(dd, n - 2));
    st2(y, n - 2, xa);
    for (int64_t i = n - 3; i >= 0; --i) {
      const z2 xi = zdiv(zsub(zsub(ld2(y, i), zmul(ld2(du, i), xa)), zmul(ld2(du2, i), xb)), ld2(dd, i));
      st2(y, i, xi);
      xb = xa;
      xa = xi;
    }
  }
}

// info: n for odd n; else 1 + the first even k with T[k] = 0; else the
// elimination's own zero pivot; else 0.
__global__ void csolve_info_kernel(int64_t n, const double* __restrict__ T, const int* __restrict__ status,
                                   int* __restrict__ dinfo) {
  if (threadIdx.x != 0) return;
  int v = 0;
  if (n % 2 == 1) v = (int)n;
  if (v == 0)
    for (int64_t k = 0; k + 1 < n; k += 2)
      if (T[2 * k] == 0.0 && T[2 * k + 1] == 0.0) {
        v = (int)(k + 1);
        break;
      }
  if (v == 0 && status) v = *status;
  *dinfo = v;
}

// First even zero pivot (or odd n) into status before anything else runs, so
// the tridiagonal and triangular steps are skipped for a singular T.
__global__ void csolve_precheck_kernel(int64_t n, const double* __restrict__ T, int* __restrict__ status) {
  if (threadIdx.x != 0) return;
  int v = (n % 2 == 1) ? (int)n : 0;
  if (v == 0)
    for (int64_t k = 0; k + 1 < n; k += 2)
      if (T[2 * k] == 0.0 && T[2 * k + 1] == 0.0) {
        v = (int)(k + 1);
        break;
      }
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
  hipLaunchKernelGGL(csolve_precheck_kernel, dim3(1), dim3(64), 0, s, n, T, w.status);
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
    hipLaunchKernelGGL(ctri_factor_kernel, dim3(1), dim3(64), 0, s, n, T, w.dd, w.du, w.du2, w.f, w.sw, w.status);
    SKF_CHECK_LAUNCH("csolve tri factor");
    hipLaunchKernelGGL(ctri_apply_kernel, dim3((unsigned)((nrhs + 63) / 64)), dim3(64), 0, s, n, nrhs, w.dd, w.du,
                       w.du2, w.f, w.sw, w.status, w.Y);
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
    hipLaunchKernelGGL(csolve_info_kernel, dim3(1), dim3(64), 0, s, n, T, w.status, dinfo);
    SKF_CHECK_LAUNCH("csolve info");
  }
  return 0;
}

}  // namespace skf
