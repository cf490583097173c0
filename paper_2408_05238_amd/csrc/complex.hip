// Pfaffian-only reduction of a complex (complex128) skew-symmetric matrix.
//
// The elimination step is the real one taken at even k only: pivot on column k
// (largest |z|^2 = re^2 + im^2 below the diagonal, each product rounded, lowest
// index on ties), interchange rows and columns k+1 and p, l = column k / alpha
// below row k+1, v = column k+1 there, and add l v^T - v l^T to the trailing
// block; rows/columns k and k+1 are then decoupled and Pf(A) = (-1)^{s + n/2}
// prod_k T[k] (Parlett-Reid congruence with a unit lower triangular matrix; the
// Pfaffian's transformation rule under congruence and interchanges).
//
// This first form is unblocked: the input's strict lower triangle is expanded
// into a full skew copy in the workspace, and every step is two launches: the
// symmetric interchange (which first reduces the pivot search's per-block
// partials) and the trailing rank-2 update over a 2-D grid, which forms l and v
// on the fly and leaves the partials of the next pivot column.  The pivot
// passes through device memory, so the host only enqueues.  The update is HBM-bound: it reads and
// writes the trailing square once per step.
#include <math.h>

#include "skf_internal.h"

// Products are rounded before they are summed (no fused multiply-add), so each
// complex product and |z|^2 are those of the textbook formulas.
#pragma clang fp contract(off)

namespace skf {
namespace {

struct c128 {
  double re, im;
};

__device__ inline c128 cmul(c128 a, c128 b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline c128 csub(c128 a, c128 b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline c128 cadd(c128 a, c128 b) { return {a.re + b.re, a.im + b.im}; }
// a / b by Smith's method (scaled by the larger component of b)
__device__ inline c128 cdiv(c128 a, c128 b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  const double r = b.re / b.im, d = b.re * r + b.im;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
// |z|^2 with each product rounded, so the pivot order is that of the plain definition
__device__ inline double cnorm2(c128 z) { return z.re * z.re + z.im * z.im; }

// W (n x n, ld n) = the skew matrix whose strict lower triangle A holds.
__global__ void form_full_kernel(int64_t n, const c128* __restrict__ A, int64_t lda, c128* __restrict__ W) {
  const int64_t j = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    c128 v = {0.0, 0.0};
    if (i > j) v = A[i + j * lda];
    else if (i < j) {
      const c128 u = A[j + i * lda];
      v = {-u.re, -u.im};
    }
    W[i + j * n] = v;
  }
}

// Pivot search, split: every 64-row block of the previous step's update (or of
// an initial pass for column 0) leaves the arg-max of |W[i,c]|^2 over its rows
// that are candidates (i > c) and a non-finite flag; the interchange kernel
// reduces those partials.  Ties go to the lowest index at both levels.
struct Best {
  double key;
  int idx;
  int bad;
};

__device__ inline void wave_best(double& key, int& idx) {
  for (int off = 32; off > 0; off >>= 1) {
    const double k2 = __shfl_xor(key, off);
    const int i2 = __shfl_xor(idx, off);
    if (k2 > key || (k2 == key && i2 < idx)) {
      key = k2;
      idx = i2;
    }
  }
}

// one 64-lane wave per block: rows i = base + 64 b + lane of column c (candidates i > c)
__device__ inline void block_partial(int64_t n, int64_t c, int64_t i, c128 z, Best* __restrict__ part, int b) {
  const bool cand = i > c && i < n;
  const bool nonfin = cand && !(isfinite(z.re) && isfinite(z.im));
  double key = (cand && !nonfin) ? cnorm2(z) : -1.0;
  int idx = cand ? (int)i : INT32_MAX;
  const uint64_t badw = __ballot(nonfin);
  wave_best(key, idx);
  if ((threadIdx.x & 63) == 0) part[b] = Best{key, idx, badw != 0};
}

// partials of column 0 (rows 64 b + lane)
__global__ void __launch_bounds__(64) init_partials_kernel(int64_t n, const c128* __restrict__ W,
                                                           Best* __restrict__ part) {
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const c128 z = (i < n) ? W[i] : c128{0.0, 0.0};
  block_partial(n, 0, i, z, part, (int)blockIdx.x);
}

// Step k's pivot p from the partials of column k (every workgroup reduces them
// the same way; ipiv[k+1] = p), then the symmetric interchange of rows/columns
// k+1 and p over the active part (index t >= k): thread t swaps (k+1, t) <-> (p, t) and (t, k+1) <-> (t, p), four
// entries no other thread touches when t is neither k+1 nor p; the 2 x 2 block
// of those two indices is permuted by one thread.  The pivot T[k] = W[k+1, k]
// after the interchange is recorded by the thread of t = k.
__global__ void __launch_bounds__(256) swap_kernel(int64_t n, int64_t k, c128* __restrict__ W,
                                                   c128* __restrict__ T, int32_t* __restrict__ ipiv,
                                                   const Best* __restrict__ part, int* __restrict__ status) {
  __shared__ double bv[256];
  __shared__ int bi[256];
  __shared__ int sbad;
  if (*status != 0) return;
  // reduce the partials of column k: blocks of rows k + 64 b + lane
  const int nblk = (int)((n - k + 63) / 64);
  const int tt = threadIdx.x;
  if (tt == 0) sbad = 0;
  __syncthreads();
  double key = -1.0;
  int idx = INT32_MAX;
  for (int b = tt; b < nblk; b += 256) {
    const Best q = part[b];
    if (q.bad) sbad = 1;
    if (q.key > key || (q.key == key && q.idx < idx)) {
      key = q.key;
      idx = q.idx;
    }
  }
  bv[tt] = key;
  bi[tt] = idx;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tt < h && (bv[tt + h] > bv[tt] || (bv[tt + h] == bv[tt] && bi[tt + h] < bi[tt]))) {
      bv[tt] = bv[tt + h];
      bi[tt] = bi[tt + h];
    }
    __syncthreads();
  }
  if (sbad) {
    if (blockIdx.x == 0 && tt == 0) atomicMin(status, SKF_ENONFINITE);
    return;
  }
  const int64_t p = bi[0], r = k + 1;
  if (blockIdx.x == 0 && tt == 0) ipiv[r] = (int32_t)p;
  for (int64_t t = k + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    if (p != r) {
      if (t == r) {
        const c128 a = W[r + r * n], b = W[r + p * n], c = W[p + r * n], d = W[p + p * n];
        W[r + r * n] = d;
        W[r + p * n] = c;
        W[p + r * n] = b;
        W[p + p * n] = a;
      } else if (t != p) {
        const c128 a = W[r + t * n], b = W[p + t * n];
        W[r + t * n] = b;
        W[p + t * n] = a;
        const c128 c = W[t + r * n], d = W[t + p * n];
        W[t + r * n] = d;
        W[t + p * n] = c;
      }
    }
    if (t == k) T[k] = W[r + k * n];  // this thread wrote (k+1, k) itself
  }
}

// W[i,j] += l_i v_j - v_i l_j for i, j >= k+2, with l = W[:,k] / alpha (0 when
// alpha = W[k+1,k] is 0) and v = W[:,k+1] formed on the fly (those two columns are
// not written here): a 64 x 16 tile per block of 64 x 4 threads, the tile's 16
// column values of l and v computed once into LDS.
__global__ void __launch_bounds__(256) update_kernel(int64_t n, int64_t k, c128* __restrict__ W,
                                                     Best* __restrict__ part, const int* __restrict__ status) {
  __shared__ c128 lj[16], vj[16];
  if (*status != 0) return;
  const c128 alpha = W[k + 1 + k * n];
  const bool zero = alpha.re == 0.0 && alpha.im == 0.0;
  const int64_t j0 = k + 2 + (int64_t)blockIdx.y * 16;
  if (threadIdx.y == 0 && threadIdx.x < 16) {
    const int64_t j = min(j0 + threadIdx.x, n - 1);
    lj[threadIdx.x] = zero ? c128{0.0, 0.0} : cdiv(W[j + k * n], alpha);
    vj[threadIdx.x] = W[j + (k + 1) * n];
  }
  __syncthreads();
  const int64_t i = k + 2 + (int64_t)blockIdx.x * 64 + threadIdx.x;
  c128 first = {0.0, 0.0};  // the new W[i, k+2] (column jj = 0 of the first tile column)
  if (i < n) {
    const c128 li = zero ? c128{0.0, 0.0} : cdiv(W[i + k * n], alpha);
    const c128 vi = W[i + (k + 1) * n];
    for (int jj = threadIdx.y; jj < 16; jj += blockDim.y) {
      const int64_t j = j0 + jj;
      if (j >= n) break;
      const c128 w = W[i + j * n];
      const c128 nw = cadd(w, csub(cmul(li, vj[jj]), cmul(vi, lj[jj])));
      W[i + j * n] = nw;
      if (jj == 0) first = nw;
    }
  }
  // the next step's pivot column is k+2: this block's partial over rows i > k+2
  if (blockIdx.y == 0 && threadIdx.y == 0) block_partial(n, k + 2, i, first, part, (int)blockIdx.x);
}

// dinfo: status if set; n for odd n; else 1 + the first even k with T[k] = 0, or 0.
__global__ void info_c128_kernel(int64_t n, const c128* __restrict__ T, const int* __restrict__ status,
                                 int* __restrict__ dinfo) {
  const int64_t z = first_zero_even_pivot(n, reinterpret_cast<const double*>(T), true);
  if (threadIdx.x != 0) return;
  int v = *status;
  if (v == 0 && (n & 1)) v = (int)n;
  if (v == 0 && z != INT64_MAX) v = (int)(z + 1);
  *dinfo = v;
}

// log|Pf| and phase = Pf / |Pf| from (ipiv, T), in index order (one thread).
__global__ void logpf_c128_kernel(int64_t n, const int32_t* __restrict__ ipiv, const c128* __restrict__ T,
                                  double* logabs, double* phase) {
  if (threadIdx.x != 0) return;
  if (n == 0) {
    *logabs = 0.0;
    phase[0] = 1.0;
    phase[1] = 0.0;
    return;
  }
  if (n & 1) {
    *logabs = -INFINITY;
    phase[0] = phase[1] = 0.0;
    return;
  }
  int64_t s = 0;
  for (int64_t j = 0; j < n; ++j) s += (ipiv[j] != j);
  c128 ph = {((s + n / 2) & 1) ? -1.0 : 1.0, 0.0};
  double la = 0.0;
  for (int64_t k = 0; k + 1 < n; k += 2) {
    const c128 t = T[k];
    const double a = hypot(t.re, t.im);
    if (a == 0.0) {
      *logabs = -INFINITY;
      phase[0] = phase[1] = 0.0;
      return;
    }
    la += log(a);
    ph = cmul(ph, c128{t.re / a, t.im / a});
  }
  *logabs = la;
  phase[0] = ph.re;
  phase[1] = ph.im;
}

struct CWork {
  c128* W;
  Best* part;
  int* status;
  size_t bytes;
};

CWork c128_carve(void* base, int64_t n) {
  CWork w{};
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = align_up(off + b, 256);
    return base ? (void*)((char*)base + o) : nullptr;
  };
  const int64_t m = std::max<int64_t>(n, 1);
  w.W = (c128*)take(sizeof(c128) * (size_t)m * m);
  w.part = (Best*)take(sizeof(Best) * (size_t)((m + 63) / 64 + 1));
  w.status = (int*)take(256);
  w.bytes = off;
  return w;
}

}  // namespace

size_t pfonly_c128_workspace_bytes(int64_t n) { return c128_carve(nullptr, n).bytes; }

int run_pfonly_c128(int64_t n, const double* A, int64_t lda, int32_t* ipiv, double* T, void* work, size_t lwork,
                    int* dinfo, hipStream_t s) {
  CWork w = c128_carve(work, n);
  if (lwork < w.bytes) return SKF_EWORK;
  if (n > 65535) return SKF_ENOTIMPL;  // one grid row per column of the copy
  int rc;
  if ((rc = launch_fill_i32(w.status, 1, 0, s))) return rc;
  if (n > 0 && (rc = launch_iota_i32(ipiv, (size_t)n, s))) return rc;
  if (n > 1 && (rc = launch_fill_u64((uint64_t*)T, (size_t)(n - 1) * 2, 0, s))) return rc;
  c128* Tc = (c128*)T;
  if (n >= 2 && n % 2 == 0) {
    const unsigned gx = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(form_full_kernel, dim3(gx, (unsigned)n), dim3(256), 0, s, n, (const c128*)A, lda, w.W);
    SKF_CHECK_LAUNCH("c128 form");
    hipLaunchKernelGGL(init_partials_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, n, w.W, w.part);
    SKF_CHECK_LAUNCH("c128 partials");
    for (int64_t k = 0; k + 1 < n; k += 2) {
      const unsigned gs = (unsigned)std::min<int64_t>((n - k + 255) / 256, 1024);
      hipLaunchKernelGGL(swap_kernel, dim3(gs), dim3(256), 0, s, n, k, w.W, Tc, ipiv, w.part, w.status);
      SKF_CHECK_LAUNCH("c128 swap");
      const int64_t m = n - k - 2;
      if (m > 0) {
        hipLaunchKernelGGL(update_kernel, dim3((unsigned)((m + 63) / 64), (unsigned)((m + 15) / 16)), dim3(64, 4), 0,
                           s, n, k, w.W, w.part, w.status);
        SKF_CHECK_LAUNCH("c128 update");
      }
    }
  }
  if (dinfo) {
    hipLaunchKernelGGL(info_c128_kernel, dim3(1), dim3(256), 0, s, n, Tc, w.status, dinfo);
    SKF_CHECK_LAUNCH("c128 info");
  }
  return 0;
}

int launch_logpf_c128(int64_t n, const int32_t* ipiv, const double* T, double* logabs, double* phase,
                      hipStream_t s) {
  hipLaunchKernelGGL(logpf_c128_kernel, dim3(1), dim3(64), 0, s, n, ipiv, (const c128*)T, logabs, phase);
  SKF_CHECK_LAUNCH("c128 logpf");
  return 0;
}

}  // namespace skf
