// Skew-symmetric rank-2k update on the matrix cores (gfx950 MFMA).
//
// The update C += alpha (P Q^T - Q P^T) of a skew matrix is one product
// [P | Q] [Q | -P]^T with inner dimension 2k; only tiles on or below the
// diagonal are computed and only the strict lower triangle is stored, so the
// work is n^2 k flops for the lower half.  In the blocked LTL^T this update
// carries nearly all of the n^3/3 flops (P = l' and Q = w of the panel's paired
// elimination steps).
//
// Tiling: 128 x 128 C tile per 256-thread workgroup, four waves in 2 x 2, each
// wave 64 x 64 = 4 x 4 MFMA blocks of 16 x 16; the operands pass through LDS in
// K-slices of 16 with the next slice prefetched into registers.  FP64 uses
// v_mfma_f64_16x16x4f64, FP32 v_mfma_f32_16x16x4f32.  Operands: A lane l holds
// (row l%16, k l/16), B lane l holds (k l/16, column l%16).  Accumulator element
// r of lane l is column l%16 and row l/16 + 4r for FP64 but row 4(l/16) + r for
// FP32 (measured on gfx950 with a lane probe).
#include "skf_internal.h"

namespace skf {
namespace {

constexpr int TM = 128;      // C tile rows / columns
constexpr int KB = 16;       // K slice per LDS stage
constexpr int NTHR = 256;
constexpr int PAD = 4;       // LDS row padding (elements)
constexpr int LDS_LD = TM + PAD;

template <typename T>
struct Mfma;

template <>
struct Mfma<double> {
  typedef d4 acc_t;
  __device__ static inline d4 op(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <>
struct Mfma<float> {
  typedef f4 acc_t;
  __device__ static inline f4 op(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Lower-triangle tile (bi >= bj) of linear index x, row-major over block rows.
__device__ inline void tri_tile(int64_t x, int64_t* bi, int64_t* bj) {
  int64_t r = (int64_t)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
  while (r * (r + 1) / 2 > x) --r;
  while ((r + 1) * (r + 2) / 2 <= x) ++r;
  *bi = r;
  *bj = x - r * (r + 1) / 2;
}

// Logical tile of a workgroup: hardware dispatches consecutive workgroups
// round-robin over the 8 XCDs; remap so that each XCD walks a contiguous band
// of tiles (shared operand rows stay in that XCD's L2).
__device__ inline int64_t xcd_remap(int64_t b, int64_t nblocks) {
  const int64_t nx = 8;
  int64_t per = nblocks / nx;
  int64_t rem = nblocks % nx;
  int64_t x = b % nx, i = b / nx;
  // XCD x owns logical tiles [start(x), start(x) + count(x))
  int64_t start = x * per + (x < rem ? x : rem);
  int64_t count = per + (x < rem ? 1 : 0);
  if (i < count) return start + i;
  return b;  // not reached when nblocks is an exact dispatch
}

struct Operands {
  const double* P;
  int64_t ldp;
  const double* Q;
  int64_t ldq;
  int64_t k;  // columns of P and Q; inner dimension is 2k
};

// Element (row, q) of X = [P | Q] and of Y = [Q | -P]; zero outside.
__device__ inline double x_elem(const Operands& o, int64_t row, int64_t q, int64_t n) {
  if (row >= n || q >= 2 * o.k) return 0.0;
  return (q < o.k) ? o.P[row + q * o.ldp] : o.Q[row + (q - o.k) * o.ldq];
}
__device__ inline double y_elem(const Operands& o, int64_t row, int64_t q, int64_t n) {
  if (row >= n || q >= 2 * o.k) return 0.0;
  return (q < o.k) ? o.Q[row + q * o.ldq] : -o.P[row + (q - o.k) * o.ldp];
}

// Tile mainloop: acc[mi][ni] for the wave's 64x64 block of tile (i0, j0).
template <typename T>
__device__ inline void tile_mainloop(const Operands& o, int64_t n, int64_t i0, int64_t j0,
                                     T* Xs, T* Ys, typename Mfma<T>::acc_t acc[4][4]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) acc[a][b] = typename Mfma<T>::acc_t{0, 0, 0, 0};

  const int64_t K = 2 * o.k;
  const int64_t nkt = (K + KB - 1) / KB;
  // each thread stages 8 elements of each operand per slice: (row = e%128, col = e/128)
  T rx[8], ry[8];
  auto fetch = [&](int64_t kt) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int idx = tid + NTHR * e;
      int col = idx / TM, row = idx % TM;
      rx[e] = (T)x_elem(o, i0 + row, kt * KB + col, n);  // X rows of the tile's row block
      ry[e] = (T)y_elem(o, j0 + row, kt * KB + col, n);  // Y rows of the tile's column block
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      int idx = tid + NTHR * e;
      int col = idx / TM, row = idx % TM;
      Xs[col * LDS_LD + row] = rx[e];
      Ys[col * LDS_LD + row] = ry[e];
    }
  };
  if (nkt > 0) fetch(0);
  for (int64_t kt = 0; kt < nkt; ++kt) {
    __syncthreads();
    stash();
    __syncthreads();
    if (kt + 1 < nkt) fetch(kt + 1);
#pragma unroll
    for (int ks = 0; ks < KB / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      T av[4], bv[4];
#pragma unroll
      for (int mi = 0; mi < 4; ++mi) av[mi] = Xs[kk * LDS_LD + wm * 64 + mi * 16 + (lane & 15)];
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) bv[ni] = Ys[kk * LDS_LD + wn * 64 + ni * 16 + (lane & 15)];
#pragma unroll
      for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = Mfma<T>::op(av[mi], bv[ni], acc[mi][ni]);
    }
  }
}

// ---------------------------------------------------------------------------
// Plain in-place update
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(NTHR) skr2k_kernel(int64_t n, Operands o, double alpha,
                                                     double beta, double* C, int64_t ldc,
                                                     int64_t ntiles) {
  __shared__ T Xs[KB * LDS_LD];
  __shared__ T Ys[KB * LDS_LD];
  int64_t t = xcd_remap(blockIdx.x, ntiles);
  int64_t bi, bj;
  tri_tile(t, &bi, &bj);
  const int64_t i0 = bi * TM, j0 = bj * TM;
  typename Mfma<T>::acc_t acc[4][4];
  tile_mainloop<T>(o, n, i0, j0, Xs, Ys, acc);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
      const int64_t j = j0 + wn * 64 + ni * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wm * 64 + mi * 16 + Mfma<T>::row(lane, r);
        if (i < n && i > j) {
          double* cp = C + i + j * ldc;
          double u = alpha * (double)acc[mi][ni][r];
          *cp = (beta == 0.0) ? u : beta * (*cp) + u;
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Out-of-place trailing update through the panel permutation
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(NTHR) skr2k_perm_kernel(int64_t n, int64_t lo, Operands o,
                                                          const double* __restrict__ src,
                                                          int64_t lds, double* __restrict__ dst,
                                                          int64_t ldd,
                                                          const int32_t* __restrict__ pi,
                                                          const double* __restrict__ cnext,
                                                          int64_t ntiles) {
  __shared__ T Xs[KB * LDS_LD];
  __shared__ T Ys[KB * LDS_LD];
  __shared__ int32_t pr[TM], pc[TM];
  int64_t t = xcd_remap(blockIdx.x, ntiles);
  int64_t bi, bj;
  tri_tile(t, &bi, &bj);
  const int64_t i0 = lo + bi * TM, j0 = lo + bj * TM;
  if (threadIdx.x < TM) {
    int64_t i = i0 + threadIdx.x;
    pr[threadIdx.x] = (i < n) ? pi[i] : 0;
  } else {
    int64_t j = j0 + (threadIdx.x - TM);
    pc[threadIdx.x - TM] = (j < n) ? pi[j] : 0;
  }
  __syncthreads();
  typename Mfma<T>::acc_t acc[4][4];
  tile_mainloop<T>(o, n, i0, j0, Xs, Ys, acc);

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
      const int jl = wn * 64 + ni * 16 + (lane & 15);
      const int64_t j = j0 + jl;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int il = wm * 64 + mi * 16 + Mfma<T>::row(lane, r);
        const int64_t i = i0 + il;
        if (i < n && i > j) {
          double v;
          if (j == lo) {
            v = cnext[i];
          } else {
            const int64_t a = pr[il], b = pc[jl];
            const double s = (a > b) ? src[a + b * lds] : -src[b + a * lds];
            v = s + (double)acc[mi][ni][r];
          }
          dst[i + j * ldd] = v;
        }
      }
    }
}

}  // namespace

template <typename T>
static int launch_plain(int64_t n, int64_t k, double alpha, const double* X, int64_t ldx,
                        const double* Y, int64_t ldy, double beta, double* C, int64_t ldc,
                        hipStream_t s) {
  if (n < 2) return 0;
  const int64_t nt = (n + TM - 1) / TM;
  const int64_t ntiles = nt * (nt + 1) / 2;
  Operands o{X, ldx, Y, ldy, k};
  if (alpha == 0.0) o.k = 0;
  hipLaunchKernelGGL(skr2k_kernel<T>, dim3((unsigned)ntiles), dim3(NTHR), 0, s, n, o, alpha, beta,
                     C, ldc, ntiles);
  SKF_CHECK_LAUNCH("skr2k");
  return 0;
}

int launch_skr2k_f64(int64_t n, int64_t k, double alpha, const double* X, int64_t ldx,
                     const double* Y, int64_t ldy, double beta, double* C, int64_t ldc,
                     hipStream_t s) {
  return launch_plain<double>(n, k, alpha, X, ldx, Y, ldy, beta, C, ldc, s);
}

int launch_skr2k_f32(int64_t n, int64_t k, double alpha, const double* X, int64_t ldx,
                     const double* Y, int64_t ldy, double beta, double* C, int64_t ldc,
                     hipStream_t s) {
  return launch_plain<float>(n, k, alpha, X, ldx, Y, ldy, beta, C, ldc, s);
}

int launch_skr2k_perm(int64_t n, int64_t lo, int64_t npairs, const double* src, int64_t ld_src,
                      double* dst, int64_t ld_dst, const int32_t* pi, const double* Lp,
                      const double* Wp, int64_t ldp, const double* cnext, bool f32, hipStream_t s) {
  const int64_t m = n - lo;
  if (m < 2) return 0;
  const int64_t nt = (m + TM - 1) / TM;
  const int64_t ntiles = nt * (nt + 1) / 2;
  Operands o{Lp, ldp, Wp, ldp, npairs};
  if (f32)
    hipLaunchKernelGGL(skr2k_perm_kernel<float>, dim3((unsigned)ntiles), dim3(NTHR), 0, s, n, lo, o,
                       src, ld_src, dst, ld_dst, pi, cnext, ntiles);
  else
    hipLaunchKernelGGL(skr2k_perm_kernel<double>, dim3((unsigned)ntiles), dim3(NTHR), 0, s, n, lo,
                       o, src, ld_src, dst, ld_dst, pi, cnext, ntiles);
  SKF_CHECK_LAUNCH("skr2k_perm");
  return 0;
}

}  // namespace skf
