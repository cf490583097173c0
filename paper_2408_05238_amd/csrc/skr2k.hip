// Skew-symmetric rank-2k update on the matrix cores (gfx950 MFMA).
//
// The update C += alpha (P Q^T - Q P^T) of a skew matrix is one product
// X Y^T with X = [P | Q], Y = [Q | -P] and inner dimension K = 2k; only tiles
// on or below the diagonal are computed and only the strict lower triangle is
// stored, so the work is n^2 k flops.  In the blocked LTL^T this update carries
// nearly all of the n^3/3 flops (P = l', Q = w of the panel's paired steps).
//
// Tiling: a 256-thread workgroup owns a 128 x 128 tile of C; each of its four
// waves owns a 64 x 64 quarter (4 x 4 MFMA blocks of 16 x 16; a quarter lying
// wholly above the diagonal is skipped).  K is short (nb = 128), so operand
// fragments are loaded straight from global memory into registers, two
// k-steps ahead, with no LDS and no barriers; the 128 x nb operand panels of a
// tile row stay in L2 because consecutive tiles of one XCD walk a band of rows.
// In the trailing-update form the accumulators start from the permuted source
// tile, so the epilogue is a plain store.
//
// MFMA lane layouts (gfx950, measured with a lane probe): operand A lane l holds
// (row l%16, k l/16), operand B lane l holds (k l/16, column l%16); accumulator
// element r of lane l is column l%16 and row l/16 + 4r for
// v_mfma_f64_16x16x4f64, row 4(l/16) + r for v_mfma_f32_16x16x4f32.
#include "skf_internal.h"

namespace skf {
namespace {

constexpr int TM = 128;    // workgroup tile
constexpr int WT = 64;     // wave tile
constexpr int NTHR = 256;

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

// Hardware dispatches consecutive workgroups round-robin over the 8 XCDs;
// remap so that each XCD walks a contiguous band of tiles (a bijection).
__device__ inline int64_t xcd_remap(int64_t b, int64_t nblocks) {
  const int64_t nx = 8;
  const int64_t per = nblocks / nx, rem = nblocks % nx;
  const int64_t x = b % nx, i = b / nx;
  return x * per + (x < rem ? x : rem) + i;
}

struct Operands {
  const double* P;
  const double* Q;
  int64_t ldp, ldq;  // leading dimensions of P and Q
  int64_t k;         // columns of P and Q; K = 2k
  int64_t n;         // rows (loads clamp to n-1; rows >= n are never stored)
};

// One k-step (4 values of the inner index) of raw FP64 operand fragments.
// Loaded values are not touched until the k-step is consumed, so the loads of
// the next steps stay in flight under the current MFMAs.
struct Frag {
  double a[4], b[4];
};

// Fragments for inner indices c = kk + lane/16 of Xb (rows ra) and Yb (rows rb);
// masked: zero past k (only for the last, partial k-step).  Offsets are 32-bit
// byte offsets from wave-uniform bases (the launcher checks they fit).
template <bool kMasked>
__device__ inline void load_frag(const double* __restrict__ Xb, int64_t ldx, const double* __restrict__ Yb,
                                 int64_t ldy, const uint32_t ra[4], const uint32_t rb[4], int64_t k,
                                 int64_t kk, int lane, Frag& f) {
  const int64_t c = kk + (lane >> 4);
  const bool in = !kMasked || c < k;
  const uint32_t cx = in ? (uint32_t)(c * ldx) : 0u;
  const uint32_t cy = in ? (uint32_t)(c * ldy) : 0u;
  const char* xb = reinterpret_cast<const char*>(Xb);
  const char* yb = reinterpret_cast<const char*>(Yb);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f.a[t] = *reinterpret_cast<const double*>(xb + ((ra[t] + cx) << 3));
    f.b[t] = *reinterpret_cast<const double*>(yb + ((rb[t] + cy) << 3));
    if (kMasked && !in) {
      f.a[t] = 0.0;
      f.b[t] = 0.0;
    }
  }
}

// acc += (+-A) B^T for one k-step; the sign and the FP32 rounding are applied here.
template <typename T>
__device__ inline void mma_step(const Frag& f, bool negA, typename Mfma<T>::acc_t acc[4][4]) {
  T a[4], b[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    a[t] = (T)(negA ? -f.a[t] : f.a[t]);
    b[t] = (T)f.b[t];
  }
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = Mfma<T>::op(a[mi], b[ni], acc[mi][ni]);
}

// acc[mi][ni] += (P Q^T - Q P^T)[rA + 16 mi + ., rB + 16 ni + .], as the
// k-steps of P Q^T followed by those of (-Q) P^T in one software pipeline with
// four k-steps of operand loads in flight (about 4000 MFMA cycles of cover).
// mid() is called once, early in the second half, to issue the loads of the C
// tile; they are consumed only in the epilogue.
template <typename T, typename Mid>
__device__ inline void wave_mainloop(const Operands& o, int64_t rA, int64_t rB,
                                     typename Mfma<T>::acc_t acc[4][4], Mid&& mid) {
  const int lane = threadIdx.x & 63;
  uint32_t ra[4], rb[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t a = rA + t * 16 + (lane & 15), b = rB + t * 16 + (lane & 15);
    ra[t] = (uint32_t)(a < o.n ? a : o.n - 1);
    rb[t] = (uint32_t)(b < o.n ? b : o.n - 1);
  }
  const int64_t nsf = o.k >> 2;  // full k-steps per half
  const int64_t total = 2 * nsf;
  // Branch-free issue: a step past the end reloads the last step (discarded), so
  // every path has the same loads in flight and no wait lands inside the loop.
  auto issue = [&](int64_t st, Frag& f) {
    st = st < total ? st : total - 1;
    const bool h2 = st >= nsf;
    const double* Xb = h2 ? o.Q : o.P;
    const double* Yb = h2 ? o.P : o.Q;
    const int64_t ldx = h2 ? o.ldq : o.ldp, ldy = h2 ? o.ldp : o.ldq;
    load_frag<false>(Xb, ldx, Yb, ldy, ra, rb, o.k, (h2 ? st - nsf : st) * 4, lane, f);
  };
  if (total > 0 && (nsf & 3) == 0) {
    // four rotating fragments; the pipeline runs across the two halves
    Frag f0, f1, f2, f3;
    issue(0, f0);
    issue(1, f1);
    issue(2, f2);
    issue(3, f3);
    auto quad = [&](int64_t st, bool neg) {
      mma_step<T>(f0, neg, acc);
      issue(st + 4, f0);
      mma_step<T>(f1, neg, acc);
      issue(st + 5, f1);
      mma_step<T>(f2, neg, acc);
      issue(st + 6, f2);
      mma_step<T>(f3, neg, acc);
      issue(st + 7, f3);
    };
    for (int64_t st = 0; st < nsf; st += 4) quad(st, false);
    mid();  // the first four k-steps of the second half are already in flight
    for (int64_t st = nsf; st < total; st += 4) quad(st, true);
  } else if (total > 0) {
    Frag f0;
    for (int64_t st = 0; st < total; ++st) {
      if (st == nsf) mid();
      issue(st, f0);
      mma_step<T>(f0, st >= nsf, acc);
    }
  } else {
    mid();
  }
  if ((o.k & 3) != 0) {  // partial last k-step of each half
    Frag f;
    load_frag<true>(o.P, o.ldp, o.Q, o.ldq, ra, rb, o.k, nsf * 4, lane, f);
    mma_step<T>(f, false, acc);
    load_frag<true>(o.Q, o.ldq, o.P, o.ldp, ra, rb, o.k, nsf * 4, lane, f);
    mma_step<T>(f, true, acc);
  }
}

// ---------------------------------------------------------------------------
// Plain in-place update: C := beta C + alpha (P Q^T - Q P^T), strict lower.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(NTHR) skr2k_kernel(Operands o, double alpha, double beta, double* C,
                                                     int64_t ldc, int64_t ntiles) {
  const int64_t n = o.n;
  int64_t bi, bj;
  tri_tile(xcd_remap(blockIdx.x, ntiles), &bi, &bj);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  if (bi == bj && wm < wn) return;  // quarter wholly above the diagonal
  const int64_t i0 = bi * TM + wm * WT, j0 = bj * TM + wn * WT;
  if (i0 >= n) return;
  typename Mfma<T>::acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = typename Mfma<T>::acc_t{0, 0, 0, 0};
  // FP32 accumulators leave room to prefetch the C tile mid-loop; FP64 reads it at the end.
  constexpr bool kPre = sizeof(T) == 4;
  double cv[4][4][4];
  auto load_c = [&]() {
    if constexpr (kPre) {
#pragma unroll
      for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
          const int64_t j = j0 + ni * 16 + (lane & 15);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t i = i0 + mi * 16 + Mfma<T>::row(lane, r);
            cv[mi][ni][r] = (beta != 0.0 && i < n && i > j) ? C[i + j * ldc] : 0.0;
          }
        }
    }
  };
  if (alpha != 0.0) wave_mainloop<T>(o, i0, j0, acc, load_c);
  else load_c();
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
      const int64_t j = j0 + ni * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + mi * 16 + Mfma<T>::row(lane, r);
        if (i < n && i > j) {
          const double u = alpha * (double)acc[mi][ni][r];
          if (beta == 0.0) C[i + j * ldc] = u;
          else C[i + j * ldc] = beta * (kPre ? cv[mi][ni][r] : C[i + j * ldc]) + u;
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Out-of-place trailing update through the panel permutation:
//   dst[i,j] = (j == lo) ? cnext[i] : S(pi[i], pi[j]) + (P Q^T - Q P^T)[i,j]
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(NTHR) skr2k_perm_kernel(Operands o, int64_t lo,
                                                          const double* __restrict__ src, int64_t lds,
                                                          double* __restrict__ dst, int64_t ldd,
                                                          const int32_t* __restrict__ pi,
                                                          const double* __restrict__ cnext,
                                                          int64_t ntiles) {
  const int64_t n = o.n;
  int64_t bi, bj;
  tri_tile(xcd_remap(blockIdx.x, ntiles), &bi, &bj);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  if (bi == bj && wm < wn) return;
  const int64_t i0 = lo + bi * TM + wm * WT, j0 = lo + bj * TM + wn * WT;
  if (i0 >= n) return;
  // permutation of the tile's rows and columns, loaded once
  int32_t pa[4][4], pb[4];
#pragma unroll
  for (int ni = 0; ni < 4; ++ni) {
    const int64_t j = j0 + ni * 16 + (lane & 15);
    pb[ni] = (j < n) ? pi[j] : 0;
  }
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = i0 + mi * 16 + Mfma<T>::row(lane, r);
      pa[mi][r] = (i < n) ? pi[i] : 0;
    }
  // S(pi[i], pi[j]) of the tile; column lo takes the panel's next column instead
  auto src_val = [&](int mi, int ni, int r) -> double {
    const int64_t j = j0 + ni * 16 + (lane & 15);
    const int64_t i = i0 + mi * 16 + Mfma<T>::row(lane, r);
    if (!(i < n && i > j)) return 0.0;
    if (j == lo) return cnext[i];
    const int64_t a = pa[mi][r], b = pb[ni];
    return (a > b) ? src[a + b * lds] : -src[b + a * lds];
  };
  typename Mfma<T>::acc_t acc[4][4];
  if constexpr (sizeof(T) == 8) {
    // FP64 accumulates straight onto the source tile
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
      for (int ni = 0; ni < 4; ++ni)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[mi][ni][r] = src_val(mi, ni, r);
    wave_mainloop<T>(o, i0, j0, acc, [] {});
  } else {
    // FP32 products are added to the FP64 source tile in the epilogue
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = typename Mfma<T>::acc_t{0, 0, 0, 0};
    wave_mainloop<T>(o, i0, j0, acc, [] {});
  }
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
      const int64_t j = j0 + ni * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + mi * 16 + Mfma<T>::row(lane, r);
        if (i < n && i > j) {
          double v;
          if (j == lo) v = cnext[i];
          else if constexpr (sizeof(T) == 8) v = (double)acc[mi][ni][r];
          else v = src_val(mi, ni, r) + (double)acc[mi][ni][r];
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
  Operands o{X, Y, ldx, ldy, (alpha == 0.0) ? 0 : k, n};
  hipLaunchKernelGGL(skr2k_kernel<T>, dim3((unsigned)ntiles), dim3(NTHR), 0, s, o, alpha, beta, C, ldc,
                     ntiles);
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
  Operands o{Lp, Wp, ldp, ldp, npairs, n};
  if (f32)
    hipLaunchKernelGGL(skr2k_perm_kernel<float>, dim3((unsigned)ntiles), dim3(NTHR), 0, s, o, lo, src,
                       ld_src, dst, ld_dst, pi, cnext, ntiles);
  else
    hipLaunchKernelGGL(skr2k_perm_kernel<double>, dim3((unsigned)ntiles), dim3(NTHR), 0, s, o, lo, src,
                       ld_src, dst, ld_dst, pi, cnext, ntiles);
  SKF_CHECK_LAUNCH("skr2k_perm");
  return 0;
}

}  // namespace skf
