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
// wholly above the diagonal skips its products but still helps to load).  The
// inner dimension is walked in chunks of 8: the chunk's 128 x 8 slices of X
// (the tile's rows) and Y (its columns) are copied from global memory straight
// into LDS (global_load_lds, no registers), into a ring of four stages, so three
// chunks are in flight while the matrix cores work on the fourth; one barrier
// per chunk.  Registers stay under 256 per lane so that two workgroups share a
// CU and cover each other's barrier and epilogue waits.
// In the trailing-update form the accumulators start from the permuted source
// tile, so the epilogue is a plain store.
//
// MFMA lane layouts (gfx950, measured with a lane probe): operand A lane l holds
// (row l%16, k l/16), operand B lane l holds (k l/16, column l%16); accumulator
// element r of lane l is column l%16 and row l/16 + 4r for
// v_mfma_f64_16x16x4f64, row 4(l/16) + r for v_mfma_f32_16x16x4f32.
// Each 16 x 16 block is formed transposed, as Y X^T (A = Y, B = X^T), so that
// accumulator element r of lane l is C row l%16 and C column row(l, r): one
// load or store instruction of the source or result tile then covers 16
// consecutive rows of four columns, i.e. four whole 128-byte lines of the
// column-major matrix, instead of 32-byte pieces of sixteen lines.
#include "skf_internal.h"

namespace skf {
namespace {

constexpr int TM = 128;     // workgroup tile
constexpr int WT = 64;      // wave tile
constexpr int NTHR = 256;
constexpr int KC = 8;       // inner terms per LDS chunk
constexpr int NSTG = 4;     // LDS stages: three chunks in flight ahead of the one multiplied
constexpr int LSTR = TM + 16;  // doubles per staged column: consecutive k-groups land 128 B apart in the banks

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

// Tile of linear index x when the lower triangle of nt x nt tiles is walked in
// bands of kBand block rows: inside a band, column block by column block, the
// band's rows at or below the diagonal.  Tiles running together then share a
// few row and column blocks of the operands, which stay in L2.  The band height
// comes from the tuning table (8 without an entry).
__device__ inline void band_tile(int64_t x, int64_t ntiles, int64_t kBand, int64_t* bi, int64_t* bj) {
  int64_t nt, r, c0;
  tri_tile(ntiles - 1, &nt, &c0);
  ++nt;
  tri_tile(x, &r, &c0);
  const int64_t t = (r / kBand) * kBand;     // first block row of the band
  const int64_t R = min(kBand, nt - t);      // block rows in the band
  int64_t y = x - t * (t + 1) / 2;           // offset inside the band
  if (y < t * R) {
    *bj = y / R;
    *bi = t + y % R;
    return;
  }
  y -= t * R;
  int64_t c = 0;
  while (y >= R - c) {
    y -= R - c;
    ++c;
  }
  *bj = t + c;
  *bi = t + c + y;
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
  const double* NP;  // -P (leading dimension ldp) or null: the second half's Y
  int64_t ldp, ldq;  // leading dimensions of P and Q
  int64_t k;         // columns of P and Q; K = 2k
  int64_t n;         // rows (loads clamp to n-1; rows >= n are never stored)
};

struct Stage {
  double X[KC][LSTR];  // X rows of the tile's row block, k-major
  double Y[KC][LSTR];  // Y rows of the tile's column block
};

// Global -> LDS copy of one wave: lane l's VEC bytes land at lds + VEC * l.
// Issued as inline assembly so that the only waits on these copies are the
// explicit vmcnt waits of the main loop (a load issued here is never consumed
// through a register).
template <int VEC>
__device__ inline void dma(const void* g, uint32_t lds) {
  if constexpr (VEC == 16)
    asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(g), "s"(lds) : "memory");
  else
    asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dword %0, off" ::"v"(g), "s"(lds) : "memory");
}

// Copies issued per wave and chunk: each wave stages 2 columns of X and 2 of Y;
// a 128-double column is one 16-byte-lane copy or four 4-byte-lane copies.
template <int VEC>
constexpr int kCopiesPerChunk = (VEC == 16) ? 4 : 16;

// Issue chunk c (inner terms 8c.. of P Q^T for c < nh, of Q (-P)^T after) into
// stage s; with o.NP the second half stages -P itself, otherwise P (negated in
// registers).  Columns past k are reloaded from a valid column and masked in
// chunk_mma; rows past n are clamped to valid rows (never stored).  VEC = 16
// needs 16-byte aligned bases, even leading dimensions and, for odd n, one
// padding row (the launcher checks).
template <int VEC>
__device__ inline void chunk_issue(const Operands& o, int64_t c, int64_t nh, int64_t rI, int64_t rJ, Stage& s) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool h2 = c >= nh;
  const int64_t kk = (h2 ? c - nh : c) * KC;
  const double* Xb = h2 ? o.Q : o.P;
  const double* Yb = h2 ? (o.NP ? o.NP : o.P) : o.Q;
  const int64_t ldx = h2 ? o.ldq : o.ldp, ldy = h2 ? o.ldp : o.ldq;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int col = 2 * wv + u;
    const int64_t kc = (kk + col < o.k) ? kk + col : kk;
    const double* xc = Xb + kc * ldx;
    const double* yc = Yb + kc * ldy;
    const uint32_t lx = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)&s.X[col][0]);
    const uint32_t ly = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)&s.Y[col][0]);
    if constexpr (VEC == 16) {
      const int64_t rmax = (o.n - 1) & ~(int64_t)1;
      const int64_t ra = min(rI + 2 * lane, rmax), rb = min(rJ + 2 * lane, rmax);
      dma<16>(xc + ra, lx);
      dma<16>(yc + rb, ly);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t ra = min(rI + 32 * i + (lane >> 1), o.n - 1), rb = min(rJ + 32 * i + (lane >> 1), o.n - 1);
        dma<4>(reinterpret_cast<const char*>(xc + ra) + 4 * (lane & 1), lx + 256 * i);
        dma<4>(reinterpret_cast<const char*>(yc + rb) + 4 * (lane & 1), ly + 256 * i);
      }
    }
  }
}

// acc += (+-X) Y^T over one staged chunk (two k-steps of 4); terms past k are
// zero.  The mask is an integer AND on the loaded bits, so no per-lane branch
// separates an LDS read from its use (and a masked value is exactly 0).
// kPlain: every term is valid and the staged operands carry their signs, so
// the fragments go from LDS to the matrix cores untouched.
template <typename T, bool kPlain>
__device__ inline void chunk_mma(const Stage& s, int wr, int wc, bool neg, int64_t kvalid,
                                 typename Mfma<T>::acc_t acc[4][4]) {
  const int lane = threadIdx.x & 63;
  const int kq = lane >> 4, rr = lane & 15;
  // both k-steps' fragments are read before the first product, so the second
  // step's LDS latency hides under the first step's products
  T a[KC / 4][4], b[KC / 4][4];
#pragma unroll
  for (int ks = 0; ks < KC / 4; ++ks) {
    const uint64_t keep = (4 * ks + kq < kvalid) ? ~0ull : 0ull;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double va = s.X[4 * ks + kq][wr + 16 * t + rr];
      if constexpr (kPlain) {
        a[ks][t] = (T)va;
      } else {
        const double sa = __longlong_as_double((long long)((uint64_t)__double_as_longlong(neg ? -va : va) & keep));
        a[ks][t] = (T)sa;
      }
      b[ks][t] = (T)s.Y[4 * ks + kq][wc + 16 * t + rr];
    }
  }
#pragma unroll
  for (int ks = 0; ks < KC / 4; ++ks)
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) acc[mi][ni] = Mfma<T>::op(b[ks][ni], a[ks][mi], acc[mi][ni]);
}

// Wait until this wave's copies of the chunk before the last `later` issued
// chunks have landed (loads complete in order).
template <int VEC>
__device__ inline void wait_chunk(int later) {
  constexpr int P = kCopiesPerChunk<VEC>;
  // s_waitcnt: vmcnt[3:0] bits 0-3, expcnt bits 4-6, lgkmcnt bits 8-11, vmcnt[5:4] bits 14-15
  constexpr int enc2 = ((2 * P) & 15) | (7 << 4) | (15 << 8) | (((2 * P) >> 4) << 14);
  constexpr int enc1 = (P & 15) | (7 << 4) | (15 << 8) | ((P >> 4) << 14);
  constexpr int enc0 = (7 << 4) | (15 << 8);
  if (later >= 2) __builtin_amdgcn_s_waitcnt(enc2);
  else if (later == 1) __builtin_amdgcn_s_waitcnt(enc1);
  else __builtin_amdgcn_s_waitcnt(enc0);
}

// The workgroup's main loop: acc[mi][ni] of the calling wave accumulates
// (P Q^T - Q P^T)[rI + wr + 16 mi + ., rJ + wc + 16 ni + .].  Every wave of the
// workgroup must call it (it contains barriers); `active` waves do the products.
// pro() runs once while the first chunks are in flight (the trailing update
// issues its source-tile gathers there, so the latencies overlap).
template <typename T, int VEC, bool kPlain, typename Pro>
__device__ inline void tile_mainloop(const Operands& o, int64_t rI, int64_t rJ, int wr, int wc, bool active,
                                     Stage* st, typename Mfma<T>::acc_t acc[4][4], Pro&& pro) {
  const int64_t nh = (o.k + KC - 1) / KC;
  const int64_t nch = 2 * nh;
  if (nch == 0) {
    pro();
    return;
  }
  const int64_t pre = nch < NSTG - 1 ? nch : NSTG - 1;
  for (int64_t c = 0; c < pre; ++c) chunk_issue<VEC>(o, c, nh, rI, rJ, st[c]);
  pro();
  for (int64_t c = 0; c < nch; ++c) {
    const int64_t later = min((int64_t)NSTG - 2, nch - 1 - c);  // chunks issued after c so far
    wait_chunk<VEC>((int)later);
    __builtin_amdgcn_s_barrier();  // chunk c visible to all waves; stage (c-1) % NSTG free
    if (c + NSTG - 1 < nch) chunk_issue<VEC>(o, c + NSTG - 1, nh, rI, rJ, st[(c + NSTG - 1) % NSTG]);
    if (active) {
      const int64_t kk = (c >= nh ? c - nh : c) * KC;
      chunk_mma<T, kPlain>(st[c % NSTG], wr, wc, c >= nh && !o.NP, o.k - kk, acc);
    }
  }
}

// ---------------------------------------------------------------------------
// Plain in-place update: C := beta C + alpha (P Q^T - Q P^T), strict lower.
// ---------------------------------------------------------------------------
template <typename T, int VEC>
__global__ void __launch_bounds__(NTHR, 2) skr2k_kernel(Operands o, double alpha, double beta, double* C,
                                                        int64_t ldc, int64_t ntiles, int64_t band) {
  __shared__ Stage st[NSTG];
  const int64_t n = o.n;
  int64_t bi, bj;
  band_tile(xcd_remap(blockIdx.x, ntiles), ntiles, band, &bi, &bj);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t rI = bi * TM, rJ = bj * TM;
  const int64_t i0 = rI + wm * WT, j0 = rJ + wn * WT;
  // a quarter wholly above the diagonal, or below the last row, has no products
  const bool active = !(bi == bj && wm < wn) && i0 < n;
  typename Mfma<T>::acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = typename Mfma<T>::acc_t{0, 0, 0, 0};
  if (alpha != 0.0) tile_mainloop<T, VEC, false>(o, rI, rJ, wm * WT, wn * WT, active, st, acc, [] {});
  if (!active) return;
  // Epilogue by 16-row slices: the slice's 16 loads of C are issued together
  // (clamped addresses, no branch around a load), then combined and stored.
#pragma unroll
  for (int mi = 0; mi < 4; ++mi) {
    double cv[4][4];
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + mi * 16 + (lane & 15), j = j0 + ni * 16 + Mfma<T>::row(lane, r);
        const bool st_ok = i < n && i > j;
        cv[ni][r] = (beta != 0.0) ? C[st_ok ? i + j * ldc : 0] : 0.0;
      }
    }
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + mi * 16 + (lane & 15), j = j0 + ni * 16 + Mfma<T>::row(lane, r);
        if (i < n && i > j) {
          const double u = alpha * (double)acc[mi][ni][r];
          C[i + j * ldc] = (beta == 0.0) ? u : beta * cv[ni][r] + u;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Out-of-place trailing update through the panel permutation:
//   dst[i,j] = (j == lo) ? cnext[i] : S(pi[i], pi[j]) + (P Q^T - Q P^T)[i,j]
// Column lo starts from cnext and gets no products because row lo of P and Q
// is zero (the panel stores it so); the epilogue is a plain masked store.
// ---------------------------------------------------------------------------
template <typename T, int VEC, bool kPlain>
__global__ void __launch_bounds__(NTHR, 2) skr2k_perm_kernel(Operands o, int64_t lo,
                                                             const double* __restrict__ src, int64_t lds,
                                                             double* __restrict__ dst, int64_t ldd,
                                                             const int32_t* __restrict__ pi,
                                                             const double* __restrict__ cnext,
                                                             int64_t ntiles, int64_t band) {
  __shared__ Stage st[NSTG];
  const int64_t n = o.n;
  int64_t bi, bj;
  band_tile(xcd_remap(blockIdx.x, ntiles), ntiles, band, &bi, &bj);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t rI = lo + bi * TM, rJ = lo + bj * TM;
  const int64_t i0 = rI + wm * WT, j0 = rJ + wn * WT;
  const bool active = !(bi == bj && wm < wn) && i0 < n;
  // Source tile S(pi[i], pi[j]) (column lo: the panel's next column).  Every
  // address is formed first and all 64 loads per lane are issued at once into
  // v; the masks (inside the strict lower triangle) and the signs (upper-storage
  // reads) are applied after a single wait.
  // The tile's permutation is loaded first and waited for before the first
  // operand copies are issued (a wait issued after them would drain them too).
  int32_t pa[4], pb[4][4];
#pragma unroll
  for (int mi = 0; mi < 4; ++mi) {
    const int64_t i = i0 + mi * 16 + (lane & 15);
    pa[mi] = pi[i < n ? i : n - 1];
  }
#pragma unroll
  for (int ni = 0; ni < 4; ++ni)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t j = j0 + ni * 16 + Mfma<T>::row(lane, r);
      pb[ni][r] = pi[j < n ? j : n - 1];
    }
  {
    int32_t all = pa[0] ^ pa[1] ^ pa[2] ^ pa[3];
#pragma unroll
    for (int ni = 0; ni < 4; ++ni) all ^= pb[ni][0] ^ pb[ni][1] ^ pb[ni][2] ^ pb[ni][3];
    asm volatile("" ::"v"(all));
  }
  uint64_t ok = 0, neg = 0;
  auto gather = [&](int m_lo, int m_hi, auto&& put) {
#pragma unroll
    for (int mi = m_lo; mi < m_hi; ++mi) {
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = i0 + mi * 16 + (lane & 15), j = j0 + ni * 16 + Mfma<T>::row(lane, r);
          const bool valid = i < n && i > j;
          const int64_t a = pa[mi], b = pb[ni][r];
          const bool lower = a > b;
          const double* p = (j == lo) ? cnext + (i < n ? i : n - 1) : src + (lower ? a + b * lds : b + a * lds);
          put(mi, ni, r, *p);
          const int e = (mi * 4 + ni) * 4 + r;
          ok |= (uint64_t)valid << e;
          neg |= (uint64_t)(j != lo && !lower) << e;
        }
      }
    }
  };
  auto fix = [&](double& x, int e) {
    const double y = ((neg >> e) & 1u) ? -x : x;
    x = ((ok >> e) & 1u) ? y : 0.0;
  };
  typename Mfma<T>::acc_t acc[4][4];
  if constexpr (sizeof(T) == 8) {
    // FP64 accumulates straight onto the source tile, gathered while the
    // first operand chunk is loading
    tile_mainloop<T, VEC, kPlain>(o, rI, rJ, wm * WT, wn * WT, active, st, acc, [&] {
      // all 64 loads per lane in flight at once, straight into the
      // accumulators (one memory latency instead of four); masks and signs
      // applied in place once they have landed
      if (active) {
        gather(0, 4, [&](int mi, int ni, int r, double x) { acc[mi][ni][r] = x; });
      } else {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = typename Mfma<T>::acc_t{0, 0, 0, 0};
      }
#pragma unroll
      for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            double x = acc[mi][ni][r];
            fix(x, (mi * 4 + ni) * 4 + r);
            acc[mi][ni][r] = x;
          }
    });
    if (!active) return;
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
      for (int ni = 0; ni < 4; ++ni) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = i0 + mi * 16 + (lane & 15), j = j0 + ni * 16 + Mfma<T>::row(lane, r);
          if (i < n && i > j) dst[i + j * ldd] = acc[mi][ni][r];
        }
      }
  } else {
    // FP32 products are added to the FP64 source tile in the epilogue
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = typename Mfma<T>::acc_t{0, 0, 0, 0};
    tile_mainloop<T, VEC, kPlain>(o, rI, rJ, wm * WT, wn * WT, active, st, acc, [] {});
    if (!active) return;
    // two halves of 32 rows: 32 source loads per lane in flight at a time
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double v[2][4][4];
      gather(2 * h, 2 * h + 2, [&](int mi, int ni, int r, double x) { v[mi - 2 * h][ni][r] = x; });
#pragma unroll
      for (int mm = 0; mm < 2; ++mm)
#pragma unroll
        for (int ni = 0; ni < 4; ++ni) {
          const int mi = 2 * h + mm;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t i = i0 + mi * 16 + (lane & 15), j = j0 + ni * 16 + Mfma<T>::row(lane, r);
            double x = v[mm][ni][r];
            fix(x, (mi * 4 + ni) * 4 + r);
            x += (double)acc[mi][ni][r];
            if (i < n && i > j) dst[i + j * ldd] = x;
          }
        }
    }
  }
}

}  // namespace

// Band height of the tile walk for a trailing order m.
int skr2k_band(int64_t m) {
  const int t = tune_lookup(SKF_TUNE_SKR2K_BAND, m);
  return t > 0 ? t : 8;
}

// 16-byte copies need 16-byte aligned operand bases, even leading dimensions and
// a readable padding row when n is odd (rows are copied in pairs).
static bool vec16_ok(const double* p, int64_t ld, int64_t n) {
  return ((uintptr_t)p & 15) == 0 && (ld & 1) == 0 && ((n & 1) == 0 || ld > n);
}

template <typename T>
static int launch_plain(int64_t n, int64_t k, double alpha, const double* X, int64_t ldx,
                        const double* Y, int64_t ldy, double beta, double* C, int64_t ldc,
                        hipStream_t s) {
  if (n < 2) return 0;
  const int64_t nt = (n + TM - 1) / TM;
  const int64_t ntiles = nt * (nt + 1) / 2;
  Operands o{X, Y, nullptr, ldx, ldy, (alpha == 0.0) ? 0 : k, n};
  if (o.k > 0 && vec16_ok(X, ldx, n) && vec16_ok(Y, ldy, n))
    hipLaunchKernelGGL((skr2k_kernel<T, 16>), dim3((unsigned)ntiles), dim3(NTHR), 0, s, o, alpha, beta, C, ldc,
                       ntiles, (int64_t)skr2k_band(n));
  else
    hipLaunchKernelGGL((skr2k_kernel<T, 4>), dim3((unsigned)ntiles), dim3(NTHR), 0, s, o, alpha, beta, C, ldc,
                       ntiles, (int64_t)skr2k_band(n));
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

template <typename T, int VEC, bool kPlain>
static void launch_perm_t(const Operands& o, int64_t lo, const double* src, int64_t ld_src, double* dst,
                          int64_t ld_dst, const int32_t* pi, const double* cnext, int64_t ntiles, hipStream_t s) {
  hipLaunchKernelGGL((skr2k_perm_kernel<T, VEC, kPlain>), dim3((unsigned)ntiles), dim3(NTHR), 0, s, o, lo, src,
                     ld_src, dst, ld_dst, pi, cnext, ntiles, (int64_t)skr2k_band(o.n - lo));
}

template <typename T>
static void launch_perm(const Operands& o, bool v16, int64_t lo, const double* src, int64_t ld_src, double* dst,
                        int64_t ld_dst, const int32_t* pi, const double* cnext, int64_t ntiles, hipStream_t s) {
  const bool plain = o.NP != nullptr;
  if (v16 && plain) launch_perm_t<T, 16, true>(o, lo, src, ld_src, dst, ld_dst, pi, cnext, ntiles, s);
  else if (v16) launch_perm_t<T, 16, false>(o, lo, src, ld_src, dst, ld_dst, pi, cnext, ntiles, s);
  else launch_perm_t<T, 4, false>(o, lo, src, ld_src, dst, ld_dst, pi, cnext, ntiles, s);
}

int launch_skr2k_perm(int64_t n, int64_t lo, int64_t npairs, const double* src, int64_t ld_src,
                      double* dst, int64_t ld_dst, const int32_t* pi, const double* Lp,
                      const double* Wp, const double* NLp, int64_t ldp, const double* cnext, bool f32,
                      hipStream_t s) {
  const int64_t m = n - lo;
  if (m < 2) return 0;
  const int64_t nt = (m + TM - 1) / TM;
  const int64_t ntiles = nt * (nt + 1) / 2;
  const bool v16 = vec16_ok(Lp, ldp, n) && vec16_ok(Wp, ldp, n) && (!NLp || vec16_ok(NLp, ldp, n));
  // the sign-free inner loop needs -Lp staged and no partial chunk
  const bool plain = NLp != nullptr && npairs % KC == 0;
  Operands o{Lp, Wp, plain ? NLp : nullptr, ldp, ldp, npairs, n};
  if (f32) launch_perm<float>(o, v16, lo, src, ld_src, dst, ld_dst, pi, cnext, ntiles, s);
  else launch_perm<double>(o, v16, lo, src, ld_src, dst, ld_dst, pi, cnext, ntiles, s);
  SKF_CHECK_LAUNCH("skr2k_perm");
  return 0;
}

}  // namespace skf
