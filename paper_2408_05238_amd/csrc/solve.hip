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
//          block I accumulates -L_IJ Y_J as each Y_J is published (tagged
//          words, no fences) and finishes with Y_I = inv(L_II) acc;
//   T^{-1} the tridiagonal's even and odd rows as two bidiagonal triangular
//          systems (zero diagonal), one substitution chain each, run together;
//   L^{-T} the same blocked scheme from the last block upwards with the
//          transposed blocks;
//   scatter B[perm[i], :] = Z[i, :].
// L[i,j] (i > j >= 1) is read from LT[i, j-1]; L[:,0] = e_0.
#include <algorithm>
#include <mutex>

#include "skf_internal.h"

namespace skf {
namespace {

constexpr int BS = 64;        // row block of the triangular solves
constexpr int RC = 16;        // right-hand sides per pass
constexpr int NT = 256;

// A block of the solution is published to the other workgroups as tagged
// words: each double travels as two 64-bit words (tag << 32 | half), written
// and read with relaxed agent-scope atomics.  A reader takes a word only when it
// carries the expected tag, so no fence (and no cache write-back or
// invalidation) is needed, and the data words are their own ready flags.
__device__ inline uint64_t ld_word(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_word(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t tagged(uint32_t tag, uint32_t half) { return ((uint64_t)tag << 32) | half; }
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
  __shared__ __align__(16) int32_t sp[CH];
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t jmax = min(n - 1, (int64_t)(blockIdx.x + 1) * blockDim.x - 1);
  int64_t pos = (j < n) ? ipiv[j] : 0;
  for (int64_t hi = jmax; hi > 1; hi -= CH) {  // chunk covers s in [max(1, hi-CH), hi)
    const int64_t lo = max((int64_t)1, hi - CH);
    __syncthreads();
    {  // all of a thread's loads in flight before the first LDS write
      constexpr int kPer = CH / 256;
      int32_t v[kPer];
#pragma unroll
      for (int q = 0; q < kPer; ++q) v[q] = ipiv[min(lo + (int64_t)threadIdx.x + 256 * q, hi - 1)];
#pragma unroll
      for (int q = 0; q < kPer; ++q) {
        const int64_t s = lo + threadIdx.x + 256 * q;
        if (s < hi) sp[s - lo] = v[q];
      }
    }
    __syncthreads();
    // the scan order matters (the last match wins), the LDS reads do not: four
    // interchanges per 16-byte read once the index is aligned, unrolled so that
    // the reads issue in batches ahead of the compare chain
    const int64_t top = min(hi, j);  // only interchanges before j count
    int idx = (int)(top - lo) - 1;   // s = lo + idx
    for (; idx >= 0 && (idx & 3) != 3; --idx)
      if (sp[idx] == pos) pos = lo + idx;
#pragma unroll 4
    for (; idx >= 3; idx -= 4) {
      const int4 q = *reinterpret_cast<const int4*>(&sp[idx - 3]);
      if (q.w == pos) pos = lo + idx;
      if (q.z == pos) pos = lo + idx - 1;
      if (q.y == pos) pos = lo + idx - 2;
      if (q.x == pos) pos = lo + idx - 3;
    }
    for (; idx >= 0; --idx)
      if (sp[idx] == pos) pos = lo + idx;
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
// I = nb-1-b (backward) and publishes Y_I in `pub` (tagged words, value (r, c)
// of block I at pub + 2 ((I RC + c) BS + r)) once it is final.  The L block
// of the next J is fetched into registers (16 loads per thread from clamped
// addresses, masks applied afterwards) while the current one is waited for and
// multiplied, and lands in the other half of a double-buffered LDS tile.
constexpr int kLdPerThread = BS * BS / NT;  // 16

// Block products out = M y (M a 64 x 64 LDS block, y 64 x 16) on the FP64
// matrix cores: wave w forms the 16 x 16 tile of rows 16w .. 16w+15 in sixteen
// 16x16x4 steps (two accumulators, even and odd steps).  Lane l supplies
// M[16w + l % 16][4s + l / 16] and y[4s + l / 16][l % 16] at step s and holds
// out[16w + l / 16 + 4r][l % 16] in element r: two LDS reads per step and wave,
// where one row and four columns per lane took twenty per eight inner terms —
// the chain-critical product went from 2.2 us (LDS-bound) to a fraction.
typedef double mf4 __attribute__((ext_vector_type(4)));

__device__ inline mf4 tile_mm(const double (&M)[BS][BS + 1], const double (&y)[BS][RC + 1], int tid) {
  static_assert(NT == 4 * 64 && BS == 64 && RC == 16, "four waves, one 16 x 16 tile each");
  const int w = tid >> 6, l = tid & 63;
  const int ra = 16 * w + (l & 15), kq = l >> 4, cb = l & 15;
  mf4 e = {0.0, 0.0, 0.0, 0.0}, o = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s2 = 0; s2 < BS / 4; s2 += 2) {
    e = __builtin_amdgcn_mfma_f64_16x16x4f64(M[ra][4 * s2 + kq], y[4 * s2 + kq][cb], e, 0, 0, 0);
    o = __builtin_amdgcn_mfma_f64_16x16x4f64(M[ra][4 * s2 + 4 + kq], y[4 * s2 + 4 + kq][cb], o, 0, 0, 0);
  }
  return e + o;
}

// The output (row, column) of element r of thread tid in tile_mm's layout.
__device__ inline int tile_row(int tid, int r) { return 16 * (tid >> 6) + ((tid & 63) >> 4) + 4 * r; }
__device__ inline int tile_col(int tid) { return tid & 15; }

// acc -= Lb y over the 64 x 16 block (each thread its four outputs).
__device__ inline void block_mv(const double (&Lb)[BS][BS + 1], const double (&y)[BS][RC + 1],
                                double (&acc)[BS][RC + 1], int tid) {
  const mf4 d = tile_mm(Lb, y, tid);
  const int c = tile_col(tid);
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[tile_row(tid, r)][c] -= d[r];
}

// Fold blocks for the last term of each block's substitution: with Db and Lb
// the diagonal inverse and the chain-neighbour block exactly as the substitution
// holds them in LDS (J = I-1 forward, I+1 backward), M_I = Db Lb, stored so that
// element e of the substitution's load pattern sits at M + I BS^2 + e.
template <bool kTrans>
__global__ void __launch_bounds__(NT) fold_kernel(int64_t n, const double* __restrict__ LT, int64_t lda,
                                                  const double* __restrict__ Dinv, double* __restrict__ M) {
  __shared__ double Db[BS][BS + 1];
  __shared__ double Lb[BS][BS + 1];
  const int64_t nb = (n + BS - 1) / BS;
  const int64_t I = blockIdx.x;
  if (kTrans ? I + 1 >= nb : I == 0) return;
  const int64_t J = kTrans ? I + 1 : I - 1;
  const int64_t r0 = I * BS, c0 = J * BS;
  const int tid = threadIdx.x;
  const double* D = Dinv + I * BS * BS;
  for (int e = tid; e < BS * BS; e += NT) {
    const int i = kTrans ? e / BS : e % BS, j = kTrans ? e % BS : e / BS;
    Db[i][j] = kTrans ? D[j + i * BS] : D[i + j * BS];
    const int64_t a = kTrans ? c0 + j : r0 + i, b = kTrans ? r0 + i : c0 + j;
    Lb[i][j] = (a < n && b >= 1) ? LT[a + (b - 1) * lda] : 0.0;
  }
  __syncthreads();
  const int i = tid % BS, g = tid / BS;
  double m[BS / 4];
#pragma unroll
  for (int t = 0; t < BS / 4; ++t) m[t] = 0.0;
  for (int k = 0; k < BS; ++k) {
    const double d = Db[i][k];
#pragma unroll
    for (int t = 0; t < BS / 4; ++t) m[t] += d * Lb[k][(BS / 4) * g + t];
  }
#pragma unroll
  for (int t = 0; t < BS / 4; ++t) {
    const int j = (BS / 4) * g + t;
    M[I * BS * BS + (kTrans ? j + i * BS : i + j * BS)] = m[t];
  }
}

template <bool kTrans>
__global__ void __launch_bounds__(NT) trsv_kernel(int64_t n, const double* __restrict__ LT, int64_t lda,
                                                  const double* __restrict__ Dinv,
                                                  const double* __restrict__ Mfold, double* __restrict__ Y,
                                                  uint64_t* __restrict__ pub, uint32_t tag, int* status) {
  __shared__ double Lb[2][BS][BS + 1];
  __shared__ double Db[BS][BS + 1];  // inv(L_II), or its transpose (backward)
  __shared__ double yJ[2][BS][RC + 1];  // double-buffered like Lb: a fast thread may unpack
                                        // the next block while others still multiply
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
  {
    // the inverse diagonal block is needed only at the end: fetched now, off the chain
    const double* D = Dinv + I * BS * BS;
    for (int t = tid; t < BS * BS; t += NT) {
      const int i = t % BS, j = t / BS;
      Db[i][j] = kTrans ? D[j + i * BS] : D[i + j * BS];
    }
  }
  // element e = tid + NT q of a block: (i, j) = (e % BS, e / BS) forward, (e / BS, e % BS)
  // backward, so consecutive threads walk down a stored column of L either way
  auto elem = [&](int q, int* i, int* j) {
    const int e = tid + NT * q;
    *i = kTrans ? e / BS : e % BS;
    *j = kTrans ? e % BS : e / BS;
  };
  // L(a, b) (a > b) sits at LT[a + (b - 1) lda] for b >= 1; column 0 of L is e_0
  auto fetch = [&](int64_t J, double (&v)[kLdPerThread]) {
    const int64_t c0 = J * BS;
#pragma unroll
    for (int q = 0; q < kLdPerThread; ++q) {
      int i, j;
      elem(q, &i, &j);
      const int64_t a = kTrans ? c0 + j : r0 + i, b = kTrans ? r0 + i : c0 + j;
      const bool ok = a < n && b >= 1;
      v[q] = LT[ok ? a + (b - 1) * lda : 0];
    }
  };
  auto put = [&](int buf, int64_t J, const double (&v)[kLdPerThread]) {
    const int64_t c0 = J * BS;
#pragma unroll
    for (int q = 0; q < kLdPerThread; ++q) {
      int i, j;
      elem(q, &i, &j);
      const int64_t a = kTrans ? c0 + j : r0 + i, b = kTrans ? r0 + i : c0 + j;
      Lb[buf][i][j] = (a < n && b >= 1) ? v[q] : 0.0;
    }
  };
  // the fold block of I (element e at Mfold + I BS^2 + e, contiguous per thread group)
  auto fetch_fold = [&](double (&w8)[kLdPerThread]) {
#pragma unroll
    for (int q = 0; q < kLdPerThread; ++q) w8[q] = Mfold[I * BS * BS + tid + NT * q];
  };
  auto put_fold = [&](int buf, const double (&w8)[kLdPerThread]) {
#pragma unroll
    for (int q = 0; q < kLdPerThread; ++q) {
      int i, j;
      elem(q, &i, &j);
      Lb[buf][i][j] = w8[q];
    }
  };
  // contributions of the other blocks J (J < I forward, J > I backward), nearest-ready first
  const int64_t count = kTrans ? nb - 1 - I : I;
  const int64_t jfirst = kTrans ? nb - 1 : 0;
  const int64_t jstep = kTrans ? -1 : 1;
  double v[kLdPerThread];
  // Y_J: thread t takes values e = t + NT q, (j, c) = (e % BS, e / BS).  The words
  // of the next J are loaded while the current J is multiplied (most blocks are
  // final long before they are needed), then checked and reloaded until all
  // carry this solve's tag (bounded wait).
  uint64_t w[4][2];
  auto load_y = [&](int64_t J) {
    const uint64_t* pj = pub + (size_t)J * RC * BS * 2;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + NT * q;
      w[q][0] = ld_word(pj + 2 * e);
      w[q][1] = ld_word(pj + 2 * e + 1);
    }
  };
  // The last block J on the chain (I-1 forward, I+1 backward) is folded into the
  // diagonal solve: its slot holds M_I = inv(L_II) L_IJ (precomputed), P =
  // inv(L_II) acc is formed from the other blocks before Y_J is awaited, and then
  // Y_I = P - M_I Y_J is a single product.
  if (count > 0) {
    load_y(jfirst);
    if (count == 1) {
      fetch_fold(v);
      put_fold(0, v);
    } else {
      fetch(jfirst, v);
      put(0, jfirst, v);
    }
  }
  __syncthreads();
  bool folded = false;
  double s4[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t idx = 0; idx < count; ++idx) {
    const int64_t J = jfirst + idx * jstep;
    const int buf = (int)(idx & 1);
    const bool more = idx + 1 < count;
    const bool next_last = idx + 2 == count;
    if (more) {
      if (next_last) fetch_fold(v);
      else fetch(J + jstep, v);
    }
    if (!more) {
      __syncthreads();  // acc complete; Lb[buf] holds M_I
      const mf4 d = tile_mm(Db, acc, tid);
#pragma unroll
      for (int r = 0; r < 4; ++r) s4[r] = d[r];
    }
    {
      auto load_all = [&]() { load_y(J); };
      uint64_t t0 = 0;
      for (int it = 0;; ++it) {
        bool ok = true;
#pragma unroll
        for (int q = 0; q < 4; ++q) ok &= ((uint32_t)(w[q][0] >> 32) == tag) & ((uint32_t)(w[q][1] >> 32) == tag);
        if (ok) break;
        poll_refresh(it);
        // only the last blocks before a workgroup's own link are urgent: one
        // waiting for a block two or more ahead of its chain neighbour's backs
        // off between rounds (about 0.4 us), leaving the newest block's lines
        // to the readers that need them first
        if (idx + 2 < count) __builtin_amdgcn_s_sleep(16);
        if ((it & 31) == 0) {
          const uint64_t now = wall_clock64();
          if (it == 0) t0 = now;
          else if (now - t0 > kWaitTicks) {
            stop = 1;
            break;
          }
        }
        load_all();
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = tid + NT * q;
        yJ[buf][e % BS][e / BS] = __longlong_as_double((long long)((w[q][0] << 32) | (uint32_t)w[q][1]));
      }
      if (more) load_y(J + jstep);
    }
    __syncthreads();
    if (stop) break;
    if (!more) {
      const mf4 m = tile_mm(Lb[buf], yJ[buf], tid);
#pragma unroll
      for (int r = 0; r < 4; ++r) s4[r] -= m[r];
      folded = true;
      break;
    }
    block_mv(Lb[buf], yJ[buf], acc, tid);
    // the other buffer was last read before this iteration's barriers
    if (next_last) put_fold(buf ^ 1, v);
    else put(buf ^ 1, J + jstep, v);
  }
  __syncthreads();
  if (stop) {
    if (tid == 0) atomicMin(status, SKF_ETIMEOUT);
    // publish anyway so that dependants finish (their result is void)
    for (int e = tid; e < BS * RC; e += NT) {
      st_word(pub + (size_t)I * RC * BS * 2 + 2 * e, tagged(tag, 0));
      st_word(pub + (size_t)I * RC * BS * 2 + 2 * e + 1, tagged(tag, 0));
    }
    return;
  }
  // Y_I = inv(L_II) acc  (forward)  or  inv(L_II)^T acc  (backward), unless folded above
  {
    // each thread its four results in tile_mm's layout; acc is read-only here
    if (!folded) {
      const mf4 d = tile_mm(Db, acc, tid);
#pragma unroll
      for (int r = 0; r < 4; ++r) s4[r] = d[r];
    }
    const int c = tile_col(tid);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = tile_row(tid, r);
      const uint64_t b = (uint64_t)__double_as_longlong(s4[r]);
      uint64_t* pw = pub + 2 * (((size_t)I * RC + c) * BS + i);
      st_word(pw, tagged(tag, (uint32_t)(b >> 32)));
      st_word(pw + 1, tagged(tag, (uint32_t)b));
      if (i < bs) Y[r0 + i + (int64_t)c * n] = s4[r];
    }
  }
}

// T^{-1} on Y (n x RC columns, n even).  T has a zero diagonal, sub-diagonal
// T[k] and super-diagonal -T[k], so its even rows hold only odd unknowns and
// its odd rows only even ones:
//   row 2i:    T[2i-1] x_{2i-1} - T[2i] x_{2i+1} = y_{2i}     (no first term at i = 0)
//   row 2i+1:  T[2i] x_{2i}     - T[2i+1] x_{2i+2} = y_{2i+1}   (no second term at 2i+1 = n-1)
// i.e. two bidiagonal triangular systems whose diagonals are the even entries
// T[2i] (all nonzero exactly when T is nonsingular).  Each is solved by
// substitution, which is componentwise backward stable:
//   odd unknowns, forward:   x_{2i+1} = a_i x_{2i-1} + b_i,  a_i = T[2i-1] r_i,  b_i = -y_{2i} r_i
//   even unknowns, backward: x_{2i}   = c_i x_{2i+2} + d_i,  c_i = T[2i+1] r_i,  d_i = y_{2i+1} r_i
// with r_i = 1/T[2i]; the coefficients of a chunk of pairs are formed by all
// threads at once, so a chain step is one fused multiply-add.  Wave 0 carries
// the forward chain and wave 1 the backward one (lane = right-hand side), over
// chunks taken from both ends; the solution goes to Z (not Y), so neither
// chain can overwrite a right-hand side the other has still to read.  A
// singular T gives non-finite values here; B is then unspecified and the info
// word reports it.
constexpr int TC = 256;       // pairs per chunk (one per thread)
constexpr int TPAD = 8;       // guard entries on each side of a chunk row
constexpr int TS = TC + 2 * TPAD + 1;  // row stride: 16 lanes' rows in distinct LDS banks

__global__ void __launch_bounds__(256) tridiag_kernel(int64_t n, int nr, const double* __restrict__ T,
                                                      const double* __restrict__ Y, double* __restrict__ Z) {
  __shared__ double sa[2][TS];
  __shared__ double sb[2][RC][TS];
  const int tid = threadIdx.x;
  const int64_t np = n / 2;
  const int64_t nch = (np + TC - 1) / TC;
  const int w = tid >> 6, c = tid & 63;
  double x = 0.0;  // x_{2i-1} (wave 0) or x_{2i+2} (wave 1) carried across chunks
  for (int64_t ch = 0; ch < nch; ++ch) {
    // coefficients of pair p at entry TPAD + tid; pairs past the end are
    // identity steps (a = 1, b = 0: x passes through unchanged)
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int64_t p = (d == 0 ? ch : nch - 1 - ch) * TC + tid;
      double av = 1.0, bv[RC];
#pragma unroll
      for (int k = 0; k < RC; ++k) bv[k] = 0.0;
      if (p < np) {
        const double r = 1.0 / T[2 * p];
        const double t = (d == 0) ? (p > 0 ? T[2 * p - 1] : 0.0) : (2 * p + 2 < n ? T[2 * p + 1] : 0.0);
#pragma unroll
        for (int k = 0; k < RC; ++k) bv[k] = (k < nr) ? Y[2 * p + d + (int64_t)k * n] : 0.0;
        av = t * r;
#pragma unroll
        for (int k = 0; k < RC; ++k) bv[k] = (d == 0) ? -(bv[k] * r) : bv[k] * r;
      }
      sa[d][TPAD + tid] = av;
#pragma unroll
      for (int k = 0; k < RC; ++k) sb[d][k][TPAD + tid] = bv[k];
    }
    __syncthreads();
    // the chains: eight steps per block, the next block's coefficients read
    // while this one runs (the guard entries absorb the reads past the row)
    constexpr int G8 = 8;
    if (w == 0 && c < nr) {
      const double* aa = sa[0] + TPAD;
      double* bb = sb[0][c] + TPAD;
      double ca[G8], cb[G8];
#pragma unroll
      for (int u = 0; u < G8; ++u) {
        ca[u] = aa[u];
        cb[u] = bb[u];
      }
      for (int j0 = 0; j0 < TC; j0 += G8) {
        double na[G8], nb2[G8];
#pragma unroll
        for (int u = 0; u < G8; ++u) {
          na[u] = aa[j0 + G8 + u];
          nb2[u] = bb[j0 + G8 + u];
        }
#pragma unroll
        for (int u = 0; u < G8; ++u) {
          x = fma(ca[u], x, cb[u]);
          bb[j0 + u] = x;
        }
#pragma unroll
        for (int u = 0; u < G8; ++u) {
          ca[u] = na[u];
          cb[u] = nb2[u];
        }
      }
    } else if (w == 1 && c < nr) {
      const double* aa = sa[1] + TPAD + TC - 1;
      double* bb = sb[1][c] + TPAD + TC - 1;
      double ca[G8], cb[G8];
#pragma unroll
      for (int u = 0; u < G8; ++u) {
        ca[u] = aa[-u];
        cb[u] = bb[-u];
      }
      for (int j0 = 0; j0 < TC; j0 += G8) {
        double na[G8], nb2[G8];
#pragma unroll
        for (int u = 0; u < G8; ++u) {
          na[u] = aa[-(j0 + G8 + u)];
          nb2[u] = bb[-(j0 + G8 + u)];
        }
#pragma unroll
        for (int u = 0; u < G8; ++u) {
          x = fma(ca[u], x, cb[u]);
          bb[-(j0 + u)] = x;
        }
#pragma unroll
        for (int u = 0; u < G8; ++u) {
          ca[u] = na[u];
          cb[u] = nb2[u];
        }
      }
    }
    __syncthreads();
    // x_{2p+1} (forward chain) and x_{2p} (backward chain) to their rows of Z
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int64_t p = (d == 0 ? ch : nch - 1 - ch) * TC + tid;
      if (p < np) {
#pragma unroll
        for (int k = 0; k < RC; ++k)
          if (k < nr) Z[2 * p + 1 - d + (int64_t)k * n] = sb[d][k][TPAD + tid];
      }
    }
    __syncthreads();  // the chunk buffers are refilled next
  }
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

// Workspace: perm (n int32) | Dinv (nb*BS*BS) | Y (n*RC) | Z (n*RC) | published blocks
// (2*nb*BS*RC words) | status
struct SolveWork {
  int32_t* perm;
  double* Dinv;
  double* Mf;  // fold blocks, forward (nb*BS*BS)
  double* Mb;  // fold blocks, backward
  double* Y;
  double* Z;  // T^{-1} Y
  uint64_t* pub;
  int* status;
  size_t bytes;
};

// Byte sizes of the workspace parts for order n (each part 256-aligned).
struct SolveSizes {
  size_t perm, Dinv, Mf, Mb, Y, Z, pub, status;
};

constexpr int64_t at_least_1(int64_t v) { return v > 1 ? v : 1; }
constexpr size_t round256(size_t b) { return (b + 255) / 256 * 256; }

constexpr SolveSizes solve_sizes(int64_t n) {
  const int64_t nb = (n + BS - 1) / BS;
  return SolveSizes{round256(sizeof(int32_t) * (size_t)at_least_1(n)),
                    round256(sizeof(double) * (size_t)at_least_1(nb) * BS * BS),
                    round256(sizeof(double) * (size_t)at_least_1(nb) * BS * BS),
                    round256(sizeof(double) * (size_t)at_least_1(nb) * BS * BS),
                    round256(sizeof(double) * (size_t)at_least_1(n) * RC),
                    round256(sizeof(double) * (size_t)at_least_1(n) * RC),
                    round256(sizeof(uint64_t) * (size_t)at_least_1(nb) * BS * RC * 2),
                    round256(256)};
}

constexpr size_t solve_bytes(int64_t n) {
  const SolveSizes z = solve_sizes(n);
  return z.perm + z.Dinv + z.Mf + z.Mb + z.Y + z.Z + z.pub + z.status;
}

static SolveWork solve_carve(void* base, int64_t n) {
  const SolveSizes z = solve_sizes(n);
  SolveWork w{};
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off += b;
    return base ? (void*)((char*)base + o) : nullptr;
  };
  w.perm = (int32_t*)take(z.perm);
  w.Dinv = (double*)take(z.Dinv);
  w.Mf = (double*)take(z.Mf);
  w.Mb = (double*)take(z.Mb);
  w.Y = (double*)take(z.Y);
  w.Z = (double*)take(z.Z);
  w.pub = (uint64_t*)take(z.pub);
  w.status = (int*)take(z.status);
  w.bytes = off;
  return w;
}

size_t solve_workspace_bytes(int64_t n, int64_t nrhs) {
  (void)nrhs;
  return solve_carve(nullptr, n).bytes + 256;
}

// perm[j] = the original row at position j after the recorded interchanges.
int launch_solve_perm(int64_t n, const int32_t* ipiv, int32_t* perm, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(perm_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, ipiv, perm);
  SKF_CHECK_LAUNCH("perm");
  return 0;
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
    hipLaunchKernelGGL(fold_kernel<false>, dim3((unsigned)nb), dim3(NT), 0, s, n, LT, lda, w.Dinv, w.Mf);
    SKF_CHECK_LAUNCH("fold fwd");
    hipLaunchKernelGGL(fold_kernel<true>, dim3((unsigned)nb), dim3(NT), 0, s, n, LT, lda, w.Dinv, w.Mb);
    SKF_CHECK_LAUNCH("fold bwd");
    if ((rc = launch_fill_u64(w.pub, (size_t)nb * BS * RC * 2, 0, s))) return rc;
    unsigned gx = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    uint32_t tag = 0;
    for (int64_t c0 = 0; c0 < nrhs; c0 += RC) {
      const int nr = (int)std::min<int64_t>(RC, nrhs - c0);
      hipLaunchKernelGGL(gather_kernel, dim3(gx, RC), dim3(256), 0, s, n, nr, w.perm, B + c0 * ldb, ldb, w.Y);
      SKF_CHECK_LAUNCH("gather");
      ++tag;
      hipLaunchKernelGGL(trsv_kernel<false>, dim3((unsigned)nb), dim3(NT), 0, s, n, LT, lda, w.Dinv, w.Mf, w.Y,
                         w.pub, tag, w.status);
      SKF_CHECK_LAUNCH("trsv fwd");
      hipLaunchKernelGGL(tridiag_kernel, dim3(1), dim3(256), 0, s, n, nr, T, w.Y, w.Z);
      SKF_CHECK_LAUNCH("tridiag");
      ++tag;
      hipLaunchKernelGGL(trsv_kernel<true>, dim3((unsigned)nb), dim3(NT), 0, s, n, LT, lda, w.Dinv, w.Mb, w.Z,
                         w.pub, tag, w.status);
      SKF_CHECK_LAUNCH("trsv bwd");
      hipLaunchKernelGGL(scatter_kernel, dim3(gx, RC), dim3(256), 0, s, n, nr, w.perm, w.Z, B + c0 * ldb, ldb);
      SKF_CHECK_LAUNCH("scatter");
    }
  }
  hipLaunchKernelGGL(solve_info_kernel, dim3(1), dim3(256), 0, s, n, T, w.status, dinfo);
  SKF_CHECK_LAUNCH("solve info");
  return 0;
}

// ---------------------------------------------------------------------------
// Allocation-free solve: the workspace is a fixed device array of this file.
// ---------------------------------------------------------------------------
// Sized for the largest order it accepts (plus the internal info word); each
// device holds its own copy at its own address for the life of the process.
// Calls on one device share it, so calls that overlap on one device race.
constexpr size_t kNoAllocScratchBytes = solve_bytes(kSolveNoAllocMaxN) + 256;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

size_t solve_noalloc_scratch_bytes() { return kNoAllocScratchBytes; }

// Device address of this device's scratch array, resolved once per device (the
// array's name is a host-side stand-in and is never passed to a kernel).
static int scratch_address(void** out) {
  static std::mutex mu;
  static void* addr[64] = {nullptr};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return note_error(e, "solve_noalloc: hipGetDevice");
  if (dev < 0 || dev >= 64) return note_error(hipErrorInvalidDevice, "solve_noalloc: device index");
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return note_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "solve_noalloc: scratch");
    addr[dev] = p;
  }
  *out = addr[dev];
  return 0;
}

// run_solve on the fixed scratch: same kernels and arithmetic as the caller-
// workspace form.  With dinfo NULL the outcome goes through the scratch's info
// word and the call waits for the stream.
int run_solve_noalloc(int64_t n, int64_t nrhs, const double* LT, int64_t lda, const int32_t* ipiv,
                      const double* T, double* B, int64_t ldb, int* dinfo, hipStream_t s) {
  if (n > kSolveNoAllocMaxN) return SKF_ESCRATCH;
  void* base = nullptr;
  int rc = scratch_address(&base);
  if (rc) return rc;
  const size_t core = solve_bytes(n);
  int* dinfo_int = (int*)((char*)base + core);
  rc = run_solve(n, nrhs, LT, lda, ipiv, T, B, ldb, base, core, dinfo ? dinfo : dinfo_int, s);
  if (rc || dinfo) return rc;
  int h = 0;
  SKF_CHECK(hipMemcpyAsync(&h, dinfo_int, sizeof(int), hipMemcpyDeviceToHost, s), "solve_noalloc info copy");
  SKF_CHECK(hipStreamSynchronize(s), "solve_noalloc sync");
  return h;
}

}  // namespace skf
