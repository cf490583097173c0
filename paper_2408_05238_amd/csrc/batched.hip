// Batched skew LTL^T + Pfaffian: many independent matrices (n <= 512) in ONE
// persistent launch.
//
// Each 512-thread workgroup takes matrix indices from a device work queue
// (largest n first, so the long factorizations start early) and factors one
// matrix at a time in its own storage, with no inter-workgroup communication:
//   * interchanges are applied eagerly to the matrix (the O(n) row/column
//     segments of the symmetric interchange, lower storage) and to the LDS rows;
//   * elimination steps are paired as in the single-matrix path: a pair (k,k+1)
//     contributes one skew rank-2 term l' w^T - w l'^T to the trailing matrix,
//     and the next pair's first column is w + alpha' (l - l_0 l');
//   * updates are delayed over a panel of nb = 16 steps: each new pivot column
//     is the stored (panel-start) column plus a skew GEMV with the panel's
//     pairs (kept in LDS), and the trailing matrix receives one rank-16 update
//     per panel;
//   * the interchange reads the pivot row/column once and thereby also obtains
//     the next column, so a step costs one memory round trip plus LDS work.
// Outputs per matrix: L in place (as skf_ltlt), T, ipiv (optional), log|Pf|,
// sign and the numerical outcome.
#include <algorithm>
#include <numeric>
#include <vector>

#include "skf_internal.h"

namespace skf {
namespace {

constexpr int BR = 512;   // largest order handled per workgroup
constexpr int BNP = 8;    // pairs per panel (nb = 16): the LDS fits two workgroups per CU
constexpr int kWgPerCu = 2;
constexpr int BT = 512;   // threads: one row per thread, two workgroups (16 waves) per CU
constexpr int RPT = BR / BT;
// two 512-thread workgroups per CU are four waves per SIMD: registers capped at
// 128 per lane (the launch-bounds form alone let them grow to 161)
constexpr int kWavesPerSimd = kWgPerCu * BT / 256;

struct BatchArgs {
  int64_t batch;
  const int64_t* order;   // matrix indices, largest first
  const int64_t* nn;      // order of each matrix
  const int64_t* lda;
  double* const* A;
  int32_t* const* ipiv;   // may be null (then scratch)
  double* const* T;       // may be null (then scratch)
  double* logabs;
  int* sign;
  int* info;
  int* queue;             // next position in `order`
  int32_t* ipiv_scratch;  // gridDim.x x BR
  double* T_scratch;      // gridDim.x x BR
};

struct Smem {
  double2 LW[BNP][BR];  // (l', w) of the panel's pairs, by current row
  double Le[BR];        // multipliers of the current pair's first step
  double cur[BR];       // current pivot column
  double rv[BT / 64];
  int rp[BT / 64];
  double sum[BT];
  int par[BT];
  int item;
  int piv;
  double alpha, l0;
  double akk;  // Pfaffian-only form: A[k+2, k+1] before the step's interchange
};

// sum over the panel's pairs q < np of l'_q[i] w_q[c] - w_q[i] l'_q[c] (the
// correction of entry (i, c) by the pairs so far).  Pairs are read four at a
// time, all eight LDS operands issued before any is used; pairs np .. 4*ceil(np/4)-1
// are the zero rows the panel start left, adding exactly nothing.
__device__ inline double skew_dot(const double2 (&LW)[BNP][BR], int i, int64_t c, int np) {
  static_assert(BNP % 4 == 0, "pairs are read in groups of four");
  double s = 0.0;
  for (int q0 = 0; q0 < np; q0 += 4) {
    double2 u[4], w[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      u[t] = LW[q0 + t][i];
      w[t] = LW[q0 + t][c];
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) s = fma(-u[t].y, w[t].x, fma(u[t].x, w[t].y, s));
  }
  return s;
}

__device__ inline bool better(double a, int pa, double b, int pb) { return (a > b) || (a == b && pa < pb); }

// block arg-max of (v, p) (larger v, then lower p); result broadcast.  The
// callers pass other barriers before the next call, so the per-wave slots need
// no barrier of their own after they are read.
__device__ inline void block_argmax(Smem& sm, double v, int p, double* ov, int* op) {
  for (int off = 32; off >= 1; off >>= 1) {
    const double v2 = __shfl_xor(v, off);
    const int p2 = __shfl_xor(p, off);
    if (better(v2, p2, v, p)) {
      v = v2;
      p = p2;
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sm.rv[w] = v;
    sm.rp[w] = p;
  }
  __syncthreads();
  double bv = sm.rv[0];
  int bp = sm.rp[0];
  for (int i = 1; i < BT / 64; ++i)
    if (better(sm.rv[i], sm.rp[i], bv, bp)) {
      bv = sm.rv[i];
      bp = sm.rp[i];
    }
  *ov = bv;
  *op = bp;
}

// Delayed trailing update of a panel: A[i,jj] += sum_q (P_q[i] Q_q[jj] - Q_q[i] P_q[jj])
// for c1 <= jj < i < n, with (P_q, Q_q) = LW[q] the panel's pairs.  The work is
// cut into items (strip of 4 columns, row): strip s (first column j0 = c1 + 4s)
// has the rows j0+1 .. n-1.  Items are numbered strip by strip and dealt to the
// threads round-robin, so every thread gets the same number of items whatever
// the triangle's shape, and consecutive threads take consecutive rows of a strip
// (coalesced).  A thread locates its first item from its index (a quadratic
// root) and each next one, BT items further, by walking on through the strips.
// Each item's 4 elements are loaded (clamped addresses) before the previous item
// is multiplied and stored.
constexpr int kStrip = 4;

__device__ inline void trailing_update(double* __restrict__ A, int64_t ld, int64_t n, int64_t c1, int npairs,
                                       const double2 (&LW)[BNP][BR]) {
  constexpr int SW = kStrip;
  const int tid = threadIdx.x;
  const int64_t a = n - 1 - c1;                        // rows of strip 0
  const int64_t ns = (n - c1 + SW - 1) / SW;           // strips
  // items before strip s: P(s) = s a - SW s (s - 1) / 2
  auto P = [&](int64_t st) { return st * a - (int64_t)SW * st * (st - 1) / 2; };
  const int64_t total = P(ns);
  auto locate = [&](int64_t x, int64_t* j0, int64_t* row) {
    // largest s with P(s) <= x: root of the quadratic, then corrected
    const double b = (double)a + SW / 2.0;
    const double disc = b * b - 2.0 * SW * (double)x;
    int64_t st = (int64_t)((b - sqrt(disc > 0.0 ? disc : 0.0)) / SW);
    st = max((int64_t)0, min(st, ns - 1));
    while (st > 0 && P(st) > x) --st;
    while (st + 1 < ns && P(st + 1) <= x) ++st;
    *j0 = c1 + SW * st;
    *row = *j0 + 1 + (x - P(st));
  };
  // the item BT further on: the rest of this strip, then whole strips (the
  // caller guarantees that it exists, so the walk ends inside the triangle)
  auto advance = [&](int64_t* j0, int64_t* row) {
    int64_t m = BT;
    while (*j0 < n) {
      const int64_t left = n - 1 - *row;  // items after this one in its strip
      if (m <= left) {
        *row += m;
        return;
      }
      m -= left + 1;
      *j0 += SW;
      *row = *j0 + 1;
    }
    *j0 = *row = n - 1;  // not reached
  };
  auto load = [&](int64_t j0, int64_t row, double (&v)[SW]) {
#pragma unroll
    for (int t = 0; t < SW; ++t) {
      const int64_t jj = j0 + t;
      v[t] = A[(row < n && jj < row) ? row + jj * ld : 1];  // unused ones read A[1, 0], strictly lower
    }
  };
  int64_t x = tid;
  if (x >= total) return;
  int64_t j0, row;
  locate(x, &j0, &row);
  double cur[SW], nxt[SW];
  load(j0, row, cur);
  for (;;) {
    const int64_t xn = x + BT;
    int64_t j0n = 0, rown = n;
    if (xn < total) {
      j0n = j0;
      rown = row;
      advance(&j0n, &rown);
      load(j0n, rown, nxt);
    }
    double acc[SW];
#pragma unroll
    for (int t = 0; t < SW; ++t) acc[t] = 0.0;
    // all of a pair's LDS operands are read before any is used (one LDS wait
    // per pair, not one per column), two fused multiply-adds per product
    for (int q = 0; q < npairs; ++q) {
      const double2 u = LW[q][row];
      double2 v[SW];
#pragma unroll
      for (int t = 0; t < SW; ++t) v[t] = LW[q][min(j0 + t, (int64_t)BR - 1)];
#pragma unroll
      for (int t = 0; t < SW; ++t) acc[t] = fma(-u.y, v[t].x, fma(u.x, v[t].y, acc[t]));
    }
#pragma unroll
    for (int t = 0; t < SW; ++t) {
      const int64_t jj = j0 + t;
      if (jj < row) A[row + jj * ld] = cur[t] + acc[t];
    }
    if (xn >= total) break;
    x = xn;
    j0 = j0n;
    row = rown;
#pragma unroll
    for (int t = 0; t < SW; ++t) cur[t] = nxt[t];
  }
}

// kFactors: also leave L in place (the Pfaffian-only form needs neither the
// finished columns of L nor their row interchanges).
template <bool kFactors>
__global__ void __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(kWavesPerSimd, kWavesPerSimd))) batched_kernel(BatchArgs a) {
  __shared__ Smem sm;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) sm.item = atomicAdd(a.queue, 1);
    __syncthreads();
    const int64_t it = sm.item;
    __syncthreads();
    if (it >= a.batch) return;
    const int64_t b = a.order[it];
    const int64_t n = a.nn[b], ld = a.lda[b];
    double* A = a.A[b];
    int32_t* ipiv = a.ipiv ? a.ipiv[b] : a.ipiv_scratch + (size_t)blockIdx.x * BR;
    double* Tv = a.T ? a.T[b] : a.T_scratch + (size_t)blockIdx.x * BR;
    if (ipiv == nullptr) ipiv = a.ipiv_scratch + (size_t)blockIdx.x * BR;
    if (Tv == nullptr) Tv = a.T_scratch + (size_t)blockIdx.x * BR;
    int status = 0;
    if (n >= 1 && tid == 0) ipiv[0] = 0;
    // column 0
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + BT * r;
      sm.cur[i] = (i >= 1 && i < n) ? A[i] : 0.0;
    }
    __syncthreads();
    for (int64_t k0 = 0; k0 < n - 1 && status == 0; k0 += 2 * BNP) {
      const int nsteps = (int)min((int64_t)2 * BNP, n - 1 - k0);
      for (int q = 0; q < BNP; ++q)
        for (int r = 0; r < RPT; ++r) sm.LW[q][tid + BT * r] = make_double2(0.0, 0.0);
      for (int r = 0; r < RPT; ++r) sm.Le[tid + BT * r] = 0.0;
      __syncthreads();
      for (int si = 0; si < nsteps; ++si) {
        const int64_t k = k0 + si, rr = k + 1;
        const int j = si >> 1, ph = si & 1;
        // loads whose addresses do not depend on the pivot, issued before its
        // search: the stored column r below r and row r of the finished columns
        // of L.  Every load of the step is issued unconditionally (an unused one
        // reads A[1, 0]) and selected where its value is used, so the loads that
        // do not depend on the pivot overlap its search.
        static_assert(BT >= BR, "one finished column per thread in the row swap");
        double colr[RPT];
        for (int r = 0; r < RPT; ++r) {
          const int i = tid + BT * r;
          const bool vr = i > rr && i < n;
          const double a0 = A[vr ? i + rr * ld : 1];
          colr[r] = vr ? a0 : 0.0;
        }
        const bool vc = kFactors && tid < k;
        const double xr = A[vc ? rr + (int64_t)tid * ld : 1];
        // pivot over rows >= k+1
        double bv = -1.0;
        int bp = INT32_MAX;
        bool nf = false;
        for (int r = 0; r < RPT; ++r) {
          const int i = tid + BT * r;
          if (i >= rr && i < n) {
            const double c = sm.cur[i];
            if (!isfinite(c)) nf = true;
            if (better(fabs(c), i, bv, bp)) {
              bv = fabs(c);
              bp = i;
            }
          }
        }
        // a non-finite entry enters the arg-max as +inf (finite |c| never is)
        if (nf) bv = INFINITY;
        double gv;
        int p;
        block_argmax(sm, bv, bp, &gv, &p);
        if (gv == INFINITY) {
          status = SKF_ENONFINITE;
          break;
        }
        const double alpha = sm.cur[p];
        // symmetric interchange r <-> p (lower storage) and the new column r below r:
        //   A[i,r] (i > r) := i < p ? -A[p,i] : (i == p ? -A[p,r] : A[i,p])
        double praw[RPT];
        for (int r = 0; r < RPT; ++r) {
          const int i = tid + BT * r;
          const bool vp = p != rr && i > rr && i < n;
          const int64_t at = (i < p) ? p + (int64_t)i * ld : (i == p ? p + rr * ld : i + (int64_t)p * ld);
          praw[r] = A[vp ? at : 1];
        }
        const bool vs = vc && p != rr;
        const double yp = A[vs ? p + (int64_t)tid * ld : 1];
        double newc[RPT];
        for (int r = 0; r < RPT; ++r) {
          const int i = tid + BT * r;
          newc[r] = (i > rr && i < n) ? (p == rr ? colr[r] : (i <= p ? -praw[r] : praw[r])) : 0.0;
        }
        if (p != rr) {
          // row segments left of r (finished columns of L; column k is carried in cur)
          if (vs) {
            A[rr + (int64_t)tid * ld] = yp;
            A[p + (int64_t)tid * ld] = xr;
          }
          // column r below r vs row p / column p (old column r moves there)
          for (int r = 0; r < RPT; ++r) {
            const int i = tid + BT * r;
            if (i > rr && i < n) {
              const double old = colr[r];
              if (i < p) A[p + (int64_t)i * ld] = -old;
              else if (i == p) A[p + rr * ld] = -old;  // A[p,r] := -A[p,r]
              else A[i + (int64_t)p * ld] = old;
            }
          }
        }
        // (column r itself is not stored: it is kept in newc and becomes the
        // pivot column through cur; the next step overwrites it with L).
        // Every thread has read alpha = cur[p] before rows r and p of the LDS
        // arrays are swapped: an LDS-only barrier (global stores stay in flight).
        // (fences on LDS only: they order the LDS accesses around the barrier for
        // the compiler too, and wait for LDS, not for the global stores)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
        if (p != rr && tid < BNP + 2) {
          // LDS rows r and p: pairs, current-pair multipliers, pivot column
          if (tid < BNP) {
            const double2 t = sm.LW[tid][rr];
            sm.LW[tid][rr] = sm.LW[tid][p];
            sm.LW[tid][p] = t;
          } else if (tid == BNP) {
            const double t = sm.Le[rr];
            sm.Le[rr] = sm.Le[p];
            sm.Le[p] = t;
          } else {
            const double t = sm.cur[rr];
            sm.cur[rr] = sm.cur[p];
            sm.cur[p] = t;
          }
        }
        if (tid == 0) {
          Tv[k] = alpha;
          ipiv[rr] = (int32_t)p;
        }
        __syncthreads();
        // multipliers; column k of the factored array = (alpha; l)
        for (int r = 0; r < RPT; ++r) {
          const int i = tid + BT * r;
          if (i == rr) {
            if (kFactors) A[i + k * ld] = alpha;
            if (ph == 0) sm.Le[i] = alpha;
            else sm.LW[j][i].x = alpha;
          } else if (i > rr && i < n) {
            const double l = (alpha != 0.0) ? sm.cur[i] / alpha : 0.0;
            if (kFactors) A[i + k * ld] = l;
            if (ph == 0) sm.Le[i] = l;
            else sm.LW[j][i].x = l;
          }
        }
        __syncthreads();
        // next column x = k+1 below its diagonal: stored value + pair corrections
        const double l0 = sm.Le[rr];
        for (int r = 0; r < RPT; ++r) {
          const int i = tid + BT * r;
          if (i < n && i > rr) {
            double corr = 0.0;
            for (int q = 0; q < j; ++q) {
              const double2 u = sm.LW[q][i], x = sm.LW[q][rr];
              corr += u.x * x.y - u.y * x.x;
            }
            const double g = newc[r] + corr;
            if (ph == 0) {
              sm.cur[i] = g;
            } else {
              sm.LW[j][i].y = g;
              sm.cur[i] = g + alpha * (sm.Le[i] - l0 * sm.LW[j][i].x);
            }
          } else if (i < n && ph == 1) {
            sm.LW[j][i].y = 0.0;
          }
        }
        __syncthreads();
      }
      if (status) break;
      // trailing update: A[i,jj] += sum_q (l'_i w_jj - w_i l'_jj) for i > jj > lo
      const int64_t lo = k0 + nsteps;
      const int npairs = nsteps / 2;
      if (nsteps % 2 == 0 && n - lo >= 3) trailing_update(A, ld, n, lo + 1, npairs, sm.LW);
      __syncthreads();
    }
    // the last column: T[n-2] was produced by the last step (its pivot search saw one row)
    // Pfaffian: log|Pf| = sum log|T[k even]|, sign from the swaps and the signs
    double acc = 0.0;
    int par = 0;
    if (status == 0 && n % 2 == 0) {
      const int64_t np2 = n / 2;
      const int64_t chunk = (np2 + BT - 1) / BT;
      for (int64_t q = tid * chunk; q < min(np2, (tid + 1) * chunk); ++q) {
        const double t = Tv[2 * q];
        if (t == 0.0) par |= 2;
        if (t < 0.0) par ^= 1;
        acc += log(fabs(t));
      }
      for (int64_t jj = tid; jj < n; jj += BT)
        if (ipiv[jj] != (int32_t)jj) par ^= 1;
    }
    sm.sum[tid] = acc;
    sm.par[tid] = par;
    __syncthreads();
    for (int s = BT / 2; s > 0; s >>= 1) {
      if (tid < s) {
        sm.sum[tid] = sm.sum[tid] + sm.sum[tid + s];
        sm.par[tid] = (sm.par[tid] ^ (sm.par[tid + s] & 1)) | (sm.par[tid + s] & 2);
      }
      __syncthreads();
    }
    if (tid == 0) {
      double la;
      int sg;
      int inf = status;
      if (status != 0) {
        la = NAN;
        sg = 0;
      } else if (n == 0) {
        la = 0.0;
        sg = 1;
      } else if (n % 2 == 1 || (sm.par[0] & 2)) {
        la = -INFINITY;
        sg = 0;
      } else {
        la = sm.sum[0];
        sg = (((sm.par[0] & 1) ^ (int)((n / 2) & 1)) != 0) ? -1 : 1;
      }
      if (inf == 0) {
        for (int64_t kk = 0; kk + 1 < n; kk += 2)
          if (Tv[kk] == 0.0) {
            inf = (int)(kk + 1);
            break;
          }
      }
      if (a.logabs) a.logabs[b] = la;
      if (a.sign) a.sign[b] = sg;
      if (a.info) a.info[b] = inf;
    }
    __syncthreads();
  }
}

// Pfaffian-only form: the elimination step taken at the even steps k only
// (the reduction the oracle's Pfaffian-only mode defines): step k pivots on
// column k, interchanges rows/columns k+1 and p, and adds l v^T - v l^T to the
// trailing matrix (l = multipliers, v = column k+1 after the interchange); rows
// and columns k, k+1 are then finished, so the next step pivots on column k+2.
// Half the pivot steps of the full factorization for the same n^3/3 flops.
// Updates are delayed over a panel of BNP steps as in the full form: each
// needed column is the stored one plus a skew GEMV with the panel's (l, v).
// Per step, the stored columns k+1 and k+2 are loaded before the pivot search
// (their addresses do not depend on it); the interchange then changes column
// k+2 at one known place (row p), or replaces it by the old column k+1 (p =
// k+2), which is patched in registers.  ipiv (if given) receives the
// interchanges (even positions stay j), T the pivots at even k.
__global__ void __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(kWavesPerSimd, kWavesPerSimd))) pfonly_kernel(BatchArgs a) {
  __shared__ Smem sm;
  const int tid = threadIdx.x;
  for (;;) {
    if (tid == 0) sm.item = atomicAdd(a.queue, 1);
    __syncthreads();
    const int64_t it = sm.item;
    __syncthreads();
    if (it >= a.batch) return;
    const int64_t b = a.order[it];
    const int64_t n = a.nn[b], ld = a.lda[b];
    double* A = a.A[b];
    int32_t* ipiv = a.ipiv ? a.ipiv[b] : nullptr;
    double* Tv = a.T ? a.T[b] : nullptr;
    if (ipiv == nullptr) ipiv = a.ipiv_scratch + (size_t)blockIdx.x * BR;
    if (Tv == nullptr) Tv = a.T_scratch + (size_t)blockIdx.x * BR;
    int status = 0;
    for (int64_t jj = tid; jj < n; jj += BT) ipiv[jj] = (int32_t)jj;
    for (int64_t jj = tid; jj + 1 < n; jj += BT) Tv[jj] = 0.0;
    if (n >= 2 && n % 2 == 0) {
      for (int r = 0; r < RPT; ++r) {
        const int i = tid + BT * r;
        sm.cur[i] = (i >= 1 && i < n) ? A[i] : 0.0;
      }
      __syncthreads();
      for (int64_t k0 = 0; k0 < n - 1 && status == 0; k0 += 2 * BNP) {
        const int np = (int)min((int64_t)BNP, (n - k0) / 2);
        for (int q = 0; q < BNP; ++q)
          for (int r = 0; r < RPT; ++r) sm.LW[q][tid + BT * r] = make_double2(0.0, 0.0);
        __syncthreads();
        int done = 0;  // steps of this panel that produced a pair
        for (int q = 0; q < np; ++q) {
          const int64_t k = k0 + 2 * q, rr = k + 1, x = k + 2;
          const bool last = x >= n;  // k = n-2: pivot only
          // stored columns k+1 (rows > k+1) and k+2 (rows > k+2), before the pivot
          // is known.  Every load here and below is issued unconditionally (an
          // unused one reads A[1, 0]) and its value selected where it is used,
          // so no wait for one load is placed before the next is issued.
          double oldr[RPT], colx[RPT];
          for (int r = 0; r < RPT; ++r) {
            const int i = tid + BT * r;
            const bool vr = !last && i > rr && i < n, vx = !last && i > x && i < n;
            const double a0 = A[vr ? i + rr * ld : 1], a1 = A[vx ? i + x * ld : 1];
            oldr[r] = vr ? a0 : 0.0;
            colx[r] = vx ? a1 : 0.0;
          }
          // pivot over rows >= k+1
          double bv = -1.0;
          int bp = INT32_MAX;
          bool nf = false;
          for (int r = 0; r < RPT; ++r) {
            const int i = tid + BT * r;
            if (i >= rr && i < n) {
              const double c = sm.cur[i];
              if (!isfinite(c)) nf = true;
              if (better(fabs(c), i, bv, bp)) {
                bv = fabs(c);
                bp = i;
              }
            }
          }
          // a non-finite entry enters the arg-max as +inf (finite |c| never is)
          if (nf) bv = INFINITY;
          double gv;
          int p;
          block_argmax(sm, bv, bp, &gv, &p);
          if (gv == INFINITY) {
            status = SKF_ENONFINITE;
            break;
          }
          const double alpha = sm.cur[p];
          // column k+1 after the interchange (rows > k+1): row p left of the
          // diagonal (negated), A[p, k+1] (negated) and column p below it; the
          // sign and the p == k+1 case are applied where the value is used
          double praw[RPT];
          for (int r = 0; r < RPT; ++r) {
            const int i = tid + BT * r;
            const bool vp = !last && p != rr && i > rr && i < n;
            const int64_t at = (i < p) ? p + (int64_t)i * ld : (i == p ? p + rr * ld : i + (int64_t)p * ld);
            praw[r] = A[vp ? at : 1];
          }
          // every thread has read alpha = cur[p] before rows r and p of the LDS
          // arrays are swapped: an LDS-only barrier (global stores stay in flight)
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
          __builtin_amdgcn_s_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
          if (p != rr && tid <= BNP) {
            if (tid < BNP) {
              const double2 t = sm.LW[tid][rr];
              sm.LW[tid][rr] = sm.LW[tid][p];
              sm.LW[tid][p] = t;
            } else {
              const double t = sm.cur[rr];
              sm.cur[rr] = sm.cur[p];
              sm.cur[p] = t;
            }
          }
          if (tid == 0) {
            Tv[k] = alpha;
            ipiv[rr] = (int32_t)p;
          }
          __syncthreads();
          if (last) break;
          // (l, v) of this step below row k+1: v = stored column k+1 + corrections.
          // The owner of row k+2 also leaves its stored A[k+2, k+1] for the next
          // column here, not where it is loaded: that LDS write waits for the
          // load, and before the arg-max barrier it would hold the whole
          // workgroup for a second memory round trip per step.
          for (int r = 0; r < RPT; ++r) {
            const int i = tid + BT * r;
            if (i == x) sm.akk = oldr[r];
            if (i > rr && i < n) {
              const double l = (alpha != 0.0) ? sm.cur[i] / alpha : 0.0;
              const double newc = (p == rr) ? oldr[r] : (i <= p ? -praw[r] : praw[r]);
              sm.LW[q][i] = make_double2(l, newc + skew_dot(sm.LW, i, rr, q));
            }
          }
          // the interchange in memory: old column k+1 moves to row p / column p.
          // Issued after the products above so that their wait (for the pivot
          // row's loads) does not also wait for these stores; the next step's
          // loads of these places come after two more barriers.
          if (p != rr) {
            for (int r = 0; r < RPT; ++r) {
              const int i = tid + BT * r;
              if (i > rr && i < n) {
                const double old = oldr[r];
                if (i < p) A[p + (int64_t)i * ld] = -old;
                else if (i == p) A[p + rr * ld] = -old;
                else A[i + (int64_t)p * ld] = old;
              }
            }
          }
          __syncthreads();
          // next pivot column k+2 below its diagonal: stored (after the interchange)
          // + corrections with the pairs so far, this one included
          const double akk = sm.akk;
          for (int r = 0; r < RPT; ++r) {
            const int i = tid + BT * r;
            if (i > x && i < n) {
              const double st = (p == x) ? oldr[r] : (i == p ? -akk : colx[r]);
              sm.cur[i] = st + skew_dot(sm.LW, i, x, q + 1);
            }
          }
          ++done;
          __syncthreads();
        }
        if (status) break;
        // trailing update: A[i,jj] += sum_q (l_i v_jj - v_i l_jj) for i > jj > lo
        const int64_t lo = k0 + 2 * done;
        if (done == np && n - lo >= 3) trailing_update(A, ld, n, lo + 1, done, sm.LW);
        __syncthreads();
      }
    }
    __syncthreads();
    // Pfaffian: log|Pf| = sum log|T[k even]|, sign from the interchanges and the signs
    double acc = 0.0;
    int par = 0;
    if (status == 0 && n % 2 == 0) {
      const int64_t np2 = n / 2;
      const int64_t chunk = (np2 + BT - 1) / BT;
      for (int64_t q = tid * chunk; q < min(np2, (tid + 1) * chunk); ++q) {
        const double t = Tv[2 * q];
        if (t == 0.0) par |= 2;
        if (t < 0.0) par ^= 1;
        acc += log(fabs(t));
      }
      for (int64_t jj = tid; jj < n; jj += BT)
        if (ipiv[jj] != (int32_t)jj) par ^= 1;
    }
    sm.sum[tid] = acc;
    sm.par[tid] = par;
    __syncthreads();
    for (int s = BT / 2; s > 0; s >>= 1) {
      if (tid < s) {
        sm.sum[tid] = sm.sum[tid] + sm.sum[tid + s];
        sm.par[tid] = (sm.par[tid] ^ (sm.par[tid + s] & 1)) | (sm.par[tid + s] & 2);
      }
      __syncthreads();
    }
    if (tid == 0) {
      double la;
      int sg;
      int inf = status;
      if (status != 0) {
        la = NAN;
        sg = 0;
      } else if (n == 0) {
        la = 0.0;
        sg = 1;
      } else if (n % 2 == 1 || (sm.par[0] & 2)) {
        la = -INFINITY;
        sg = 0;
      } else {
        la = sm.sum[0];
        sg = (((sm.par[0] & 1) ^ (int)((n / 2) & 1)) != 0) ? -1 : 1;
      }
      if (inf == 0) {
        if (n % 2 == 1) inf = (int)n;
        else
          for (int64_t kk = 0; kk + 1 < n; kk += 2)
            if (Tv[kk] == 0.0) {
              inf = (int)(kk + 1);
              break;
            }
      }
      if (a.logabs) a.logabs[b] = la;
      if (a.sign) a.sign[b] = sg;
      if (a.info) a.info[b] = inf;
    }
    __syncthreads();
  }
}

struct BatchedWork {
  int64_t* order;
  int64_t* nn;
  int64_t* lda;
  int* queue;
  int32_t* ipiv_scratch;
  double* T_scratch;
  size_t bytes;
};

int batched_grid() { return kWgPerCu * device_info().num_cus; }

BatchedWork batched_carve(void* base, int64_t batch) {
  BatchedWork w{};
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = align_up(off + b, 256);
    return base ? (void*)((char*)base + o) : nullptr;
  };
  const int64_t bb = std::max<int64_t>(batch, 1);
  w.order = (int64_t*)take(sizeof(int64_t) * bb);
  w.nn = (int64_t*)take(sizeof(int64_t) * bb);
  w.lda = (int64_t*)take(sizeof(int64_t) * bb);
  w.queue = (int*)take(256);
  w.ipiv_scratch = (int32_t*)take(sizeof(int32_t) * (size_t)batched_grid() * BR);
  w.T_scratch = (double*)take(sizeof(double) * (size_t)batched_grid() * BR);
  w.bytes = off;
  return w;
}

}  // namespace

size_t batched_workspace_bytes(int64_t batch) { return batched_carve(nullptr, batch).bytes; }

int batched_max_n() { return BR; }

// Host arrays n_host, lda_host are staged into the workspace (synchronous copy
// of O(batch) words); everything else is asynchronous on `s`.
int run_batched(int64_t batch, const int64_t* n_host, double* const* A, const int64_t* lda_host,
                int32_t* const* ipiv, double* const* T, double* logabs, int* sign, int* info, void* work,
                size_t lwork, bool want_L, hipStream_t s) {
  // want_L: the full factorization (L, T, ipiv); otherwise the Pfaffian-only
  // reduction (ipiv / T, if given, receive its interchanges and pivots)
  BatchedWork w = batched_carve(work, batch);
  if (lwork < w.bytes) return SKF_EWORK;
  if (batch == 0) return 0;
  std::vector<int64_t> order((size_t)batch);
  std::iota(order.begin(), order.end(), (int64_t)0);
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return n_host[x] > n_host[y]; });
  SKF_CHECK(hipMemcpyAsync(w.order, order.data(), sizeof(int64_t) * batch, hipMemcpyHostToDevice, s), "order");
  SKF_CHECK(hipMemcpyAsync(w.nn, n_host, sizeof(int64_t) * batch, hipMemcpyHostToDevice, s), "n");
  SKF_CHECK(hipMemcpyAsync(w.lda, lda_host, sizeof(int64_t) * batch, hipMemcpyHostToDevice, s), "lda");
  SKF_CHECK(hipStreamSynchronize(s), "stage");  // the host vectors go out of scope
  int rc;
  if ((rc = launch_fill_i32(w.queue, 1, 0, s))) return rc;
  BatchArgs args{batch, w.order, w.nn, w.lda, A, ipiv, T, logabs, sign, info, w.queue, w.ipiv_scratch, w.T_scratch};
  if (want_L)
    hipLaunchKernelGGL(batched_kernel<true>, dim3((unsigned)batched_grid()), dim3(BT), 0, s, args);
  else
    hipLaunchKernelGGL(pfonly_kernel, dim3((unsigned)batched_grid()), dim3(BT), 0, s, args);
  SKF_CHECK_LAUNCH("batched");
  return 0;
}

}  // namespace skf
