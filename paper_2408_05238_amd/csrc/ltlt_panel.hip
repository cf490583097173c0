// Persistent panel kernel of the blocked skew LTL^T.
//
// One panel = nb consecutive elimination steps k0 .. k0+nb-1, taken two at a
// time.  Steps k and k+1 (a "pair") pivot on column k, then on column k+1, and
// together change the trailing matrix by ONE skew rank-2 term
//     A[k+3:, k+3:] += l' w^T - w l'^T,
// where l' = multipliers of step k+1 and w = column k+2 after both interchanges
// and before the pair (derivation: write out both congruence steps; the terms
// built from step k's multipliers cancel because v = alpha' l' below row k+2).
// Column k+2 itself, the first pivot column of the next pair, is
//     c = w + alpha' (l - l_0 l'),  l = multipliers of step k, l_0 = l[k+2].
// Summed over the panel's nb/2 pairs the trailing update is a skew rank-nb
// product, applied afterwards on the matrix cores; inside the panel, each new
// pivot column is rebuilt from the panel-start matrix plus the pairs so far
// (column recompute = a skew GEMV pair per row).
//
// Interchanges are never applied to memory during the panel.  Every row of the
// active part lives in a "slot" of one workgroup (LDS), and a slot carries its
// current index psi and the row of the panel-start matrix it came from (hbm).
// Interchanging rows/columns r and p only relabels two slots; a needed column x
// of the current matrix is gathered as S(hbm(i), hbm(x)) with S(a,b) = src[a,b]
// for a > b and -src[b,a] otherwise (strict lower storage).
//
// Grid synchronisation: once per step every workgroup publishes its best
// candidate (largest |c|, lowest current index on ties) and that row's pair
// coefficients as 64-bit words (step tag << 32 | 32 payload bits), written and
// read with agent-scope relaxed atomics.  A reader accepts a word only when its
// tag matches, so no fence is needed and a torn record cannot be used; records
// are double-buffered by step parity.  All waits are bounded: past the limit the
// workgroup records SKF_ETIMEOUT and leaves, so every wave of the grid ends.
#include "skf_internal.h"

namespace skf {

constexpr int kPanelThreads = 256;
constexpr int kRecHeader = 8;
constexpr int kRecStride = 8 + 4 * 64 + 8;  // words per record (nb <= 128)
constexpr uint32_t kNoCand = 0xFFFFFFFFu;
constexpr uint32_t kNonFinite = 0xFFFFFFFEu;
constexpr uint32_t kTimeout = 0xFFFFFFFDu;

namespace {

__device__ inline uint64_t ld_word(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_word(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t mk(uint32_t tag, uint32_t payload) {
  return ((uint64_t)tag << 32) | payload;
}
__device__ inline uint32_t hi32(double x) { return (uint32_t)(__double_as_longlong(x) >> 32); }
__device__ inline uint32_t lo32(double x) { return (uint32_t)(__double_as_longlong(x)); }
__device__ inline double from32(uint32_t h, uint32_t l) {
  return __longlong_as_double((long long)(((uint64_t)h << 32) | l));
}

// Candidate ordering: larger |c| first, then lower current index.
__device__ inline bool better(double a, uint32_t pa, double b, uint32_t pb) {
  return (a > b) || (a == b && pa < pb);
}

// Wall-clock limit for one wait (the constant 100 MHz counter): 2 s.
constexpr uint64_t kWaitTicks = 200000000ull;

template <int NB, int SMAX>
struct PanelSmem {
  static constexpr int TPR = kPanelThreads / SMAX;  // threads per slot
  static constexpr int LWLD = NB + 2;               // interleaved Lp/Wp, padded
  static constexpr int LELD = NB / 2 + 1;
  double LW[SMAX * LWLD];
  double LE[SMAX * LELD];
  double cur[SMAX];
  int32_t psi[SMAX];
  int32_t hbm[SMAX];
  double coef[NB + 8];       // winner's Lp/Wp (interleaved) for pairs < j
  double red_v[kPanelThreads / 64];
  uint32_t red_p[kPanelThreads / 64];
  int32_t red_s[kPanelThreads / 64];
  int flag;                  // nonzero: non-finite seen locally
  uint32_t win_psi, win_hbm;
  int win_g;
  double win_c, win_l0;
  int stop;
  uint32_t cand_hbm[kPanelThreads];
  double cand_c[kPanelThreads];
};

// Block-wide arg-best over (v, p, s) held by every thread; result broadcast.
template <int NT>
__device__ inline void block_best(double& v, uint32_t& p, int& s, double* rv, uint32_t* rp,
                                  int32_t* rs) {
  for (int off = 32; off >= 1; off >>= 1) {
    double ov = __shfl_xor(v, off);
    uint32_t op = __shfl_xor(p, off);
    int os = __shfl_xor(s, off);
    if (better(ov, op, v, p)) {
      v = ov;
      p = op;
      s = os;
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    rv[w] = v;
    rp[w] = p;
    rs[w] = s;
  }
  __syncthreads();
  v = rv[0];
  p = rp[0];
  s = rs[0];
  for (int i = 1; i < NT / 64; ++i)
    if (better(rv[i], rp[i], v, p)) {
      v = rv[i];
      p = rp[i];
      s = rs[i];
    }
  __syncthreads();
}

template <int NB, int SMAX>
__global__ void __launch_bounds__(kPanelThreads) panel_kernel(PanelParams P) {
  typedef PanelSmem<NB, SMAX> Sm;
  __shared__ Sm sm;
  constexpr int TPR = Sm::TPR;
  constexpr int LWLD = Sm::LWLD;
  constexpr int LELD = Sm::LELD;

  const int tid = threadIdx.x;
  const int g = blockIdx.x;
  if (*P.status != 0) return;  // an earlier panel failed: every workgroup leaves at once
  const int64_t n = P.n, k0 = P.k0, ld = P.ld;
  const double* __restrict__ src = P.src;
  const int64_t rowbase = k0 + 1 + (int64_t)g * P.S;
  const int nslots = (int)max((int64_t)0, min((int64_t)P.S, n - rowbase));

  // ---- panel start: slots, zeroed pair storage, column k0 ----
  for (int i = tid; i < SMAX * LWLD; i += kPanelThreads) sm.LW[i] = 0.0;
  for (int i = tid; i < SMAX * LELD; i += kPanelThreads) sm.LE[i] = 0.0;
  if (tid < SMAX) {
    const int64_t row = rowbase + tid;
    const bool v = tid < nslots;
    sm.psi[tid] = v ? (int32_t)row : INT32_MAX;
    sm.hbm[tid] = v ? (int32_t)row : 0;
    sm.cur[tid] = v ? src[row + k0 * ld] : 0.0;
  }
  if (tid == 0) {
    sm.flag = 0;
    sm.stop = 0;
  }
  if (g == 0)
    for (int64_t i = tid; i <= k0; i += kPanelThreads) P.pi[i] = (int32_t)i;
  __syncthreads();

  const int slot = tid / TPR;   // slot handled by this thread in per-slot work
  const int part = tid % TPR;   // which pairs q = part (mod TPR) it sums

  for (int si = 0; si < P.nsteps; ++si) {
    const int64_t k = k0 + si;
    const int j = si >> 1;
    const int ph = si & 1;
    const uint32_t tag = P.tag_base + (uint32_t)si + 1u;
    uint64_t* rec_mine = P.rec + ((size_t)(si & 1) * P.G + g) * kRecStride;

    // (A) local candidate over active slots (current index >= k+1)
    double cv = -1.0;
    uint32_t cp = kNoCand;
    int cs = -1;
    if (tid < SMAX && tid < nslots && sm.psi[tid] >= k + 1) {
      double c = sm.cur[tid];
      if (!isfinite(c)) sm.flag = 1;
      cv = fabs(c);
      cp = (uint32_t)sm.psi[tid];
      cs = tid;
    }
    block_best<kPanelThreads>(cv, cp, cs, sm.red_v, sm.red_p, sm.red_s);
    const bool nonfinite = sm.flag != 0;

    // (B) publish: header words + the candidate row's pair coefficients
    {
      const int nwords = kRecHeader + 4 * j;
      for (int w = tid; w < nwords; w += kPanelThreads) {
        uint32_t pay = 0;
        if (w == 0) {
          pay = nonfinite ? kNonFinite : cp;
        } else if (w == 1) {
          pay = (cs >= 0) ? (uint32_t)sm.hbm[cs] : 0u;
        } else if (w == 2 || w == 3) {
          double c = (cs >= 0) ? sm.cur[cs] : 0.0;
          pay = (w == 2) ? hi32(c) : lo32(c);
        } else if (w == 4 || w == 5) {
          double l0 = (cs >= 0) ? sm.LE[cs * LELD + j] : 0.0;
          pay = (w == 4) ? hi32(l0) : lo32(l0);
        } else if (w >= kRecHeader) {
          const int q = (w - kRecHeader) >> 2, e = (w - kRecHeader) & 3;
          double x = (cs >= 0) ? sm.LW[cs * LWLD + 2 * q + (e >> 1)] : 0.0;
          pay = (e & 1) ? lo32(x) : hi32(x);
        }
        st_word(rec_mine + w, mk(tag, pay));
      }
    }

    // (C) gather every workgroup's candidate; reduce to the global pivot
    {
      double v = -1.0;
      uint32_t p = kNoCand;
      int s = -1;
      bool bad = false, tout = false;
      if (tid < P.G) {
        const uint64_t* r = P.rec + ((size_t)(si & 1) * P.G + tid) * kRecStride;
        uint64_t w0, w1, w2, w3;
        const uint64_t t0 = wall_clock64();
        for (;;) {
          w0 = ld_word(r + 0);
          w1 = ld_word(r + 1);
          w2 = ld_word(r + 2);
          w3 = ld_word(r + 3);
          if ((uint32_t)(w0 >> 32) == tag && (uint32_t)(w1 >> 32) == tag &&
              (uint32_t)(w2 >> 32) == tag && (uint32_t)(w3 >> 32) == tag)
            break;
          if (wall_clock64() - t0 > kWaitTicks) {
            tout = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        if (!tout) {
          const uint32_t ps = (uint32_t)w0;
          if (ps == kNonFinite) {
            bad = true;
          } else if (ps != kNoCand) {
            const double c = from32((uint32_t)w2, (uint32_t)w3);
            v = fabs(c);
            p = ps;
            s = tid;
            sm.cand_hbm[tid] = (uint32_t)w1;
            sm.cand_c[tid] = c;
          }
        }
      }
      if (bad) atomicOr(&sm.flag, 2);
      if (tout) atomicOr(&sm.flag, 4);
      block_best<kPanelThreads>(v, p, s, sm.red_v, sm.red_p, sm.red_s);
      if (tid == 0) {
        sm.win_g = s;
        sm.win_psi = p;
        sm.stop = (sm.flag & 6) ? sm.flag : (s < 0 ? 4 : 0);
      }
      __syncthreads();
    }
    if (sm.stop) break;
    const int wg = sm.win_g;  // >= 0: rows k+1.. are nonempty for every step of a panel
    const uint64_t* rec_win = P.rec + ((size_t)(si & 1) * P.G + wg) * kRecStride;
    const int64_t pidx = sm.win_psi;        // pivot row p
    const int64_t r = k + 1;
    const double alpha = sm.cand_c[wg];
    const int64_t hx = sm.cand_hbm[wg];     // panel-start row of the new row r = column x

    // (D) relabel the two slots; record the step
    if (tid < nslots && pidx != r) {
      const int32_t ps = sm.psi[tid];
      if (ps == (int32_t)r) sm.psi[tid] = (int32_t)pidx;
      else if (ps == (int32_t)pidx) sm.psi[tid] = (int32_t)r;
    }
    if (g == 0 && tid == 0) {
      P.ipiv[r] = (int32_t)pidx;
      P.T[k] = alpha;
    }
    __syncthreads();

    // (E) multipliers: l = c / alpha below row k+1; alpha itself at row k+1
    if (tid < nslots) {
      const int32_t ps = sm.psi[tid];
      double val;
      bool wr = true;
      if (ps >= k + 2) val = (alpha != 0.0) ? sm.cur[tid] / alpha : 0.0;
      else if (ps == r) val = alpha;
      else wr = false;
      if (wr) {
        if (ph == 0) sm.LE[tid * LELD + j] = val;
        else sm.LW[tid * LWLD + 2 * j] = val;
      }
    }

    // (F) the next needed column x = k+1 of the current matrix (the new row r): gather + pair
    // corrections.  Step k of a pair yields v (pivot column of step k+1); step k+1 yields w
    // and, through the pair's extra term, the next pair's first pivot column.
    const int64_t x = k + 1;
    double gval = 0.0;
    bool active = false;
    if (slot < nslots) {
      const int64_t ps = sm.psi[slot];
      active = ps >= x + 1;
      if (active && part == 0) {
        const int64_t a = sm.hbm[slot];
        gval = (a > hx) ? src[a + hx * ld] : -src[hx + a * ld];
      }
    }
    // winner's coefficients (pairs < j) and, in the second step, its l_0
    {
      const int nw = 4 * j + 2;
      for (int w = tid; w < nw; w += kPanelThreads) {
        const int widx = (w < 2) ? 4 + w : kRecHeader + (w - 2);
        const uint64_t t0 = wall_clock64();
        uint64_t word;
        bool tout = false;
        for (;;) {
          word = ld_word(rec_win + widx);
          if ((uint32_t)(word >> 32) == tag) break;
          if (wall_clock64() - t0 > kWaitTicks) {
            tout = true;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        if (tout) atomicOr(&sm.flag, 4);
        // assemble doubles pairwise in LDS: even word = hi, odd word = lo
        uint32_t* c32 = reinterpret_cast<uint32_t*>(sm.coef);
        // coef[0] = l0; coef[1 + 2q] = Lx[q], coef[2 + 2q] = Wx[q]
        const int d = (w < 2) ? 0 : 1 + ((w - 2) >> 1);
        const int half = (w & 1) ? 0 : 1;  // little endian: hi word at [2d+1]
        c32[2 * d + half] = (uint32_t)word;
      }
    }
    __syncthreads();
    if (sm.flag & 4) {
      if (tid == 0) sm.stop = 4;
      __syncthreads();
      break;
    }
    double corr = 0.0;
    if (active) {
      const double* lw = &sm.LW[slot * LWLD];
      for (int q = part; q < j; q += TPR) corr += lw[2 * q] * sm.coef[2 + 2 * q] - lw[2 * q + 1] * sm.coef[1 + 2 * q];
    }
#pragma unroll
    for (int off = 1; off < TPR; off <<= 1) corr += __shfl_xor(corr, off);
    if (part == 0 && slot < nslots) {
      if (ph == 0) {
        if (active) sm.cur[slot] = gval + corr;
      } else {
        if (active) {
          const double w = gval + corr;
          sm.LW[slot * LWLD + 2 * j + 1] = w;
          const double l = sm.LE[slot * LELD + j];
          const double lp = sm.LW[slot * LWLD + 2 * j];
          sm.cur[slot] = w + alpha * (l - sm.coef[0] * lp);
        } else {
          sm.LW[slot * LWLD + 2 * j + 1] = 0.0;
        }
      }
    }
    __syncthreads();
  }

  // ---- panel end ----
  if (sm.stop) {
    if (tid == 0) {
      int code = (sm.stop & 4) ? SKF_ETIMEOUT : SKF_ENONFINITE;
      atomicMin(P.status, code);
    }
    return;
  }
  const int npairs = P.nsteps / 2;
  const int64_t lo = k0 + P.nsteps;
  for (int idx = tid; idx < nslots * P.nsteps; idx += kPanelThreads) {
    const int t = idx / P.nsteps, c = idx % P.nsteps;
    const int64_t ps = sm.psi[t];
    const double v = (c & 1) ? sm.LW[t * LWLD + (c - 1)] : sm.LE[t * LELD + (c >> 1)];
    P.Lbuf[ps + (int64_t)c * n] = v;
  }
  for (int idx = tid; idx < nslots * npairs; idx += kPanelThreads) {
    const int t = idx / npairs, q = idx % npairs;
    const int64_t ps = sm.psi[t];
    P.Lp[ps + (int64_t)q * n] = sm.LW[t * LWLD + 2 * q];
    P.Wp[ps + (int64_t)q * n] = sm.LW[t * LWLD + 2 * q + 1];
  }
  if (tid < nslots) {
    const int64_t ps = sm.psi[tid];
    P.pi[ps] = sm.hbm[tid];
    if ((P.nsteps & 1) == 0 && ps >= lo + 1) P.cnext[ps] = sm.cur[tid];
  }
}

template <int NB, int SMAX>
int launch_panel_t(const PanelParams& p, hipStream_t s) {
  hipLaunchKernelGGL((panel_kernel<NB, SMAX>), dim3(p.G), dim3(kPanelThreads), 0, s, p);
  SKF_CHECK_LAUNCH("panel");
  return 0;
}

}  // namespace

int launch_panel(const PanelParams& p, hipStream_t s) {
  if (p.nb == 128 && p.S <= 64) return launch_panel_t<128, 64>(p, s);
  if (p.nb == 64 && p.S <= 128) return launch_panel_t<64, 128>(p, s);
  if (p.nb == 64 && p.S <= 64) return launch_panel_t<64, 64>(p, s);
  return SKF_ENOTIMPL;
}

size_t panel_record_words(int G) { return (size_t)2 * G * kRecStride; }

}  // namespace skf
