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
// active part lives in a "slot" of one workgroup (LDS columns; lane s%64 of the
// control wave holds its scalars) and carries its current index psi and the row
// of the panel-start matrix it came from (hbm).  Interchanging rows/columns r
// and p only relabels two slots; a needed column x of the current matrix is
// gathered as S(hbm(i), hbm(x)) with S(a,b) = src[a,b] for a > b and
// -src[b,a] otherwise (strict lower storage).
//
// One step:
//   control wave: local arg-max (largest |c|, lowest current index on ties) ->
//   publish a 6-word record -> read every workgroup's record -> global pivot ->
//   relabel, scale -> gather the new column and fetch the pivot row's pair
//   coefficients from its workgroup's coefficient mirror;
//   barrier; all four waves: partial skew GEMV over the pairs so far; barrier;
//   control wave: finish the column (on a pair's second step also w, the next
//   pair's first column and the mirror entries of the pair).
// Cross-workgroup words are 64-bit (tag << 32 | payload), written and read with
// agent-scope relaxed atomics; a reader accepts a word only when it carries the
// expected step's tag, so no fence is needed and a torn record is never used.
// Records are double-buffered by step parity.  Every wait is bounded: past the
// limit the workgroup records SKF_ETIMEOUT and leaves, so every wave ends.
#include "skf_internal.h"

namespace skf {

constexpr int kPanelThreads = 256;
constexpr int kRecWords = 8;  // psi, (slot<<24 | hbm), c hi, c lo, l0 hi, l0 lo, -, -
constexpr uint32_t kNoCand = 0xFFFFFFFFu;
constexpr uint32_t kNonFinite = 0xFFFFFFFEu;

namespace {

__device__ inline uint64_t ld_word(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_word(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t mk(uint32_t tag, uint32_t payload) { return ((uint64_t)tag << 32) | payload; }
__device__ inline uint32_t tag_of(uint64_t w) { return (uint32_t)(w >> 32); }
__device__ inline uint32_t hi32(double x) { return (uint32_t)((uint64_t)__double_as_longlong(x) >> 32); }
__device__ inline uint32_t lo32(double x) { return (uint32_t)(__double_as_longlong(x)); }
__device__ inline double from32(uint32_t h, uint32_t l) {
  return __longlong_as_double((long long)(((uint64_t)h << 32) | l));
}

// Candidate ordering: larger |c| first, then lower current index.
__device__ inline bool better(double a, uint32_t pa, double b, uint32_t pb) {
  return (a > b) || (a == b && pa < pb);
}

// Wave-wide arg-best over (v, p, s); every lane ends with the result.
__device__ inline void wave_best(double& v, uint32_t& p, int& s) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(v, off);
    const uint32_t op = __shfl_xor(p, off);
    const int os = __shfl_xor(s, off);
    if (better(ov, op, v, p)) {
      v = ov;
      p = op;
      s = os;
    }
  }
}

// Wall-clock limit for one wait (the constant 100 MHz counter): 2 s.
constexpr uint64_t kWaitTicks = 200000000ull;

template <int NB, int SPL>
struct PanelSmem {
  static constexpr int SMAX = 64 * SPL;  // slots per workgroup
  double Lp[NB / 2][SMAX];               // l' of each pair, per slot
  double Wp[NB / 2][SMAX];               // w of each pair, per slot
  double Le[NB / 2][SMAX];               // l of each pair's first step, per slot
  double part[4][SMAX];                  // partial GEMV sums of the four waves
  double coefL[NB / 2], coefW[NB / 2];   // pivot row's l', w of the pairs so far
  int32_t psi[SMAX], hbm[SMAX];
  double cur[SMAX];
  int stop;
};

template <int NB, int SPL>
__global__ void __launch_bounds__(kPanelThreads) panel_kernel(PanelParams P) {
  typedef PanelSmem<NB, SPL> Sm;
  constexpr int SMAX = Sm::SMAX;
  constexpr int NP = NB / 2;
  __shared__ Sm sm;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = blockIdx.x;
  if (*P.status != 0) return;  // an earlier panel failed: every workgroup leaves at once
  const int64_t n = P.n, k0 = P.k0, ld = P.ld;
  const double* __restrict__ src = P.src;
  const int64_t rowbase = k0 + 1 + (int64_t)g * P.S;
  const int nslots = (int)max((int64_t)0, min((int64_t)P.S, n - rowbase));
  const int G = P.G;
  uint64_t* const my_mirror = P.mirror + (size_t)g * SMAX * NP * 4;

  for (int i = tid; i < NP * SMAX; i += kPanelThreads) {
    (&sm.Lp[0][0])[i] = 0.0;
    (&sm.Wp[0][0])[i] = 0.0;
    (&sm.Le[0][0])[i] = 0.0;
  }
  if (g == 0)
    for (int64_t i = tid; i <= k0; i += kPanelThreads) P.pi[i] = (int32_t)i;

  // control-wave state of slot s = lane + 64 e
  int32_t psi[SPL], hbm[SPL];
  double cur[SPL], gat[SPL];
  double alpha = 0.0, l0 = 0.0;
  if (wave == 0) {
#pragma unroll
    for (int e = 0; e < SPL; ++e) {
      const int s = lane + 64 * e;
      const bool v = s < nslots;
      psi[e] = v ? (int32_t)(rowbase + s) : INT32_MAX;
      hbm[e] = v ? (int32_t)(rowbase + s) : 0;
      cur[e] = v ? src[rowbase + s + k0 * ld] : 0.0;
      gat[e] = 0.0;
    }
    if (lane == 0) sm.stop = 0;
  }
  __syncthreads();

  for (int si = 0; si < P.nsteps; ++si) {
    const int64_t k = k0 + si;
    const int j = si >> 1;
    const int ph = si & 1;
    const uint32_t tag = P.tag_base + (uint32_t)si + 1u;
    uint64_t* const recs = P.rec + (size_t)(si & 1) * G * kRecWords;

    if (wave == 0) {
      // (A) local candidate over active slots (current index >= k+1)
      double bv = -1.0;
      uint32_t bp = kNoCand;
      int bs = -1;
      bool nonfin = false;
#pragma unroll
      for (int e = 0; e < SPL; ++e) {
        if (lane + 64 * e < nslots && psi[e] >= k + 1) {
          const double c = cur[e];
          if (!isfinite(c)) nonfin = true;
          if (better(fabs(c), (uint32_t)psi[e], bv, bp)) {
            bv = fabs(c);
            bp = (uint32_t)psi[e];
            bs = lane + 64 * e;
          }
        }
      }
      wave_best(bv, bp, bs);
      nonfin = __any(nonfin);

      // (B) publish this workgroup's record (the owning lane supplies c and hbm)
      {
        const int owner = (bs >= 0) ? (bs & 63) : 0;
        const int oe = (bs >= 0) ? (bs >> 6) : 0;
        double cval = 0.0;
        int32_t h = 0;
#pragma unroll
        for (int e = 0; e < SPL; ++e)
          if (e == oe) {
            cval = cur[e];
            h = hbm[e];
          }
        cval = __shfl(cval, owner);
        h = __shfl(h, owner);
        const double lz = (bs >= 0) ? sm.Le[j][bs] : 0.0;
        uint32_t pay = 0;
        if (lane == 0) pay = nonfin ? kNonFinite : bp;
        else if (lane == 1) pay = ((uint32_t)(bs < 0 ? 0 : bs) << 24) | (uint32_t)h;
        else if (lane == 2) pay = hi32(cval);
        else if (lane == 3) pay = lo32(cval);
        else if (lane == 4) pay = hi32(lz);
        else if (lane == 5) pay = lo32(lz);
        if (lane < 6) st_word(recs + (size_t)g * kRecWords + lane, mk(tag, pay));
      }

      // (C) every workgroup's record (lane t reads records t, t+64, ...) -> global pivot
      double gv = -1.0;
      uint32_t gp = kNoCand;
      int gs = -1;
      bool bad = false, tout = false;
      double cc[4];
      uint32_t ch[4];
      {
        // all four words of every record this lane reads, re-issued together
        // while any is stale, so one poll costs one memory round trip
        uint64_t w[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rr = lane + 64 * q;
#pragma unroll
          for (int t = 0; t < 4; ++t) w[q][t] = (rr < G) ? ld_word(recs + (size_t)rr * kRecWords + t) : mk(tag, 0);
        }
        uint64_t t0 = 0;
        for (int it = 0;; ++it) {
          bool ok = true;
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int t = 0; t < 4; ++t) ok = ok && tag_of(w[q][t]) == tag;
          if (__all(ok)) break;
          if ((it & 31) == 0) {
            const uint64_t now = wall_clock64();
            if (it == 0) t0 = now;
            else if (now - t0 > kWaitTicks) {
              tout = true;
              break;
            }
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int rr = lane + 64 * q;
#pragma unroll
            for (int t = 0; t < 4; ++t)
              if (tag_of(w[q][t]) != tag) w[q][t] = ld_word(recs + (size_t)rr * kRecWords + t);
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rr = lane + 64 * q;
          cc[q] = 0.0;
          ch[q] = 0;
          if (rr < G && !tout) {
            const uint32_t ps = (uint32_t)w[q][0];
            if (ps == kNonFinite) {
              bad = true;
            } else if (ps != kNoCand) {
              const double c = from32((uint32_t)w[q][2], (uint32_t)w[q][3]);
              cc[q] = c;
              ch[q] = (uint32_t)w[q][1];
              if (better(fabs(c), ps, gv, gp)) {
                gv = fabs(c);
                gp = ps;
                gs = rr;
              }
            }
          }
        }
      }
      wave_best(gv, gp, gs);
      bad = __any(bad);
      tout = __any(tout);
      int stop = tout ? 4 : (bad ? 2 : (gs < 0 ? 4 : 0));
      if (!stop) {
        const int wl = gs & 63, wq = gs >> 6;
        double wc = 0.0;
        uint32_t wh = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q == wq) {
            wc = cc[q];
            wh = ch[q];
          }
        alpha = __shfl(wc, wl);
        const uint32_t hw = __shfl(wh, wl);
        const int64_t hx = hw & 0xFFFFFFu;  // panel-start row of the new row r (= column x)
        const int wslot = (int)(hw >> 24);  // its slot inside workgroup gs
        const int64_t pidx = gp, r = k + 1;

        // (D) relabel the two slots; record the step
#pragma unroll
        for (int e = 0; e < SPL; ++e) {
          if (lane + 64 * e < nslots && pidx != r) {
            if (psi[e] == (int32_t)r) psi[e] = (int32_t)pidx;
            else if (psi[e] == (int32_t)pidx) psi[e] = (int32_t)r;
          }
        }
        if (g == 0 && lane == 0) {
          P.ipiv[r] = (int32_t)pidx;
          P.T[k] = alpha;
        }

        // (F, issued first) gather column x = k+1 below its diagonal
#pragma unroll
        for (int e = 0; e < SPL; ++e) {
          gat[e] = 0.0;
          if (lane + 64 * e < nslots && psi[e] >= k + 2) {
            const int64_t a = hbm[e];
            gat[e] = (a > hx) ? src[a + hx * ld] : -src[hx + a * ld];
          }
        }
        // pivot row's coefficients (pairs q < j) from its workgroup's mirror, and its l0
        {
          const uint64_t* wm = P.mirror + ((size_t)gs * SMAX + wslot) * NP * 4;
          const int nw = 4 * j;
          uint64_t cw[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int t = lane + 64 * i;
            cw[i] = (t < nw) ? ld_word(wm + t) : 0;
          }
          const uint64_t* lwp = recs + (size_t)gs * kRecWords + 4 + (lane & 1);
          uint64_t lw = (lane < 2) ? ld_word(lwp) : mk(tag, 0);
          uint64_t t0 = 0;
          for (int it = 0;; ++it) {
            bool ok = tag_of(lw) == tag;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int t = lane + 64 * i;
              ok = ok && (t >= nw || tag_of(cw[i]) == P.tag_base + 2u * (uint32_t)(t >> 2) + 2u);
            }
            if (__all(ok)) break;
            if ((it & 31) == 0) {
              const uint64_t now = wall_clock64();
              if (it == 0) t0 = now;
              else if (now - t0 > kWaitTicks) {
                tout = true;
                break;
              }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int t = lane + 64 * i;
              if (t < nw && tag_of(cw[i]) != P.tag_base + 2u * (uint32_t)(t >> 2) + 2u) cw[i] = ld_word(wm + t);
            }
            if (lane < 2 && tag_of(lw) != tag) lw = ld_word(lwp);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int t = lane + 64 * i;
            // words of pair q: L hi, L lo, W hi, W lo in lanes 4q' .. 4q'+3
            const uint32_t lo = (uint32_t)__shfl_down((unsigned)(uint32_t)cw[i], 1);
            if (t < nw && (t & 1) == 0) {
              const double v = from32((uint32_t)cw[i], lo);
              if ((t & 3) == 0) sm.coefL[t >> 2] = v;
              else sm.coefW[t >> 2] = v;
            }
          }
          const uint32_t l0lo = (uint32_t)__shfl((unsigned)(uint32_t)lw, 1);
          const uint32_t l0hi = (uint32_t)__shfl((unsigned)(uint32_t)lw, 0);
          l0 = from32(l0hi, l0lo);
          tout = __any(tout);
          if (tout) stop = 4;
        }

        // (E) multipliers below row k+1, alpha at row k+1
#pragma unroll
        for (int e = 0; e < SPL; ++e) {
          const int s = lane + 64 * e;
          if (s < nslots) {
            double val = 0.0;
            bool wr = true;
            if (psi[e] >= k + 2) val = (alpha != 0.0) ? cur[e] / alpha : 0.0;
            else if (psi[e] == (int32_t)r) val = alpha;
            else wr = false;
            if (wr) {
              if (ph == 0) sm.Le[j][s] = val;
              else sm.Lp[j][s] = val;
            }
          }
        }
      }
      if (lane == 0) sm.stop = stop;
    }
    __syncthreads();
    if (sm.stop) break;

    // partial skew GEMV of every slot with the pivot row over pairs q = wave (mod 4), q < j
#pragma unroll
    for (int e = 0; e < SPL; ++e) {
      const int s = lane + 64 * e;
      double acc = 0.0;
      for (int q = wave; q < j; q += 4) acc += sm.Lp[q][s] * sm.coefW[q] - sm.Wp[q][s] * sm.coefL[q];
      sm.part[wave][s] = acc;
    }
    __syncthreads();

    if (wave == 0) {
#pragma unroll
      for (int e = 0; e < SPL; ++e) {
        const int s = lane + 64 * e;
        if (s < nslots) {
          const double corr = ((sm.part[0][s] + sm.part[1][s]) + sm.part[2][s]) + sm.part[3][s];
          const bool act = psi[e] >= k + 2;
          if (ph == 0) {
            if (act) cur[e] = gat[e] + corr;
          } else {
            const double w = act ? gat[e] + corr : 0.0;
            sm.Wp[j][s] = w;
            if (act) cur[e] = w + alpha * (sm.Le[j][s] - l0 * sm.Lp[j][s]);
            // mirror entries of pair j for this slot (read by other workgroups' later steps)
            const double lp = sm.Lp[j][s];
            const uint32_t mt = P.tag_base + 2u * (uint32_t)j + 2u;
            uint64_t* m = my_mirror + ((size_t)s * NP + j) * 4;
            st_word(m + 0, mk(mt, hi32(lp)));
            st_word(m + 1, mk(mt, lo32(lp)));
            st_word(m + 2, mk(mt, hi32(w)));
            st_word(m + 3, mk(mt, lo32(w)));
          }
        }
      }
    }
  }

  // ---- panel end ----
  if (sm.stop) {
    if (tid == 0) atomicMin(P.status, (sm.stop & 4) ? SKF_ETIMEOUT : SKF_ENONFINITE);
    return;
  }
  if (wave == 0) {
#pragma unroll
    for (int e = 0; e < SPL; ++e) {
      const int s = lane + 64 * e;
      sm.psi[s] = psi[e];
      sm.hbm[s] = hbm[e];
      sm.cur[s] = cur[e];
    }
  }
  __syncthreads();
  const int npairs = P.nsteps / 2;
  const int64_t lo = k0 + P.nsteps;
  for (int idx = tid; idx < nslots * P.nsteps; idx += kPanelThreads) {
    const int c = idx / nslots, s = idx % nslots;
    const double v = (c & 1) ? sm.Lp[c >> 1][s] : sm.Le[c >> 1][s];
    P.Lbuf[sm.psi[s] + (int64_t)c * n] = v;
  }
  for (int idx = tid; idx < nslots * npairs; idx += kPanelThreads) {
    const int q = idx / nslots, s = idx % nslots;
    const int64_t ps = sm.psi[s];
    P.Lp[ps + (int64_t)q * n] = sm.Lp[q][s];
    P.Wp[ps + (int64_t)q * n] = sm.Wp[q][s];
  }
  for (int s = tid; s < nslots; s += kPanelThreads) {
    const int64_t ps = sm.psi[s];
    P.pi[ps] = sm.hbm[s];
    if ((P.nsteps & 1) == 0 && ps >= lo + 1) P.cnext[ps] = sm.cur[s];
  }
}

template <int NB, int SPL>
int launch_panel_t(const PanelParams& p, hipStream_t s) {
  hipLaunchKernelGGL((panel_kernel<NB, SPL>), dim3(p.G), dim3(kPanelThreads), 0, s, p);
  SKF_CHECK_LAUNCH("panel");
  return 0;
}

}  // namespace

int launch_panel(const PanelParams& p, hipStream_t s) {
  if (p.G > 256 || p.n >= (1 << 24)) return SKF_ENOTIMPL;
  if (p.nb == 128 && p.S <= 64) return launch_panel_t<128, 1>(p, s);
  if (p.nb == 64 && p.S <= 128) return launch_panel_t<64, 2>(p, s);
  return SKF_ENOTIMPL;
}

size_t panel_record_words(int G) { return (size_t)2 * G * kRecWords; }

size_t panel_mirror_words(int G, int nb) { return (size_t)G * 128 * (nb / 2) * 4; }

}  // namespace skf
