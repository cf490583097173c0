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
// Interchanges are never applied to memory during the panel.  Each workgroup is
// ONE wave; lane s owns "slot" s, a row of the active part, with its current
// index psi, the row of the panel-start matrix it came from (hbm), its current
// column value, and (in LDS) its multipliers and pair vectors.  Interchanging
// rows/columns r and p only relabels two slots; a needed column x of the
// current matrix is gathered as S(hbm(i), hbm(x)) with S(a,b) = src[a,b] for
// a > b and -src[b,a] otherwise (strict lower storage).
//
// One step, all inside the wave (no barriers): local arg-max (largest |c|,
// lowest current index on ties; DPP butterflies) -> publish a 6-word record ->
// read every workgroup's record -> global pivot -> relabel, record T[k] and the
// interchange -> gather the new column and fetch the pivot row's pair
// coefficients from its workgroup's coefficient mirror -> multipliers -> skew
// GEMV over the pairs so far -> finish the column (on a pair's second step also
// w, the next pair's first column and this wave's mirror entries of the pair).
// Cross-workgroup words are 64-bit (tag << 32 | payload), written and read with
// agent-scope relaxed atomics; a reader accepts a word only when it carries the
// expected step's tag, so no fence is needed and a torn record is never used.
// Records are double-buffered by step parity.  Every wait is bounded: past the
// limit the workgroup records SKF_ETIMEOUT and leaves, so every wave ends.
#include "skf_internal.h"

namespace skf {

constexpr int kPanelThreads = 64;
constexpr int kRecWords = 8;  // psi, (slot<<24 | hbm), c hi, c lo, l0 hi, l0 lo, -, -
constexpr int kMaxG = 512;    // workgroups of one panel launch
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

// Lane exchanges: DPP for fixed patterns, readlane for a uniform source lane.
template <int CTRL>
__device__ inline uint32_t dpp32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ inline double dppd(double x) {
  return from32(dpp32<CTRL>(hi32(x)), dpp32<CTRL>(lo32(x)));
}
__device__ inline uint32_t rl32(uint32_t x, int lane) { return (uint32_t)__builtin_amdgcn_readlane((int)x, lane); }
__device__ inline double rld(double x, int lane) { return from32(rl32(hi32(x), lane), rl32(lo32(x), lane)); }

// Candidate ordering: larger |c| first, then lower current index.
__device__ inline bool better(double a, uint32_t pa, double b, uint32_t pb) {
  return (a > b) || (a == b && pa < pb);
}

template <int CTRL>
__device__ inline void best_step(double& v, uint32_t& p, int& s) {
  const double ov = dppd<CTRL>(v);
  const uint32_t op = dpp32<CTRL>(p);
  const int os = (int)dpp32<CTRL>((uint32_t)s);
  if (better(ov, op, v, p)) {
    v = ov;
    p = op;
    s = os;
  }
}

// Wave-wide arg-best over (v, p, s); every lane ends with the result.  Within a
// row of 16 lanes: xor-1, xor-2, rotate-4, rotate-8 (DPP); across the four rows:
// readlane of lanes 0, 16, 32, 48.
__device__ inline void wave_best(double& v, uint32_t& p, int& s) {
  best_step<0xB1>(v, p, s);   // quad_perm [1,0,3,2]
  best_step<0x4E>(v, p, s);   // quad_perm [2,3,0,1]
  best_step<0x124>(v, p, s);  // row_ror:4
  best_step<0x128>(v, p, s);  // row_ror:8
  double bv = rld(v, 0);
  uint32_t bp = rl32(p, 0);
  int bs = (int)rl32((uint32_t)s, 0);
#pragma unroll
  for (int r = 1; r < 4; ++r) {
    const double ov = rld(v, 16 * r);
    const uint32_t op = rl32(p, 16 * r);
    const int os = (int)rl32((uint32_t)s, 16 * r);
    if (better(ov, op, bv, bp)) {
      bv = ov;
      bp = op;
      bs = os;
    }
  }
  v = bv;
  p = bp;
  s = bs;
}

// Wall-clock limit for one wait (the constant 100 MHz counter): 2 s.
constexpr uint64_t kWaitTicks = 200000000ull;

template <int NB>
struct PanelSmem {
  double2 LW[NB / 2][64];  // (l', w) of each pair, per slot
  double Le[NB / 2][64];   // l of each pair's first step, per slot
  double2 coef[NB / 2];    // the pivot row's (l', w) of the pairs so far
};

template <int NB, int NQ>
__global__ void __launch_bounds__(kPanelThreads) panel_kernel(PanelParams P) {
  constexpr int NP = NB / 2;
  __shared__ PanelSmem<NB> sm;

  const int lane = threadIdx.x;
  const int g = blockIdx.x;
  if (*P.status != 0) return;  // an earlier panel failed: every workgroup leaves at once
  const int64_t n = P.n, k0 = P.k0, ld = P.ld;
  const double* __restrict__ src = P.src;
  const int64_t rowbase = k0 + 1 + (int64_t)g * P.S;
  const int nslots = (int)max((int64_t)0, min((int64_t)P.S, n - rowbase));
  const int G = P.G;
  const bool mine = lane < nslots;
  uint64_t* const my_mirror = P.mirror + ((size_t)g * 64 + lane) * NP * 4;

  for (int q = 0; q < NP; ++q) {
    sm.LW[q][lane] = make_double2(0.0, 0.0);
    sm.Le[q][lane] = 0.0;
  }
  if (g == 0)
    for (int64_t i = lane; i <= k0; i += kPanelThreads) P.pi[i] = (int32_t)i;

  int32_t psi = mine ? (int32_t)(rowbase + lane) : INT32_MAX;
  const int32_t hbm = mine ? (int32_t)(rowbase + lane) : 0;
  double cur = mine ? src[rowbase + lane + k0 * ld] : 0.0;
  int stop = 0;

  for (int si = 0; si < P.nsteps; ++si) {
    const int64_t k = k0 + si;
    const int j = si >> 1;
    const int ph = si & 1;
    const uint32_t tag = P.tag_base + (uint32_t)si + 1u;
    uint64_t* const recs = P.rec + (size_t)(si & 1) * G * kRecWords;

    // (A) local candidate: this lane's slot if its current index is >= k+1
    const bool act = mine && psi >= k + 1;
    double bv = act ? fabs(cur) : -1.0;
    uint32_t bp = act ? (uint32_t)psi : kNoCand;
    int bs = act ? lane : -1;
    const bool nonfin = __any(act && !isfinite(cur));
    wave_best(bv, bp, bs);

    // (B) publish this workgroup's record (read the candidate's data by readlane)
    {
      const int owner = (bs >= 0) ? bs : 0;
      const double cval = rld(cur, owner);
      const uint32_t h = rl32((uint32_t)hbm, owner);
      const double lz = (bs >= 0) ? sm.Le[j][owner] : 0.0;
      uint32_t pay = 0;
      if (lane == 0) pay = nonfin ? kNonFinite : bp;
      else if (lane == 1) pay = ((uint32_t)owner << 24) | h;
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
    double cc[NQ];
    uint32_t ch[NQ];
    {
      uint64_t w[NQ][4];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int rr = lane + 64 * q;
#pragma unroll
        for (int t = 0; t < 4; ++t) w[q][t] = (rr < G) ? ld_word(recs + (size_t)rr * kRecWords + t) : mk(tag, 0);
      }
      uint64_t t0 = 0;
      for (int it = 0;; ++it) {
        bool ok = true;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
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
        for (int q = 0; q < NQ; ++q) {
          const int rr = lane + 64 * q;
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (tag_of(w[q][t]) != tag) w[q][t] = ld_word(recs + (size_t)rr * kRecWords + t);
        }
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
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
    tout = __any(tout);
    bad = __any(bad);
    wave_best(gv, gp, gs);
    stop = tout ? 4 : (bad ? 2 : (gs < 0 ? 4 : 0));
    if (stop) break;

    // pivot's value and origin: in lane gs % 64, entry gs / 64 of its records
    const int wl = gs & 63, wq = gs >> 6;
    double wc = 0.0;
    uint32_t wh = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (q == wq) {
        wc = cc[q];
        wh = ch[q];
      }
    const double alpha = rld(wc, wl);
    const uint32_t hw = rl32(wh, wl);
    const int64_t hx = hw & 0xFFFFFFu;  // panel-start row of the new row r (= column x)
    const int wslot = (int)(hw >> 24);  // its slot inside workgroup gs
    const int64_t pidx = gp, r = k + 1;

    // (D) relabel the two slots; record the step
    if (mine && pidx != r) {
      if (psi == (int32_t)r) psi = (int32_t)pidx;
      else if (psi == (int32_t)pidx) psi = (int32_t)r;
    }
    if (g == 0 && lane == 0) {
      P.ipiv[r] = (int32_t)pidx;
      P.T[k] = alpha;
    }
    const bool below = mine && psi >= k + 2;  // rows of the new column x = k+1

    // (F) gather column x below its diagonal; fetch the pivot row's coefficients
    double gat = 0.0;
    if (below) {
      const int64_t a = hbm;
      gat = (a > hx) ? src[a + hx * ld] : -src[hx + a * ld];
    }
    // lane t holds coefficient d = t (and d = t + 64): d = 2q -> l'[q], d = 2q+1 -> w[q]
    double cA = 0.0, cB = 0.0, l0 = 0.0;
    {
      const uint64_t* wm = P.mirror + ((size_t)gs * 64 + wslot) * NP * 4;
      const int nd = 2 * j;
      const uint32_t tA = P.tag_base + 2u * (uint32_t)(lane >> 1) + 2u;
      const uint32_t tB = P.tag_base + 2u * (uint32_t)((lane + 64) >> 1) + 2u;
      const bool hasA = lane < nd, hasB = lane + 64 < nd;
      uint64_t a0 = hasA ? ld_word(wm + 2 * lane) : mk(tA, 0);
      uint64_t a1 = hasA ? ld_word(wm + 2 * lane + 1) : mk(tA, 0);
      uint64_t b0 = hasB ? ld_word(wm + 2 * (lane + 64)) : mk(tB, 0);
      uint64_t b1 = hasB ? ld_word(wm + 2 * (lane + 64) + 1) : mk(tB, 0);
      const uint64_t* lwp = recs + (size_t)gs * kRecWords + 4;
      uint64_t z0 = (lane == 0) ? ld_word(lwp) : mk(tag, 0);
      uint64_t z1 = (lane == 0) ? ld_word(lwp + 1) : mk(tag, 0);
      uint64_t t0 = 0;
      for (int it = 0;; ++it) {
        const bool ok = tag_of(a0) == tA && tag_of(a1) == tA && tag_of(b0) == tB && tag_of(b1) == tB &&
                        tag_of(z0) == tag && tag_of(z1) == tag;
        if (__all(ok)) break;
        if ((it & 31) == 0) {
          const uint64_t now = wall_clock64();
          if (it == 0) t0 = now;
          else if (now - t0 > kWaitTicks) {
            tout = true;
            break;
          }
        }
        if (tag_of(a0) != tA) a0 = ld_word(wm + 2 * lane);
        if (tag_of(a1) != tA) a1 = ld_word(wm + 2 * lane + 1);
        if (tag_of(b0) != tB) b0 = ld_word(wm + 2 * (lane + 64));
        if (tag_of(b1) != tB) b1 = ld_word(wm + 2 * (lane + 64) + 1);
        if (tag_of(z0) != tag) z0 = ld_word(lwp);
        if (tag_of(z1) != tag) z1 = ld_word(lwp + 1);
      }
      cA = from32((uint32_t)a0, (uint32_t)a1);
      cB = from32((uint32_t)b0, (uint32_t)b1);
      // coefficient d sits in component d % 2 of pair d / 2
      if (hasA) reinterpret_cast<double*>(&sm.coef[0])[lane] = cA;
      if (hasB) reinterpret_cast<double*>(&sm.coef[0])[lane + 64] = cB;
      l0 = rld(from32((uint32_t)z0, (uint32_t)z1), 0);
      if (__any(tout)) {
        stop = 4;
        break;
      }
    }

    // (E) multipliers below row k+1, alpha at row k+1
    if (mine) {
      double val = 0.0;
      bool wr = true;
      if (psi >= k + 2) val = (alpha != 0.0) ? cur / alpha : 0.0;
      else if (psi == (int32_t)r) val = alpha;
      else wr = false;
      if (wr) {
        if (ph == 0) sm.Le[j][lane] = val;
        else sm.LW[j][lane].x = val;
      }
    }

    // skew GEMV with the pivot row over the pairs so far
    double corr = 0.0, corr2 = 0.0;
    {
      int q = 0;
      for (; q + 1 < j; q += 2) {
        const double2 a = sm.LW[q][lane], b = sm.LW[q + 1][lane];
        const double2 ca = sm.coef[q], cb = sm.coef[q + 1];
        corr += a.x * ca.y - a.y * ca.x;
        corr2 += b.x * cb.y - b.y * cb.x;
      }
      if (q < j) {
        const double2 a = sm.LW[q][lane];
        const double2 ca = sm.coef[q];
        corr += a.x * ca.y - a.y * ca.x;
      }
      corr += corr2;
    }

    // finish the column
    if (ph == 0) {
      if (below) cur = gat + corr;
    } else {
      const double w = below ? gat + corr : 0.0;
      sm.LW[j][lane].y = w;
      const double lp = sm.LW[j][lane].x;
      if (below) cur = w + alpha * (sm.Le[j][lane] - l0 * lp);
      // mirror entries of pair j for this slot (read by other workgroups' later steps)
      if (mine) {
        const uint32_t mt = P.tag_base + 2u * (uint32_t)j + 2u;
        uint64_t* m = my_mirror + (size_t)j * 4;
        st_word(m + 0, mk(mt, hi32(lp)));
        st_word(m + 1, mk(mt, lo32(lp)));
        st_word(m + 2, mk(mt, hi32(w)));
        st_word(m + 3, mk(mt, lo32(w)));
      }
    }
  }

  // ---- panel end ----
  if (stop) {
    if (lane == 0) atomicMin(P.status, (stop & 4) ? SKF_ETIMEOUT : SKF_ENONFINITE);
    return;
  }
  if (!mine) return;
  const int npairs = P.nsteps / 2;
  const int64_t lo = k0 + P.nsteps;
  for (int c = 0; c < P.nsteps; ++c)
    P.Lbuf[psi + (int64_t)c * n] = (c & 1) ? sm.LW[c >> 1][lane].x : sm.Le[c >> 1][lane];
  for (int q = 0; q < npairs; ++q) {
    const double2 v = sm.LW[q][lane];
    P.Lp[psi + (int64_t)q * n] = v.x;
    P.Wp[psi + (int64_t)q * n] = v.y;
  }
  P.pi[psi] = hbm;
  if ((P.nsteps & 1) == 0 && psi >= lo + 1) P.cnext[psi] = cur;
}

template <int NB, int NQ>
int launch_panel_t(const PanelParams& p, hipStream_t s) {
  hipLaunchKernelGGL((panel_kernel<NB, NQ>), dim3(p.G), dim3(kPanelThreads), 0, s, p);
  SKF_CHECK_LAUNCH("panel");
  return 0;
}

}  // namespace

int launch_panel(const PanelParams& p, hipStream_t s) {
  if (p.G > kMaxG || p.S > 64 || p.n >= (1 << 24)) return SKF_ENOTIMPL;
  const int nq = (p.G + 63) / 64;
  if (p.nb == 128) {
    if (nq <= 1) return launch_panel_t<128, 1>(p, s);
    if (nq <= 2) return launch_panel_t<128, 2>(p, s);
    if (nq <= 4) return launch_panel_t<128, 4>(p, s);
    return launch_panel_t<128, 8>(p, s);
  }
  if (p.nb == 64) {
    if (nq <= 1) return launch_panel_t<64, 1>(p, s);
    if (nq <= 2) return launch_panel_t<64, 2>(p, s);
    if (nq <= 4) return launch_panel_t<64, 4>(p, s);
    return launch_panel_t<64, 8>(p, s);
  }
  return SKF_ENOTIMPL;
}

size_t panel_record_words(int G) { return (size_t)2 * G * kRecWords; }

size_t panel_mirror_words(int G, int nb) { return (size_t)G * 64 * (nb / 2) * 4; }

}  // namespace skf
