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
#include <algorithm>

#include "panel_common.h"

namespace skf {

using namespace panel;

namespace {


// LE: each slot's first-step multipliers l kept in LDS (the faster form) or,
// when the grid needs more workgroups per CU than that footprint allows, in a
// slot-major global scratch (one coalesced line per pair, stored with the
// pair's mirror entries and read back by the same lane at the panel's end).
template <int NB, bool LE>
struct PanelSmem {
  double2 LW[NB / 2][64];        // (l', w) of each pair, per slot
  double Le[LE ? NB / 2 : 1][64];  // l of each pair's first step, per slot (LE)
  double2 coef[NB / 2];          // the pivot row's (l', w) of the pairs so far
};

template <int NB, int NQ, bool LE>
__global__ void __launch_bounds__(kPanelThreads) panel_kernel(PanelParams P) {
  constexpr int NP = NB / 2;
  __shared__ PanelSmem<NB, LE> sm;

  const int lane = threadIdx.x;
  const int g = blockIdx.x;
  const int64_t n = P.n, k0 = P.k0, ld = P.ld;
  const double* __restrict__ src = P.src;
  const int64_t rowbase = k0 + 1 + (int64_t)g * P.S;
  const int nslots = (int)max((int64_t)0, min((int64_t)P.S, n - rowbase));
  const int G = P.G;
  const bool mine = lane < nslots;
  if (g == 0)
    for (int64_t i = lane; i <= k0; i += kPanelThreads) P.pi[i] = (int32_t)i;
  if (*P.status != 0) {
    // an earlier panel failed: every workgroup leaves at once, with this
    // panel's permutation the identity (later kernels index rows through it)
    if (mine) P.pi[rowbase + lane] = (int32_t)(rowbase + lane);
    return;
  }
  uint64_t* const my_mirror = P.mirror + ((size_t)g * 64 + lane) * NP * 4;

  for (int q = 0; q < NP; ++q) {
    sm.LW[q][lane] = make_double2(0.0, 0.0);
    if constexpr (LE) sm.Le[q][lane] = 0.0;
  }
  for (int q = lane; q < NP; q += 64) sm.coef[q] = make_double2(0.0, 0.0);
  double* const my_le = P.Lscr + (size_t)g * 64 + lane;  // !LE: slot-major scratch
  const size_t le_stride = (size_t)G * 64;

  int32_t psi = mine ? (int32_t)(rowbase + lane) : INT32_MAX;
  const int32_t hbm = mine ? (int32_t)(rowbase + lane) : 0;
  double cur = mine ? src[rowbase + lane + k0 * ld] : 0.0;
  // wait for this load here: left pending into the step loop, its wait sat at
  // the loop head and, vmcnt counting stores too, made every step wait for the
  // previous step's mirror and record stores
  asm volatile("" : "+v"(cur));
  double lj = 0.0;  // this slot's l of the current pair
  int stop = 0;

  for (int si = 0; si < P.nsteps; ++si) {
    const int64_t k = k0 + si;
    const int j = si >> 1;
    const int ph = si & 1;
    const uint32_t tag = P.tag_base + (uint32_t)si + 1u;
    const uint32_t t16 = tag16(tag);
    uint64_t* const recs0 = P.rec + (size_t)(si & 1) * G * kRecCopies * (kRecStride + 2);
    // l0 words of record g, copy c, at 2 (c G + g) and the next word
    uint64_t* const lzs = recs0 + (size_t)kRecCopies * G * kRecStride;
    uint64_t* const recs = recs0 + (size_t)(g % kRecCopies) * G * kRecStride;  // the copy this workgroup reads

    // (A) local candidate: this lane's slot if its current index is >= k+1
    const bool act = mine && psi >= k + 1;
    const bool nonfin = __any(act && !isfinite(cur));
    const int bs = wave_argbest(fabs(cur), (uint32_t)psi, act);

    // (B) publish this workgroup's record (the candidate's data by readlane);
    // lanes 0..3 each store one word, the payloads picked without branches
    {
      const int owner = (bs >= 0) ? bs : 0;
      const double cval = rld(cur, owner);
      const double lz = rld(lj, owner);  // readers ignore it when there is no candidate
      const uint32_t meta = nonfin ? kFlagNonFinite
                                   : (bs < 0 ? kFlagNoCand : (rl32((uint32_t)psi, owner) | ((uint32_t)owner << 24)));
      const uint64_t cb = (uint64_t)__double_as_longlong(cval);
      const uint64_t mag = cb & ~(1ull << 63);
      const uint64_t th = (uint64_t)t16 << 48;
      const uint64_t w0 = th | ((uint64_t)meta << 16) | (mag >> 47);
      const uint64_t w1 = th | ((cb >> 63) << 47) | (mag & kLow47);
      // lanes 0 .. 2 kRecCopies - 1: word lane % 2 of record copy lane / 2; the next
      // 2 kRecCopies lanes: word lane % 2 of l0 copy (lane - kW) / 2
      constexpr int kW = 2 * kRecCopies;
      const int cw = (lane < kW ? lane : lane - kW) >> 1;
      const uint64_t v = (lane < kW) ? ((lane & 1) ? w1 : w0) : ((lane & 1) ? mk(tag, lo32(lz)) : mk(tag, hi32(lz)));
      uint64_t* const dstw = (lane < kW) ? recs0 + ((size_t)cw * G + g) * kRecStride + (lane & 1)
                                         : lzs + 2 * ((size_t)cw * G + g) + (lane & 1);
      if (lane < 2 * kW) st_word(dstw, v);
    }

    // (C) every workgroup's record (lane t reads records t, t+64, ...) -> global pivot.
    // Each round reloads both words of every record of a block (addresses always
    // valid; lanes past G read record 0 and ignore it) until all carry this step's
    // tag.  One block holds up to 16 records per lane, so up to 1024 workgroups
    // are read in one round; beyond, the blocks are waited for one after the other
    // (a record with this step's tag stays until every workgroup has read it).
    double gv = -1.0, gc = 0.0;
    uint32_t gp = kNoCand, gslot = 0;
    int gs = -1;
    bool bad = false, tout = false;
    {
      constexpr int QB = NQ < 16 ? NQ : 16;
      const int nblk = (G + 64 * QB - 1) / (64 * QB);
#pragma unroll 1
      for (int b = 0; b < nblk && !tout; ++b) {
        const int rb = 64 * QB * b;
        uint64_t w[QB][2];
        const uint64_t* rp[QB];
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          const int rr = rb + lane + 64 * q;
          rp[q] = recs + (size_t)(rr < G ? rr : 0) * kRecStride;
        }
        auto load_all = [&]() {
#pragma unroll
          for (int q = 0; q < QB; ++q) {
            w[q][0] = ld_word(rp[q]);
            w[q][1] = ld_word(rp[q] + 1);
          }
        };
        load_all();
        uint64_t t0 = 0;
        for (int it = 0;; ++it) {
          bool ok = true;
#pragma unroll
          for (int q = 0; q < QB; ++q) {
            const bool need = rb + lane + 64 * q < G;
            ok &= !need | ((tag16_of(w[q][0]) == t16) & (tag16_of(w[q][1]) == t16));  // no short-circuit branches
          }
          if (__all(ok)) break;
          poll_refresh<(NQ > 16)>(it);
          if ((it & 31) == 0) {
            const uint64_t now = wall_clock64();
            if (it == 0) t0 = now;
            else if (now - t0 > kWaitTicks) {
              tout = true;
              break;
            }
          }
          load_all();
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          landed(w[q][0]);
          landed(w[q][1]);
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          const int rr = rb + lane + 64 * q;
          const uint32_t meta = (uint32_t)(w[q][0] >> 16);
          const bool use = rr < G && !tout;
          bad |= use && (meta & kFlagNonFinite);
          if (use && !(meta & (kFlagNonFinite | kFlagNoCand))) {
            const uint64_t mag = ((w[q][0] & 0xFFFFull) << 47) | (w[q][1] & kLow47);
            const double a = __longlong_as_double((long long)mag);
            const uint32_t ps = meta & 0xFFFFFFu;
            if (better(a, ps, gv, gp)) {
              gv = a;
              gc = __longlong_as_double((long long)(mag | (((w[q][1] >> 47) & 1ull) << 63)));
              gp = ps;
              gs = rr;
              gslot = meta >> 24 & 63u;
            }
          }
        }
        tout = __any(tout);
      }
    }
    tout = __any(tout);
    bad = __any(bad);
    const int wl = wave_argbest(gv, gp, gs >= 0);
    stop = tout ? 4 : (bad ? 2 : (wl < 0 ? 4 : 0));
    if (stop) break;

    // the pivot: its value, current index, workgroup and slot (from lane wl)
    const double alpha = rld(gc, wl);
    gp = rl32(gp, wl);
    gs = (int)rl32((uint32_t)gs, wl);
    const int wslot = (int)rl32(gslot, wl);
    const int64_t hx = k0 + 1 + (int64_t)gs * P.S + wslot;  // panel-start row of the new row r (= column x)
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

    // (F) gather column x below its diagonal (every lane loads from a valid
    // address; the sign and the mask are applied afterwards); fetch the pivot
    // row's coefficients and l0
    const bool lowr = (int64_t)hbm > hx;
    const double graw = src[lowr ? (int64_t)hbm + hx * ld : hx + (int64_t)hbm * ld];
    // lane t holds coefficients d = t + 64 c (c < CPL): d = 2q -> l'[q], d = 2q+1 -> w[q]
    double l0 = 0.0;
    {
      constexpr int CPL = (2 * NP + 63) / 64;  // coefficients per lane
      const uint64_t* wm = P.mirror + ((size_t)gs * 64 + wslot) * NP * 4;
      const int nd = 2 * j;
      uint32_t tc[CPL];
      bool has[CPL];
      int ic[CPL];
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int d = lane + 64 * c;
        tc[c] = P.tag_base + 2u * (uint32_t)(d >> 1) + 2u;
        has[c] = d < nd;
        ic[c] = (d < 2 * NP) ? 2 * d : 0;  // a valid address for every lane
      }
      const uint64_t* lwp = lzs + 2 * ((size_t)(g % kRecCopies) * G + gs);
      uint64_t cw[CPL][2], z0, z1;
      auto load_all = [&]() {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          cw[c][0] = ld_word(wm + ic[c]);
          cw[c][1] = ld_word(wm + ic[c] + 1);
        }
        z0 = ld_word(lwp);
        z1 = ld_word(lwp + 1);
      };
      load_all();
      // (E) multipliers below row k+1, alpha at row k+1: formed while the
      // gather and the coefficient words are in flight
      if (mine) {
        double val = 0.0;
        bool wr = true;
        if (psi >= k + 2) val = (alpha != 0.0) ? cur / alpha : 0.0;
        else if (psi == (int32_t)r) val = alpha;
        else wr = false;
        if (wr) {
          if (ph == 1) sm.LW[j][lane].x = val;
          else if constexpr (LE) sm.Le[j][lane] = val;
        }
        if (ph == 0) lj = wr ? val : 0.0;
      }
      uint64_t t0 = 0;
      for (int it = 0;; ++it) {
        bool ok = (tag_of(z0) == tag) & (tag_of(z1) == tag);
#pragma unroll
        for (int c = 0; c < CPL; ++c) ok &= !has[c] | ((tag_of(cw[c][0]) == tc[c]) & (tag_of(cw[c][1]) == tc[c]));
        if (__all(ok)) break;
        poll_refresh<(NQ > 16)>(it);
        if ((it & 31) == 0) {
          const uint64_t now = wall_clock64();
          if (it == 0) t0 = now;
          else if (now - t0 > kWaitTicks) {
            tout = true;
            break;
          }
        }
        load_all();
      }
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        landed(cw[c][0]);
        landed(cw[c][1]);
      }
      landed(z0);
      landed(z1);
      // coefficient d sits in component d % 2 of pair d / 2
#pragma unroll
      for (int c = 0; c < CPL; ++c)
        if (has[c])
          reinterpret_cast<double*>(&sm.coef[0])[lane + 64 * c] = from32((uint32_t)cw[c][0], (uint32_t)cw[c][1]);
      l0 = from32((uint32_t)z0, (uint32_t)z1);
      // form l0 in its own registers here, while the coefficient loads are
      // known to have landed: formed lazily at its use after this step's
      // mirror stores, it made the compiler wait for those stores too
      asm volatile("" : "+v"(l0));
      if (__any(tout)) {
        stop = 4;
        break;
      }
    }
    const double gat = below ? (lowr ? graw : -graw) : 0.0;

    // skew GEMV with the pivot row over the pairs so far: sixteen pairs per
    // pass (all of them for the narrowest panel), their LDS reads issued
    // together (coefficients of pairs >= j are zero)
    double corr = 0.0;
    {
      // l' w-terms and w l'-terms summed separately (one fused multiply-add per
      // product, four independent chains each)
      double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
      constexpr int GW = NP < 16 ? NP : 16;
      const int jr = (j + GW - 1) / GW * GW;
      for (int q = 0; q < jr; q += GW) {
        double2 a[GW], c[GW];
        const double2* cb = &sm.coef[q];
#pragma unroll
        for (int t = 0; t < GW; ++t) {
          a[t] = sm.LW[q + t][lane];
          c[t] = cb[t];
        }
#pragma unroll
        for (int t = 0; t < GW; t += 4) {
          p0 = fma(a[t].x, c[t].y, p0);
          m0 = fma(a[t].y, c[t].x, m0);
          p1 = fma(a[t + 1].x, c[t + 1].y, p1);
          m1 = fma(a[t + 1].y, c[t + 1].x, m1);
          p2 = fma(a[t + 2].x, c[t + 2].y, p2);
          m2 = fma(a[t + 2].y, c[t + 2].x, m2);
          p3 = fma(a[t + 3].x, c[t + 3].y, p3);
          m3 = fma(a[t + 3].y, c[t + 3].x, m3);
        }
      }
      corr = ((p0 + p1) + (p2 + p3)) - ((m0 + m1) + (m2 + m3));
    }

    // finish the column
    if (ph == 0) {
      if (below) cur = gat + corr;
    } else {
      const double w = below ? gat + corr : 0.0;
      sm.LW[j][lane].y = w;
      const double lp = sm.LW[j][lane].x;
      if (below) cur = w + alpha * (lj - l0 * lp);
      // mirror entries of pair j for this slot (read by other workgroups' later steps)
      if (mine) {
        const uint32_t mt = P.tag_base + 2u * (uint32_t)j + 2u;
        uint64_t* m = my_mirror + (size_t)j * 4;
        st_word(m + 0, mk(mt, hi32(lp)));
        st_word(m + 1, mk(mt, lo32(lp)));
        st_word(m + 2, mk(mt, hi32(w)));
        st_word(m + 3, mk(mt, lo32(w)));
        if constexpr (!LE) my_le[(size_t)j * le_stride] = lj;  // beside the mirror stores
      }
    }
  }

  // ---- panel end ----
  if (stop) {
    if (lane == 0) atomicMin(P.status, (stop & 4) ? SKF_ETIMEOUT : SKF_ENONFINITE);
    // the permutation stays in range (row indices of this panel) for the kernels after it
    if (mine) P.pi[psi] = hbm;
    return;
  }
  if (!mine) return;
  const int npairs = P.nsteps / 2;
  const int64_t lo = k0 + P.nsteps;
  // !LE: an unpaired last step's l is still in lj (pairs store theirs at the pair's end)
  for (int c = 0; c < P.nsteps; ++c) {
    double le;
    if constexpr (LE) le = sm.Le[c >> 1][lane];
    else le = (c + 1 == P.nsteps) ? lj : my_le[(size_t)(c >> 1) * le_stride];
    P.Lbuf[psi + (int64_t)c * n] = (c & 1) ? sm.LW[c >> 1][lane].x : le;
  }
  // the pair vectors are the trailing update's operands; row lo is stored as
  // zero, so the update leaves column lo (the next panel's first column, taken
  // from cnext as it stands) without products
  for (int q = 0; q < npairs; ++q) {
    const double2 v = sm.LW[q][lane];
    const double lp = (psi == lo) ? 0.0 : v.x;
    P.Lp[psi + (int64_t)q * n] = lp;
    P.Wp[psi + (int64_t)q * n] = (psi == lo) ? 0.0 : v.y;
    P.NLp[psi + (int64_t)q * n] = -lp;
  }
  P.pi[psi] = hbm;
  if ((P.nsteps & 1) == 0 && psi >= lo + 1) P.cnext[psi] = cur;
}

// ---------------------------------------------------------------------------
// Pfaffian-only panel: NB/2 elimination steps at even k only (k = k0, k0+2, ...),
// each giving one pair (l, v): l = multipliers of column k, v = column k+1 after
// the interchange, and the trailing change l v^T - v l^T.  The machinery is the
// full panel's (slots, relabelling, records, mirrors, gathers from the
// panel-start matrix S plus the panel's pairs); what differs is the next pivot
// column: it is column k+2, i.e. the row y standing at index k+2 after the
// interchange (the old row k+1 when p = k+2, else the old row k+2), which is in
// general not the winner.  So the owners of the rows at indices k+1 and k+2
// publish (workgroup, slot, current value) in two tagged front entries beside
// the records, and after the exchange every workgroup fetches the coefficient
// rows of both x (the winner) and y, gathers S(., x) and S(., y) for its slots,
// and forms, per slot i with index >= k+2:
//   l_i = c_i / alpha,  v_i = S(i, x) + sum_{q<s} (l_q[i] v_q[x] - v_q[i] l_q[x]),
// the scalars l_y = c_y / alpha and v_y = S(y, x) + sum_{q<s} (l_q[y] v_q[x] - v_q[y] l_q[x]),
// and the next column  c'_i = S(i, y) + sum_{q<s} (l_q[i] v_q[y] - v_q[i] l_q[y])
//                             + l_i v_y - v_i l_y.
// Pair q's mirror words carry the tag of step q.  No L is produced.
template <int NB>
struct PanelPfSmem {
  double2 LW[NB / 2][64];  // (l, v) of each step, per slot
  double2 cx[NB / 2];      // the winner's (l, v) of the steps so far
  double2 cy[NB / 2];      // the row at index k+2: its (l, v) of the steps so far
};

template <int NB, int NQ>
__global__ void __launch_bounds__(kPanelThreads) panel_pf_kernel(PanelParams P) {
  constexpr int NP = NB / 2;
  __shared__ PanelPfSmem<NB> sm;

  const int lane = threadIdx.x;
  const int g = blockIdx.x;
  const int64_t n = P.n, k0 = P.k0, ld = P.ld;
  const double* __restrict__ src = P.src;
  const int64_t rowbase = k0 + 1 + (int64_t)g * P.S;
  const int nslots = (int)max((int64_t)0, min((int64_t)P.S, n - rowbase));
  const int G = P.G;
  const bool mine = lane < nslots;
  if (g == 0)
    for (int64_t i = lane; i <= k0; i += kPanelThreads) P.pi[i] = (int32_t)i;
  if (*P.status != 0) {
    if (mine) P.pi[rowbase + lane] = (int32_t)(rowbase + lane);
    return;
  }
  uint64_t* const my_mirror = P.mirror + ((size_t)g * 64 + lane) * NP * 4;

  for (int q = 0; q < NP; ++q) sm.LW[q][lane] = make_double2(0.0, 0.0);
  for (int q = lane; q < NP; q += 64) {
    sm.cx[q] = make_double2(0.0, 0.0);
    sm.cy[q] = make_double2(0.0, 0.0);
  }

  int32_t psi = mine ? (int32_t)(rowbase + lane) : INT32_MAX;
  const int32_t hbm = mine ? (int32_t)(rowbase + lane) : 0;
  double cur = mine ? src[rowbase + lane + k0 * ld] : 0.0;
  // wait for this load here: left pending into the step loop, its wait sat at
  // the loop head and, vmcnt counting stores too, made every step wait for the
  // previous step's mirror and record stores
  asm volatile("" : "+v"(cur));
  int stop = 0;
  int done = 0;  // steps that produced a pair

  for (int si = 0; si < P.nsteps; ++si) {
    const int64_t k = k0 + 2 * si;
    const int64_t r = k + 1;
    const bool last = k + 2 > n - 1;  // k = n-2: pivot only
    const uint32_t tag = P.tag_base + (uint32_t)si + 1u;
    const uint32_t t16 = tag16(tag);
    uint64_t* const recs0 = P.rec + (size_t)(si & 1) * G * kRecCopies * (kRecStride + 2);
    uint64_t* const recs = recs0 + (size_t)(g % kRecCopies) * G * kRecStride;
    uint64_t* const front = P.front + (size_t)(si & 1) * 8;  // entry e (index k+1+e) at 4e: ws, hi, lo

    // (A) local candidate
    const bool act = mine && psi >= k + 1;
    const bool nonfin = __any(act && !isfinite(cur));
    const int bs = wave_argbest(fabs(cur), (uint32_t)psi, act);

    // (B) record (as the full panel) and, by the owners of indices k+1 and k+2,
    // the front entries (workgroup << 6 | slot, current value)
    {
      const int owner = (bs >= 0) ? bs : 0;
      const double cval = rld(cur, owner);
      const uint32_t meta = nonfin ? kFlagNonFinite
                                   : (bs < 0 ? kFlagNoCand : (rl32((uint32_t)psi, owner) | ((uint32_t)owner << 24)));
      const uint64_t cb = (uint64_t)__double_as_longlong(cval);
      const uint64_t mag = cb & ~(1ull << 63);
      const uint64_t th = (uint64_t)t16 << 48;
      const uint64_t w0 = th | ((uint64_t)meta << 16) | (mag >> 47);
      const uint64_t w1 = th | ((cb >> 63) << 47) | (mag & kLow47);
      constexpr int kW = 2 * kRecCopies;
      const uint64_t v = (lane & 1) ? w1 : w0;
      uint64_t* const dstw = recs0 + ((size_t)(lane >> 1) * G + g) * kRecStride + (lane & 1);
      if (lane < kW) st_word(dstw, v);
      const int64_t e = (int64_t)psi - (k + 1);
      if (mine && (e == 0 || (e == 1 && !last))) {
        uint64_t* fe = front + 4 * e;
        st_word(fe, mk(tag, ((uint32_t)g << 6) | (uint32_t)lane));
        st_word(fe + 1, mk(tag, hi32(cur)));
        st_word(fe + 2, mk(tag, lo32(cur)));
      }
    }

    // (C) records -> global pivot; front entries (every lane reads the same words).
    // Records are read in blocks of up to 16 per lane as in the full panel; the
    // front entries are polled with every block.
    double gv = -1.0, gc = 0.0;
    uint32_t gp = kNoCand, gslot = 0;
    int gs = -1;
    bool bad = false, tout = false;
    uint64_t f0a = 0, f0b = 0, f0c = 0, f1a = 0, f1b = 0, f1c = 0;
    {
      constexpr int QB = NQ < 16 ? NQ : 16;
      const int nblk = (G + 64 * QB - 1) / (64 * QB);
#pragma unroll 1
      for (int b = 0; b < nblk && !tout; ++b) {
        const int rb = 64 * QB * b;
        uint64_t w[QB][2];
        const uint64_t* rp[QB];
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          const int rr = rb + lane + 64 * q;
          rp[q] = recs + (size_t)(rr < G ? rr : 0) * kRecStride;
        }
        auto load_recs = [&]() {
#pragma unroll
          for (int q = 0; q < QB; ++q) {
            w[q][0] = ld_word(rp[q]);
            w[q][1] = ld_word(rp[q] + 1);
          }
          f0a = ld_word(front);
          f0b = ld_word(front + 1);
          f0c = ld_word(front + 2);
          f1a = ld_word(front + 4);
          f1b = ld_word(front + 5);
          f1c = ld_word(front + 6);
        };
        load_recs();
        uint64_t t0 = 0;
        for (int it = 0;; ++it) {
          bool ok = (tag_of(f0a) == tag) & (tag_of(f0b) == tag) & (tag_of(f0c) == tag);
          ok &= last | ((tag_of(f1a) == tag) & (tag_of(f1b) == tag) & (tag_of(f1c) == tag));
#pragma unroll
          for (int q = 0; q < QB; ++q) {
            const bool need = rb + lane + 64 * q < G;
            ok &= !need | ((tag16_of(w[q][0]) == t16) & (tag16_of(w[q][1]) == t16));
          }
          if (__all(ok)) break;
          poll_refresh<(NQ > 16)>(it);
          if ((it & 31) == 0) {
            const uint64_t now = wall_clock64();
            if (it == 0) t0 = now;
            else if (now - t0 > kWaitTicks) {
              tout = true;
              break;
            }
          }
          load_recs();
        }
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          landed(w[q][0]);
          landed(w[q][1]);
        }
        landed(f0a);
        landed(f0b);
        landed(f0c);
        landed(f1a);
        landed(f1b);
        landed(f1c);
#pragma unroll
        for (int q = 0; q < QB; ++q) {
          const int rr = rb + lane + 64 * q;
          const uint32_t meta = (uint32_t)(w[q][0] >> 16);
          const bool use = rr < G && !tout;
          bad |= use && (meta & kFlagNonFinite);
          if (use && !(meta & (kFlagNonFinite | kFlagNoCand))) {
            const uint64_t mag = ((w[q][0] & 0xFFFFull) << 47) | (w[q][1] & kLow47);
            const double a = __longlong_as_double((long long)mag);
            const uint32_t ps = meta & 0xFFFFFFu;
            if (better(a, ps, gv, gp)) {
              gv = a;
              gc = __longlong_as_double((long long)(mag | (((w[q][1] >> 47) & 1ull) << 63)));
              gp = ps;
              gs = rr;
              gslot = meta >> 24 & 63u;
            }
          }
        }
        tout = __any(tout);
      }
    }
    tout = __any(tout);
    bad = __any(bad);
    const int wl = wave_argbest(gv, gp, gs >= 0);
    stop = tout ? 4 : (bad ? 2 : (wl < 0 ? 4 : 0));
    if (stop) break;

    const double alpha = rld(gc, wl);
    gp = rl32(gp, wl);
    gs = (int)rl32((uint32_t)gs, wl);
    const int wslot = (int)rl32(gslot, wl);
    const int64_t hx = k0 + 1 + (int64_t)gs * P.S + wslot;
    const int64_t pidx = gp;

    // the row at index k+2 after the interchange: the old row k+1 when p = k+2
    const bool yfrom0 = pidx == k + 2;
    const uint32_t fws = (uint32_t)(yfrom0 ? f0a : f1a);
    const int ygs = (int)(fws >> 6), yslot = (int)(fws & 63u);
    const double ycur = yfrom0 ? from32((uint32_t)f0b, (uint32_t)f0c) : from32((uint32_t)f1b, (uint32_t)f1c);
    const int64_t hy = k0 + 1 + (int64_t)ygs * P.S + yslot;

    // (D) relabel; record the step
    if (mine && pidx != r) {
      if (psi == (int32_t)r) psi = (int32_t)pidx;
      else if (psi == (int32_t)pidx) psi = (int32_t)r;
    }
    if (g == 0 && lane == 0) {
      P.ipiv[r] = (int32_t)pidx;
      P.T[k] = alpha;
    }
    if (last) break;
    const bool below = mine && psi >= k + 2;

    // (F) gathers S(i, x), S(i, y), S(y, x) (valid addresses everywhere; signs and
    // masks afterwards) and the coefficient rows of x and y
    const bool lowx = (int64_t)hbm > hx, lowy = (int64_t)hbm > hy, lowyx = hy > hx;
    const double grx = src[lowx ? (int64_t)hbm + hx * ld : hx + (int64_t)hbm * ld];
    const double gry = src[lowy ? (int64_t)hbm + hy * ld : hy + (int64_t)hbm * ld];
    const double gyx = src[lowyx ? hy + hx * ld : hx + hy * ld];
    {
      constexpr int CPL = (2 * NP + 63) / 64;  // coefficients per lane: d = lane + 64 c
      const uint64_t* wx = P.mirror + ((size_t)gs * 64 + wslot) * NP * 4;
      const uint64_t* wy = P.mirror + ((size_t)ygs * 64 + yslot) * NP * 4;
      const int nd = 2 * si;
      uint32_t tc[CPL];
      bool has[CPL];
      int ic[CPL];
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int d = lane + 64 * c;
        tc[c] = P.tag_base + (uint32_t)(d >> 1) + 1u;
        has[c] = d < nd;
        ic[c] = (d < 2 * NP) ? 2 * d : 0;  // a valid address for every lane
      }
      uint64_t xw[CPL][2], yw[CPL][2];
      auto load_coef = [&]() {
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          xw[c][0] = ld_word(wx + ic[c]);
          xw[c][1] = ld_word(wx + ic[c] + 1);
          yw[c][0] = ld_word(wy + ic[c]);
          yw[c][1] = ld_word(wy + ic[c] + 1);
        }
      };
      load_coef();
      uint64_t t0 = 0;
      for (int it = 0;; ++it) {
        bool ok = true;
#pragma unroll
        for (int c = 0; c < CPL; ++c)
          ok &= !has[c] | ((tag_of(xw[c][0]) == tc[c]) & (tag_of(xw[c][1]) == tc[c]) & (tag_of(yw[c][0]) == tc[c]) &
                           (tag_of(yw[c][1]) == tc[c]));
        if (__all(ok)) break;
        poll_refresh<(NQ > 16)>(it);
        if ((it & 31) == 0) {
          const uint64_t now = wall_clock64();
          if (it == 0) t0 = now;
          else if (now - t0 > kWaitTicks) {
            tout = true;
            break;
          }
        }
        load_coef();
      }
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        landed(xw[c][0]);
        landed(xw[c][1]);
        landed(yw[c][0]);
        landed(yw[c][1]);
      }
      // coefficient d sits in component d % 2 of step d / 2
#pragma unroll
      for (int c = 0; c < CPL; ++c)
        if (has[c]) {
          reinterpret_cast<double*>(&sm.cx[0])[lane + 64 * c] = from32((uint32_t)xw[c][0], (uint32_t)xw[c][1]);
          reinterpret_cast<double*>(&sm.cy[0])[lane + 64 * c] = from32((uint32_t)yw[c][0], (uint32_t)yw[c][1]);
        }
      if (__any(tout)) {
        stop = 4;
        break;
      }
    }
    const double gx = below ? (lowx ? grx : -grx) : 0.0;
    const double gy = (mine && psi >= k + 3) ? (lowy ? gry : -gry) : 0.0;
    const double syx = lowyx ? gyx : -gyx;  // S(y, x); y != x (y stands at index k+2, x at k+1)

    // skew GEMVs over the steps so far (coefficients of steps >= si are zero)
    double ax = 0.0, ay = 0.0, axy = 0.0;
    {
      const int jr = (si + 7) & ~7;
      for (int q = 0; q < jr; q += 8) {
        double2 a[8], cxv[8], cyv[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          a[t] = sm.LW[q + t][lane];
          cxv[t] = sm.cx[q + t];
          cyv[t] = sm.cy[q + t];
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          ax += a[t].x * cxv[t].y - a[t].y * cxv[t].x;
          ay += a[t].x * cyv[t].y - a[t].y * cyv[t].x;
          axy += cyv[t].x * cxv[t].y - cyv[t].y * cxv[t].x;
        }
      }
    }
    // l_y is formed exactly as its owner forms it, so every workgroup uses the same bits
    const double li = below ? ((alpha != 0.0) ? cur / alpha : 0.0) : 0.0;
    const double vi = below ? gx + ax : 0.0;
    const double ly = (alpha != 0.0) ? ycur / alpha : 0.0;
    const double vy = syx + axy;
    sm.LW[si][lane] = make_double2(li, vi);
    cur = (mine && psi >= k + 3) ? gy + ay + (li * vy - vi * ly) : 0.0;
    ++done;
    if (mine) {
      const uint32_t mt = tag;  // pair si carries the tag of step si
      uint64_t* m = my_mirror + (size_t)si * 4;
      st_word(m + 0, mk(mt, hi32(li)));
      st_word(m + 1, mk(mt, lo32(li)));
      st_word(m + 2, mk(mt, hi32(vi)));
      st_word(m + 3, mk(mt, lo32(vi)));
    }
  }

  // ---- panel end ----
  if (stop) {
    if (lane == 0) atomicMin(P.status, (stop & 4) ? SKF_ETIMEOUT : SKF_ENONFINITE);
    if (mine) P.pi[psi] = hbm;
    return;
  }
  if (!mine) return;
  const int64_t lo = k0 + 2 * done;
  for (int q = 0; q < done; ++q) {
    const double2 v = sm.LW[q][lane];
    const double lp = (psi == lo) ? 0.0 : v.x;
    P.Lp[psi + (int64_t)q * n] = lp;
    P.Wp[psi + (int64_t)q * n] = (psi == lo) ? 0.0 : v.y;
    P.NLp[psi + (int64_t)q * n] = -lp;
  }
  P.pi[psi] = hbm;
  if (psi >= lo + 1) P.cnext[psi] = cur;
}

template <int NB, int NQ>
int launch_panel_pf_t(const PanelParams& p, hipStream_t s) {
  hipLaunchKernelGGL((panel_pf_kernel<NB, NQ>), dim3(p.G), dim3(kPanelThreads), 0, s, p);
  SKF_CHECK_LAUNCH("panel_pf");
  return 0;
}

template <int NB, int NQ, bool LE>
int launch_panel_t(const PanelParams& p, hipStream_t s) {
  hipLaunchKernelGGL((panel_kernel<NB, NQ, LE>), dim3(p.G), dim3(kPanelThreads), 0, s, p);
  SKF_CHECK_LAUNCH("panel");
  return 0;
}

}  // namespace

int launch_panel(const PanelParams& p, hipStream_t s) {
  if (p.G > kMaxG || p.S > 64 || p.n >= (1 << 24)) return SKF_ENOTIMPL;
  const int nq = (p.G + 63) / 64;
  // multipliers in LDS whenever the grid fits at that footprint
  const bool le = p.G <= panel_wgs_per_cu_form(p.nb, true) * device_info().num_cus;
  switch (p.nb) {
    case 256: return nq <= 1 ? launch_panel_t<256, 1, false>(p, s) : nq <= 2 ? launch_panel_t<256, 2, false>(p, s)
                     : nq <= 4 ? launch_panel_t<256, 4, false>(p, s) : SKF_ENOTIMPL;
    case 128:
      if (le)
        return nq <= 1 ? launch_panel_t<128, 1, true>(p, s) : nq <= 2 ? launch_panel_t<128, 2, true>(p, s)
               : nq <= 4 ? launch_panel_t<128, 4, true>(p, s) : launch_panel_t<128, 8, true>(p, s);
      return nq <= 4 ? launch_panel_t<128, 4, false>(p, s) : launch_panel_t<128, 8, false>(p, s);
    case 64:
      if (le)
        return nq <= 1 ? launch_panel_t<64, 1, true>(p, s) : nq <= 2 ? launch_panel_t<64, 2, true>(p, s)
               : nq <= 4 ? launch_panel_t<64, 4, true>(p, s) : nq <= 8 ? launch_panel_t<64, 8, true>(p, s)
               : launch_panel_t<64, 16, true>(p, s);
      return nq <= 8 ? launch_panel_t<64, 8, false>(p, s) : launch_panel_t<64, 16, false>(p, s);
    case 32: return nq <= 2 ? launch_panel_t<32, 2, true>(p, s) : nq <= 8 ? launch_panel_t<32, 8, true>(p, s)
                    : nq <= 16 ? launch_panel_t<32, 16, true>(p, s) : launch_panel_t<32, 32, true>(p, s);
    case 16: return nq <= 2 ? launch_panel_t<16, 2, true>(p, s) : nq <= 8 ? launch_panel_t<16, 8, true>(p, s)
                    : nq <= 16 ? launch_panel_t<16, 16, true>(p, s) : launch_panel_t<16, 32, true>(p, s);
    default: return SKF_ENOTIMPL;
  }
}

int launch_panel_pf(const PanelParams& p, hipStream_t s) {
  if (p.G > kMaxG || p.S > 64 || p.n >= (1 << 24) || !p.front) return SKF_ENOTIMPL;
  const int nq = (p.G + 63) / 64;
  switch (p.nb) {
    case 256: return nq <= 1 ? launch_panel_pf_t<256, 1>(p, s) : nq <= 2 ? launch_panel_pf_t<256, 2>(p, s)
                     : nq <= 4 ? launch_panel_pf_t<256, 4>(p, s) : SKF_ENOTIMPL;
    case 128: return nq <= 1 ? launch_panel_pf_t<128, 1>(p, s) : nq <= 2 ? launch_panel_pf_t<128, 2>(p, s)
                     : nq <= 4 ? launch_panel_pf_t<128, 4>(p, s) : launch_panel_pf_t<128, 8>(p, s);
    case 64: return nq <= 1 ? launch_panel_pf_t<64, 1>(p, s) : nq <= 2 ? launch_panel_pf_t<64, 2>(p, s)
                    : nq <= 4 ? launch_panel_pf_t<64, 4>(p, s) : nq <= 8 ? launch_panel_pf_t<64, 8>(p, s) : launch_panel_pf_t<64, 16>(p, s);
    case 32: return nq <= 2 ? launch_panel_pf_t<32, 2>(p, s) : nq <= 8 ? launch_panel_pf_t<32, 8>(p, s)
                    : nq <= 16 ? launch_panel_pf_t<32, 16>(p, s) : launch_panel_pf_t<32, 32>(p, s);
    case 16: return nq <= 2 ? launch_panel_pf_t<16, 2>(p, s) : nq <= 8 ? launch_panel_pf_t<16, 8>(p, s)
                    : nq <= 16 ? launch_panel_pf_t<16, 16>(p, s) : launch_panel_pf_t<16, 32>(p, s);
    default: return SKF_ENOTIMPL;
  }
}

// At most six panel workgroups per CU: measured with every polling round fenced,
// 1536 workgroups (six per CU) exchange their records correctly, while with
// 2032 (eight per CU) some readers still never saw records already written and
// the bounded wait ended in SKF_ETIMEOUT.
constexpr int kMaxPanelPerCu = 6;

size_t panel_record_words(int G) { return (size_t)2 * G * kRecCopies * (kRecStride + 2); }

size_t panel_mirror_words(int G, int nb) { return (size_t)G * 64 * (nb / 2) * 4; }

int panel_slots() { return 64; }

// Panel workgroups that may share one CU for width nb, per kernel form (the
// full panel with its multipliers in LDS or in scratch, or the Pfaffian-only
// panel): the occupancy of its largest record-pass instantiation (registers
// and wave slots), capped by the LDS it holds rounded up to 1 KB per workgroup
// (the occupancy query counts the exact byte size, and one workgroup more than
// the rounded bound, 13 of 12416 bytes on a 160 KB CU, was measured not to
// fit), and by kMaxPanelPerCu; 0 for a form that is not built.  Cached.
static int wgs_per_cu(int nb, int form) {  // form 0: full, LE; 1: full, scratch; 2: Pfaffian-only
  static int cache[3][6] = {{0}};
  const int w = nb == 128 ? 0 : nb == 64 ? 1 : nb == 32 ? 2 : nb == 16 ? 3 : nb == 256 ? 4 : 5;
  if (w == 5) return 0;
  if (form == 0 && w == 4) return 0;       // 256 with l in LDS: beyond a CU's LDS
  if (form == 1 && (w == 2 || w == 3)) return 0;  // 32, 16: the LDS form already reaches the cap
  int& c = cache[form][w];
  if (c) return c;
  const void* k = nullptr;
  size_t lds = 0;
  switch (form * 8 + w) {
    case 0: k = (const void*)panel_kernel<128, 8, true>; lds = sizeof(PanelSmem<128, true>); break;
    case 1: k = (const void*)panel_kernel<64, 16, true>; lds = sizeof(PanelSmem<64, true>); break;
    case 2: k = (const void*)panel_kernel<32, 32, true>; lds = sizeof(PanelSmem<32, true>); break;
    case 3: k = (const void*)panel_kernel<16, 32, true>; lds = sizeof(PanelSmem<16, true>); break;
    case 8: k = (const void*)panel_kernel<128, 8, false>; lds = sizeof(PanelSmem<128, false>); break;
    case 9: k = (const void*)panel_kernel<64, 16, false>; lds = sizeof(PanelSmem<64, false>); break;
    case 12: k = (const void*)panel_kernel<256, 4, false>; lds = sizeof(PanelSmem<256, false>); break;
    case 16: k = (const void*)panel_pf_kernel<128, 8>; lds = sizeof(PanelPfSmem<128>); break;
    case 17: k = (const void*)panel_pf_kernel<64, 16>; lds = sizeof(PanelPfSmem<64>); break;
    case 18: k = (const void*)panel_pf_kernel<32, 32>; lds = sizeof(PanelPfSmem<32>); break;
    case 19: k = (const void*)panel_pf_kernel<16, 32>; lds = sizeof(PanelPfSmem<16>); break;
    default: k = (const void*)panel_pf_kernel<256, 4>; lds = sizeof(PanelPfSmem<256>); break;
  }
  size_t lds_cu = 163840;
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) == hipSuccess && v > 0)
    lds_cu = (size_t)v;
  (void)hipGetLastError();
  const int by_lds = (int)(lds_cu / align_up(lds, 1024));
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k, kPanelThreads, 0) != hipSuccess || b < 1) {
    // no device to ask (host-only use of the planner): the LDS bound alone
    (void)hipGetLastError();
    b = by_lds;
  }
  c = std::min(std::min(b, by_lds), kMaxPanelPerCu);
  return c;
}

int panel_wgs_per_cu_form(int nb, bool le) { return wgs_per_cu(nb, le ? 0 : 1); }

// The most panel workgroups per CU any form of the panel reaches at width nb.
int panel_wgs_per_cu(int nb, bool pf) {
  if (pf) return wgs_per_cu(nb, 2);
  return std::max(wgs_per_cu(nb, 0), wgs_per_cu(nb, 1));
}

size_t panel_scratch_doubles(int G, int nb) { return (size_t)(nb / 2) * G * 64; }

}  // namespace skf
