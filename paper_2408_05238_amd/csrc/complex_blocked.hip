// Blocked Pfaffian-only reduction of a complex (complex128) skew-symmetric
// matrix on the real panel machinery and the real matrix cores.
//
// The elimination is the one of the unblocked form (complex.hip): at even steps
// k only, pivot on the largest |z|^2 = re^2 + im^2 below the diagonal of column
// k (each product rounded, lowest index on ties), interchange rows and columns
// k+1 and p, l = column k / alpha, v = column k+1, add l v^T - v l^T.  Taken in
// panels of nb/2 steps as the real Pfaffian-only reduction does (panel_pf_kernel
// in ltlt_panel.hip): a persistent panel kernel with one row slot per lane,
// interchanges applied as relabellings, each new column rebuilt from the
// panel-start matrix plus the panel's pairs (complex skew GEMVs), one tagged
// record per workgroup and step for the pivot search, and the panel's pairs
// applied afterwards as one skew rank-nb update.
//
// The working matrix is kept as two real planes (real and imaginary parts, each
// in strict lower storage).  Then the complex update splits into two real skew
// rank-2k updates that share one operand: with P = [Lr | Li],
//   Re(L V^T - V L^T) = P Qr^T - Qr P^T,  Qr = [Vr | -Vi],
//   Im(L V^T - V L^T) = P Qi^T - Qi P^T,  Qi = [Vi |  Vr],
// i.e. the real trailing update (FP64 matrix cores, permuted source tiles) run
// once per plane with inner dimension 2 nb: four real products per complex one.
#include <stdlib.h>

#include <algorithm>

#include "panel_common.h"

namespace skf {

using namespace panel;

namespace {

struct cd {
  double re, im;
};

__device__ inline cd cmulz(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cd caddz(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cd csubz(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline cd cnegz(cd a) { return {-a.re, -a.im}; }
// a / b by Smith's method (scaled by the larger component of b)
__device__ inline cd cdivz(cd a, cd b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  const double r = b.re / b.im, d = b.re * r + b.im;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
// |z|^2 with both products rounded: the pivot key of the definition
__device__ inline double cnorm2z(cd z) {
#pragma clang fp contract(off)
  return z.re * z.re + z.im * z.im;
}
__device__ inline bool cfinite(cd z) { return isfinite(z.re) && isfinite(z.im); }
__device__ inline cd rldz(cd z, int lane) { return {rld(z.re, lane), rld(z.im, lane)}; }

struct CPanelParams {
  int64_t n;
  int64_t k0;         // first step of the panel
  int nsteps;         // steps (even k) of this panel
  int G, S;           // workgroups, slots per workgroup
  const double* sre;  // panel-start matrix, real plane (strict lower storage, ld)
  const double* sim;  // imaginary plane
  int64_t ld;
  double* P;          // n x 2 nsteps: [Lr | Li] (column c at c n)
  double* NP;         // -P
  double* Qre;        // [Vr | -Vi]
  double* Qim;        // [Vi | Vr]
  int32_t* pi;        // panel permutation (current index -> panel-start row)
  double* cnre;       // next panel's first column, real part
  double* cnim;       // imaginary part
  double* T;          // complex128 interleaved: T[k] at 2k, 2k+1
  int32_t* ipiv;
  uint64_t* rec;      // records, double-buffered by step parity
  uint64_t* mirror;   // per slot and step: (lr, li, vr, vi) as 8 tagged words
  uint64_t* zc;       // per workgroup and step parity: its candidate's value (4 tagged words)
  uint64_t* front;    // per step parity: owners of indices k+1, k+2 (8 words each)
  int* status;
  uint32_t tag_base;  // tag of step si is tag_base + si + 1
};

template <int NB>
struct CSmem {
  double2 L[NB / 2][64];  // l of each step, per slot (re, im)
  double2 V[NB / 2][64];  // v of each step, per slot
  double2 xl[NB / 2];     // the winner's l and v of the steps so far
  double2 xv[NB / 2];
  double2 yl[NB / 2];     // the row at index k+2: its l and v of the steps so far
  double2 yv[NB / 2];
};

__device__ inline double2 d2(cd z) { return make_double2(z.re, z.im); }
__device__ inline cd cz(double2 v) { return {v.x, v.y}; }

template <int NB, int NQ>
__global__ void __launch_bounds__(kPanelThreads) cpanel_kernel(CPanelParams P) {
  constexpr int NP = NB / 2;
  __shared__ CSmem<NB> sm;

  const int lane = threadIdx.x;
  const int g = blockIdx.x;
  const int64_t n = P.n, k0 = P.k0, ld = P.ld;
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
  uint64_t* const my_mirror = P.mirror + ((size_t)g * 64 + lane) * NP * 8;

  for (int q = 0; q < NP; ++q) {
    sm.L[q][lane] = make_double2(0.0, 0.0);
    sm.V[q][lane] = make_double2(0.0, 0.0);
  }
  if (lane < NP) {
    sm.xl[lane] = sm.xv[lane] = sm.yl[lane] = sm.yv[lane] = make_double2(0.0, 0.0);
  }

  int32_t psi = mine ? (int32_t)(rowbase + lane) : INT32_MAX;
  const int32_t hbm = mine ? (int32_t)(rowbase + lane) : 0;
  cd cur = {0.0, 0.0};
  if (mine) cur = {P.sre[rowbase + lane + k0 * ld], P.sim[rowbase + lane + k0 * ld]};
  asm volatile("" : "+v"(cur.re), "+v"(cur.im));  // landed here, not at the loop head
  int stop = 0;
  int done = 0;

  for (int si = 0; si < P.nsteps; ++si) {
    const int64_t k = k0 + 2 * si;
    const int64_t r = k + 1;
    const bool last = k + 2 > n - 1;  // k = n-2: pivot only
    const uint32_t tag = P.tag_base + (uint32_t)si + 1u;
    const uint32_t t16 = tag16(tag);
    uint64_t* const recs0 = P.rec + (size_t)(si & 1) * G * kRecCopies * kRecStride;
    uint64_t* const recs = recs0 + (size_t)(g % kRecCopies) * G * kRecStride;
    uint64_t* const zcs = P.zc + (size_t)(si & 1) * G * 4;
    uint64_t* const front = P.front + (size_t)(si & 1) * 16;  // entry e at 8e: ws, re hi, re lo, im hi, im lo

    // (A) local candidate: largest |z|^2 of this workgroup's rows at index >= k+1
    const bool act = mine && psi >= k + 1;
    const bool nonfin = __any(act && !cfinite(cur));
    const double key = act ? cnorm2z(cur) : 0.0;
    const int bs = wave_argbest(key, (uint32_t)psi, act);

    // (B) record (key, index, slot), the candidate's value, and by the owners of
    // indices k+1 and k+2 the front entries
    {
      const int owner = (bs >= 0) ? bs : 0;
      const double kv = rld(key, owner);
      const cd zv = rldz(cur, owner);
      const uint32_t meta = nonfin ? kFlagNonFinite
                                   : (bs < 0 ? kFlagNoCand : (rl32((uint32_t)psi, owner) | ((uint32_t)owner << 24)));
      const uint64_t kb = (uint64_t)__double_as_longlong(kv) & ~(1ull << 63);
      const uint64_t th = (uint64_t)t16 << 48;
      const uint64_t w0 = th | ((uint64_t)meta << 16) | (kb >> 47);
      const uint64_t w1 = th | (kb & kLow47);
      constexpr int kW = 2 * kRecCopies;
      if (lane < kW) st_word(recs0 + ((size_t)(lane >> 1) * G + g) * kRecStride + (lane & 1), (lane & 1) ? w1 : w0);
      if (lane >= kW && lane < kW + 4) {
        const int t = lane - kW;
        const uint32_t pay = (t == 0) ? hi32(zv.re) : (t == 1) ? lo32(zv.re) : (t == 2) ? hi32(zv.im) : lo32(zv.im);
        st_word(zcs + (size_t)g * 4 + t, mk(tag, pay));
      }
      const int64_t e = (int64_t)psi - (k + 1);
      if (mine && (e == 0 || (e == 1 && !last))) {
        uint64_t* fe = front + 8 * e;
        st_word(fe, mk(tag, ((uint32_t)g << 6) | (uint32_t)lane));
        st_word(fe + 1, mk(tag, hi32(cur.re)));
        st_word(fe + 2, mk(tag, lo32(cur.re)));
        st_word(fe + 3, mk(tag, hi32(cur.im)));
        st_word(fe + 4, mk(tag, lo32(cur.im)));
      }
    }

    // (C) records -> global pivot; front entries
    double gv = -1.0;
    uint32_t gp = kNoCand, gslot = 0;
    int gs = -1;
    bool bad = false, tout = false;
    uint64_t fw[2][5];
    {
      uint64_t w[NQ][2];
      const uint64_t* rp[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int rr = lane + 64 * q;
        rp[q] = recs + (size_t)(rr < G ? rr : 0) * kRecStride;
      }
      auto load_recs = [&]() {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          w[q][0] = ld_word(rp[q]);
          w[q][1] = ld_word(rp[q] + 1);
        }
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
          for (int t = 0; t < 5; ++t) fw[e][t] = ld_word(front + 8 * e + t);
      };
      load_recs();
      uint64_t t0 = 0;
      for (int it = 0;; ++it) {
        bool ok = true, ok1 = true;
#pragma unroll
        for (int t = 0; t < 5; ++t) {
          ok &= tag_of(fw[0][t]) == tag;
          ok1 &= tag_of(fw[1][t]) == tag;
        }
        ok &= last | ok1;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const bool need = lane + 64 * q < G;
          ok &= !need | ((tag16_of(w[q][0]) == t16) & (tag16_of(w[q][1]) == t16));
        }
        if (__all(ok)) break;
        poll_refresh(it);
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
      for (int q = 0; q < NQ; ++q) {
        landed(w[q][0]);
        landed(w[q][1]);
      }
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int t = 0; t < 5; ++t) landed(fw[e][t]);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int rr = lane + 64 * q;
        const uint32_t meta = (uint32_t)(w[q][0] >> 16);
        const bool use = rr < G && !tout;
        bad |= use && (meta & kFlagNonFinite);
        if (use && !(meta & (kFlagNonFinite | kFlagNoCand))) {
          const uint64_t kb = ((w[q][0] & 0xFFFFull) << 47) | (w[q][1] & kLow47);
          const double a = __longlong_as_double((long long)kb);
          const uint32_t ps = meta & 0xFFFFFFu;
          if (better(a, ps, gv, gp)) {
            gv = a;
            gp = ps;
            gs = rr;
            gslot = meta >> 24 & 63u;
          }
        }
      }
    }
    tout = __any(tout);
    bad = __any(bad);
    const int wl = wave_argbest(gv, gp, gs >= 0);
    stop = tout ? 4 : (bad ? 2 : (wl < 0 ? 4 : 0));
    if (stop) break;
    gp = rl32(gp, wl);
    gs = (int)rl32((uint32_t)gs, wl);
    const int wslot = (int)rl32(gslot, wl);
    const int64_t hx = k0 + 1 + (int64_t)gs * P.S + wslot;
    const int64_t pidx = gp;

    // the row at index k+2 after the interchange: the old row k+1 when p = k+2
    const bool yfrom0 = pidx == k + 2;
    const uint32_t fws = (uint32_t)(yfrom0 ? fw[0][0] : fw[1][0]);
    const int ygs = (int)(fws >> 6), yslot = (int)(fws & 63u);
    const cd ycur = yfrom0 ? cd{from32((uint32_t)fw[0][1], (uint32_t)fw[0][2]), from32((uint32_t)fw[0][3], (uint32_t)fw[0][4])}
                           : cd{from32((uint32_t)fw[1][1], (uint32_t)fw[1][2]), from32((uint32_t)fw[1][3], (uint32_t)fw[1][4])};
    const int64_t hy = k0 + 1 + (int64_t)ygs * P.S + yslot;

    // (D) relabel
    if (mine && pidx != r) {
      if (psi == (int32_t)r) psi = (int32_t)pidx;
      else if (psi == (int32_t)pidx) psi = (int32_t)r;
    }
    const bool below = mine && psi >= k + 2;

    // (F) the winner's value (alpha), gathers S(i, x), S(i, y), S(y, x) (valid
    // addresses everywhere; signs and masks afterwards) and the coefficient
    // rows of x and y: lane q fetches step q's (l, v) of both rows
    const bool lowx = (int64_t)hbm > hx, lowy = (int64_t)hbm > hy, lowyx = hy > hx;
    const int64_t ax_ = lowx ? (int64_t)hbm + hx * ld : hx + (int64_t)hbm * ld;
    const int64_t ay_ = lowy ? (int64_t)hbm + hy * ld : hy + (int64_t)hbm * ld;
    const int64_t axy_ = lowyx ? hy + hx * ld : hx + hy * ld;
    const cd grx = {P.sre[ax_], P.sim[ax_]};
    const cd gry = {P.sre[ay_], P.sim[ay_]};
    const cd gyx = {P.sre[axy_], P.sim[axy_]};
    cd alpha;
    {
      const bool has = lane < si;
      const uint64_t* wx = P.mirror + (((size_t)gs * 64 + wslot) * NP + (has ? lane : 0)) * 8;
      const uint64_t* wy = P.mirror + (((size_t)ygs * 64 + yslot) * NP + (has ? lane : 0)) * 8;
      const uint64_t* za = zcs + (size_t)gs * 4;
      const uint32_t tq = P.tag_base + (uint32_t)lane + 1u;  // pair q carries the tag of step q
      uint64_t cx[8], cy[8], z[4];
      auto load_all = [&]() {
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          cx[t] = ld_word(wx + t);
          cy[t] = ld_word(wy + t);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) z[t] = ld_word(za + t);
      };
      load_all();
      uint64_t t0 = 0;
      for (int it = 0;; ++it) {
        bool ok = true, okc = true;
#pragma unroll
        for (int t = 0; t < 4; ++t) ok &= tag_of(z[t]) == tag;
#pragma unroll
        for (int t = 0; t < 8; ++t) okc &= (tag_of(cx[t]) == tq) & (tag_of(cy[t]) == tq);
        ok &= !has | okc;
        if (__all(ok)) break;
        poll_refresh(it);
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
      for (int t = 0; t < 8; ++t) {
        landed(cx[t]);
        landed(cy[t]);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) landed(z[t]);
      if (__any(tout)) {
        stop = 4;
        break;
      }
      alpha = {from32((uint32_t)z[0], (uint32_t)z[1]), from32((uint32_t)z[2], (uint32_t)z[3])};
      if (has) {
        sm.xl[lane] = make_double2(from32((uint32_t)cx[0], (uint32_t)cx[1]), from32((uint32_t)cx[2], (uint32_t)cx[3]));
        sm.xv[lane] = make_double2(from32((uint32_t)cx[4], (uint32_t)cx[5]), from32((uint32_t)cx[6], (uint32_t)cx[7]));
        sm.yl[lane] = make_double2(from32((uint32_t)cy[0], (uint32_t)cy[1]), from32((uint32_t)cy[2], (uint32_t)cy[3]));
        sm.yv[lane] = make_double2(from32((uint32_t)cy[4], (uint32_t)cy[5]), from32((uint32_t)cy[6], (uint32_t)cy[7]));
      }
    }
    if (g == 0 && lane == 0) {
      P.ipiv[r] = (int32_t)pidx;
      P.T[2 * k] = alpha.re;
      P.T[2 * k + 1] = alpha.im;
    }
    if (last) break;
    const cd gx = below ? (lowx ? grx : cnegz(grx)) : cd{0.0, 0.0};
    const cd gy = (mine && psi >= k + 3) ? (lowy ? gry : cnegz(gry)) : cd{0.0, 0.0};
    const cd syx = lowyx ? gyx : cnegz(gyx);  // S(y, x); y != x

    // complex skew GEMVs over the steps so far; the y-x sum in the same order as
    // the owner of y forms its own, so v_y has the same bits everywhere
    cd ax = {0.0, 0.0}, ay = {0.0, 0.0}, axy = {0.0, 0.0};
    for (int q = 0; q < si; ++q) {
      const cd l = cz(sm.L[q][lane]), v = cz(sm.V[q][lane]);
      const cd xl = cz(sm.xl[q]), xv = cz(sm.xv[q]), yl = cz(sm.yl[q]), yv = cz(sm.yv[q]);
      ax = caddz(ax, csubz(cmulz(l, xv), cmulz(v, xl)));
      ay = caddz(ay, csubz(cmulz(l, yv), cmulz(v, yl)));
      axy = caddz(axy, csubz(cmulz(yl, xv), cmulz(yv, xl)));
    }
    const bool anz = alpha.re != 0.0 || alpha.im != 0.0;
    const cd li = (below && anz) ? cdivz(cur, alpha) : cd{0.0, 0.0};
    const cd vi = below ? caddz(gx, ax) : cd{0.0, 0.0};
    const cd ly = anz ? cdivz(ycur, alpha) : cd{0.0, 0.0};
    const cd vy = caddz(syx, axy);
    sm.L[si][lane] = d2(li);
    sm.V[si][lane] = d2(vi);
    cur = (mine && psi >= k + 3) ? caddz(caddz(gy, ay), csubz(cmulz(li, vy), cmulz(vi, ly))) : cd{0.0, 0.0};
    ++done;
    if (mine) {
      uint64_t* m = my_mirror + (size_t)si * 8;
      st_word(m + 0, mk(tag, hi32(li.re)));
      st_word(m + 1, mk(tag, lo32(li.re)));
      st_word(m + 2, mk(tag, hi32(li.im)));
      st_word(m + 3, mk(tag, lo32(li.im)));
      st_word(m + 4, mk(tag, hi32(vi.re)));
      st_word(m + 5, mk(tag, lo32(vi.re)));
      st_word(m + 6, mk(tag, hi32(vi.im)));
      st_word(m + 7, mk(tag, lo32(vi.im)));
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
  const bool z0 = psi == lo;  // row lo of the operands is zero: column lo gets no products
  for (int q = 0; q < done; ++q) {
    const double2 l = sm.L[q][lane], v = sm.V[q][lane];
    const int64_t a = psi + (int64_t)q * n, b = psi + (int64_t)(done + q) * n;
    const double lr = z0 ? 0.0 : l.x, lim = z0 ? 0.0 : l.y, vr = z0 ? 0.0 : v.x, vim = z0 ? 0.0 : v.y;
    P.P[a] = lr;
    P.P[b] = lim;
    P.NP[a] = -lr;
    P.NP[b] = -lim;
    P.Qre[a] = vr;
    P.Qre[b] = -vim;
    P.Qim[a] = vim;
    P.Qim[b] = vr;
  }
  P.pi[psi] = hbm;
  if (psi >= lo + 1) {
    P.cnre[psi] = cur.re;
    P.cnim[psi] = cur.im;
  }
}

// Real and imaginary planes (strict lower triangle) of the interleaved input.
__global__ void split_kernel(int64_t n, const double* __restrict__ A, int64_t lda, double* __restrict__ R,
                             double* __restrict__ I) {
  const int64_t j = blockIdx.y;
  for (int64_t i = j + 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double* z = A + 2 * (i + j * lda);
    R[i + j * n] = z[0];
    I[i + j * n] = z[1];
  }
}

// dinfo: status if set; n for odd n; else 1 + the first even k with T[k] = 0, or 0.
__global__ void cinfo_kernel(int64_t n, const double* __restrict__ T, const int* __restrict__ status,
                             int* __restrict__ dinfo) {
  const int64_t z = first_zero_even_pivot(n, T, true);
  if (threadIdx.x != 0) return;
  int v = *status;
  if (v == 0 && (n & 1)) v = (int)n;
  if (v == 0 && z != INT64_MAX) v = (int)(z + 1);
  *dinfo = v;
}

template <int NB, int NQ>
int launch_cpanel_t(const CPanelParams& p, hipStream_t s) {
  hipLaunchKernelGGL((cpanel_kernel<NB, NQ>), dim3(p.G), dim3(kPanelThreads), 0, s, p);
  SKF_CHECK_LAUNCH("complex panel");
  return 0;
}

int launch_cpanel(const CPanelParams& p, int nb, hipStream_t s) {
  const int nq = (p.G + 63) / 64;
  if (nb == 128) {
    if (nq <= 1) return launch_cpanel_t<128, 1>(p, s);
    if (nq <= 2) return launch_cpanel_t<128, 2>(p, s);
    if (nq <= 4) return launch_cpanel_t<128, 4>(p, s);
  } else if (nb == 64) {
    if (nq <= 1) return launch_cpanel_t<64, 1>(p, s);
    if (nq <= 2) return launch_cpanel_t<64, 2>(p, s);
    if (nq <= 4) return launch_cpanel_t<64, 4>(p, s);
    if (nq <= 8) return launch_cpanel_t<64, 8>(p, s);
  }
  return SKF_ENOTIMPL;
}

// ---------------------------------------------------------------------------
// Complex LTL^T panel: steps k = k0 .. k0 + nsteps - 1, every one of them (the
// real factorization's step with the complex pivot key).  Step k gives the pair
// (l, v): l = column k / alpha below row k+1, v = column k+1 after the
// interchange there; the update l v^T - v l^T touches only rows and columns
// >= k+2, so v is itself the next step's pivot column: a step gathers one
// column of the panel-start matrix, S(., x) for the winner x, and adds the GEMV
// over the panel's pairs so far (the winner's coefficients from its mirror).
// The panel leaves the pairs as the operands of the two real trailing updates
// (as the Pfaffian-only panel does), and its L columns (alpha at the pivot row,
// l below) in the slots' panel-end order.
// ---------------------------------------------------------------------------
template <int NB>
struct CLSmem {
  double2 L[NB][64];  // l of each step, per slot
  double2 V[NB][64];  // v of each step, per slot
  double2 xl[NB];     // the winner's l and v of the steps so far
  double2 xv[NB];
  double2 al[NB];     // alpha of each step
};

struct CLtltParams {
  CPanelParams c;
  double* Lre;  // n x nsteps: the panel's L columns, real plane (slot rows in panel-end order)
  double* Lim;  // imaginary plane
  int npairs;   // steps with a pair (k <= n-3)
};

template <int NB, int NQ>
__global__ void __launch_bounds__(kPanelThreads) cltlt_panel_kernel(CLtltParams Q) {
  const CPanelParams& P = Q.c;
  __shared__ CLSmem<NB> sm;

  const int lane = threadIdx.x;
  const int g = blockIdx.x;
  const int64_t n = P.n, k0 = P.k0, ld = P.ld;
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
  uint64_t* const my_mirror = P.mirror + ((size_t)g * 64 + lane) * NB * 8;
  for (int q = 0; q < NB; ++q) {
    sm.L[q][lane] = make_double2(0.0, 0.0);
    sm.V[q][lane] = make_double2(0.0, 0.0);
  }
  if (lane < NB) sm.xl[lane] = sm.xv[lane] = sm.al[lane] = make_double2(0.0, 0.0);

  int32_t psi = mine ? (int32_t)(rowbase + lane) : INT32_MAX;
  const int32_t hbm = mine ? (int32_t)(rowbase + lane) : 0;
  cd cur = {0.0, 0.0};
  if (mine) cur = {P.sre[rowbase + lane + k0 * ld], P.sim[rowbase + lane + k0 * ld]};
  asm volatile("" : "+v"(cur.re), "+v"(cur.im));  // landed here, not at the loop head
  int stop = 0;
  int done = 0;      // steps with a pair
  int recorded = 0;  // steps whose pivot is recorded

  for (int si = 0; si < P.nsteps; ++si) {
    const int64_t k = k0 + si;
    const int64_t r = k + 1;
    const bool last = si >= Q.npairs;  // k = n-2: pivot only
    const uint32_t tag = P.tag_base + (uint32_t)si + 1u;
    const uint32_t t16 = tag16(tag);
    uint64_t* const recs0 = P.rec + (size_t)(si & 1) * G * kRecCopies * kRecStride;
    uint64_t* const recs = recs0 + (size_t)(g % kRecCopies) * G * kRecStride;
    uint64_t* const zcs = P.zc + (size_t)(si & 1) * G * 4;

    // (A) local candidate: largest |z|^2 of this workgroup's rows at index >= k+1
    const bool act = mine && psi >= k + 1;
    const bool nonfin = __any(act && !cfinite(cur));
    const double key = act ? cnorm2z(cur) : 0.0;
    const int bs = wave_argbest(key, (uint32_t)psi, act);

    // (B) record (key, index, slot) and the candidate's value
    {
      const int owner = (bs >= 0) ? bs : 0;
      const double kv = rld(key, owner);
      const cd zv = rldz(cur, owner);
      const uint32_t meta = nonfin ? kFlagNonFinite
                                   : (bs < 0 ? kFlagNoCand : (rl32((uint32_t)psi, owner) | ((uint32_t)owner << 24)));
      const uint64_t kb = (uint64_t)__double_as_longlong(kv) & ~(1ull << 63);
      const uint64_t th = (uint64_t)t16 << 48;
      const uint64_t w0 = th | ((uint64_t)meta << 16) | (kb >> 47);
      const uint64_t w1 = th | (kb & kLow47);
      constexpr int kW = 2 * kRecCopies;
      if (lane < kW) st_word(recs0 + ((size_t)(lane >> 1) * G + g) * kRecStride + (lane & 1), (lane & 1) ? w1 : w0);
      if (lane >= kW && lane < kW + 4) {
        const int t = lane - kW;
        const uint32_t pay = (t == 0) ? hi32(zv.re) : (t == 1) ? lo32(zv.re) : (t == 2) ? hi32(zv.im) : lo32(zv.im);
        st_word(zcs + (size_t)g * 4 + t, mk(tag, pay));
      }
    }

    // (C) records -> global pivot
    double gv = -1.0;
    uint32_t gp = kNoCand, gslot = 0;
    int gs = -1;
    bool bad = false, tout = false;
    {
      uint64_t w[NQ][2];
      const uint64_t* rp[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int rr = lane + 64 * q;
        rp[q] = recs + (size_t)(rr < G ? rr : 0) * kRecStride;
      }
      auto load_recs = [&]() {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          w[q][0] = ld_word(rp[q]);
          w[q][1] = ld_word(rp[q] + 1);
        }
      };
      load_recs();
      uint64_t t0 = 0;
      for (int it = 0;; ++it) {
        bool ok = true;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const bool need = lane + 64 * q < G;
          ok &= !need | ((tag16_of(w[q][0]) == t16) & (tag16_of(w[q][1]) == t16));
        }
        if (__all(ok)) break;
        poll_refresh(it);
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
      for (int q = 0; q < NQ; ++q) {
        landed(w[q][0]);
        landed(w[q][1]);
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int rr = lane + 64 * q;
        const uint32_t meta = (uint32_t)(w[q][0] >> 16);
        const bool use = rr < G && !tout;
        bad |= use && (meta & kFlagNonFinite);
        if (use && !(meta & (kFlagNonFinite | kFlagNoCand))) {
          const uint64_t kb = ((w[q][0] & 0xFFFFull) << 47) | (w[q][1] & kLow47);
          const double a = __longlong_as_double((long long)kb);
          const uint32_t ps = meta & 0xFFFFFFu;
          if (better(a, ps, gv, gp)) {
            gv = a;
            gp = ps;
            gs = rr;
            gslot = meta >> 24 & 63u;
          }
        }
      }
    }
    tout = __any(tout);
    bad = __any(bad);
    const int wl = wave_argbest(gv, gp, gs >= 0);
    stop = tout ? 4 : (bad ? 2 : (wl < 0 ? 4 : 0));
    if (stop) break;
    gp = rl32(gp, wl);
    gs = (int)rl32((uint32_t)gs, wl);
    const int wslot = (int)rl32(gslot, wl);
    const int64_t hx = k0 + 1 + (int64_t)gs * P.S + wslot;
    const int64_t pidx = gp;

    // (D) relabel
    if (mine && pidx != r) {
      if (psi == (int32_t)r) psi = (int32_t)pidx;
      else if (psi == (int32_t)pidx) psi = (int32_t)r;
    }
    const bool below = mine && psi >= k + 2;

    // (F) the winner's value (alpha), the gather S(i, x) (valid addresses
    // everywhere; sign and mask afterwards) and the winner's coefficient rows:
    // lane q fetches step q's (l, v) of row x
    const bool lowx = (int64_t)hbm > hx;
    const int64_t ax_ = lowx ? (int64_t)hbm + hx * ld : hx + (int64_t)hbm * ld;
    const cd grx = {P.sre[ax_], P.sim[ax_]};
    cd alpha;
    {
      const bool has = lane < si;
      const uint64_t* wx = P.mirror + (((size_t)gs * 64 + wslot) * NB + (has ? lane : 0)) * 8;
      const uint64_t* za = zcs + (size_t)gs * 4;
      const uint32_t tq = P.tag_base + (uint32_t)lane + 1u;  // pair q carries the tag of step q
      uint64_t cx[8], z[4];
      auto load_all = [&]() {
#pragma unroll
        for (int t = 0; t < 8; ++t) cx[t] = ld_word(wx + t);
#pragma unroll
        for (int t = 0; t < 4; ++t) z[t] = ld_word(za + t);
      };
      load_all();
      uint64_t t0 = 0;
      for (int it = 0;; ++it) {
        bool ok = true, okc = true;
#pragma unroll
        for (int t = 0; t < 4; ++t) ok &= tag_of(z[t]) == tag;
#pragma unroll
        for (int t = 0; t < 8; ++t) okc &= tag_of(cx[t]) == tq;
        ok &= !has | okc;
        if (__all(ok)) break;
        poll_refresh(it);
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
      for (int t = 0; t < 8; ++t) landed(cx[t]);
#pragma unroll
      for (int t = 0; t < 4; ++t) landed(z[t]);
      if (__any(tout)) {
        stop = 4;
        break;
      }
      alpha = {from32((uint32_t)z[0], (uint32_t)z[1]), from32((uint32_t)z[2], (uint32_t)z[3])};
      if (has) {
        sm.xl[lane] = make_double2(from32((uint32_t)cx[0], (uint32_t)cx[1]), from32((uint32_t)cx[2], (uint32_t)cx[3]));
        sm.xv[lane] = make_double2(from32((uint32_t)cx[4], (uint32_t)cx[5]), from32((uint32_t)cx[6], (uint32_t)cx[7]));
      }
    }
    if (g == 0 && lane == 0) {
      P.ipiv[r] = (int32_t)pidx;
      P.T[2 * k] = alpha.re;
      P.T[2 * k + 1] = alpha.im;
    }
    if (lane == 0) sm.al[si] = d2(alpha);
    recorded = si + 1;
    if (last) break;
    const cd gx = below ? (lowx ? grx : cnegz(grx)) : cd{0.0, 0.0};

    // complex skew GEMV over the steps so far
    cd ax = {0.0, 0.0};
    for (int q = 0; q < si; ++q) {
      const cd l = cz(sm.L[q][lane]), v = cz(sm.V[q][lane]);
      ax = caddz(ax, csubz(cmulz(l, cz(sm.xv[q])), cmulz(v, cz(sm.xl[q]))));
    }
    const bool anz = alpha.re != 0.0 || alpha.im != 0.0;
    const cd li = (below && anz) ? cdivz(cur, alpha) : cd{0.0, 0.0};
    const cd vi = below ? caddz(gx, ax) : cd{0.0, 0.0};
    sm.L[si][lane] = d2(li);
    sm.V[si][lane] = d2(vi);
    cur = vi;  // the next pivot column (rows at index >= k+2)
    ++done;
    if (mine) {
      uint64_t* m = my_mirror + (size_t)si * 8;
      st_word(m + 0, mk(tag, hi32(li.re)));
      st_word(m + 1, mk(tag, lo32(li.re)));
      st_word(m + 2, mk(tag, hi32(li.im)));
      st_word(m + 3, mk(tag, lo32(li.im)));
      st_word(m + 4, mk(tag, hi32(vi.re)));
      st_word(m + 5, mk(tag, lo32(vi.re)));
      st_word(m + 6, mk(tag, hi32(vi.im)));
      st_word(m + 7, mk(tag, lo32(vi.im)));
    }
  }

  // ---- panel end ----
  if (stop) {
    if (lane == 0) atomicMin(P.status, (stop & 4) ? SKF_ETIMEOUT : SKF_ENONFINITE);
    if (mine) P.pi[psi] = hbm;
    return;
  }
  __syncthreads();  // sm.al written by lane 0
  if (!mine) return;
  const int64_t lo = k0 + done;
  const bool z0 = psi == lo;  // row lo of the operands is zero: column lo gets no products
  for (int q = 0; q < done; ++q) {
    const double2 l = sm.L[q][lane], v = sm.V[q][lane];
    const int64_t a = psi + (int64_t)q * n, b = psi + (int64_t)(done + q) * n;
    const double lr = z0 ? 0.0 : l.x, lim = z0 ? 0.0 : l.y, vr = z0 ? 0.0 : v.x, vim = z0 ? 0.0 : v.y;
    P.P[a] = lr;
    P.P[b] = lim;
    P.NP[a] = -lr;
    P.NP[b] = -lim;
    P.Qre[a] = vr;
    P.Qre[b] = -vim;
    P.Qim[a] = vim;
    P.Qim[b] = vr;
  }
  // L columns: alpha at the step's pivot row, l below it
  for (int q = 0; q < recorded; ++q) {
    const int64_t kq = k0 + q;
    const double2 x = ((int64_t)psi == kq + 1) ? sm.al[q] : sm.L[q][lane];
    Q.Lre[psi + (int64_t)q * n] = x.x;
    Q.Lim[psi + (int64_t)q * n] = x.y;
  }
  P.pi[psi] = hbm;
  if (psi >= lo + 1) {
    P.cnre[psi] = cur.re;
    P.cnim[psi] = cur.im;
  }
}

template <int NB, int NQ>
int launch_cltlt_t(const CLtltParams& p, hipStream_t s) {
  hipLaunchKernelGGL((cltlt_panel_kernel<NB, NQ>), dim3(p.c.G), dim3(kPanelThreads), 0, s, p);
  SKF_CHECK_LAUNCH("complex ltlt panel");
  return 0;
}

int launch_cltlt(const CLtltParams& p, int nb, hipStream_t s) {
  const int nq = (p.c.G + 63) / 64;
  if (nb == 64) {
    if (nq <= 1) return launch_cltlt_t<64, 1>(p, s);
    if (nq <= 2) return launch_cltlt_t<64, 2>(p, s);
    if (nq <= 4) return launch_cltlt_t<64, 4>(p, s);
  } else if (nb == 32) {
    if (nq <= 1) return launch_cltlt_t<32, 1>(p, s);
    if (nq <= 2) return launch_cltlt_t<32, 2>(p, s);
    if (nq <= 4) return launch_cltlt_t<32, 4>(p, s);
    if (nq <= 8) return launch_cltlt_t<32, 8>(p, s);
  } else if (nb == 16) {
    if (nq <= 2) return launch_cltlt_t<16, 2>(p, s);
    if (nq <= 8) return launch_cltlt_t<16, 8>(p, s);
    if (nq <= 16) return launch_cltlt_t<16, 16>(p, s);
  }
  return SKF_ENOTIMPL;
}

// W[i, k0+c] = L[i, c] (both planes) for the rows below the diagonal of column k0+c.
__global__ void park_L_kernel(int64_t n, int64_t k0, const double* __restrict__ Lre, const double* __restrict__ Lim,
                              double* __restrict__ Wre, double* __restrict__ Wim) {
  const int c = blockIdx.y;
  const int64_t col = k0 + c;
  for (int64_t i = col + 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    Wre[i + col * n] = Lre[i + (int64_t)c * n];
    Wim[i + col * n] = Lim[i + (int64_t)c * n];
  }
}

// A[i, c] (interleaved) = W[sigma_P(i), c] for i > c, P the panel of column c.
__global__ void final_L_c128_kernel(int64_t n, int nb, const double* __restrict__ Wre, const double* __restrict__ Wim,
                                    const int32_t* __restrict__ sigma, double* __restrict__ A, int64_t lda) {
  const int64_t c = blockIdx.y;
  const int32_t* sg = sigma + (c / nb) * n;
  for (int64_t i = c + 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t src = (int64_t)sg[i] + c * n;
    A[2 * (i + c * lda)] = Wre[src];
    A[2 * (i + c * lda) + 1] = Wim[src];
  }
}

// dinfo: status if set; else 1 + the first even k with T[k] = 0, or 0 (the
// real factorization's rule: odd n completes, Pf = 0 follows from n).
__global__ void cltlt_info_kernel(int64_t n, const double* __restrict__ T, const int* __restrict__ status,
                                  int* __restrict__ dinfo) {
  const int64_t z = first_zero_even_pivot(n, T, true);
  if (threadIdx.x != 0) return;
  int v = *status;
  if (v == 0 && z != INT64_MAX) v = (int)(z + 1);
  *dinfo = v;
}

constexpr int kCSlots = 64;

// Panel width for order n: 128 (132 KB of LDS per workgroup, one per CU) when
// its workgroups fit on the device, else 64 (two per CU), else 0.
// SKF_NB=64 selects the narrow panel wherever it fits.
int cplan_nb(int64_t n) {
  const int64_t g0 = std::max<int64_t>(1, (n - 1 + kCSlots - 1) / kCSlots);
  const int64_t cus = device_info().num_cus;
  const char* e = getenv("SKF_NB");
  const bool narrow = e && atoi(e) == 64;
  if (!narrow && g0 <= std::min<int64_t>(256, cus)) return 128;
  if (g0 <= std::min<int64_t>(512, 2 * cus)) return 64;
  return 0;
}

struct CBWork {
  double* re[2];
  double* im[2];
  double *P, *NP, *Qre, *Qim, *cnre, *cnim;
  int32_t* pi;
  uint64_t *rec, *mirror, *zc, *front;
  int* status;
  size_t bytes;
};

CBWork cb_carve(void* base, int64_t n, int nb) {
  CBWork w{};
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = align_up(off + b, 256);
    return base ? (void*)((char*)base + o) : nullptr;
  };
  const size_t m = (size_t)std::max<int64_t>(n, 1);
  const int64_t G = std::max<int64_t>(1, (n - 1 + kCSlots - 1) / kCSlots);
  for (int t = 0; t < 2; ++t) {
    w.re[t] = (double*)take(sizeof(double) * m * m);
    w.im[t] = (double*)take(sizeof(double) * m * m);
  }
  w.P = (double*)take(sizeof(double) * m * nb);
  w.NP = (double*)take(sizeof(double) * m * nb);
  w.Qre = (double*)take(sizeof(double) * m * nb);
  w.Qim = (double*)take(sizeof(double) * m * nb);
  w.cnre = (double*)take(sizeof(double) * m);
  w.cnim = (double*)take(sizeof(double) * m);
  w.pi = (int32_t*)take(sizeof(int32_t) * m);
  w.rec = (uint64_t*)take(sizeof(uint64_t) * 2 * (size_t)G * kRecCopies * kRecStride);
  w.mirror = (uint64_t*)take(sizeof(uint64_t) * (size_t)G * 64 * (nb / 2) * 8);
  w.zc = (uint64_t*)take(sizeof(uint64_t) * 2 * (size_t)G * 4);
  w.front = (uint64_t*)take(sizeof(uint64_t) * 32);
  w.status = (int*)take(256);
  w.bytes = off;
  return w;
}

// Panel width (steps per panel) of the complex LTL^T for order n: 64 (134 KB
// of LDS per workgroup, one per CU) when its workgroups fit on the device, else
// 32 (67 KB, two per CU), else 16 (34 KB, four per CU), else 0.  SKF_NB=32 or 16
// selects that narrower panel wherever it fits.
int clplan_nb(int64_t n) {
  const int64_t g0 = std::max<int64_t>(1, (n - 1 + kCSlots - 1) / kCSlots);
  const int64_t cus = device_info().num_cus;
  const char* e = getenv("SKF_NB");
  const int want = e ? atoi(e) : 0;
  if (want != 32 && want != 16 && g0 <= std::min<int64_t>(256, cus)) return 64;
  if (want != 16 && g0 <= std::min<int64_t>(512, 2 * cus)) return 32;
  if (g0 <= std::min<int64_t>(1024, 4 * cus)) return 16;
  return 0;
}

struct CLWork {
  double* re[2];
  double* im[2];
  double *P, *NP, *Qre, *Qim, *Lre, *Lim, *cnre, *cnim;
  int32_t *pis, *sigma;
  uint64_t *rec, *mirror, *zc;
  int* status;
  size_t bytes;
};

CLWork cl_carve(void* base, int64_t n, int nb) {
  CLWork w{};
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = align_up(off + b, 256);
    return base ? (void*)((char*)base + o) : nullptr;
  };
  const size_t m = (size_t)std::max<int64_t>(n, 1);
  const int64_t G = std::max<int64_t>(1, (n - 1 + kCSlots - 1) / kCSlots);
  const size_t np = (size_t)std::max<int64_t>(1, (n - 1 + nb - 1) / nb);
  for (int t = 0; t < 2; ++t) {
    w.re[t] = (double*)take(sizeof(double) * m * m);
    w.im[t] = (double*)take(sizeof(double) * m * m);
  }
  w.P = (double*)take(sizeof(double) * m * 2 * nb);
  w.NP = (double*)take(sizeof(double) * m * 2 * nb);
  w.Qre = (double*)take(sizeof(double) * m * 2 * nb);
  w.Qim = (double*)take(sizeof(double) * m * 2 * nb);
  w.Lre = (double*)take(sizeof(double) * m * nb);
  w.Lim = (double*)take(sizeof(double) * m * nb);
  w.cnre = (double*)take(sizeof(double) * m);
  w.cnim = (double*)take(sizeof(double) * m);
  w.pis = (int32_t*)take(sizeof(int32_t) * np * m);
  w.sigma = (int32_t*)take(sizeof(int32_t) * np * m);
  w.rec = (uint64_t*)take(sizeof(uint64_t) * 2 * (size_t)G * kRecCopies * kRecStride);
  w.mirror = (uint64_t*)take(sizeof(uint64_t) * (size_t)G * 64 * nb * 8);
  w.zc = (uint64_t*)take(sizeof(uint64_t) * 2 * (size_t)G * 4);
  w.status = (int*)take(256);
  w.bytes = off;
  return w;
}

}  // namespace

size_t pfonly_c128_blocked_workspace_bytes(int64_t n) {
  const int nb = cplan_nb(n);
  return nb ? cb_carve(nullptr, n, nb).bytes : 0;
}

int pfonly_c128_blocked_nb(int64_t n) { return cplan_nb(n); }

int run_pfonly_c128_blocked(int64_t n, const double* A, int64_t lda, int32_t* ipiv, double* T, void* work,
                            size_t lwork, int* dinfo, hipStream_t s) {
  const int nb = cplan_nb(n);
  if (!nb) return SKF_ENOTIMPL;
  CBWork w = cb_carve(work, n, nb);
  if (lwork < w.bytes) return SKF_EWORK;
  int rc;
  if ((rc = launch_fill_i32(w.status, 1, 0, s))) return rc;
  if (n > 0 && (rc = launch_iota_i32(ipiv, (size_t)n, s))) return rc;
  if (n > 1 && (rc = launch_fill_u64((uint64_t*)T, (size_t)(n - 1) * 2, 0, s))) return rc;
  if (n >= 2 && n % 2 == 0) {
    const int64_t G0 = std::max<int64_t>(1, (n - 1 + kCSlots - 1) / kCSlots);
    const unsigned gx = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(split_kernel, dim3(gx, (unsigned)n), dim3(256), 0, s, n, A, lda, w.re[0], w.im[0]);
    SKF_CHECK_LAUNCH("complex split");
    if ((rc = launch_fill_u64(w.rec, 2 * (size_t)G0 * kRecCopies * kRecStride, 0, s))) return rc;
    if ((rc = launch_fill_u64(w.mirror, (size_t)G0 * 64 * (nb / 2) * 8, 0, s))) return rc;
    if ((rc = launch_fill_u64(w.zc, 2 * (size_t)G0 * 4, 0, s))) return rc;
    if ((rc = launch_fill_u64(w.front, 32, 0, s))) return rc;
    const int64_t np = (n + nb - 1) / nb;
    for (int64_t Pn = 0; Pn < np; ++Pn) {
      const int64_t k0 = Pn * nb;
      const int nsteps = (int)std::min<int64_t>(nb / 2, (n - k0) / 2);
      if (nsteps <= 0) break;
      CPanelParams pp{};
      pp.n = n;
      pp.k0 = k0;
      pp.nsteps = nsteps;
      pp.S = kCSlots;
      pp.G = (int)std::max<int64_t>(1, (n - k0 - 1 + kCSlots - 1) / kCSlots);
      pp.sre = w.re[Pn % 2];
      pp.sim = w.im[Pn % 2];
      pp.ld = n;
      pp.P = w.P;
      pp.NP = w.NP;
      pp.Qre = w.Qre;
      pp.Qim = w.Qim;
      pp.pi = w.pi;
      pp.cnre = w.cnre;
      pp.cnim = w.cnim;
      pp.T = T;
      pp.ipiv = ipiv;
      pp.rec = w.rec;
      pp.mirror = w.mirror;
      pp.zc = w.zc;
      pp.front = w.front;
      pp.status = w.status;
      pp.tag_base = (uint32_t)k0;
      prof_begin(s);
      if ((rc = launch_cpanel(pp, nb, s))) return rc;
      prof_end(s, 0, 0.0);
      const int64_t lo = k0 + 2 * (int64_t)nsteps;
      if (lo < n) {  // the panel did not reach the last step: the trailing planes get the panel's pairs
        const int64_t m = n - lo;
        prof_begin(s);
        rc = launch_skr2k_perm(n, lo, 2 * nsteps, w.re[Pn % 2], n, w.re[(Pn + 1) % 2], n, w.pi, w.P, w.Qre, w.NP, n,
                               w.cnre, false, s);
        if (rc) return rc;
        rc = launch_skr2k_perm(n, lo, 2 * nsteps, w.im[Pn % 2], n, w.im[(Pn + 1) % 2], n, w.pi, w.P, w.Qim, w.NP, n,
                               w.cnim, false, s);
        if (rc) return rc;
        prof_end(s, 1, 2.0 * 2.0 * (2.0 * nsteps) * (double)m * (double)(m - 1) / 2.0);
      }
    }
  }
  if (dinfo) {
    hipLaunchKernelGGL(cinfo_kernel, dim3(1), dim3(256), 0, s, n, T, w.status, dinfo);
    SKF_CHECK_LAUNCH("complex info");
  }
  return 0;
}


size_t ltlt_c128_workspace_bytes(int64_t n) {
  const int nb = clplan_nb(n);
  return nb ? cl_carve(nullptr, n, nb).bytes : 0;
}

int ltlt_c128_nb(int64_t n) { return clplan_nb(n); }

// Blocked complex LTL^T: per panel of nb steps the panel kernel, the trailing
// update of both planes on the matrix cores (the panel's pairs as in the
// Pfaffian-only reduction), and the panel's L columns parked in plane set 1;
// at the end the later panels' interchanges are composed and L is gathered into
// A (interleaved) in final row order.
int run_ltlt_c128(int64_t n, double* A, int64_t lda, int32_t* ipiv, double* T, void* work, size_t lwork,
                  int* dinfo, hipStream_t s) {
  if (n == 0) return dinfo ? launch_fill_i32(dinfo, 1, 0, s) : 0;
  const int nb = clplan_nb(n);
  if (!nb) return SKF_ENOTIMPL;
  CLWork w = cl_carve(work, n, nb);
  if (lwork < w.bytes) return SKF_EWORK;
  int rc;
  if ((rc = launch_fill_i32(w.status, 1, 0, s))) return rc;
  if ((rc = launch_fill_i32(ipiv, 1, 0, s))) return rc;  // ipiv[0] = 0
  if (n >= 2) {
    if ((rc = launch_fill_u64((uint64_t*)T, (size_t)(n - 1) * 2, 0, s))) return rc;
    const int64_t G0 = std::max<int64_t>(1, (n - 1 + kCSlots - 1) / kCSlots);
    const unsigned gx = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(split_kernel, dim3(gx, (unsigned)n), dim3(256), 0, s, n, A, lda, w.re[0], w.im[0]);
    SKF_CHECK_LAUNCH("complex split");
    if ((rc = launch_fill_u64(w.rec, 2 * (size_t)G0 * kRecCopies * kRecStride, 0, s))) return rc;
    if ((rc = launch_fill_u64(w.mirror, (size_t)G0 * 64 * nb * 8, 0, s))) return rc;
    if ((rc = launch_fill_u64(w.zc, 2 * (size_t)G0 * 4, 0, s))) return rc;
    const int64_t np = (n - 1 + nb - 1) / nb;
    for (int64_t Pn = 0; Pn < np; ++Pn) {
      const int64_t k0 = Pn * nb;
      const int nsteps = (int)std::min<int64_t>(nb, n - 1 - k0);
      const int npairs = (int)std::max<int64_t>(0, std::min<int64_t>(nsteps, n - 2 - k0));
      CLtltParams q{};
      CPanelParams& pp = q.c;
      pp.n = n;
      pp.k0 = k0;
      pp.nsteps = nsteps;
      pp.S = kCSlots;
      pp.G = (int)std::max<int64_t>(1, (n - k0 - 1 + kCSlots - 1) / kCSlots);
      pp.sre = w.re[Pn % 2];
      pp.sim = w.im[Pn % 2];
      pp.ld = n;
      pp.P = w.P;
      pp.NP = w.NP;
      pp.Qre = w.Qre;
      pp.Qim = w.Qim;
      pp.pi = w.pis + Pn * n;
      pp.cnre = w.cnre;
      pp.cnim = w.cnim;
      pp.T = T;
      pp.ipiv = ipiv;
      pp.rec = w.rec;
      pp.mirror = w.mirror;
      pp.zc = w.zc;
      pp.front = nullptr;
      pp.status = w.status;
      pp.tag_base = (uint32_t)k0;
      q.Lre = w.Lre;
      q.Lim = w.Lim;
      q.npairs = npairs;
      prof_begin(s);
      if ((rc = launch_cltlt(q, nb, s))) return rc;
      prof_end(s, 0, 0.0);
      const int64_t lo = k0 + npairs;
      if (npairs == nsteps) {  // not the last panel: the trailing planes get the panel's pairs
        const int64_t m = n - lo;
        prof_begin(s);
        rc = launch_skr2k_perm(n, lo, 2 * npairs, w.re[Pn % 2], n, w.re[(Pn + 1) % 2], n, pp.pi, w.P, w.Qre, w.NP,
                               n, w.cnre, false, s);
        if (rc) return rc;
        rc = launch_skr2k_perm(n, lo, 2 * npairs, w.im[Pn % 2], n, w.im[(Pn + 1) % 2], n, pp.pi, w.P, w.Qim, w.NP,
                               n, w.cnim, false, s);
        if (rc) return rc;
        prof_end(s, 1, 2.0 * 2.0 * (2.0 * npairs) * (double)m * (double)(m - 1) / 2.0);
      }
      hipLaunchKernelGGL(park_L_kernel, dim3(gx, (unsigned)nsteps), dim3(256), 0, s, n, k0, w.Lre, w.Lim, w.re[1],
                         w.im[1]);
      SKF_CHECK_LAUNCH("complex park L");
    }
    if ((rc = launch_compose_sigma(n, (int)np, w.pis, w.sigma, s))) return rc;
    hipLaunchKernelGGL(final_L_c128_kernel, dim3(gx, (unsigned)(n - 1)), dim3(256), 0, s, n, nb, w.re[1], w.im[1],
                       w.sigma, A, lda);
    SKF_CHECK_LAUNCH("complex final L");
  }
  if (dinfo) {
    hipLaunchKernelGGL(cltlt_info_kernel, dim3(1), dim3(256), 0, s, n, T, w.status, dinfo);
    SKF_CHECK_LAUNCH("complex ltlt info");
  }
  return 0;
}

}  // namespace skf
