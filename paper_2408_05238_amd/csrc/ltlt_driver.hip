// Host driver of the blocked, right-looking skew LTL^T.
//
// For each panel P of nb paired elimination steps (k0 = P*nb):
//   1. panel kernel on the panel-start matrix buf[P%2] (persistent grid, one
//      pivot search per step on the device; emits L, l', w, T, ipiv, the
//      panel's permutation and the next panel's first column);
//   2. trailing update buf[P%2] -> buf[(P+1)%2] through that permutation
//      (skew rank-nb on the matrix cores, FP64 or FP32);
//   3. the panel's L columns parked in the workspace copy W.
// buf[0] is the caller's A, buf[1] the workspace W.  At the end the later
// panels' permutations are composed and L is copied into A in final row order.
// The host only enqueues; nothing waits on the device inside the loop.
#include <algorithm>
#include <stdlib.h>

#include "skf_internal.h"

namespace skf {

// The panel kernel is one wave per workgroup with 64 row slots; LDS holds the
// (nb/2) x 64 pair vectors per workgroup and, in the faster form, the
// first-step multipliers (97 KB at nb = 128, 49 KB at 64, 24 KB at 32, 12 KB at
// 16: one, three, six, six per CU); the other form keeps the multipliers in
// global scratch (131 KB at 256, 66 KB at 128, 33 KB at 64: one, two, four per
// CU), and a launch takes it only when its grid needs that residency (the
// occupancy query and the cap of six per CU also apply).  Every workgroup of a
// panel launch must be resident together, so the narrower widths carry larger
// orders: up to 256, 512, 1024 and 1536 workgroups of 64 rows on 256 CUs.
static constexpr int kMaxPanelG = 2048;

static int slots() { return panel_slots(); }

static int64_t max_panel_groups(int nb, bool pf = false) {
  return std::min<int64_t>(kMaxPanelG, (int64_t)panel_wgs_per_cu(nb, pf) * device_info().num_cus);
}

// Panel width for order n: SKF_NB override, else the tuning table's entry
// (256 only from there: its one-per-CU panel is not always the faster), else the
// widest of 128, 64, 32, 16 whose workgroups fit on the device; an infeasible
// choice falls through to the next rule.  -1: no width fits.
static int plan_nb(int64_t n, int param) {
  const int64_t g0 = std::max<int64_t>(1, (n - 1 + slots() - 1) / slots());
  const bool pf = param == SKF_TUNE_PFONLY_NB;
  auto fits = [&](int nb) {
    return (nb == 256 || nb == 128 || nb == 64 || nb == 32 || nb == 16) && g0 <= max_panel_groups(nb, pf);
  };
  if (const char* e = getenv("SKF_NB")) {
    const int want = atoi(e);
    if (fits(want)) return want;
  }
  const int t = tune_lookup(param, n);
  if (fits(t)) return t;
  for (int nb : {128, 64, 32, 16})
    if (fits(nb)) return nb;
  return -1;
}

int ltlt_plan_nb(int64_t n) { return plan_nb(n, SKF_TUNE_LTLT_NB); }
int pfonly_plan_nb(int64_t n) { return plan_nb(n, SKF_TUNE_PFONLY_NB); }

int ltlt_panel_grid(int64_t m, int nb, int* G, int* S, bool pf) {
  const int64_t g = std::max<int64_t>(1, (m + slots() - 1) / slots());
  if (g > max_panel_groups(nb, pf)) return SKF_ENOTIMPL;
  *G = (int)g;
  *S = slots();
  return 0;
}

static int64_t npanels_of(int64_t n, int nb) { return n >= 2 ? (n - 1 + nb - 1) / nb : 0; }

static size_t carve(LtltWork* w, char* base, int64_t n, int nb) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes, 256);
    return base ? (void*)(base + o) : nullptr;
  };
  const int64_t np = npanels_of(n, nb);
  const int gmax = (int)std::max<int64_t>(1, (n - 1 + slots() - 1) / slots());  // first (largest) panel
  w->W = (double*)take(sizeof(double) * (size_t)n * n);
  w->Lbuf = (double*)take(sizeof(double) * (size_t)n * nb);
  w->Lp = (double*)take(sizeof(double) * (size_t)n * (nb / 2));
  w->Wp = (double*)take(sizeof(double) * (size_t)n * (nb / 2));
  w->NLp = (double*)take(sizeof(double) * (size_t)n * (nb / 2));
  w->cnext = (double*)take(sizeof(double) * (size_t)n);
  w->pis = (int32_t*)take(sizeof(int32_t) * (size_t)std::max<int64_t>(np, 1) * n);
  w->sigma = (int32_t*)take(sizeof(int32_t) * (size_t)std::max<int64_t>(np, 1) * n);
  w->rec = (uint64_t*)take(sizeof(uint64_t) * panel_record_words(gmax));
  w->mirror = (uint64_t*)take(sizeof(uint64_t) * panel_mirror_words(gmax, nb));
  w->front = (uint64_t*)take(sizeof(uint64_t) * 16);
  w->Lscr = (double*)take(sizeof(double) * panel_scratch_doubles(gmax, nb));
  w->status = (int*)take(256);
  w->bytes = off;
  return off;
}

// Workspace for order n: the larger of the two panel widths' layouts (when
// feasible), so a workspace sized once stays valid whichever width the tuning
// table or the environment selects later.
size_t ltlt_workspace_bytes(int64_t n, int prec) {
  (void)prec;
  if (ltlt_plan_nb(n) < 0 && pfonly_plan_nb(n) < 0) return 0;
  const int64_t g0 = std::max<int64_t>(1, (n - 1 + slots() - 1) / slots());
  size_t b = 0;
  for (int nb : {16, 32, 64, 128, 256}) {
    if (g0 > max_panel_groups(nb, false) && g0 > max_panel_groups(nb, true)) continue;
    LtltWork w;
    b = std::max(b, carve(&w, nullptr, n, nb));
  }
  return b;
}

static LtltWork carve_nb(void* work, int64_t n, int nb) {
  LtltWork w{};
  carve(&w, (char*)work, n, nb);
  return w;
}

LtltWork ltlt_carve(void* work, int64_t n, int prec) {
  (void)prec;
  return carve_nb(work, n, ltlt_plan_nb(n));
}

int run_ltlt(int64_t n, double* A, int64_t lda, int32_t* ipiv, double* T, int prec, void* work,
             size_t lwork, int* dinfo_dev, hipStream_t s) {
  if (n == 0) return dinfo_dev ? launch_fill_i32(dinfo_dev, 1, 0, s) : 0;
  const int nb = ltlt_plan_nb(n);
  if (nb < 0) return SKF_ENOTIMPL;
  LtltWork w = ltlt_carve(work, n, prec);
  if (lwork < w.bytes) return SKF_EWORK;
  const int gmax = (int)std::max<int64_t>(1, (n - 1 + slots() - 1) / slots());
  int rc;
  if ((rc = launch_fill_i32(w.status, 1, 0, s))) return rc;
  if ((rc = launch_fill_i32(ipiv, 1, 0, s))) return rc;  // ipiv[0] = 0
  if (n == 1) {
    if (dinfo_dev) return launch_ltlt_info(n, T, w.status, dinfo_dev, s);
    return 0;
  }
  if ((rc = launch_fill_u64(w.rec, panel_record_words(gmax), 0, s))) return rc;
  if ((rc = launch_fill_u64(w.mirror, panel_mirror_words(gmax, nb), 0, s))) return rc;

  const int64_t np = npanels_of(n, nb);
  double* buf[2] = {A, w.W};
  const int64_t ldb[2] = {lda, n};
  for (int64_t P = 0; P < np; ++P) {
    const int64_t k0 = P * nb;
    const int nsteps = (int)std::min<int64_t>(nb, n - 1 - k0);
    const int64_t m = n - k0 - 1;
    PanelParams pp{};
    pp.n = n;
    pp.k0 = k0;
    pp.nsteps = nsteps;
    pp.nb = nb;
    if ((rc = ltlt_panel_grid(m, nb, &pp.G, &pp.S, false))) return rc;
    pp.src = buf[P % 2];
    pp.ld = ldb[P % 2];
    pp.Lbuf = w.Lbuf;
    pp.Lp = w.Lp;
    pp.Wp = w.Wp;
    pp.NLp = w.NLp;
    pp.pi = w.pis + P * n;
    pp.cnext = w.cnext;
    pp.T = T;
    pp.ipiv = ipiv;
    pp.rec = w.rec;
    pp.mirror = w.mirror;
    pp.Lscr = w.Lscr;
    pp.status = w.status;
    pp.tag_base = (uint32_t)k0;
    prof_begin(s);
    if ((rc = launch_panel(pp, s))) return rc;
    prof_end(s, 0, 0.0);
    const int64_t lo = k0 + nsteps;
    if (n - lo >= 2 && nsteps % 2 == 0) {
      prof_begin(s);
      rc = launch_skr2k_perm(n, lo, nsteps / 2, buf[P % 2], ldb[P % 2], buf[(P + 1) % 2],
                             ldb[(P + 1) % 2], pp.pi, w.Lp, w.Wp, w.NLp, n, w.cnext,
                             prec == SKF_PREC_F32_TRAILING, s);
      if (rc) return rc;
      const double mt = (double)(n - lo);
      prof_end(s, 1, 2.0 * (double)nsteps * mt * (mt - 1.0) / 2.0);
    }
    if ((rc = launch_copy_panel_L(n, k0, nsteps, w.Lbuf, w.W, n, s))) return rc;
  }
  if ((rc = launch_compose_sigma(n, (int)np, w.pis, w.sigma, s))) return rc;
  if ((rc = launch_final_L(n, nb, (int)np, w.W, n, w.sigma, A, lda, s))) return rc;
  if (dinfo_dev) return launch_ltlt_info(n, T, w.status, dinfo_dev, s);
  return 0;
}

// Pfaffian-only reduction: the same panel/update loop with steps at even k only.
// Panel P covers k0 = P*nb .. k0+nb-1 with nb/2 steps; each step's pair (l, v)
// enters the same skew rank-nb trailing update.  No L is kept, so there is no
// write-back or final permutation of L; ipiv starts as the identity (the even
// entries stay so) and T as zero (the odd entries stay so).
int run_pfonly(int64_t n, double* A, int64_t lda, int32_t* ipiv, double* T, int prec, void* work,
               size_t lwork, int* dinfo_dev, hipStream_t s) {
  if (n == 0) return dinfo_dev ? launch_fill_i32(dinfo_dev, 1, 0, s) : 0;
  const int nb = pfonly_plan_nb(n);
  if (nb < 0) return SKF_ENOTIMPL;
  LtltWork w = carve_nb(work, n, nb);
  if (lwork < w.bytes) return SKF_EWORK;
  int rc;
  if ((rc = launch_iota_i32(ipiv, (size_t)n, s))) return rc;
  if (n > 1 && (rc = launch_fill_u64((uint64_t*)T, (size_t)(n - 1), 0, s))) return rc;
  if (n % 2 == 1) return dinfo_dev ? launch_fill_i32(dinfo_dev, 1, (int32_t)n, s) : 0;
  const int gmax = (int)std::max<int64_t>(1, (n - 1 + slots() - 1) / slots());
  if ((rc = launch_fill_i32(w.status, 1, 0, s))) return rc;
  if ((rc = launch_fill_u64(w.rec, panel_record_words(gmax), 0, s))) return rc;
  if ((rc = launch_fill_u64(w.mirror, panel_mirror_words(gmax, nb), 0, s))) return rc;
  if ((rc = launch_fill_u64(w.front, 16, 0, s))) return rc;

  const int64_t np = (n + nb - 1) / nb;
  double* buf[2] = {A, w.W};
  const int64_t ldb[2] = {lda, n};
  for (int64_t P = 0; P < np; ++P) {
    const int64_t k0 = P * nb;
    const int nsteps = (int)std::min<int64_t>(nb / 2, (n - k0) / 2);
    PanelParams pp{};
    pp.n = n;
    pp.k0 = k0;
    pp.nsteps = nsteps;
    pp.nb = nb;
    if ((rc = ltlt_panel_grid(n - k0 - 1, nb, &pp.G, &pp.S, true))) return rc;
    pp.src = buf[P % 2];
    pp.ld = ldb[P % 2];
    pp.Lp = w.Lp;
    pp.Wp = w.Wp;
    pp.NLp = w.NLp;
    pp.pi = w.pis;
    pp.cnext = w.cnext;
    pp.T = T;
    pp.ipiv = ipiv;
    pp.rec = w.rec;
    pp.mirror = w.mirror;
    pp.front = w.front;
    pp.status = w.status;
    pp.tag_base = (uint32_t)k0;
    prof_begin(s);
    if ((rc = launch_panel_pf(pp, s))) return rc;
    prof_end(s, 0, 0.0);
    const int64_t lo = k0 + 2 * (int64_t)nsteps;
    if (lo < n) {  // the panel did not reach the last step (k = n-2): n - lo >= 2 and even
      prof_begin(s);
      rc = launch_skr2k_perm(n, lo, nsteps, buf[P % 2], ldb[P % 2], buf[(P + 1) % 2], ldb[(P + 1) % 2],
                             pp.pi, w.Lp, w.Wp, w.NLp, n, w.cnext, prec == SKF_PREC_F32_TRAILING, s);
      if (rc) return rc;
      const double mt = (double)(n - lo);
      prof_end(s, 1, 2.0 * (double)nsteps * mt * (mt - 1.0));
    }
  }
  if (dinfo_dev) return launch_ltlt_info(n, T, w.status, dinfo_dev, s);
  return 0;
}

}  // namespace skf
