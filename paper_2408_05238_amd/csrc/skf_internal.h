// Internal declarations shared by the HIP translation units of libskf.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "skf.h"

namespace skf {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// Records the last HIP error for skf_last_error(); returns SKF_EDEVICE if err != success.
int note_error(hipError_t err, const char* where);

#define SKF_CHECK_LAUNCH(where)                              \
  do {                                                       \
    hipError_t e_ = hipGetLastError();                       \
    if (e_ != hipSuccess) return ::skf::note_error(e_, where); \
  } while (0)

#define SKF_CHECK(call, where)                                  \
  do {                                                          \
    hipError_t e_ = (call);                                     \
    if (e_ != hipSuccess) return ::skf::note_error(e_, where);  \
  } while (0)

struct DeviceInfo {
  int device;
  int num_cus;
  size_t lds_per_block;
};
// Properties of the current device (cached per device).
const DeviceInfo& device_info();

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Cross-workgroup words are polled with relaxed device-scope loads.  Those are
// not bound to observe a store from another XCD within any time: a reader's
// cached copy of the line can keep answering (measured: with a fourth panel
// workgroup on some CUs, a record stayed invisible to a third of the readers for
// the full two-second wait bound).  A device-scope acquire fence, which
// invalidates the reader's non-coherent cache lines, ends that.  With up to four
// polling workgroups per CU one fence every eighth round was enough (measured up
// to 1094 panel workgroups) and the common case, where the word lands within a
// few rounds, pays nothing; with six per CU stale lines outlived that cadence, so
// the widest grids (kEveryRound) fence before every reload.
template <bool kEveryRound = false>
__device__ inline void poll_refresh(int it) {
  if (kEveryRound || (it & 7) == 7) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// First even k (k + 1 < n) with T[k] == 0 -- complex interleaved T when cplx --
// found by the whole workgroup (blockDim.x a multiple of 64, at most 1024);
// INT64_MAX when there is none.  Every thread gets the result.
__device__ inline int64_t first_zero_even_pivot(int64_t n, const double* __restrict__ T, bool cplx) {
  __shared__ int64_t red[16];
  int64_t b = INT64_MAX;
  for (int64_t k = 2 * (int64_t)threadIdx.x; k + 1 < n; k += 2 * (int64_t)blockDim.x) {
    const bool z = cplx ? (T[2 * k] == 0.0 && T[2 * k + 1] == 0.0) : (T[k] == 0.0);
    if (z) {
      b = k;
      break;
    }
  }
  for (int s = 32; s >= 1; s >>= 1) {
    const int64_t o = __shfl_xor(b, s);
    b = o < b ? o : b;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
  __syncthreads();
  int64_t r = INT64_MAX;
  for (unsigned w = 0; w < (blockDim.x + 63) / 64; ++w) r = red[w] < r ? red[w] : r;
  __syncthreads();
  return r;
}

// Tuning table (tune.hip)
int tune_lookup(int param, int64_t n);
int tune_set(int param, int64_t lo, int64_t hi, int value);
void tune_clear();
int pfonly_plan_nb(int64_t n);
int skr2k_band(int64_t m);

// Solve with the factors (solve.hip): workspace bytes, and the solve in place over B.
size_t solve_workspace_bytes(int64_t n, int64_t nrhs);
int run_solve(int64_t n, int64_t nrhs, const double* LT, int64_t lda, const int32_t* ipiv, const double* T,
              double* B, int64_t ldb, void* work, size_t lwork, int* dinfo, hipStream_t s);
// perm[j] = the original row at position j after the interchanges ipiv (solve.hip).
int launch_solve_perm(int64_t n, const int32_t* ipiv, int32_t* perm, hipStream_t s);
// Solve with complex factors (csolve.hip).
size_t solve_c128_workspace_bytes(int64_t n, int64_t nrhs);
int run_solve_c128(int64_t n, int64_t nrhs, const double* LT, int64_t lda, const int32_t* ipiv, const double* T,
                   double* B, int64_t ldb, void* work, size_t lwork, int* dinfo, hipStream_t s);
// Batched solves in one launch (solve_batched.hip); orders above 1024 fall back
// to run_solve per matrix.
size_t solve_batched_workspace_bytes(int64_t batch, const int64_t* n_host, const int64_t* nrhs_host);
int run_solve_batched(int64_t batch, const int64_t* n_host, const double* const* LT, const int64_t* lda_host,
                      const int32_t* const* ipiv, const double* const* T, const int64_t* nrhs_host,
                      double* const* B, const int64_t* ldb_host, int* info, void* work, size_t lwork,
                      hipStream_t s);

// Allocation-free solve (solve.hip): fixed device scratch for n <= kSolveNoAllocMaxN.
constexpr int64_t kSolveNoAllocMaxN = SKF_SOLVE_NOALLOC_MAX_N;
size_t solve_noalloc_scratch_bytes();
int run_solve_noalloc(int64_t n, int64_t nrhs, const double* LT, int64_t lda, const int32_t* ipiv,
                      const double* T, double* B, int64_t ldb, int* dinfo, hipStream_t s);

// ---------------------------------------------------------------------------
// skr2k (trailing update) launchers
// ---------------------------------------------------------------------------

// Plain in-place update of the strict lower triangle of C (n x n):
//   C := beta C + alpha (X Y^T - Y X^T), X, Y: n x k.
int launch_skr2k_f64(int64_t n, int64_t k, double alpha, const double* X, int64_t ldx,
                     const double* Y, int64_t ldy, double beta, double* C, int64_t ldc,
                     hipStream_t s);
int launch_skr2k_f32(int64_t n, int64_t k, double alpha, const double* X, int64_t ldx,
                     const double* Y, int64_t ldy, double beta, double* C, int64_t ldc,
                     hipStream_t s);

// Trailing update of the blocked factorization, out of place and through the
// panel's row/column permutation pi (current index -> row index in src):
//   for lo <= j < i < n:
//     dst[i,j] = (j == lo) ? cnext[i]
//              : S(pi[i], pi[j]) + sum_q (Lp[i,q] Wp[j,q] - Wp[i,q] Lp[j,q]),
//   where S(a,b) = src[a,b] if a > b else -src[b,a] (strict lower storage).
// Lp, Wp: n x npairs (ld = ldp, rows indexed by the current index); their row
// lo must be zero (column lo then receives no products and equals cnext).
// NLp: -Lp with the same layout, or null; when given (and npairs is a multiple
// of 8) the products need no sign changes in registers.
int launch_skr2k_perm(int64_t n, int64_t lo, int64_t npairs, const double* src, int64_t ld_src,
                      double* dst, int64_t ld_dst, const int32_t* pi, const double* Lp,
                      const double* Wp, const double* NLp, int64_t ldp, const double* cnext, bool f32,
                      hipStream_t s);

// ---------------------------------------------------------------------------
// Blocked factorization pieces
// ---------------------------------------------------------------------------
struct PanelParams {
  int64_t n;
  int64_t k0;        // first step of the panel
  int nsteps;        // elimination steps in this panel (<= nb)
  int nb;            // panel width (even)
  int G;             // workgroups of the persistent panel kernel
  int S;             // rows (slots) per workgroup
  const double* src; // current trailing matrix (strict lower storage)
  int64_t ld;
  double* Lbuf;      // n x nb: L columns of the panel, current order at panel end
  double* Lp;        // n x nb/2: l' of each pair
  double* Wp;        // n x nb/2: w of each pair
  double* NLp;       // n x nb/2: -l' of each pair
  int32_t* pi;       // n: panel permutation (current index -> src row)
  double* cnext;     // n: first column of the next panel
  double* T;         // global T output
  int32_t* ipiv;     // global ipiv output
  uint64_t* rec;     // sync records, double-buffered by step parity
  uint64_t* mirror;  // per-workgroup tagged copy of each slot's pair coefficients
  uint64_t* front;   // Pfaffian-only panel: owners of indices k+1, k+2 (16 words)
  double* Lscr;      // (nb/2) x G x slots: first-step multipliers, slot-indexed
  int* status;       // device status word (0 ok)
  uint32_t tag_base; // tag of step k is tag_base + (k - k0) + 1
};

int launch_panel(const PanelParams& p, hipStream_t s);
int launch_panel_pf(const PanelParams& p, hipStream_t s);
int panel_slots();
int panel_wgs_per_cu(int nb, bool pf);
int panel_wgs_per_cu_form(int nb, bool le);  // the full panel with its multipliers in LDS (le) or scratch
size_t panel_record_words(int G);
size_t panel_mirror_words(int G, int nb);
size_t panel_scratch_doubles(int G, int nb);

// Workspace layout of the blocked path.
struct LtltWork {
  double* W;       // n x n ping-pong copy (ld n)
  double* Lbuf;    // n x nb
  double* Lp;      // n x nb/2
  double* Wp;      // n x nb/2
  double* NLp;     // n x nb/2
  double* cnext;   // n
  int32_t* pis;    // npanels x n: per-panel permutations
  int32_t* sigma;  // npanels x n: composed later permutations
  uint64_t* rec;   // sync records
  uint64_t* mirror;  // panel coefficient mirrors
  uint64_t* front;   // Pfaffian-only panel exchange words (16)
  double* Lscr;    // panel multiplier scratch
  int* status;     // 1 int (+ padding)
  size_t bytes;
};

int ltlt_plan_nb(int64_t n);
int ltlt_panel_grid(int64_t m, int nb, int* G, int* S, bool pf);
size_t ltlt_workspace_bytes(int64_t n, int prec);
LtltWork ltlt_carve(void* work, int64_t n, int prec);

int run_ltlt(int64_t n, double* A, int64_t lda, int32_t* ipiv, double* T, int prec, void* work,
             size_t lwork, int* dinfo_dev, hipStream_t s);
// Pfaffian-only reduction (interchanges and the even-step pivots), same workspace.
int run_pfonly(int64_t n, double* A, int64_t lda, int32_t* ipiv, double* T, int prec, void* work,
               size_t lwork, int* dinfo_dev, hipStream_t s);

// Pfaffian ratio of a low-rank skew update with resident factors (ratio.hip).
int pf_ratio_max_rank();
size_t pf_ratio_workspace_bytes(int64_t n, int r);
int run_pf_ratio(int64_t n, int r, const double* LT, int64_t lda, const int32_t* ipiv, const double* T,
                 const double* U, int64_t ldu, const double* V, int64_t ldv, double* logabs, int* sign,
                 void* work, size_t lwork, int* dinfo, hipStream_t s);

// Complex (complex128) Pfaffian-only reduction (complex.hip); A and T interleaved re, im.
size_t pfonly_c128_workspace_bytes(int64_t n);
int run_pfonly_c128(int64_t n, const double* A, int64_t lda, int32_t* ipiv, double* T, void* work, size_t lwork,
                    int* dinfo, hipStream_t s);
int launch_logpf_c128(int64_t n, const int32_t* ipiv, const double* T, double* logabs, double* phase,
                      hipStream_t s);
// Blocked form (complex_blocked.hip): panel width for n (0 when its panel does not fit the device).
int pfonly_c128_blocked_nb(int64_t n);
// Complex LTL^T (complex_blocked.hip): steps per panel (0: order too large), workspace, run.
int ltlt_c128_nb(int64_t n);
size_t ltlt_c128_workspace_bytes(int64_t n);
int run_ltlt_c128(int64_t n, double* A, int64_t lda, int32_t* ipiv, double* T, void* work, size_t lwork,
                  int* dinfo, hipStream_t s);
size_t pfonly_c128_blocked_workspace_bytes(int64_t n);
int run_pfonly_c128_blocked(int64_t n, const double* A, int64_t lda, int32_t* ipiv, double* T, void* work,
                            size_t lwork, int* dinfo, hipStream_t s);

// Kernel timing hooks (api.hip): no-ops unless skf_profile_enable(1).
void prof_begin(hipStream_t s);
void prof_end(hipStream_t s, int cls, double flops);

// Helpers (ltlt_aux.hip)
int launch_fill_u64(uint64_t* p, size_t count, uint64_t v, hipStream_t s);
int launch_fill_i32(int32_t* p, size_t count, int32_t v, hipStream_t s);
int launch_iota_i32(int32_t* p, size_t count, hipStream_t s);
int launch_copy_panel_L(int64_t n, int64_t k0, int nsteps, const double* Lbuf, double* W, int64_t ldw,
                        hipStream_t s);
int launch_compose_sigma(int64_t n, int npanels, const int32_t* pis, int32_t* sigma, hipStream_t s);
int launch_final_L(int64_t n, int nb, int npanels, const double* W, int64_t ldw, const int32_t* sigma,
                   double* A, int64_t lda, hipStream_t s);
int launch_ltlt_info(int64_t n, const double* T, const int* status, int* dinfo, hipStream_t s);
int launch_logpf(int64_t n, const int32_t* ipiv, const double* T, double* logabs, int* sign,
                 double* pf, hipStream_t s);

}  // namespace skf
