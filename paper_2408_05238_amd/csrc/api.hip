// extern "C" entry points of libskf: argument checks on the host, then the
// stream-ordered launches.  See include/skf.h for the contract of each call.
#include <mutex>
#include <stdio.h>
#include <algorithm>
#include <vector>
#include <string.h>
#include <stdlib.h>

#include "skf_internal.h"

namespace skf {

static thread_local char g_last_error[256] = "";

int note_error(hipError_t err, const char* where) {
  snprintf(g_last_error, sizeof g_last_error, "%s: %s", where, hipGetErrorString(err));
  return SKF_EDEVICE;
}

const DeviceInfo& device_info() {
  static std::mutex mu;
  static DeviceInfo cache[64];
  static bool have[64] = {false};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  std::lock_guard<std::mutex> lk(mu);
  if (!have[dev]) {
    DeviceInfo d{};
    d.device = dev;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
    d.num_cus = cus;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      lds = 65536;
    d.lds_per_block = (size_t)lds;
    cache[dev] = d;
    have[dev] = true;
  }
  return cache[dev];
}

// Synchronous completion: when the caller gave no device info word, use one
// inside the workspace, wait for the stream and return the outcome.
static int finish_sync(int rc, int* dinfo_internal, hipStream_t s) {
  if (rc) return rc;
  int h = 0;
  SKF_CHECK(hipMemcpyAsync(&h, dinfo_internal, sizeof(int), hipMemcpyDeviceToHost, s), "info copy");
  SKF_CHECK(hipStreamSynchronize(s), "sync");
  return h;
}

// ---------------------------------------------------------------------------
// Kernel timing hooks
// ---------------------------------------------------------------------------
namespace {
struct ProfRec {
  hipEvent_t a, b;
  int cls;
  double flops;
};
struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t pending = nullptr;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
Profiler& prof() {
  static Profiler p;
  return p;
}
}  // namespace

void prof_begin(hipStream_t s) {
  Profiler& p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  if (!p.on) return;
  p.pending = p.get();
  if (p.pending) (void)hipEventRecord(p.pending, s);
}

void prof_end(hipStream_t s, int cls, double flops) {
  Profiler& p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  if (!p.on || !p.pending) return;
  hipEvent_t b = p.get();
  if (!b) return;
  (void)hipEventRecord(b, s);
  p.recs.push_back(ProfRec{p.pending, b, cls, flops});
  p.pending = nullptr;
}

size_t batched_workspace_bytes(int64_t batch);
int batched_max_n();
int run_batched(int64_t batch, const int64_t* n_host, double* const* A, const int64_t* lda_host,
                int32_t* const* ipiv, double* const* T, double* logabs, int* sign, int* info, void* work,
                size_t lwork, bool want_L, hipStream_t s);
size_t refine_workspace_bytes(int64_t n, int64_t nrhs);
int run_refine(int64_t n, int64_t nrhs, const double* A0, int64_t lda0, const double* LT, int64_t lda,
               const int32_t* ipiv, const double* T, const double* B, int64_t ldb, double* X, int64_t ldx,
               double tol, int maxit, int* iters, double* berr, void* work, size_t lwork, hipStream_t s);

}  // namespace skf

using namespace skf;

extern "C" {

const char* skf_version(void) { return "skf 0.1 (gfx950)"; }

const char* skf_last_error(void) { return g_last_error; }

size_t skf_ltlt_workspace(skf_int n, int prec) {
  if (n < 0 || (prec != SKF_PREC_F64 && prec != SKF_PREC_F32_TRAILING)) return 0;
  return ltlt_workspace_bytes(n, prec) + 256;  // + internal info word
}

static int check_ltlt_args(skf_int n, const double* A, skf_int lda, const int32_t* ipiv,
                           const double* T, int prec, const void* work, size_t lwork) {
  if (n < 0) return -1;
  if (n > 0 && !A) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (n > 0 && !ipiv) return -4;
  if (n > 1 && !T) return -5;
  if (prec != SKF_PREC_F64 && prec != SKF_PREC_F32_TRAILING) return -6;
  if (n > 0 && !work) return -7;
  if (((uintptr_t)work & 255) != 0) return -7;
  if (n > 0 && lwork < skf_ltlt_workspace(n, prec)) return SKF_EWORK;
  if (n > INT32_MAX - 2) return -1;
  return 0;
}

int skf_ltlt(skf_int n, double* A, skf_int lda, int32_t* ipiv, double* T, int prec, void* work,
             size_t lwork, int* dinfo, void* stream) {
  int rc = check_ltlt_args(n, A, lda, ipiv, T, prec, work, lwork);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (n == 0) {
    if (dinfo) return launch_fill_i32(dinfo, 1, 0, s);
    return 0;
  }
  const size_t core = ltlt_workspace_bytes(n, prec);
  int* dinfo_int = (int*)((char*)work + core);
  rc = run_ltlt(n, A, lda, ipiv, T, prec, work, core, dinfo ? dinfo : dinfo_int, s);
  if (dinfo) return rc;
  return finish_sync(rc, dinfo_int, s);
}

int skf_pfonly(skf_int n, double* A, skf_int lda, int32_t* ipiv, double* T, int prec, void* work,
               size_t lwork, int* dinfo, void* stream) {
  int rc = check_ltlt_args(n, A, lda, ipiv, T, prec, work, lwork);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (n == 0) {
    if (dinfo) return launch_fill_i32(dinfo, 1, 0, s);
    return 0;
  }
  const size_t core = ltlt_workspace_bytes(n, prec);
  int* dinfo_int = (int*)((char*)work + core);
  rc = run_pfonly(n, A, lda, ipiv, T, prec, work, core, dinfo ? dinfo : dinfo_int, s);
  if (dinfo) return rc;
  return finish_sync(rc, dinfo_int, s);
}

int skf_logpf_from_factors(skf_int n, const int32_t* ipiv, const double* T, double* logabs, int* sign,
                           void* stream) {
  if (n < 0) return -1;
  if (n > 0 && !ipiv) return -2;
  if (n > 1 && !T) return -3;
  if (!logabs) return -4;
  if (!sign) return -5;
  return launch_logpf(n, ipiv, T, logabs, sign, nullptr, (hipStream_t)stream);
}

// Pfaffian-only reduction, then the product; ipiv and T live at the end of the
// caller's workspace.
static size_t pf_extra(skf_int n) { return align_up(sizeof(int32_t) * (n + 1), 256) + align_up(sizeof(double) * (n + 1), 256); }

static int logpf_common(skf_int n, double* A, skf_int lda, double* logabs, int* sign, double* pf, int prec,
                        void* work, size_t lwork, int* dinfo, void* stream) {
  if (n < 0) return -1;
  if (n > 0 && !A) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (!work && n > 0) return -7;
  const size_t need = skf_ltlt_workspace(n, prec);
  if (n > 0 && lwork < need + pf_extra(n)) return SKF_EWORK;
  hipStream_t s = (hipStream_t)stream;
  char* extra = (char*)work + need;
  int32_t* ipiv = (int32_t*)extra;
  double* T = (double*)(extra + align_up(sizeof(int32_t) * (n + 1), 256));
  int rc = 0;
  if (n > 0) {
    const size_t core = ltlt_workspace_bytes(n, prec);
    int* dinfo_int = (int*)((char*)work + core);
    rc = run_pfonly(n, A, lda, ipiv, T, prec, work, core, dinfo ? dinfo : dinfo_int, s);
    if (rc) return rc;
    rc = launch_logpf(n, ipiv, T, logabs, sign, pf, s);
    if (rc) return rc;
    if (!dinfo) return finish_sync(0, dinfo_int, s);
    return 0;
  }
  rc = launch_logpf(0, nullptr, nullptr, logabs, sign, pf, s);
  if (rc) return rc;
  if (dinfo) return launch_fill_i32(dinfo, 1, 0, s);
  SKF_CHECK(hipStreamSynchronize(s), "sync");
  return 0;
}

size_t skf_logpf_workspace(skf_int n, int prec) { return skf_ltlt_workspace(n, prec) + pf_extra(n); }

int skf_logpf(skf_int n, double* A, skf_int lda, double* logabs, int* sign, int prec, void* work,
              size_t lwork, int* dinfo, void* stream) {
  if (!logabs) return -4;
  if (!sign) return -5;
  return logpf_common(n, A, lda, logabs, sign, nullptr, prec, work, lwork, dinfo, stream);
}

int skf_pfaffian(skf_int n, double* A, skf_int lda, double* pf, int prec, void* work, size_t lwork,
                 int* dinfo, void* stream) {
  if (!pf) return -4;
  return logpf_common(n, A, lda, nullptr, nullptr, pf, prec, work, lwork, dinfo, stream);
}

static int check_skr2k(skf_int n, skf_int k, const double* A, skf_int lda, const double* B, skf_int ldb,
                       const double* C, skf_int ldc) {
  if (n < 0) return -1;
  if (k < 0) return -2;
  if (n > 0 && k > 0 && !A) return -4;
  if (lda < (n > 1 ? n : 1)) return -5;
  if (n > 0 && k > 0 && !B) return -6;
  if (ldb < (n > 1 ? n : 1)) return -7;
  if (n > 1 && !C) return -9;
  if (ldc < (n > 1 ? n : 1)) return -10;
  return 0;
}

int skf_skr2k(skf_int n, skf_int k, double alpha, const double* A, skf_int lda, const double* B, skf_int ldb,
              double beta, double* C, skf_int ldc, void* stream) {
  int rc = check_skr2k(n, k, A, lda, B, ldb, C, ldc);
  if (rc) return rc;
  return launch_skr2k_f64(n, k, alpha, A, lda, B, ldb, beta, C, ldc, (hipStream_t)stream);
}

int skf_skr2k_f32(skf_int n, skf_int k, double alpha, const double* A, skf_int lda, const double* B,
                  skf_int ldb, double beta, double* C, skf_int ldc, void* stream) {
  int rc = check_skr2k(n, k, A, lda, B, ldb, C, ldc);
  if (rc) return rc;
  return launch_skr2k_f32(n, k, alpha, A, lda, B, ldb, beta, C, ldc, (hipStream_t)stream);
}

size_t skf_solve_workspace(skf_int n, skf_int nrhs) {
  if (n < 0 || nrhs < 0) return 0;
  return solve_workspace_bytes(n, nrhs) + 256;
}

int skf_solve(skf_int n, skf_int nrhs, const double* LT, skf_int lda, const int32_t* ipiv, const double* T,
              double* B, skf_int ldb, void* work, size_t lwork, int* dinfo, void* stream) {
  if (n < 0) return -1;
  if (nrhs < 0) return -2;
  if (n > 0 && !LT) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (n > 0 && !ipiv) return -5;
  if (n > 1 && !T) return -6;
  if (n > 0 && nrhs > 0 && !B) return -7;
  if (ldb < (n > 1 ? n : 1)) return -8;
  if (!work || ((uintptr_t)work & 255)) return -9;
  if (lwork < skf_solve_workspace(n, nrhs)) return SKF_EWORK;
  hipStream_t s = (hipStream_t)stream;
  const size_t core = solve_workspace_bytes(n, nrhs);
  int* dinfo_int = (int*)((char*)work + core);
  int rc = run_solve(n, nrhs, LT, lda, ipiv, T, B, ldb, work, core, dinfo ? dinfo : dinfo_int, s);
  if (dinfo) return rc;
  return finish_sync(rc, dinfo_int, s);
}

int skf_solve_noalloc(skf_int n, skf_int nrhs, const double* LT, skf_int lda, const int32_t* ipiv,
                      const double* T, double* B, skf_int ldb, int* dinfo, void* stream) {
  if (n < 0) return -1;
  if (nrhs < 0) return -2;
  if (n > 0 && !LT) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (n > 0 && !ipiv) return -5;
  if (n > 1 && !T) return -6;
  if (n > 0 && nrhs > 0 && !B) return -7;
  if (ldb < (n > 1 ? n : 1)) return -8;
  if (n > kSolveNoAllocMaxN) {
    snprintf(g_last_error, sizeof g_last_error,
             "skf_solve_noalloc: n = %lld exceeds the fixed scratch limit n <= %lld (%zu bytes)", (long long)n,
             (long long)kSolveNoAllocMaxN, solve_noalloc_scratch_bytes());
    return SKF_ESCRATCH;
  }
  return run_solve_noalloc(n, nrhs, LT, lda, ipiv, T, B, ldb, dinfo, (hipStream_t)stream);
}

// The blocked reduction runs when its panel fits on the device (n up to 256 or
// 512 panel workgroups of 64 rows) and SKF_C128_UNBLOCKED is unset; otherwise
// the unblocked one.  The workspace covers whichever of the two is larger.
static bool c128_blocked(skf_int n) {
  return pfonly_c128_blocked_nb(n) > 0 && !getenv("SKF_C128_UNBLOCKED");
}

static size_t c128_core_bytes(skf_int n) {
  return std::max(pfonly_c128_workspace_bytes(n), pfonly_c128_blocked_workspace_bytes(n));
}

size_t skf_pfonly_c128_workspace(skf_int n) {
  if (n < 0) return 0;
  return c128_core_bytes(n) + 256;
}

int skf_pfonly_c128(skf_int n, const double* A, skf_int lda, int32_t* ipiv, double* T, void* work, size_t lwork,
                    int* dinfo, void* stream) {
  if (n < 0) return -1;
  if (n > 0 && !A) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (n > 0 && !ipiv) return -4;
  if (n > 1 && !T) return -5;
  if (!work || ((uintptr_t)work & 255)) return -6;
  if (lwork < skf_pfonly_c128_workspace(n)) return SKF_EWORK;
  hipStream_t s = (hipStream_t)stream;
  const size_t core = c128_core_bytes(n);
  int* dinfo_int = (int*)((char*)work + core);
  int rc = c128_blocked(n) ? run_pfonly_c128_blocked(n, A, lda, ipiv, T, work, core, dinfo ? dinfo : dinfo_int, s)
                           : run_pfonly_c128(n, A, lda, ipiv, T, work, core, dinfo ? dinfo : dinfo_int, s);
  if (dinfo) return rc;
  return finish_sync(rc, dinfo_int, s);
}

size_t skf_ltlt_c128_workspace(skf_int n) {
  if (n < 0) return 0;
  const size_t core = ltlt_c128_workspace_bytes(n);
  return (core || n == 0) ? core + 256 : 0;
}

int skf_ltlt_c128(skf_int n, double* A, skf_int lda, int32_t* ipiv, double* T, void* work, size_t lwork, int* dinfo,
                  void* stream) {
  if (n < 0) return -1;
  if (n > 0 && !A) return -2;
  if (lda < (n > 1 ? n : 1)) return -3;
  if (n > 0 && !ipiv) return -4;
  if (n > 1 && !T) return -5;
  if (!work || ((uintptr_t)work & 255)) return -6;
  if (n > 0 && ltlt_c128_nb(n) == 0) return SKF_ENOTIMPL;
  if (lwork < skf_ltlt_c128_workspace(n)) return SKF_EWORK;
  hipStream_t s = (hipStream_t)stream;
  const size_t core = ltlt_c128_workspace_bytes(n);
  int* dinfo_int = (int*)((char*)work + core);
  int rc = run_ltlt_c128(n, A, lda, ipiv, T, work, core, dinfo ? dinfo : dinfo_int, s);
  if (dinfo) return rc;
  return finish_sync(rc, dinfo_int, s);
}

size_t skf_solve_c128_workspace(skf_int n, skf_int nrhs) {
  if (n < 0 || nrhs < 0) return 0;
  return solve_c128_workspace_bytes(n, nrhs) + 256;
}

int skf_solve_c128(skf_int n, skf_int nrhs, const double* LT, skf_int lda, const int32_t* ipiv, const double* T,
                   double* B, skf_int ldb, void* work, size_t lwork, int* dinfo, void* stream) {
  if (n < 0) return -1;
  if (nrhs < 0) return -2;
  if (n > 0 && !LT) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (n > 0 && !ipiv) return -5;
  if (n > 1 && !T) return -6;
  if (n > 0 && nrhs > 0 && !B) return -7;
  if (ldb < (n > 1 ? n : 1)) return -8;
  if (!work || ((uintptr_t)work & 255)) return -9;
  if (lwork < skf_solve_c128_workspace(n, nrhs)) return SKF_EWORK;
  hipStream_t s = (hipStream_t)stream;
  const size_t core = solve_c128_workspace_bytes(n, nrhs);
  int* dinfo_int = (int*)((char*)work + core);
  int rc = run_solve_c128(n, nrhs, LT, lda, ipiv, T, B, ldb, work, core, dinfo ? dinfo : dinfo_int, s);
  if (dinfo) return rc;
  return finish_sync(rc, dinfo_int, s);
}

int skf_logpf_c128_from_factors(skf_int n, const int32_t* ipiv, const double* T, double* logabs, double* phase,
                                void* stream) {
  if (n < 0) return -1;
  if (n > 0 && !ipiv) return -2;
  if (n > 1 && !T) return -3;
  if (!logabs) return -4;
  if (!phase) return -5;
  return launch_logpf_c128(n, ipiv, T, logabs, phase, (hipStream_t)stream);
}

size_t skf_pf_ratio_workspace(skf_int n, skf_int r) {
  if (n < 0 || r < 0 || r > pf_ratio_max_rank()) return 0;
  return pf_ratio_workspace_bytes(n, (int)r) + 256;
}

int skf_pf_ratio(skf_int n, skf_int r, const double* LT, skf_int lda, const int32_t* ipiv, const double* T,
                 const double* U, skf_int ldu, const double* V, skf_int ldv, double* logabs, int* sign,
                 void* work, size_t lwork, int* dinfo, void* stream) {
  if (n < 0) return -1;
  if (r < 0 || r > pf_ratio_max_rank()) return -2;
  if (n > 0 && !LT) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (n > 0 && !ipiv) return -5;
  if (n > 1 && !T) return -6;
  if (n > 0 && r > 0 && !U) return -7;
  if (ldu < (n > 1 ? n : 1)) return -8;
  if (n > 0 && r > 0 && !V) return -9;
  if (ldv < (n > 1 ? n : 1)) return -10;
  if (!logabs) return -11;
  if (!sign) return -12;
  if (!work || ((uintptr_t)work & 255)) return -13;
  if (lwork < skf_pf_ratio_workspace(n, r)) return SKF_EWORK;
  hipStream_t s = (hipStream_t)stream;
  const size_t core = pf_ratio_workspace_bytes(n, (int)r);
  int* dinfo_int = (int*)((char*)work + core);
  int rc = run_pf_ratio(n, (int)r, LT, lda, ipiv, T, U, ldu, V, ldv, logabs, sign, work, core,
                        dinfo ? dinfo : dinfo_int, s);
  if (dinfo) return rc;
  return finish_sync(rc, dinfo_int, s);
}

size_t skf_refine_workspace(skf_int n, skf_int nrhs) {
  if (n < 0 || nrhs < 0) return 0;
  return refine_workspace_bytes(n, nrhs);
}

int skf_solve_refine(skf_int n, skf_int nrhs, const double* A0, skf_int lda0, const double* LT, skf_int lda,
                     const int32_t* ipiv, const double* T, const double* B, skf_int ldb, double* X, skf_int ldx,
                     double tol, int maxit, int* iters, double* berr, void* work, size_t lwork, void* stream) {
  if (n < 0) return -1;
  if (nrhs < 0) return -2;
  if (n > 0 && !A0) return -3;
  if (lda0 < (n > 1 ? n : 1)) return -4;
  if (n > 0 && !LT) return -5;
  if (lda < (n > 1 ? n : 1)) return -6;
  if (n > 0 && !ipiv) return -7;
  if (n > 1 && !T) return -8;
  if (n > 0 && nrhs > 0 && !B) return -9;
  if (ldb < (n > 1 ? n : 1)) return -10;
  if (n > 0 && nrhs > 0 && !X) return -11;
  if (ldx < (n > 1 ? n : 1)) return -12;
  if (!(tol >= 0.0)) return -13;
  if (maxit < 0) return -14;
  if (!work || ((uintptr_t)work & 255)) return -17;
  if (lwork < skf_refine_workspace(n, nrhs)) return SKF_EWORK;
  return run_refine(n, nrhs, A0, lda0, LT, lda, ipiv, T, B, ldb, X, ldx, tol, maxit, iters, berr, work, lwork,
                    (hipStream_t)stream);
}

size_t skf_batched_workspace(skf_int batch, const skf_int* n_host) {
  if (batch < 0) return 0;
  size_t solve = 0;
  if (n_host && batch > 0) {
    // the factors' batched solve with up to 16 right-hand sides each
    std::vector<skf_int> nr((size_t)batch, 16);
    solve = solve_batched_workspace_bytes(batch, n_host, nr.data());
  }
  return std::max(align_up(batched_workspace_bytes(batch), 256), solve);
}

static int check_batched(skf_int batch, const skf_int* n_host, double* const* A, const skf_int* lda_host,
                         void* work, size_t lwork) {
  if (batch < 0) return -1;
  if (batch > 0 && !n_host) return -2;
  if (batch > 0 && !A) return -3;
  if (batch > 0 && !lda_host) return -4;
  for (skf_int b = 0; b < batch; ++b) {
    if (n_host[b] < 0 || n_host[b] > batched_max_n()) return -2;
    if (lda_host[b] < (n_host[b] > 1 ? n_host[b] : 1)) return -4;
  }
  if (batch > 0 && (!work || ((uintptr_t)work & 255))) return SKF_EWORK;
  if (lwork < batched_workspace_bytes(batch)) return SKF_EWORK;
  return 0;
}

int skf_ltlt_batched(skf_int batch, const skf_int* n_host, double* const* A, const skf_int* lda_host,
                     int32_t* const* ipiv, double* const* T, double* logabs, int* sign, int* info, void* work,
                     size_t lwork, void* stream) {
  int rc = check_batched(batch, n_host, A, lda_host, work, lwork);
  if (rc) return rc;
  return run_batched(batch, n_host, A, lda_host, ipiv, T, logabs, sign, info, work, lwork, true, (hipStream_t)stream);
}

int skf_pfonly_batched(skf_int batch, const skf_int* n_host, double* const* A, const skf_int* lda_host,
                       int32_t* const* ipiv, double* const* T, double* logabs, int* sign, int* info,
                       void* work, size_t lwork, void* stream) {
  int rc = check_batched(batch, n_host, A, lda_host, work, lwork);
  if (rc) return rc;
  if (batch > 0 && (!logabs || !sign)) return -7;
  return run_batched(batch, n_host, A, lda_host, ipiv, T, logabs, sign, info, work, lwork, false,
                     (hipStream_t)stream);
}

int skf_logpf_batched(skf_int batch, const skf_int* n_host, double* const* A, const skf_int* lda_host,
                      double* logabs, int* sign, int* info, void* work, size_t lwork, void* stream) {
  int rc = check_batched(batch, n_host, A, lda_host, work, lwork);
  if (rc) return rc;
  if (batch > 0 && (!logabs || !sign)) return -5;
  return run_batched(batch, n_host, A, lda_host, nullptr, nullptr, logabs, sign, info, work, lwork, false,
                     (hipStream_t)stream);
}

size_t skf_solve_batched_workspace(skf_int batch, const skf_int* n_host, const skf_int* nrhs_host) {
  if (batch < 0 || (batch > 0 && (!n_host || !nrhs_host))) return 0;
  return solve_batched_workspace_bytes(batch, n_host, nrhs_host);
}

int skf_solve_batched(skf_int batch, const skf_int* n_host, double* const* LT, const skf_int* lda_host,
                      int32_t* const* ipiv, double* const* T, const skf_int* nrhs_host, double* const* B,
                      const skf_int* ldb_host, int* info, void* work, size_t lwork, void* stream) {
  if (batch < 0) return -1;
  if (batch == 0) return 0;
  if (!n_host || !LT || !lda_host || !ipiv || !T || !nrhs_host || !B || !ldb_host || !info) return -2;
  for (skf_int b = 0; b < batch; ++b)
    if (n_host[b] < 0 || nrhs_host[b] < 0 || lda_host[b] < std::max<skf_int>(1, n_host[b]) ||
        ldb_host[b] < std::max<skf_int>(1, n_host[b]))
      return -2;
  if (!work || ((uintptr_t)work & 255)) return SKF_EWORK;
  return run_solve_batched(batch, n_host, (const double* const*)LT, lda_host, (const int32_t* const*)ipiv,
                           (const double* const*)T, nrhs_host, B, ldb_host, info, work, lwork,
                           (hipStream_t)stream);
}

int skf_profile_enable(int on) {
  Profiler& p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  p.on = on != 0;
  return 0;
}

int skf_profile_read(double* ms, double* flops, int64_t* launches, int reset) {
  Profiler& p = prof();
  std::lock_guard<std::mutex> lk(p.mu);
  double t[2] = {0, 0}, f[2] = {0, 0};
  int64_t c[2] = {0, 0};
  for (const ProfRec& r : p.recs) {
    SKF_CHECK(hipEventSynchronize(r.b), "profile sync");
    float e = 0.f;
    SKF_CHECK(hipEventElapsedTime(&e, r.a, r.b), "profile elapsed");
    if (r.cls >= 0 && r.cls < 2) {
      t[r.cls] += e;
      f[r.cls] += r.flops;
      c[r.cls] += 1;
    }
  }
  for (int i = 0; i < 2; ++i) {
    if (ms) ms[i] = t[i];
    if (flops) flops[i] = f[i];
    if (launches) launches[i] = c[i];
  }
  if (reset) {
    for (const ProfRec& r : p.recs) {
      p.pool.push_back(r.a);
      p.pool.push_back(r.b);
    }
    p.recs.clear();
  }
  return 0;
}

int skf_tune_set(int param, skf_int n_lo, skf_int n_hi, int value) { return tune_set(param, n_lo, n_hi, value); }

int skf_tune_get(int param, skf_int n) {
  switch (param) {
    case SKF_TUNE_LTLT_NB: {
      const int nb = ltlt_plan_nb(n);
      return nb < 0 ? 0 : nb;
    }
    case SKF_TUNE_PFONLY_NB: {
      const int nb = pfonly_plan_nb(n);
      return nb < 0 ? 0 : nb;
    }
    case SKF_TUNE_SKR2K_BAND:
      return skr2k_band(n);
    default:
      return -1;
  }
}

int skf_tune_clear(void) {
  tune_clear();
  return 0;
}

}  // extern "C"
