// extern "C" entry points of libskf: argument checks on the host, then the
// stream-ordered launches.  See include/skf.h for the contract of each call.
#include <mutex>
#include <stdio.h>
#include <string.h>

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

int skf_logpf_from_factors(skf_int n, const int32_t* ipiv, const double* T, double* logabs, int* sign,
                           void* stream) {
  if (n < 0) return -1;
  if (n > 0 && !ipiv) return -2;
  if (n > 1 && !T) return -3;
  if (!logabs) return -4;
  if (!sign) return -5;
  return launch_logpf(n, ipiv, T, logabs, sign, nullptr, (hipStream_t)stream);
}

// Factor, then reduce; ipiv and T live at the end of the caller's workspace.
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
    rc = run_ltlt(n, A, lda, ipiv, T, prec, work, core, dinfo ? dinfo : dinfo_int, s);
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

}  // extern "C"

// ---------------------------------------------------------------------------
// Entry points whose kernels live in later translation units are declared in
// skf.h; until a unit provides them these definitions report SKF_ENOTIMPL.
// ---------------------------------------------------------------------------
