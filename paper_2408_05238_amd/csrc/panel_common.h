// Device helpers shared by the persistent panel kernels (real and complex):
// cross-workgroup tagged words, lane exchanges and the wave arg-max.
#pragma once

#include "skf_internal.h"

namespace skf {
namespace panel {

constexpr int kPanelThreads = 64;
// A workgroup's record for one step is two 64-bit words, each carrying a 16-bit
// step tag and 48 payload bits:
//   w0 = tag | flags:2 | slot:6 | psi:24 | |c| bits 62..47
//   w1 = tag | sign of c | |c| bits 46..0
// (flags: bit 31 of the 32-bit field = no candidate, bit 30 = non-finite
// column), so a reader needs two atomic 64-bit loads per record.  Records sit
// kRecStride words apart; the candidate's l0 (read only from the winner) is kept
// in a separate pair of 32-bit-tagged words.
constexpr int kRecStride = 16;
// Every record and l0 pair is written in kRecCopies copies; workgroup g reads
// copy g % kRecCopies (consecutive workgroups are dispatched round-robin over
// the XCDs), so each line has G / kRecCopies readers instead of G.  (Copies of
// the coefficient mirror were measured too: the extra stores at every pair end
// delay the next loads, which wait behind them, and the step got slower.)
constexpr int kRecCopies = 8;
constexpr uint32_t kFlagNonFinite = 1u << 30;
constexpr uint32_t kFlagNoCand = 1u << 31;
constexpr uint64_t kLow47 = (1ull << 47) - 1;
constexpr int kMaxG = 2048;   // workgroups of one panel launch
constexpr uint32_t kNoCand = 0xFFFFFFFFu;


__device__ inline uint64_t ld_word(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_word(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t mk(uint32_t tag, uint32_t payload) { return ((uint64_t)tag << 32) | payload; }
__device__ inline uint32_t tag_of(uint64_t w) { return (uint32_t)(w >> 32); }
__device__ inline uint32_t tag16(uint32_t tag) { return (tag - 1u) % 65535u + 1u; }  // never 0
__device__ inline uint32_t tag16_of(uint64_t w) { return (uint32_t)(w >> 48); }
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

// Marks a polled word as consumed where its loads are known to have landed (a
// wait loop's exit), so the compiler never places a later wait for it after
// stores it cannot tell apart (vmcnt counts stores too).
__device__ inline void landed(uint64_t& w) { asm volatile("" : "+v"(w)); }

// Candidate ordering: larger |c| first, then lower current index.
__device__ inline bool better(double a, uint32_t pa, double b, uint32_t pb) {
  return (a > b) || (a == b && pa < pb);
}

// Wave-wide maximum / minimum of u; every lane ends with the result.  Inside
// each row of 16 lanes: xor-1, xor-2, rotate-4, rotate-8 (DPP); across the four
// rows: readlane of lanes 0, 16, 32, 48 (scalar, uniform).
__device__ inline uint32_t wave_max_u32(uint32_t u) {
  u = max(u, dpp32<0xB1>(u));   // quad_perm [1,0,3,2]
  u = max(u, dpp32<0x4E>(u));   // quad_perm [2,3,0,1]
  u = max(u, dpp32<0x124>(u));  // row_ror:4
  u = max(u, dpp32<0x128>(u));  // row_ror:8
  return max(max(rl32(u, 0), rl32(u, 16)), max(rl32(u, 32), rl32(u, 48)));
}
__device__ inline uint32_t wave_min_u32(uint32_t u) {
  u = min(u, dpp32<0xB1>(u));
  u = min(u, dpp32<0x4E>(u));
  u = min(u, dpp32<0x124>(u));
  u = min(u, dpp32<0x128>(u));
  return min(min(rl32(u, 0), rl32(u, 16)), min(rl32(u, 32), rl32(u, 48)));
}

// Lane of the best candidate (largest v, then lowest p) among the lanes with
// `cand` set (their v >= 0, +0 for zero), or -1 if there is none.  For
// non-negative doubles the bit patterns order as the values, so the maximum is
// found on 32-bit keys: the high word (+1, so that every candidate beats a
// non-candidate's 0), then, only if several lanes share it, the low word among
// them; the lanes holding it by a ballot; only an exact tie of values needs the
// index reduction.
__device__ inline int wave_argbest(double v, uint32_t p, bool cand) {
  const uint64_t bits = (uint64_t)__double_as_longlong(v);
  const uint32_t hk = cand ? (uint32_t)(bits >> 32) + 1u : 0u;
  const uint32_t mh = wave_max_u32(hk);
  if (mh == 0) return -1;
  uint64_t at = __ballot(hk == mh);
  if ((at & (at - 1)) == 0) return (int)__builtin_ctzll(at);
  const bool in_hi = (at >> threadIdx.x) & 1ull;
  const uint32_t ml = wave_max_u32(in_hi ? (uint32_t)bits : 0u);
  at = __ballot(in_hi && (uint32_t)bits == ml);
  if ((at & (at - 1)) == 0) return (int)__builtin_ctzll(at);
  const bool mine = (at >> threadIdx.x) & 1ull;
  const uint32_t q = wave_min_u32(mine ? p : 0xFFFFFFFFu);
  return (int)__builtin_ctzll(__ballot(mine && p == q));
}

// Wall-clock limit for one wait (the constant 100 MHz counter): 2 s.
constexpr uint64_t kWaitTicks = 200000000ull;

}  // namespace panel
}  // namespace skf
