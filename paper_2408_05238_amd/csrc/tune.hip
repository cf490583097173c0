// Tuning table: block sizes and tile-walk parameters chosen by measurement.
//
// Entries map (parameter, range of orders) to a value.  The table starts empty
// (built-in feasibility rules apply); the Python tuner measures the candidates
// on the device, persists its choices as JSON, and the binding loads them into
// this table through skf_tune_set when the library is first used.  A later
// entry covering the same order takes precedence over an earlier one.
#include <mutex>
#include <vector>

#include "skf_internal.h"

namespace skf {
namespace {

struct TuneEntry {
  int param;
  int64_t lo, hi;  // orders lo <= n <= hi
  int value;
};

std::mutex& tune_mu() {
  static std::mutex m;
  return m;
}
std::vector<TuneEntry>& tune_table() {
  static std::vector<TuneEntry> t;
  return t;
}

}  // namespace

bool tune_value_ok(int param, int value) {
  switch (param) {
    case SKF_TUNE_LTLT_NB:
    case SKF_TUNE_PFONLY_NB:
      return value == 16 || value == 32 || value == 64 || value == 128 || value == 256;
    case SKF_TUNE_SKR2K_BAND:
      return value >= 1 && value <= 64;

    default:
      return false;
  }
}

// The table's value for (param, n), or 0 when no entry covers n.
int tune_lookup(int param, int64_t n) {
  std::lock_guard<std::mutex> lk(tune_mu());
  const std::vector<TuneEntry>& t = tune_table();
  for (size_t i = t.size(); i-- > 0;)
    if (t[i].param == param && t[i].lo <= n && n <= t[i].hi) return t[i].value;
  return 0;
}

int tune_set(int param, int64_t lo, int64_t hi, int value) {
  if (param < 0 || param >= SKF_TUNE_NPARAMS) return -1;
  if (lo < 0) return -2;
  if (hi < lo) return -3;
  if (!tune_value_ok(param, value)) return -4;
  std::lock_guard<std::mutex> lk(tune_mu());
  tune_table().push_back(TuneEntry{param, lo, hi, value});
  return 0;
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(tune_mu());
  tune_table().clear();
}

}  // namespace skf
