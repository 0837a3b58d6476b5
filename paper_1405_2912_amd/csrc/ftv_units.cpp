// ftv_units.cpp -- fault-aware runtime estimation fed by the voter's results
// (Kicherer & Karl, Sec. IV-B).  Host arithmetic only.
#include <algorithm>
#include <cmath>
#include <limits>
#include <vector>

#include "ftv.h"
#include "ftv_common.hpp"

using namespace ftv;

extern "C" {

double ftv_fault_aware_runtime(const ftv_unit *u) {
  if (!u || !(u->runtime > 0.0) || u->valid > u->total) return std::numeric_limits<double>::quiet_NaN();
  if (u->total == 0) return u->runtime;  // no history yet
  if (u->valid == 0) return std::numeric_limits<double>::infinity();
  // R / (1 - p) with 1 - p = v / t
  return u->runtime * ((double)u->total / (double)u->valid);
}

int ftv_rank_units(const ftv_unit *units, uint32_t n, int probe, uint32_t *order) {
  if ((n && (!units || !order))) return fail(FTV_E_INVALID, "NULL argument");
  std::vector<double> f(n);
  for (uint32_t i = 0; i < n; ++i) {
    f[i] = ftv_fault_aware_runtime(&units[i]);
    if (std::isnan(f[i])) return fail(FTV_E_INVALID, "unit with runtime <= 0 or valid > total");
    order[i] = i;
  }
  std::stable_sort(order, order + n, [&](uint32_t a, uint32_t b) { return f[a] < f[b]; });
  if (probe) {
    for (uint32_t j = 0; j < n; ++j)
      if (std::isinf(f[order[j]])) {
        const uint32_t u = order[j];
        for (uint32_t q = j; q > 0; --q) order[q] = order[q - 1];
        order[0] = u;
        break;
      }
  }
  return FTV_OK;
}

int ftv_record_vote(ftv_unit *units, uint32_t nunits, const uint32_t *unit_of_replica, uint32_t k,
                    const ftv_stats *stats) {
  if (!units || !unit_of_replica || !stats) return fail(FTV_E_INVALID, "NULL argument");
  if (k < 2 || k > FTV_MAX_K) return fail(FTV_E_K, "k must be in [2, 7]");
  for (uint32_t r = 0; r < k; ++r)
    if (unit_of_replica[r] >= nunits) return fail(FTV_E_INVALID, "unit index out of range");
  if (stats->verdict == FTV_UNRESOLVED) return FTV_OK;
  for (uint32_t r = 0; r < k; ++r) {
    ftv_unit &u = units[unit_of_replica[r]];
    u.total += 1;
    u.valid += stats->disagree[r] == 0 ? 1 : 0;
  }
  return FTV_OK;
}

}  // extern "C"
