// subtrips.cpp -- sub-trip shortcuts (Section II-G), a data enhancement done
// before the preprocessing of Section III-A.
//
// A trip is the sequence of connections one vehicle runs: connection i leaves
// stop v_i at t_i and reaches v_{i+1} at t_i + lam_i, and the next one leaves
// v_{i+1} no earlier (t_i + lam_i <= t_{i+1}).  Each trip of k connections is
// cut into consecutive, non-overlapping sub-trips of r connections (the last
// one holds what is left), and every sub-trip i..j of at least two
// connections gets one artificial connection v_i -> v_{j+1} leaving at t_i
// and arriving at t_j + lam_j.  Staying on the vehicle along the sub-trip
// reaches v_{j+1} at exactly that time, so the earliest arrival times never
// change; a relaxation round covers the whole sub-trip at once, so fewer
// rounds are needed (the temporal diameter shrinks).
// Sub-trip length (Section IV-B): r = sqrt(mean trip length) by default (the
// paper's preferred rule), r = sqrt(k) per trip, or a fixed r.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "internal.hpp"
#include "layout.hpp"

namespace eat {

eat_status add_subtrip_shortcuts(const int32_t *u, const int32_t *v, const int32_t *t, const int32_t *lam,
                                 const int32_t *trip, int64_t n, int32_t subtrip_len, SubtripConns &out,
                                 std::string *err) {
  auto fail = [&](eat_status s, const std::string &m) {
    if (err) *err = m;
    return s;
  };
  if (subtrip_len < -1) return fail(EAT_ERR_INVALID_ARGUMENT, "subtrip_len must be >= -1");
  if (n > 0 && !trip) return fail(EAT_ERR_INVALID_ARGUMENT, "trip array is NULL");
  // the connections of each trip, in departure order
  std::vector<int64_t> idx;
  idx.reserve((size_t)n);
  for (int64_t i = 0; i < n; ++i)
    if (trip[i] >= 0) idx.push_back(i);
  std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
    return trip[a] != trip[b] ? trip[a] < trip[b] : (t[a] != t[b] ? t[a] < t[b] : a < b);
  });
  // trips as ranges of idx, each checked to be one vehicle's run
  std::vector<std::pair<size_t, size_t>> trips;
  for (size_t i = 0; i < idx.size();) {
    size_t j = i + 1;
    while (j < idx.size() && trip[idx[j]] == trip[idx[i]]) ++j;
    for (size_t k = i; k + 1 < j; ++k) {
      const int64_t a = idx[k], b = idx[k + 1];
      if (v[a] != u[b] || (int64_t)t[a] + lam[a] > (int64_t)t[b])
        return fail(EAT_ERR_INVALID_ARGUMENT,
                    "trip " + std::to_string(trip[a]) + " is not one vehicle's run: connection " + std::to_string(a) +
                        " arrives at stop " + std::to_string(v[a]) + " at " + std::to_string((int64_t)t[a] + lam[a]) +
                        ", the next leaves stop " + std::to_string(u[b]) + " at " + std::to_string(t[b]));
    }
    trips.emplace_back(i, j);
    i = j;
  }
  out = SubtripConns();
  out.n_trips = (int64_t)trips.size();
  if (trips.empty() || subtrip_len == 1) return EAT_OK;
  int64_t fixed_r = subtrip_len;
  if (subtrip_len == 0) {  // sqrt of the mean trip length
    const double mean = (double)idx.size() / (double)trips.size();
    fixed_r = std::max<int64_t>(1, std::llround(std::sqrt(mean)));
  }
  out.subtrip_len = subtrip_len == -1 ? -1 : (int32_t)fixed_r;
  for (const auto &tr : trips) {
    const int64_t k = (int64_t)(tr.second - tr.first);
    const int64_t r = subtrip_len == -1 ? std::max<int64_t>(1, std::llround(std::sqrt((double)k))) : fixed_r;
    for (int64_t b = 0; b < k; b += r) {
      const int64_t e = std::min(k, b + r) - 1;  // last connection of the sub-trip
      if (e <= b) continue;                      // a single connection: nothing to add
      const int64_t ci = idx[tr.first + (size_t)b], cj = idx[tr.first + (size_t)e];
      out.u.push_back(u[ci]);
      out.v.push_back(v[cj]);
      out.t.push_back(t[ci]);
      out.lam.push_back((int32_t)((int64_t)t[cj] + lam[cj] - t[ci]));
    }
  }
  return EAT_OK;
}

}  // namespace eat
