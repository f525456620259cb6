// layout.hpp -- host-side timetable layout (the preprocessing of Section III-A).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "eat.h"

struct eat_layout {
  int32_t kind = EAT_LAYOUT_HYBRID;
  int32_t n_vertices = 0;
  int32_t cluster_seconds = 3600;
  int32_t n_clusters = 1;
  int32_t max_departure = 0;
  int32_t max_types_per_vertex = 0;
  int64_t n_conn_input = 0, n_self_loops = 0, n_duplicates = 0, n_conn = 0;
  int64_t n_edges = 0, n_types = 0, n_headers = 0, n_ap = 0, n_array = 0;
  int64_t n_trips = 0, n_shortcuts = 0;  // sub-trip shortcuts added (Section II-G)
  int32_t subtrip_len = 0;               // their sub-trip length (-1: sqrt of each trip's)
  std::vector<int32_t> vt;        // [2V] per stop: first type, type count
  std::vector<int32_t> order;     // [V] the stops in layout order
  std::vector<int32_t> ty;        // [4*T]
  std::vector<uint32_t> mask_hi;  // [T] (hybrid)
  std::vector<int32_t> hdr;       // [2*K] (hybrid)
  std::vector<int32_t> pool;      // departures
};

namespace eat {

// Words of infinity after the last pool entry.
constexpr int64_t kPoolTail = 16;

// Shortcut connections of the sub-trips of every trip (subtrips.cpp).
struct SubtripConns {
  std::vector<int32_t> u, v, t, lam;
  int64_t n_trips = 0;
  int32_t subtrip_len = 0;
};
// trip[i] >= 0: the vehicle trip of connection i (-1: none).  subtrip_len: 0 =
// sqrt of the mean trip length, -1 = sqrt of each trip's length, r >= 1 =
// fixed (1 adds nothing).  EAT_ERR_INVALID_ARGUMENT if a trip's connections,
// in departure order, do not chain (head = next tail, arrival <= next
// departure).
eat_status add_subtrip_shortcuts(const int32_t *u, const int32_t *v, const int32_t *t, const int32_t *lam,
                                 const int32_t *trip, int64_t n, int32_t subtrip_len, SubtripConns &out,
                                 std::string *err);

// Builds the layout; on failure returns a status and sets *err.
eat_status build_layout(const int32_t *u, const int32_t *v, const int32_t *t,
                        const int32_t *lam, int64_t n, int32_t nv,
                        const eat_build_options &opt, eat_layout &out,
                        std::string *err);

}  // namespace eat
