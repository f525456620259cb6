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

// Builds the layout; on failure returns a status and sets *err.
eat_status build_layout(const int32_t *u, const int32_t *v, const int32_t *t,
                        const int32_t *lam, int64_t n, int32_t nv,
                        const eat_build_options &opt, eat_layout &out,
                        std::string *err);

}  // namespace eat
