// internal.hpp -- declarations shared by the C ABI sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "device.hpp"
#include "eat.h"

struct eat_graph {
  int device = 0;
  eat_graph_info_t info{};
  eat::GraphDev desc{};            // device pointers
  eat::GraphDev *d_desc = nullptr; // device copy of desc
  void *d_buf = nullptr;
  std::mutex mu;                   // guards the single-query scratch
  eat_query_stats *d_stats = nullptr;
  int32_t *d_failed = nullptr;
  std::vector<int32_t> rank;       // position of each stop in the layout order
};

namespace eat {

// Thread-local error text returned by eat_last_error().
eat_status set_err(eat_status s, const std::string &msg);
eat_status hip_err(hipError_t e, const char *what);

#define HIP_TRY(call)                                 \
  do {                                                \
    hipError_t e_ = (call);                           \
    if (e_ != hipSuccess) return eat::hip_err(e_, #call); \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct DeviceLimits {
  int cus = 0;
  int xccs = 1;  // L2 domains (XCDs) that work-groups are dealt to in turn
  size_t lds = 0;
  int64_t ns_per_tick = 10 << 10;  // wall clock period in ns, fixed point x 1024
};
eat_status device_limits(int dev, DeviceLimits *out);

// Launch plan of the relaxation kernel for a set of graphs.
struct Plan {
  int tpv = 0;
  int ub = 1;  // connection types in flight per lane (load-balanced expansion)
  int mode = EAT_MODE_AUTO;
  int max_rounds = 0;
  int fcap = 0;
  int bm_words = 0;
  int table_cap = 0;
  int table_bits = 0;
  int headers = EAT_HEADERS_AUTO;
  int window = 0;  // seconds, 0 = none
  int block = 1024; // threads per query
  int64_t ns_per_tick = 0;
  size_t lds = 0;
};

// Kernel variant (kKindCompact / kKindFlat / kKindGrid) for graphs g[0..n)
// and a requested eat_headers form; all graphs must share one layout kind.
eat_status exec_kind(const eat_graph *const *g, int32_t n, int headers, int *kind);
// max_v: the largest graph the kernel will see.
eat_status make_plan(const eat_run_options *ro, int32_t max_v, int device, Plan *pl);
// RunArgs fields that come from a plan.
void apply_plan(const Plan &pl, RunArgs *a);

// Orders queries for a launch: larger graphs first, then by the layout
// position of the source (nearby sources touch nearby data), and splits them
// into n_buckets contiguous buckets of nearly equal size; off receives
// n_buckets + 1 offsets.
void order_queries(const std::vector<const eat_graph *> &graphs, std::vector<QueryDev> &qs,
                   int n_buckets, std::vector<int32_t> &off);

}  // namespace eat
