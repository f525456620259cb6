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

// A prepared batch: device descriptors of its graphs and queries, per-query
// statistics, launch counters, and the launch shape.
struct eat_batch {
  int device = 0;
  int32_t n_q = 0;
  int tpv = 0, ub = 1, kind = 0, block = 1024, grid = 0;
  size_t lds = 0;
  eat::RunArgs args{};
  eat_run_options options{};  // the options the batch was created with (after tuning lookup)
  void *d_buf = nullptr;
  hipEvent_t done = nullptr;
  bool ran = false;
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
  char name[64] = {};              // architecture name (tuning key)
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
  int order = EAT_ORDER_AUTO;
  bool bits_global = false;  // slab-mode activity bits in HBM (they do not fit the LDS)
  int bits_stride = 0;       // words of HBM bits per work-group
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

// Tuned launch options recorded by eat_batch_tune for a device, a set of
// graphs and a batch size (tune.cpp): true and *out filled if there is a record.
bool tuned_options(int device, const eat_graph *const *graphs, int32_t n_graphs, int32_t n_q,
                   eat_run_options *out);
// Launch options eat_batch_create uses when the caller passes none and no
// tuning record exists: 768-thread queries (two per CU) when the batch has
// more queries than the device has CUs and its largest graph (max_v stops)
// fits a half-LDS plan, else 1024-thread ones.
eat_run_options default_batch_options(int device, int32_t n_q, int32_t max_v);

// Launch order of two queries (see order_queries); ties broken by the query
// index, so any sort gives the same order.
bool query_before(const eat_graph *const *graphs, const QueryDev &a, const QueryDev &b);
// Splits n ordered queries into min(n_buckets, n) (at least 1) contiguous
// buckets of nearly equal size: off[0..nb] receives the offsets; returns nb.
int32_t bucket_offsets(int64_t n, int n_buckets, int32_t *off);

// Orders queries for a launch: larger graphs first, then by the layout
// position of the source (nearby sources touch nearby data), and splits them
// into n_buckets contiguous buckets of nearly equal size; off receives
// n_buckets + 1 offsets.
// Then each bucket's queries are reordered as order_in_buckets says.
void order_queries(const std::vector<const eat_graph *> &graphs, std::vector<QueryDev> &qs,
                   int n_buckets, std::vector<int32_t> &off, int bands);
// Inside each bucket of qs (offsets off[0..nb]): bands < 0 keeps the locality
// order; bands = 0 orders by departure time, earliest first; bands > 0 splits
// the departure-time order into that many bands of equal size, earliest band
// first, each band in the locality order.
void order_in_buckets(const eat_graph *const *graphs, QueryDev *qs, const int32_t *off, int32_t nb, int bands);
// The bands argument of order_in_buckets for a launch of n_q queries on
// `slots` work-groups in flight (resolves EAT_ORDER_AUTO).
int order_bands(int order, int32_t n_q, int64_t slots);

}  // namespace eat
