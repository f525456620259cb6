// device.hpp -- descriptors shared by the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "eat.h"

namespace eat {

// One device-resident timetable (see eat_layout_view in eat.h for the arrays).
struct GraphDev {
  const int2 *vt;          // [V] per stop: first type, type count
  // [2T] per type two int4: {v, lam, a, b} as in the host layout, then
  // {first type of v, type count of v, cluster-occupancy bits 32..63, 0}.  The
  // second half lets a lane that improves v push it without another read.
  const int4 *ty;
  const int2 *hdr;         // [K + 1] hybrid (one padding entry)
  const int32_t *pool;     // departures
  // Hybrid header grid (nullptr when not built): side[T] per type
  // {v, lam, first type of v, type count of v}; grid[T * n_clusters]: one
  // int4 per (type, cluster), {t0, c, next, m}, stop-blocked and cluster-major
  // (spelled out at eat_graph_upload in eat.h);
  // tail[T] the tail stop of each type (diagnostics only).
  const int4 *side;
  const int4 *grid;
  const int32_t *tail;
  int64_t n_types;
  int32_t n_vertices;
  int32_t cluster_seconds;
  int32_t n_clusters;
  int32_t kind;            // eat_layout_kind
  int32_t horizon;         // n_clusters * cluster_seconds (< 2^24)
  float inv_cw;            // 1 / cluster_seconds, for the cluster index of a time
};

// Kernel variants by the timetable form they read: the hybrid layout's
// compact headers, the flat layout, the hybrid layout's header grid.
constexpr int kKindCompact = EAT_LAYOUT_HYBRID;
constexpr int kKindFlat = EAT_LAYOUT_FLAT;
constexpr int kKindGrid = 2;

// One query: the graph index, the source, the departure time, the caller's
// result slab, and the query's index in the caller's order (for its stats).
struct QueryDev {
  int32_t graph;
  int32_t s;
  int32_t ts;
  int32_t index;
  int32_t *arr;
};

// Arguments of one launch of the relaxation kernel.
struct RunArgs {
  const GraphDev *graphs;    // device array
  const QueryDev *queries;   // device array of nq, or nullptr: use `single`
  QueryDev single;           // the one query when queries == nullptr
  int32_t nq;
  int32_t max_rounds;        // 0: n_vertices + 2 (8 * n_vertices + 64 with a window)
  int32_t mode;              // eat_mode
  int32_t fcap;              // frontier list capacity (entries, multiple of 32)
  int32_t bm_words;          // activity bitmap words (>= ceil(V / 32) of every graph)
  // Slab-mode activity bits in HBM (nullable: in LDS): work-group w uses
  // bits_global[w * bits_stride ..], bits_stride >= bm_words.
  uint32_t *bits_global;
  int32_t bits_stride;
  int32_t table_cap;         // on-chip arrival table slots (power of two), 0 = none
  int32_t table_bits;        // log2(table_cap)
  int32_t window;            // arrival window of a round in seconds, 0 = none
  // Queries are split into n_buckets contiguous buckets (queries[buckets[b]]
  // .. queries[buckets[b+1]-1]); work-group w takes queries from bucket
  // w % n_buckets first (work-groups are dealt to the XCDs in turn, so a
  // bucket's queries share one XCD's L2), then helps the other buckets.
  const int32_t *buckets;    // device array of n_buckets + 1 offsets (batch only)
  int32_t n_buckets;
  // Batch counters (batch only; zero before the first launch, re-armed by the
  // last work-group of every launch): [0] work-groups done, [1] queries of
  // this launch that hit the round limit, [2] that count for the previous
  // completed launch, [4 + b] next query of bucket b.
  int32_t *work;
  eat_query_stats *stats;    // per query, indexed by QueryDev::index; nullable
  int32_t *n_failed;         // == work + 1 in a batch; nullable
  int64_t ns_per_tick;       // device wall clock period in ns (x 1024)
  // Per-query completion words (serving sessions; nullable): when a query has
  // finished -- its slab and statistics written and released at system scope
  // -- done[QueryDev::index] = epoch.  Host-visible (pinned) memory.
  int32_t *done;
  int32_t epoch;
  // Goal-directed queries (nonzero: the goal-directed kernel variant runs):
  // the destination of query i is targets[QueryDev::index] in a batch, or
  // single_target, -1 for every stop (answered in full by that variant too).
  int32_t goal;
  int32_t single_target;
  const int32_t *targets;    // device array (batch only)
};

constexpr int kBlock = 1024;        // threads per query (work-group), default
constexpr int kBlockSmall = 512;    // the alternatives: two queries per CU ...
constexpr int kBlockMid = 768;      // ... with 8 or 12 waves each,
constexpr int kBlockQuarter = 384;  // four queries per CU with 6 waves each,
constexpr int kBlockSixth = 256;    // six queries per CU with 4 waves each
// Queries (work-groups) of a block size that share one CU, each with that
// share of the LDS.
constexpr int queries_per_cu(int block) {
  return block == kBlock ? 1 : block == kBlockQuarter ? 4 : block == kBlockSixth ? 6 : 2;
}
// LDS a relaxation work-group holds besides the dynamic part the plan sizes
// (its counters and the start bits of the type windows).
constexpr size_t kStaticLds = 2048;
constexpr int kMaxBuckets = 32;
constexpr int kCounterWords = 4 + kMaxBuckets;

// Host-side launchers (kernels.hip).
// The kernel variant follows a.goal.
hipError_t launch_relax(const RunArgs &a, int tpv, int ub, int kind, int block, int grid, size_t lds_bytes,
                        hipStream_t stream);
hipError_t launch_zero(int32_t *p, int n, hipStream_t stream);
hipError_t launch_next_departure(const GraphDev *g_dev, int kind, const int32_t *type_ids,
                                 const int32_t *x, int32_t *out, int32_t n, hipStream_t stream);
// Fills g.grid from the compact headers (g as on the host: device pointers).
hipError_t launch_build_grid(const GraphDev &g, hipStream_t stream);
// out[qs[q].index] += fingerprint of query q's result slab (qs, graphs: device).
hipError_t launch_slab_hash(const QueryDev *qs, const GraphDev *graphs, int32_t nq, unsigned long long *out,
                            hipStream_t stream);
// Work-groups of the relaxation kernel that fit on one CU with lds_bytes of LDS.
int relax_blocks_per_cu(int tpv, int ub, int kind, int block, size_t lds_bytes, bool goal = false);

}  // namespace eat
