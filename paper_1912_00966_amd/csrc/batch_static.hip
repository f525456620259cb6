// batch_static.hip -- eat_query_batch_static: eat_query_batch without any
// device or host allocation, for callers that cannot allocate.
//
// The batch's device-side state -- graph and query descriptors, launch
// counters, bucket offsets, per-query statistics -- lives in `scratch`, a
// file-scope device array of kStaticBytes that each GPU the library runs on
// holds until the process ends; its host-side staging lives in static host
// arrays.  In host code the array's name is only a stand-in: its device
// address is fetched once per device with hipGetSymbolAddress (on the first
// call made on that device) and that address is what kernels and copies use.
// Every call on a GPU shares that GPU's array, so calls that overlap on one
// GPU race (a host mutex serializes the calls of one process); each call
// rewrites the descriptors and clears the counters before its launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "device.hpp"
#include "eat.h"
#include "internal.hpp"

using eat::GraphDev;
using eat::QueryDev;
using eat::RunArgs;

namespace {

constexpr int32_t kStaticMaxQueries = 8192;
constexpr int32_t kStaticMaxGraphs = 64;
constexpr int kMaxDevices = 64;

// Layout of the scratch array (byte offsets, each 256-byte aligned).
constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t kOffGraphs = 0;
constexpr size_t kOffQueries = kOffGraphs + align256(sizeof(GraphDev) * kStaticMaxGraphs);
constexpr size_t kOffStats = kOffQueries + align256(sizeof(QueryDev) * kStaticMaxQueries);
constexpr size_t kOffCounters = kOffStats + align256(sizeof(eat_query_stats) * kStaticMaxQueries);
constexpr size_t kOffBuckets = kOffCounters + align256(sizeof(int32_t) * eat::kCounterWords);
constexpr size_t kStaticBytes = kOffBuckets + align256(sizeof(int32_t) * (eat::kMaxBuckets + 1));

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

struct HostStage {
  GraphDev graphs[kStaticMaxGraphs];
  QueryDev queries[kStaticMaxQueries];
  int32_t buckets[eat::kMaxBuckets + 1];
  int32_t failed;
};

std::mutex g_mu;              // serializes the calls of this process
HostStage g_stage;            // host staging (no allocation per call)
unsigned char *g_scratch[kMaxDevices] = {};  // device address of `scratch` per device

}  // namespace

extern "C" eat_status eat_query_batch_static(const eat_graph *const *graphs, int32_t n_graphs,
                                             const int32_t *q_graph, const int32_t *q_src,
                                             const int32_t *q_ts, int32_t n_q, int32_t *const *arr,
                                             void *stream, const eat_run_options *ro,
                                             eat_query_stats *stats) {
  if (!graphs || n_graphs < 1) return eat::set_err(EAT_ERR_INVALID_ARGUMENT, "need at least one graph");
  if (n_graphs > kStaticMaxGraphs)
    return eat::set_err(EAT_ERR_INVALID_ARGUMENT, "at most " + std::to_string(kStaticMaxGraphs) + " graphs");
  if (n_q < 0) return eat::set_err(EAT_ERR_INVALID_ARGUMENT, "n_q must be >= 0");
  if (n_q > kStaticMaxQueries)
    return eat::set_err(EAT_ERR_INVALID_ARGUMENT, "at most " + std::to_string(kStaticMaxQueries) + " queries");
  if (n_q > 0 && (!q_graph || !q_src || !q_ts || !arr)) return eat::set_err(EAT_ERR_INVALID_ARGUMENT, "NULL query array");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return eat::set_err(EAT_ERR_DEVICE, "device index out of range");
  int32_t max_v = 1;
  for (int32_t i = 0; i < n_graphs; ++i) {
    if (!graphs[i]) return eat::set_err(EAT_ERR_INVALID_ARGUMENT, "graph " + std::to_string(i) + " is NULL");
    if (graphs[i]->device != dev)
      return eat::set_err(EAT_ERR_INVALID_ARGUMENT, "graph " + std::to_string(i) + " lives on another device");
    max_v = std::max(max_v, graphs[i]->info.n_vertices);
  }
  std::lock_guard<std::mutex> lk(g_mu);
  QueryDev *qs = g_stage.queries;
  for (int32_t i = 0; i < n_q; ++i) {
    const int32_t gi = q_graph[i];
    if (gi < 0 || gi >= n_graphs)
      return eat::set_err(EAT_ERR_INVALID_ARGUMENT, "query " + std::to_string(i) + ": graph index out of range");
    if (q_src[i] < 0 || q_src[i] >= graphs[gi]->info.n_vertices)
      return eat::set_err(EAT_ERR_INVALID_ARGUMENT, "query " + std::to_string(i) + ": source out of range");
    if (q_ts[i] < 0) return eat::set_err(EAT_ERR_INVALID_ARGUMENT, "query " + std::to_string(i) + ": ts < 0");
    if (!arr[i]) return eat::set_err(EAT_ERR_INVALID_ARGUMENT, "query " + std::to_string(i) + ": arr is NULL");
    qs[i] = QueryDev{gi, q_src[i], q_ts[i], i, arr[i]};
  }
  if (n_q == 0) return EAT_OK;
  eat_run_options chosen{};
  if (ro) chosen = *ro;
  else if (!eat::tuned_options(dev, graphs, n_graphs, n_q, &chosen)) chosen = eat::default_batch_options(dev, n_q, max_v);
  eat::Plan pl;
  eat_status st = eat::make_plan(&chosen, max_v, dev, &pl);
  if (st != EAT_OK) return st;
  int kind = 0;
  st = eat::exec_kind(graphs, n_graphs, pl.headers, &kind);
  if (st != EAT_OK) return st;
  eat::DeviceLimits lim;
  st = eat::device_limits(dev, &lim);
  if (st != EAT_OK) return st;
  if (pl.bits_global)
    return eat::set_err(EAT_ERR_UNSUPPORTED, "a graph's activity bitmap does not fit the LDS; this entry point "
                                             "has no room for it in its fixed scratch (use eat_query_batch)");

  // set-up, once per device: the device address of this device's array
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return eat::hip_err(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
    g_scratch[dev] = static_cast<unsigned char *>(p);
  }
  unsigned char *base = g_scratch[dev];
  GraphDev *d_g = reinterpret_cast<GraphDev *>(base + kOffGraphs);
  QueryDev *d_q = reinterpret_cast<QueryDev *>(base + kOffQueries);
  eat_query_stats *d_s = reinterpret_cast<eat_query_stats *>(base + kOffStats);
  int32_t *d_c = reinterpret_cast<int32_t *>(base + kOffCounters);
  int32_t *d_b = reinterpret_cast<int32_t *>(base + kOffBuckets);

  // the same launch order as eat_batch_create (in-place sorts: no allocation)
  const int per_cu = std::max(1, eat::relax_blocks_per_cu(pl.tpv, pl.ub, kind, pl.block, pl.lds));
  const int slots = lim.cus * per_cu;
  std::sort(qs, qs + n_q, [&](const QueryDev &a, const QueryDev &b) { return eat::query_before(graphs, a, b); });
  const int32_t nb = eat::bucket_offsets(n_q, std::min(lim.xccs, eat::kMaxBuckets), g_stage.buckets);
  eat::order_in_buckets(graphs, qs, g_stage.buckets, nb, eat::order_bands(pl.order, n_q, slots));
  for (int32_t i = 0; i < n_graphs; ++i) g_stage.graphs[i] = graphs[i]->desc;

  hipStream_t hs = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(d_g, g_stage.graphs, sizeof(GraphDev) * (size_t)n_graphs, hipMemcpyHostToDevice, hs));
  HIP_TRY(hipMemcpyAsync(d_q, qs, sizeof(QueryDev) * (size_t)n_q, hipMemcpyHostToDevice, hs));
  HIP_TRY(hipMemcpyAsync(d_b, g_stage.buckets, sizeof(int32_t) * (size_t)(nb + 1), hipMemcpyHostToDevice, hs));
  // the launch counters start at zero (a fill kernel, no memset node)
  HIP_TRY(eat::launch_zero(d_c, eat::kCounterWords, hs));

  RunArgs a{};
  a.graphs = d_g;
  a.queries = d_q;
  a.nq = n_q;
  eat::apply_plan(pl, &a);
  a.buckets = d_b;
  a.n_buckets = nb;
  a.work = d_c;
  a.stats = stats ? d_s : nullptr;
  a.n_failed = d_c + 1;
  const int grid = std::max(1, std::min<int>(n_q, slots));
  const hipError_t le = eat::launch_relax(a, pl.tpv, pl.ub, kind, pl.block, grid, pl.lds, hs);
  if (le != hipSuccess) return eat::hip_err(le, "relaxation launch");
  // the last work-group moved the failure count to counter word 2
  HIP_TRY(hipMemcpyAsync(&g_stage.failed, d_c + 2, sizeof(int32_t), hipMemcpyDeviceToHost, hs));
  if (stats)
    HIP_TRY(hipMemcpyAsync(stats, d_s, sizeof(eat_query_stats) * (size_t)n_q, hipMemcpyDeviceToHost, hs));
  HIP_TRY(hipStreamSynchronize(hs));
  if (g_stage.failed)
    return eat::set_err(EAT_ERR_NOT_CONVERGED, std::to_string(g_stage.failed) + " queries hit their round limit");
  return EAT_OK;
}
