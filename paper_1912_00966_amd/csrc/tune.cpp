// tune.cpp -- the autotuner of batched launches (eat_batch_tune) and the
// per-process record of its choices that eat_batch_create consults when it is
// given no run options.
//
// The launch options (threads per query, types in flight per lane, virtual
// warps, arrival window, schedule, header form) change the speed of a batch,
// never its answers: the answer of a query is unique.  The tuner runs the
// caller's batch under each candidate, fingerprints every result slab on the
// device and requires all candidates to agree, times each with HIP events on
// the caller's stream, and records the fastest under a key made of the device
// (architecture, CU count), the graphs' shapes and the batch size.  With the
// environment variable EAT_TUNE_FILE set, records are also appended to that
// file and read back by later processes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "device.hpp"
#include "eat.h"
#include "internal.hpp"

using eat::hip_err;
using eat::set_err;

namespace {

std::mutex g_mu;
std::map<std::string, eat_run_options> g_records;
bool g_file_loaded = false;

std::string tune_key(int device, const eat_graph *const *graphs, int32_t n_graphs, int32_t n_q) {
  eat::DeviceLimits lim;
  if (eat::device_limits(device, &lim) != EAT_OK) return std::string();
  std::ostringstream k;
  k << lim.name << ":" << lim.cus << "|q=" << n_q << "|g=";
  for (int32_t i = 0; i < n_graphs; ++i) {
    const eat_graph_info_t &f = graphs[i]->info;
    k << f.n_vertices << "," << f.n_types << "," << f.n_headers << "," << f.n_conn << "," << f.layout << ","
      << f.cluster_seconds << "," << (f.n_grid_entries > 0) << ";";
  }
  return k.str();
}

// One record per line: key, a tab, the ten option fields.
std::string options_text(const eat_run_options &o) {
  std::ostringstream t;
  t << o.threads_per_vertex << " " << o.mode << " " << o.max_rounds << " " << o.frontier_cap << " " << o.table_cap
    << " " << o.types_per_lane << " " << o.headers << " " << o.time_window << " " << o.threads_per_query << " "
    << o.query_order;
  return t.str();
}

void load_file_locked() {
  if (g_file_loaded) return;
  g_file_loaded = true;
  const char *path = std::getenv("EAT_TUNE_FILE");
  if (!path || !*path) return;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    const size_t tab = line.find('\t');
    if (tab == std::string::npos) continue;
    eat_run_options o{};
    std::istringstream t(line.substr(tab + 1));
    if (t >> o.threads_per_vertex >> o.mode >> o.max_rounds >> o.frontier_cap >> o.table_cap >> o.types_per_lane >>
        o.headers >> o.time_window >> o.threads_per_query >> o.query_order)
      g_records[line.substr(0, tab)] = o;
  }
}

void record(const std::string &key, const eat_run_options &o) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_file_locked();
  g_records[key] = o;
  const char *path = std::getenv("EAT_TUNE_FILE");
  if (path && *path) {
    std::ofstream out(path, std::ios::app);
    out << key << "\t" << options_text(o) << "\n";
  }
}

eat_run_options cand(int threads, int ub, int window, int tpv = 0, int mode = EAT_MODE_AUTO,
                     int headers = EAT_HEADERS_AUTO, int order = EAT_ORDER_AUTO) {
  eat_run_options o{};
  o.query_order = order;
  o.threads_per_query = threads;
  o.types_per_lane = ub;
  o.time_window = window;
  o.threads_per_vertex = tpv;
  o.mode = mode;
  o.headers = headers;
  return o;
}

// The candidates: work-group size (one query per 1024-thread work-group, two
// per CU at 768 / 512 threads, four at 384, six at 256), connection types in
// flight per lane (a wave evaluates 64 x that many (type, cluster) lookups at
// once), virtual warps of 16 / 32 lanes per active stop, the arrival window of
// a round, the topology-driven schedule, the compact header form, and the
// order in which the work-groups take the queries (locality, departure-time
// bands; timed over the caller's streams, where a launch's tail overlaps the
// next launch).
std::vector<eat_run_options> candidates() {
  return {cand(1024, 1, 7200), cand(1024, 1, 3600), cand(1024, 1, -1), cand(1024, 2, 7200),
          cand(768, 1, 7200),  cand(768, 1, 3600),  cand(512, 1, 7200), cand(512, 2, 7200),
          cand(384, 1, 7200),  cand(384, 1, 3600),  cand(256, 1, 7200),
          cand(768, 1, 7200, 0, EAT_MODE_AUTO, EAT_HEADERS_AUTO, EAT_ORDER_LOCALITY),
          cand(768, 1, 7200, 0, EAT_MODE_AUTO, EAT_HEADERS_AUTO, EAT_ORDER_BANDED),
          cand(1024, 1, 7200, 0, EAT_MODE_AUTO, EAT_HEADERS_AUTO, EAT_ORDER_LOCALITY),
          cand(1024, 1, 7200, 16), cand(1024, 1, 7200, 32),
          cand(1024, 1, 7200, 0, EAT_MODE_TOPOLOGY), cand(1024, 1, 7200, 0, EAT_MODE_AUTO, EAT_HEADERS_COMPACT)};
}

struct Cleanup {
  std::vector<eat_batch *> batches;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  unsigned long long *d_hash = nullptr;
  ~Cleanup() {
    for (auto s : streams) (void)hipStreamSynchronize(s);
    for (auto b : batches) eat_batch_free(b);
    for (auto s : streams) (void)hipStreamDestroy(s);
    for (auto e : events) (void)hipEventDestroy(e);
    if (d_hash) (void)hipFree(d_hash);
  }
};

}  // namespace

namespace eat {

bool tuned_options(int device, const eat_graph *const *graphs, int32_t n_graphs, int32_t n_q,
                   eat_run_options *out) {
  const std::string key = tune_key(device, graphs, n_graphs, n_q);
  if (key.empty()) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  load_file_locked();
  auto it = g_records.find(key);
  if (it == g_records.end()) return false;
  *out = it->second;
  return true;
}

eat_run_options default_batch_options(int device, int32_t n_q, int32_t max_v) {
  eat_run_options o{};
  o.threads_per_query = kBlockMid;
  Plan pl;
  DeviceLimits lim;
  // two queries per CU only when the batch outnumbers the CUs and the graphs
  // fit a half-LDS plan
  if (device_limits(device, &lim) != EAT_OK || n_q <= lim.cus || make_plan(&o, max_v, device, &pl) != EAT_OK)
    o.threads_per_query = 0;
  return o;
}

}  // namespace eat

extern "C" eat_status eat_batch_tune(const eat_graph *const *graphs, int32_t n_graphs, const int32_t *q_graph,
                                     const int32_t *q_src, const int32_t *q_ts, int32_t n_q, int32_t *const *arr,
                                     void *stream, const eat_tune_options *opt, eat_run_options *best,
                                     eat_tune_result *results, int32_t results_cap, int32_t *n_results) {
  if (!best) return set_err(EAT_ERR_INVALID_ARGUMENT, "best is NULL");
  if (n_results) *n_results = 0;
  if (results_cap < 0 || (results_cap > 0 && !results))
    return set_err(EAT_ERR_INVALID_ARGUMENT, "bad results array");
  eat_tune_options o{};
  if (opt) o = *opt;
  for (int r : o.reserved)
    if (r != 0) return set_err(EAT_ERR_INVALID_ARGUMENT, "reserved tune options must be zero");
  if (o.reps < 0 || o.n_streams < 0 || o.n_streams > 4)
    return set_err(EAT_ERR_INVALID_ARGUMENT, "reps must be >= 0 and n_streams 0..4");
  const int reps = o.reps ? o.reps : 3;
  const int S = o.n_streams ? o.n_streams : 1;
  if (n_q < 1) return set_err(EAT_ERR_INVALID_ARGUMENT, "need at least one query");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  hipStream_t s0 = static_cast<hipStream_t>(stream);

  Cleanup c;
  for (int k = 1; k < S; ++k) {
    hipStream_t st = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    c.streams.push_back(st);
  }
  std::vector<hipStream_t> streams{s0};
  streams.insert(streams.end(), c.streams.begin(), c.streams.end());
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  HIP_TRY(hipEventCreate(&ev0));
  c.events.push_back(ev0);
  HIP_TRY(hipEventCreate(&ev1));
  c.events.push_back(ev1);
  std::vector<hipEvent_t> joins;
  for (int k = 1; k < S; ++k) {
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c.events.push_back(e);
    joins.push_back(e);
  }
  HIP_TRY(hipMalloc(&c.d_hash, sizeof(unsigned long long) * (size_t)n_q));
  std::vector<unsigned long long> ref, got((size_t)n_q);

  float best_ms = -1.0f;
  int32_t n_done = 0;
  for (const eat_run_options &cd : candidates()) {
    // S prepared batches over the caller's slabs (runs of one batch must not overlap)
    std::vector<eat_batch *> bs;
    eat_status st = EAT_OK;
    for (int k = 0; k < S && st == EAT_OK; ++k) {
      eat_batch *b = nullptr;
      st = eat_batch_create(graphs, n_graphs, q_graph, q_src, q_ts, n_q, arr, &cd, &b);
      if (st == EAT_OK) bs.push_back(b);
    }
    if (st == EAT_ERR_UNSUPPORTED) {  // not available for these graphs (LDS, header form)
      for (auto b : bs) eat_batch_free(b);
      continue;
    }
    if (st != EAT_OK) {
      for (auto b : bs) eat_batch_free(b);
      return st;
    }
    c.batches.insert(c.batches.end(), bs.begin(), bs.end());
    // a run alone, then the fingerprints of its answers
    st = eat_batch_run(bs[0], s0);
    if (st != EAT_OK) return st;
    HIP_TRY(hipMemsetAsync(c.d_hash, 0, sizeof(unsigned long long) * (size_t)n_q, s0));
    HIP_TRY(eat::launch_slab_hash(bs[0]->args.queries, bs[0]->args.graphs, n_q, c.d_hash, s0));
    HIP_TRY(hipMemcpyAsync(got.data(), c.d_hash, sizeof(unsigned long long) * (size_t)n_q, hipMemcpyDeviceToHost,
                           s0));
    HIP_TRY(hipStreamSynchronize(s0));
    st = eat_batch_wait(bs[0], nullptr);
    if (st != EAT_OK) return st;
    if (ref.empty()) {
      ref = got;
    } else if (got != ref) {
      return set_err(EAT_ERR_DEVICE, "autotune: the options {" + std::string(options_text(cd)) +
                                         "} gave different answers than the first candidate");
    }
    // timed runs, alternating over the streams
    HIP_TRY(hipEventRecord(ev0, s0));
    for (int k = 1; k < S; ++k) HIP_TRY(hipStreamWaitEvent(streams[(size_t)k], ev0, 0));
    for (int r = 0; r < reps * S; ++r) {
      st = eat_batch_run(bs[(size_t)(r % S)], streams[(size_t)(r % S)]);
      if (st != EAT_OK) return st;
    }
    for (int k = 1; k < S; ++k) {
      HIP_TRY(hipEventRecord(joins[(size_t)k - 1], streams[(size_t)k]));
      HIP_TRY(hipStreamWaitEvent(s0, joins[(size_t)k - 1], 0));
    }
    HIP_TRY(hipEventRecord(ev1, s0));
    HIP_TRY(hipEventSynchronize(ev1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
    ms /= (float)(reps * S);
    for (auto b : bs) {
      st = eat_batch_wait(b, nullptr);
      if (st != EAT_OK) return st;
    }
    if (n_done < results_cap) results[n_done] = eat_tune_result{cd, ms, 0};
    ++n_done;
    if (best_ms < 0.0f || ms < best_ms) {
      best_ms = ms;
      *best = cd;
    }
    // the batches' device memory goes back before the next candidate
    for (auto b : bs) {
      c.batches.erase(std::find(c.batches.begin(), c.batches.end(), b));
      eat_batch_free(b);
    }
  }
  if (best_ms < 0.0f) return set_err(EAT_ERR_UNSUPPORTED, "autotune: no candidate runs on these graphs");
  if (n_results) *n_results = std::min(n_done, results_cap);
  record(tune_key(dev, graphs, n_graphs, n_q), *best);
  // leave the answers of the chosen options in the slabs (the timed runs may
  // have overlapped on the same slabs)
  eat_batch *b = nullptr;
  eat_status st = eat_batch_create(graphs, n_graphs, q_graph, q_src, q_ts, n_q, arr, best, &b);
  if (st != EAT_OK) return st;
  c.batches.push_back(b);
  st = eat_batch_run(b, s0);
  if (st == EAT_OK) st = eat_batch_wait(b, nullptr);
  return st;
}
