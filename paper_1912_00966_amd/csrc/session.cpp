// session.cpp -- serving sessions (continuous batching) of the C ABI.
//
// Slot memory: one device pool, carved first-fit into result slots (one
// n_vertices int32 slab per admitted query), with coalescing on release.
// Launches: each step copies the descriptors of the newly admitted queries from
// pinned host memory to the device and launches the relaxation kernel over
// them on one of n_streams streams; a step block (descriptors, counters,
// completion words, statistics, event) is reused only after its previous
// launch has finished.  When every block is in flight, a step returns
// EAT_ERR_BUSY instead of waiting.
// Completion: each query's work-group writes its statistics and then its
// completion word (system-scope release) into pinned host memory as soon as
// the query is done, so a slot finishes on its own, not when its whole step
// launch does; eat_session_poll reads those words without any HIP call.
// Result copies: eat_session_copy records an event on the caller's stream; a
// slot released before that event has passed keeps its slab range out of the
// pool until it has, so no later query overwrites a slab still being copied.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "device.hpp"
#include "eat.h"
#include "internal.hpp"

using eat::GraphDev;
using eat::QueryDev;
using eat::RunArgs;
using eat::hip_err;
using eat::set_err;

namespace {

enum SlotState : int32_t { kFree = 0, kAdmitted = 1, kLaunched = 2, kDone = 3 };

struct Slot {
  int32_t state = kFree;
  int32_t graph = 0, s = 0, ts = 0;
  int64_t off = 0;    // words into the pool
  int64_t words = 0;  // reserved words
  eat_query_stats stats{};
  hipEvent_t copy = nullptr;  // recorded by eat_session_copy on the caller's stream
};

struct StepBlock {
  QueryDev *d_q = nullptr;
  uint32_t *d_bits = nullptr;           // HBM activity bits per work-group (when they do not fit the LDS)
  int32_t *d_ctr = nullptr;
  int32_t *d_b = nullptr;               // bucket offsets
  QueryDev *h_q = nullptr;              // pinned
  int32_t *h_b = nullptr;               // pinned
  eat_query_stats *h_stats = nullptr;   // pinned, written by the kernel
  eat_query_stats *k_stats = nullptr;   // ... its device-side address
  int32_t *h_done = nullptr;            // pinned completion words, written by the kernel
  int32_t *k_done = nullptr;            // ... their device-side address
  int32_t epoch = 0;                    // value of a completion word of the current launch
  hipEvent_t done = nullptr;
  hipStream_t stream = nullptr;
  std::vector<int32_t> slots;
  std::vector<char> retired;
  size_t n_retired = 0;
  bool in_flight = false;
};

// A released slot's slab range whose result copy may still be pending.
struct Deferred {
  int64_t off, words;
  hipEvent_t copy;
};

constexpr int64_t kSlotAlignWords = 64;  // 256-byte aligned slabs

}  // namespace

struct eat_session {
  int device = 0;
  std::vector<const eat_graph *> graphs;
  GraphDev *d_graphs = nullptr;
  eat::Plan plan;
  int kind = 0;  // kernel variant
  int grid_cap = 1;
  int n_buckets = 1;
  int32_t max_step = 4096;
  int32_t *d_pool = nullptr;
  int64_t pool_words = 0;
  std::map<int64_t, int64_t> free_ranges;  // offset -> length (words)
  std::vector<Slot> slots;
  std::vector<int32_t> free_ids;
  std::deque<int32_t> admitted;
  std::deque<int32_t> finished;
  std::vector<StepBlock> blocks;
  size_t next_block = 0;
  std::vector<size_t> order;  // in-flight blocks, oldest first
  std::vector<Deferred> deferred;
  std::vector<hipEvent_t> spare_events;
};

namespace {

void destroy(eat_session *S) {
  if (!S) return;
  (void)hipSetDevice(S->device);
  (void)hipDeviceSynchronize();
  for (auto &b : S->blocks) {
    if (b.done) (void)hipEventDestroy(b.done);
    if (b.stream) (void)hipStreamDestroy(b.stream);
    if (b.h_q) (void)hipHostFree(b.h_q);
    if (b.h_b) (void)hipHostFree(b.h_b);
    if (b.h_stats) (void)hipHostFree(b.h_stats);
    if (b.h_done) (void)hipHostFree(b.h_done);
    if (b.d_q) (void)hipFree(b.d_q);
    if (b.d_bits) (void)hipFree(b.d_bits);
  }
  for (auto &sl : S->slots)
    if (sl.copy) (void)hipEventDestroy(sl.copy);
  for (auto &d : S->deferred) (void)hipEventDestroy(d.copy);
  for (auto e : S->spare_events) (void)hipEventDestroy(e);
  if (S->d_graphs) (void)hipFree(S->d_graphs);
  if (S->d_pool) (void)hipFree(S->d_pool);
  delete S;
}

void pool_give(eat_session *S, int64_t off, int64_t words);

// Returns to the pool the deferred ranges whose result copies have passed.
void reclaim(eat_session *S) {
  size_t k = 0;
  for (size_t i = 0; i < S->deferred.size(); ++i) {
    Deferred &d = S->deferred[i];
    if (hipEventQuery(d.copy) == hipSuccess) {
      pool_give(S, d.off, d.words);
      S->spare_events.push_back(d.copy);
    } else {
      S->deferred[k++] = d;
    }
  }
  S->deferred.resize(k);
}

// First-fit allocation of `words` from the pool; -1 if nothing fits.
int64_t pool_take(eat_session *S, int64_t words) {
  if (!S->deferred.empty()) reclaim(S);
  for (auto it = S->free_ranges.begin(); it != S->free_ranges.end(); ++it) {
    if (it->second < words) continue;
    const int64_t off = it->first, len = it->second;
    S->free_ranges.erase(it);
    if (len > words) S->free_ranges.emplace(off + words, len - words);
    return off;
  }
  return -1;
}

void pool_give(eat_session *S, int64_t off, int64_t words) {
  auto it = S->free_ranges.emplace(off, words).first;
  auto next = std::next(it);
  if (next != S->free_ranges.end() && it->first + it->second == next->first) {
    it->second += next->second;
    S->free_ranges.erase(next);
  }
  if (it != S->free_ranges.begin()) {
    auto prev = std::prev(it);
    if (prev->first + prev->second == it->first) {
      prev->second += it->second;
      S->free_ranges.erase(it);
    }
  }
}

void retire_slot(eat_session *S, StepBlock &b, size_t i) {
  Slot &sl = S->slots[(size_t)b.slots[i]];
  sl.stats = b.h_stats[i];
  sl.state = kDone;
  S->finished.push_back(b.slots[i]);
  b.retired[i] = 1;
  ++b.n_retired;
}

// Retires every slot whose completion word the kernel has written, and frees
// the blocks whose launches have ended.  Never blocks.
eat_status retire_ready(eat_session *S) {
  size_t k = 0;
  for (size_t oi = 0; oi < S->order.size(); ++oi) {
    StepBlock &b = S->blocks[S->order[oi]];
    for (size_t i = 0; i < b.slots.size() && b.n_retired < b.slots.size(); ++i)
      if (!b.retired[i] && __atomic_load_n(&b.h_done[i], __ATOMIC_ACQUIRE) == b.epoch) retire_slot(S, b, i);
    bool free_now = false;
    if (b.n_retired == b.slots.size()) {
      const hipError_t e = hipEventQuery(b.done);
      if (e == hipSuccess) free_now = true;
      else if (e != hipErrorNotReady) return hip_err(e, "step completion");
    }
    if (free_now) {
      b.slots.clear();
      b.in_flight = false;
    } else {
      S->order[k++] = S->order[oi];
    }
  }
  S->order.resize(k);
  return EAT_OK;
}

// Waits for every launch, then retires everything.
eat_status retire_all(eat_session *S) {
  for (size_t bi : S->order) {
    StepBlock &b = S->blocks[bi];
    const hipError_t e = hipEventSynchronize(b.done);
    if (e != hipSuccess) return hip_err(e, "step completion");
    for (size_t i = 0; i < b.slots.size(); ++i)
      if (!b.retired[i]) retire_slot(S, b, i);
    b.slots.clear();
    b.in_flight = false;
  }
  S->order.clear();
  return EAT_OK;
}

}  // namespace

extern "C" eat_status eat_session_create(const eat_graph *const *graphs, int32_t n_graphs,
                                         const eat_session_options *opt, eat_session **out) {
  if (!out) return set_err(EAT_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (!graphs || n_graphs < 1) return set_err(EAT_ERR_INVALID_ARGUMENT, "need at least one graph");
  eat_session_options o{};
  if (opt) o = *opt;
  for (int r : o.reserved)
    if (r != 0) return set_err(EAT_ERR_INVALID_ARGUMENT, "reserved session options must be zero");
  if (o.pool_bytes < 0 || o.n_streams < 0 || o.n_streams > 8 || o.max_step_queries < 0)
    return set_err(EAT_ERR_INVALID_ARGUMENT, "invalid session options");
  const int64_t pool_bytes = o.pool_bytes ? o.pool_bytes : (int64_t)256 << 20;
  const int n_streams = o.n_streams ? o.n_streams : 2;
  const int32_t max_step = o.max_step_queries ? o.max_step_queries : 4096;
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  int32_t max_v = 1;
  for (int32_t i = 0; i < n_graphs; ++i) {
    if (!graphs[i]) return set_err(EAT_ERR_INVALID_ARGUMENT, "graph " + std::to_string(i) + " is NULL");
    if (graphs[i]->device != dev) return set_err(EAT_ERR_INVALID_ARGUMENT, "graph on another device");
    max_v = std::max(max_v, graphs[i]->info.n_vertices);
  }
  eat::Plan pl;
  eat_status st = eat::make_plan(&o.run, max_v, dev, &pl);
  if (st != EAT_OK) return st;
  int kind = 0;
  st = eat::exec_kind(graphs, n_graphs, pl.headers, &kind);
  if (st != EAT_OK) return st;
  eat::DeviceLimits lim;
  st = eat::device_limits(dev, &lim);
  if (st != EAT_OK) return st;

  eat_session *S = new (std::nothrow) eat_session();
  if (!S) return set_err(EAT_ERR_OUT_OF_MEMORY, "host allocation failed");
  S->device = dev;
  S->graphs.assign(graphs, graphs + n_graphs);
  S->plan = pl;
  S->kind = kind;
  S->max_step = max_step;
  const int per_cu = std::max(1, eat::relax_blocks_per_cu(pl.tpv, pl.ub, kind, pl.block, pl.lds));
  S->grid_cap = lim.cus * per_cu;
  S->n_buckets = std::min(lim.xccs, eat::kMaxBuckets);
  S->pool_words = pool_bytes / 4 / kSlotAlignWords * kSlotAlignWords;
  auto fail = [&](eat_status s2, const std::string &m) {
    destroy(S);
    return set_err(s2, m);
  };
  if (S->pool_words < kSlotAlignWords) return fail(EAT_ERR_INVALID_ARGUMENT, "pool_bytes too small");
  if (hipMalloc(&S->d_pool, (size_t)S->pool_words * 4) != hipSuccess)
    return fail(EAT_ERR_OUT_OF_MEMORY, "hipMalloc of the slot pool failed");
  S->free_ranges.emplace(0, S->pool_words);
  std::vector<GraphDev> gd((size_t)n_graphs);
  for (int32_t i = 0; i < n_graphs; ++i) gd[(size_t)i] = graphs[i]->desc;
  if (hipMalloc(&S->d_graphs, gd.size() * sizeof(GraphDev)) != hipSuccess ||
      hipMemcpy(S->d_graphs, gd.data(), gd.size() * sizeof(GraphDev), hipMemcpyHostToDevice) != hipSuccess)
    return fail(EAT_ERR_OUT_OF_MEMORY, "graph descriptors");
  S->blocks.resize((size_t)n_streams);
  const size_t bq = eat::align_up((size_t)max_step * sizeof(QueryDev));
  const size_t bs = eat::align_up((size_t)max_step * sizeof(eat_query_stats));
  const size_t bd = eat::align_up((size_t)max_step * sizeof(int32_t));
  for (auto &b : S->blocks) {
    void *p = nullptr;
    if (hipMalloc(&p, bq + 512) != hipSuccess) return fail(EAT_ERR_OUT_OF_MEMORY, "step block");
    b.d_q = static_cast<QueryDev *>(p);
    b.d_ctr = reinterpret_cast<int32_t *>(static_cast<char *>(p) + bq);
    b.d_b = reinterpret_cast<int32_t *>(static_cast<char *>(p) + bq + 256);
    if (hipMemset(b.d_ctr, 0, 256) != hipSuccess) return fail(EAT_ERR_DEVICE, "step counters");
    if (pl.bits_global &&
        hipMalloc((void **)&b.d_bits, (size_t)S->grid_cap * (size_t)pl.bits_stride * 4) != hipSuccess)
      return fail(EAT_ERR_OUT_OF_MEMORY, "activity bits of a step");
    // statistics and completion words: coherent pinned memory the kernel writes
    const unsigned mapped = hipHostMallocMapped | hipHostMallocCoherent;
    if (hipHostMalloc((void **)&b.h_b, 256, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&b.h_q, bq, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&b.h_stats, bs, mapped) != hipSuccess ||
        hipHostMalloc((void **)&b.h_done, bd, mapped) != hipSuccess)
      return fail(EAT_ERR_OUT_OF_MEMORY, "pinned step staging");
    if (hipHostGetDevicePointer((void **)&b.k_stats, b.h_stats, 0) != hipSuccess ||
        hipHostGetDevicePointer((void **)&b.k_done, b.h_done, 0) != hipSuccess)
      return fail(EAT_ERR_DEVICE, "device address of pinned step memory");
    std::memset(b.h_done, 0, bd);
    if (hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b.done, hipEventDisableTiming) != hipSuccess)
      return fail(EAT_ERR_DEVICE, "stream or event creation");
  }
  *out = S;
  return EAT_OK;
}

extern "C" eat_status eat_session_admit(eat_session *S, int32_t graph, int32_t s, int32_t ts,
                                        int32_t *slot) {
  if (!S || !slot) return set_err(EAT_ERR_INVALID_ARGUMENT, "NULL argument");
  if (graph < 0 || graph >= (int32_t)S->graphs.size()) return set_err(EAT_ERR_INVALID_ARGUMENT, "graph index out of range");
  const int32_t V = S->graphs[(size_t)graph]->info.n_vertices;
  if (s < 0 || s >= V) return set_err(EAT_ERR_INVALID_ARGUMENT, "source out of range");
  if (ts < 0) return set_err(EAT_ERR_INVALID_ARGUMENT, "ts must be >= 0");
  const int64_t words = ((int64_t)V + kSlotAlignWords - 1) / kSlotAlignWords * kSlotAlignWords;
  const int64_t off = pool_take(S, words);
  if (off < 0) return set_err(EAT_ERR_BUSY, "no free result slot of that size");
  int32_t id;
  if (!S->free_ids.empty()) {
    id = S->free_ids.back();
    S->free_ids.pop_back();
  } else {
    id = (int32_t)S->slots.size();
    S->slots.emplace_back();
  }
  Slot &sl = S->slots[(size_t)id];
  sl.state = kAdmitted;
  sl.graph = graph;
  sl.s = s;
  sl.ts = ts;
  sl.off = off;
  sl.words = words;
  std::memset(&sl.stats, 0, sizeof(sl.stats));
  S->admitted.push_back(id);
  *slot = id;
  return EAT_OK;
}

static eat_status step_impl(eat_session *S, int32_t *n_launched);

extern "C" eat_status eat_session_step(eat_session *S, int32_t *n_launched) {
  try {
    return step_impl(S, n_launched);
  } catch (const std::bad_alloc &) {  // nothing throws across the C ABI
    return set_err(EAT_ERR_OUT_OF_MEMORY, "host allocation failed in a step");
  }
}

static eat_status step_impl(eat_session *S, int32_t *n_launched) {
  if (!S) return set_err(EAT_ERR_INVALID_ARGUMENT, "session is NULL");
  if (n_launched) *n_launched = 0;
  if (S->admitted.empty()) return EAT_OK;
  HIP_TRY(hipSetDevice(S->device));
  // a free block: the next one in turn; none free: busy (never waits)
  eat_status st = retire_ready(S);
  if (st != EAT_OK) return st;
  size_t bi = S->blocks.size();
  for (size_t k = 0; k < S->blocks.size(); ++k) {
    const size_t c = (S->next_block + k) % S->blocks.size();
    if (!S->blocks[c].in_flight) {
      bi = c;
      break;
    }
  }
  if (bi == S->blocks.size()) return set_err(EAT_ERR_BUSY, "every step of the session is in flight");
  S->next_block = (bi + 1) % S->blocks.size();
  StepBlock &b = S->blocks[bi];
  const int32_t n = (int32_t)std::min<size_t>(S->admitted.size(), (size_t)S->max_step);
  b.slots.assign(S->admitted.begin(), S->admitted.begin() + n);
  b.retired.assign((size_t)n, 0);
  b.n_retired = 0;
  b.epoch = b.epoch == INT32_MAX ? 1 : b.epoch + 1;
  S->admitted.erase(S->admitted.begin(), S->admitted.begin() + n);
  std::vector<QueryDev> qs((size_t)n);
  for (int32_t i = 0; i < n; ++i) {
    Slot &sl = S->slots[(size_t)b.slots[(size_t)i]];
    sl.state = kLaunched;
    qs[(size_t)i] = QueryDev{sl.graph, sl.s, sl.ts, i, S->d_pool + sl.off};
  }
  std::vector<int32_t> boff;
  eat::order_queries(S->graphs, qs, S->n_buckets, boff, eat::order_bands(S->plan.order, n, S->grid_cap));
  std::copy(qs.begin(), qs.end(), b.h_q);
  std::copy(boff.begin(), boff.end(), b.h_b);
  HIP_TRY(hipMemcpyAsync(b.d_q, b.h_q, sizeof(QueryDev) * (size_t)n, hipMemcpyHostToDevice, b.stream));
  HIP_TRY(hipMemcpyAsync(b.d_b, b.h_b, sizeof(int32_t) * boff.size(), hipMemcpyHostToDevice, b.stream));
  RunArgs a{};
  a.graphs = S->d_graphs;
  a.queries = b.d_q;
  a.nq = n;
  eat::apply_plan(S->plan, &a);
  a.buckets = b.d_b;
  a.n_buckets = (int32_t)boff.size() - 1;
  a.work = b.d_ctr;
  a.stats = b.k_stats;
  a.n_failed = b.d_ctr + 1;
  a.done = b.k_done;
  a.epoch = b.epoch;
  a.bits_global = b.d_bits;
  const int grid = std::max(1, std::min(n, S->grid_cap));
  hipError_t e = eat::launch_relax(a, S->plan.tpv, S->plan.ub, S->kind, S->plan.block, grid, S->plan.lds, b.stream);
  if (e != hipSuccess) return hip_err(e, "relaxation launch");
  HIP_TRY(hipEventRecord(b.done, b.stream));
  b.in_flight = true;
  S->order.push_back(bi);
  if (n_launched) *n_launched = n;
  return EAT_OK;
}

extern "C" eat_status eat_session_poll(eat_session *S, int32_t *done, int32_t cap, int32_t *n) {
  if (!S || !n || cap < 0 || (cap > 0 && !done)) return set_err(EAT_ERR_INVALID_ARGUMENT, "bad argument");
  *n = 0;
  eat_status st = retire_ready(S);
  if (st != EAT_OK) return st;
  while (*n < cap && !S->finished.empty()) {
    done[(*n)++] = S->finished.front();
    S->finished.pop_front();
  }
  return EAT_OK;
}

extern "C" eat_status eat_session_sync(eat_session *S) {
  if (!S) return set_err(EAT_ERR_INVALID_ARGUMENT, "session is NULL");
  return retire_all(S);
}

extern "C" eat_status eat_session_result(eat_session *S, int32_t slot, const int32_t **arr,
                                         int32_t *n_vertices) {
  if (!S || !arr) return set_err(EAT_ERR_INVALID_ARGUMENT, "NULL argument");
  if (slot < 0 || slot >= (int32_t)S->slots.size() || S->slots[(size_t)slot].state != kDone)
    return set_err(EAT_ERR_INVALID_ARGUMENT, "slot is not a finished query");
  const Slot &sl = S->slots[(size_t)slot];
  *arr = S->d_pool + sl.off;
  if (n_vertices) *n_vertices = S->graphs[(size_t)sl.graph]->info.n_vertices;
  return EAT_OK;
}

extern "C" eat_status eat_session_copy(eat_session *S, int32_t slot, int32_t *dst, void *stream) {
  const int32_t *src = nullptr;
  int32_t n = 0;
  eat_status st = eat_session_result(S, slot, &src, &n);
  if (st != EAT_OK) return st;
  if (!dst) return set_err(EAT_ERR_INVALID_ARGUMENT, "dst is NULL");
  HIP_TRY(hipMemcpyAsync(dst, src, (size_t)n * 4, hipMemcpyDefault, static_cast<hipStream_t>(stream)));
  Slot &sl = S->slots[(size_t)slot];
  if (!sl.copy) {
    if (!S->spare_events.empty()) {
      sl.copy = S->spare_events.back();
      S->spare_events.pop_back();
    } else {
      HIP_TRY(hipEventCreateWithFlags(&sl.copy, hipEventDisableTiming));
    }
  }
  HIP_TRY(hipEventRecord(sl.copy, static_cast<hipStream_t>(stream)));
  return EAT_OK;
}

extern "C" eat_status eat_session_query_stats(eat_session *S, int32_t slot, eat_query_stats *out) {
  if (!S || !out) return set_err(EAT_ERR_INVALID_ARGUMENT, "NULL argument");
  if (slot < 0 || slot >= (int32_t)S->slots.size() || S->slots[(size_t)slot].state != kDone)
    return set_err(EAT_ERR_INVALID_ARGUMENT, "slot is not a finished query");
  *out = S->slots[(size_t)slot].stats;
  return EAT_OK;
}

extern "C" eat_status eat_session_release(eat_session *S, int32_t slot) {
  if (!S) return set_err(EAT_ERR_INVALID_ARGUMENT, "session is NULL");
  if (slot < 0 || slot >= (int32_t)S->slots.size()) return set_err(EAT_ERR_INVALID_ARGUMENT, "slot out of range");
  Slot &sl = S->slots[(size_t)slot];
  if (sl.state == kAdmitted) {
    auto it = std::find(S->admitted.begin(), S->admitted.end(), slot);
    if (it != S->admitted.end()) S->admitted.erase(it);
  } else if (sl.state != kDone) {
    return set_err(EAT_ERR_INVALID_ARGUMENT, "slot is not finished (or already free)");
  }
  // a finished slot may still be listed as finished if it was never polled
  auto f = std::find(S->finished.begin(), S->finished.end(), slot);
  if (f != S->finished.end()) S->finished.erase(f);
  if (sl.copy && hipEventQuery(sl.copy) == hipErrorNotReady) {
    // a result copy may still read the slab: keep the range until it has passed
    S->deferred.push_back(Deferred{sl.off, sl.words, sl.copy});
    sl.copy = nullptr;
  } else {
    pool_give(S, sl.off, sl.words);
  }
  sl.state = kFree;
  S->free_ids.push_back(slot);
  return EAT_OK;
}

extern "C" void eat_session_free(eat_session *S) { destroy(S); }

// ---------------------------------------------------------------------------
// The request loop of a server, natively: open-loop arrivals, first-come
// admission, steps by the batching policy, completions polled, copied and
// released.
// ---------------------------------------------------------------------------
static eat_status serve_loop(eat_session *S, int32_t n, const int32_t *graph, const int32_t *src,
                             const int32_t *ts, const double *arrival_s, int32_t min_batch, double max_delay_s,
                             int32_t *const *copy_dst, void *copy_stream, double *latency_s,
                             eat_serve_report *rep) {
  if (!S) return set_err(EAT_ERR_INVALID_ARGUMENT, "session is NULL");
  if (n < 0 || min_batch < 1 || !(max_delay_s >= 0.0))
    return set_err(EAT_ERR_INVALID_ARGUMENT, "n >= 0, min_batch >= 1 and max_delay_s >= 0 are required");
  if (n > 0 && (!graph || !src || !ts || !arrival_s || !latency_s))
    return set_err(EAT_ERR_INVALID_ARGUMENT, "NULL request array");
  for (const Slot &sl : S->slots)
    if (sl.state == kAdmitted || sl.state == kLaunched)
      return set_err(EAT_ERR_INVALID_ARGUMENT, "the session holds admitted or unfinished queries");
  for (int32_t i = 0; i < n; ++i) {
    if (graph[i] < 0 || graph[i] >= (int32_t)S->graphs.size())
      return set_err(EAT_ERR_INVALID_ARGUMENT, "request " + std::to_string(i) + ": bad graph index");
    const int32_t V = S->graphs[(size_t)graph[i]]->info.n_vertices;
    if (src[i] < 0 || src[i] >= V || ts[i] < 0)
      return set_err(EAT_ERR_INVALID_ARGUMENT, "request " + std::to_string(i) + ": bad source or time");
    // a slot larger than the whole pool could never be admitted
    if (((int64_t)V + kSlotAlignWords - 1) / kSlotAlignWords * kSlotAlignWords > S->pool_words)
      return set_err(EAT_ERR_INVALID_ARGUMENT, "request " + std::to_string(i) + ": its result slot exceeds the pool");
    if (!(arrival_s[i] >= 0.0) || (i > 0 && arrival_s[i] < arrival_s[i - 1]))
      return set_err(EAT_ERR_INVALID_ARGUMENT, "arrival_s must be >= 0 and non-decreasing");
  }
  using Clock = std::chrono::steady_clock;
  const Clock::time_point t0 = Clock::now();
  auto now_s = [&]() { return std::chrono::duration<double>(Clock::now() - t0).count(); };
  std::deque<int32_t> waiting;                      // arrived, not admitted
  std::deque<std::pair<int32_t, double>> pending;   // admitted, not launched: (slot, admit time)
  std::vector<int32_t> req_of(S->slots.size(), -1);  // slot -> request
  std::vector<int32_t> fin(1024);
  int64_t unfinished = 0, steps = 0, launched = 0, busy = 0;
  int32_t done = 0, next = 0;
  while (done < n) {
    const double now = now_s();
    while (next < n && arrival_s[next] <= now) waiting.push_back(next++);
    while (!waiting.empty()) {
      const int32_t r = waiting.front();
      int32_t slot = -1;
      const eat_status st = eat_session_admit(S, graph[r], src[r], ts[r], &slot);
      if (st == EAT_ERR_BUSY) {
        ++busy;
        break;
      }
      if (st != EAT_OK) return st;
      waiting.pop_front();
      if ((size_t)slot >= req_of.size()) req_of.resize((size_t)slot + 1, -1);
      req_of[(size_t)slot] = r;
      pending.emplace_back(slot, now);
    }
    if (!pending.empty() &&
        (unfinished == 0 || (int32_t)pending.size() >= min_batch || now - pending.front().second >= max_delay_s)) {
      int32_t k = 0;
      const eat_status st = eat_session_step(S, &k);
      if (st != EAT_OK && st != EAT_ERR_BUSY) return st;
      if (st == EAT_OK && k > 0) {  // the oldest k admitted queries
        pending.erase(pending.begin(), pending.begin() + k);
        unfinished += k;
        launched += k;
        ++steps;
      }
    }
    int32_t nf = 0;
    eat_status st = eat_session_poll(S, fin.data(), (int32_t)fin.size(), &nf);
    if (st != EAT_OK) return st;
    if (nf > 0) {
      const double t_done = now_s();
      for (int32_t j = 0; j < nf; ++j) {
        const int32_t slot = fin[(size_t)j];
        const int32_t r = req_of[(size_t)slot];
        req_of[(size_t)slot] = -1;
        latency_s[r] = t_done - arrival_s[r];
        if (copy_dst && copy_dst[r]) {
          st = eat_session_copy(S, slot, copy_dst[r], copy_stream);
          if (st != EAT_OK) return st;
        }
        st = eat_session_release(S, slot);
        if (st != EAT_OK) return st;
        --unfinished;
        ++done;
      }
    } else if (unfinished == 0 && pending.empty() && waiting.empty() && next < n) {
      const double gap = arrival_s[next] - now_s();  // idle until the next arrival
      if (gap > 200e-6) std::this_thread::sleep_for(std::chrono::duration<double>(gap - 100e-6));
    }
  }
  if (rep) {
    rep->steps = steps;
    rep->launched = launched;
    rep->busy_waits = busy;
    rep->wall_s = now_s();
  }
  return EAT_OK;
}

extern "C" eat_status eat_session_serve(eat_session *S, int32_t n, const int32_t *graph, const int32_t *src,
                                        const int32_t *ts, const double *arrival_s, int32_t min_batch,
                                        double max_delay_s, int32_t *const *copy_dst, void *copy_stream,
                                        double *latency_s, eat_serve_report *rep) {
  try {
    return serve_loop(S, n, graph, src, ts, arrival_s, min_batch, max_delay_s, copy_dst, copy_stream, latency_s,
                      rep);
  } catch (const std::bad_alloc &) {  // nothing throws across the C ABI
    return set_err(EAT_ERR_OUT_OF_MEMORY, "host allocation failed in the request loop");
  }
}
