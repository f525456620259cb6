// capi.cpp -- the C ABI of libeat (declared in include/eat.h): graph objects,
// single queries, prepared batches, diagnostics and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "device.hpp"
#include "eat.h"
#include "internal.hpp"
#include "layout.hpp"

using eat::GraphDev;
using eat::QueryDev;
using eat::RunArgs;

namespace {
thread_local std::string g_last_error;
bool valid_tpv(int t) { return t == 1 || t == 2 || t == 4 || t == 8 || t == 16 || t == 32 || t == 64; }
}  // namespace

namespace eat {

eat_status set_err(eat_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

eat_status hip_err(hipError_t e, const char *what) {
  return set_err(EAT_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Device properties are read once per device and kept for the process: a
// plain query then costs no property query (hipGetDeviceProperties is slow).
eat_status device_limits(int dev, DeviceLimits *out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static DeviceLimits cache[kMaxDevices];
  static bool known[kMaxDevices] = {};
  if (dev < 0) return set_err(EAT_ERR_DEVICE, "no current HIP device");
  if (dev < kMaxDevices) {
    std::lock_guard<std::mutex> lk(mu);
    if (known[dev]) {
      *out = cache[dev];
      return EAT_OK;
    }
  }
  hipDeviceProp_t p;
  HIP_TRY(hipGetDeviceProperties(&p, dev));
  DeviceLimits lim;
  lim.cus = p.multiProcessorCount;
  // leave room for the kernel's static shared variables
  lim.lds = p.sharedMemPerBlock > 1024 ? p.sharedMemPerBlock - 1024 : p.sharedMemPerBlock;
  int xcc = 0;
  if (hipDeviceGetAttribute(&xcc, hipDeviceAttributeNumberOfXccs, dev) == hipSuccess && xcc > 0) lim.xccs = xcc;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
    lim.ns_per_tick = (int64_t)((1000000.0 / khz) * 1024.0);
  std::snprintf(lim.name, sizeof(lim.name), "%s", p.gcnArchName);
  if (dev < kMaxDevices) {
    std::lock_guard<std::mutex> lk(mu);
    cache[dev] = lim;
    known[dev] = true;
  }
  *out = lim;
  return EAT_OK;
}

}  // namespace eat

using eat::Plan;
using eat::set_err;
using eat::hip_err;
using eat::align_up;
using eat::DeviceLimits;
using eat::device_limits;
using eat::make_plan;



// ---------------------------------------------------------------------------
// status / version
// ---------------------------------------------------------------------------
extern "C" const char *eat_status_string(eat_status s) {
  switch (s) {
    case EAT_OK: return "ok";
    case EAT_ERR_INVALID_ARGUMENT: return "invalid argument";
    case EAT_ERR_OUT_OF_MEMORY: return "out of memory";
    case EAT_ERR_DEVICE: return "device error";
    case EAT_ERR_NOT_CONVERGED: return "not converged";
    case EAT_ERR_BUSY: return "busy";
    case EAT_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

extern "C" const char *eat_last_error(void) { return g_last_error.c_str(); }

extern "C" int32_t eat_version(void) { return 100; }

// ---------------------------------------------------------------------------
// host layout
// ---------------------------------------------------------------------------
static void fill_info(const eat_layout &L, eat_graph_info_t *o) {
  std::memset(o, 0, sizeof(*o));
  o->n_vertices = L.n_vertices;
  o->layout = L.kind;
  o->cluster_seconds = L.cluster_seconds;
  o->n_clusters = L.n_clusters;
  o->max_departure = L.max_departure;
  o->max_types_per_vertex = L.max_types_per_vertex;
  o->n_conn_input = L.n_conn_input;
  o->n_self_loops = L.n_self_loops;
  o->n_duplicates = L.n_duplicates;
  o->n_conn = L.n_conn;
  o->n_edges = L.n_edges;
  o->n_types = L.n_types;
  o->n_headers = L.n_headers;
  o->n_ap_clusters = L.n_ap;
  o->n_array_clusters = L.n_array;
  o->n_pool = (int64_t)L.pool.size() - eat::kPoolTail;
  o->n_trips = L.n_trips;
  o->n_shortcuts = L.n_shortcuts;
  o->subtrip_len = L.subtrip_len;
}

extern "C" eat_status eat_layout_build(const int32_t *u, const int32_t *v, const int32_t *t,
                                       const int32_t *lam, int64_t n_conn, int32_t n_vertices,
                                       const eat_build_options *opt, eat_layout **out) {
  if (!out) return set_err(EAT_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  eat_build_options o{};
  if (opt) o = *opt;
  eat_layout *L = new (std::nothrow) eat_layout();
  if (!L) return set_err(EAT_ERR_OUT_OF_MEMORY, "host allocation failed");
  std::string err;
  eat_status s;
  try {
    s = eat::build_layout(u, v, t, lam, n_conn, n_vertices, o, *L, &err);
  } catch (const std::bad_alloc &) {
    s = EAT_ERR_OUT_OF_MEMORY;
    err = "host allocation failed";
  }
  if (s != EAT_OK) {
    delete L;
    return set_err(s, err);
  }
  *out = L;
  return EAT_OK;
}

extern "C" eat_status eat_layout_build_trips(const int32_t *u, const int32_t *v, const int32_t *t,
                                             const int32_t *lam, const int32_t *trip, int64_t n_conn,
                                             int32_t n_vertices, const eat_build_options *opt, eat_layout **out) {
  if (!out) return set_err(EAT_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (n_conn < 0) return set_err(EAT_ERR_INVALID_ARGUMENT, "n_conn must be >= 0");
  if (n_conn > 0 && (!u || !v || !t || !lam)) return set_err(EAT_ERR_INVALID_ARGUMENT, "null connection array");
  eat_build_options o{};
  if (opt) o = *opt;
  std::string err;
  eat::SubtripConns sc;
  eat_status s;
  std::vector<int32_t> au, av, at, al;
  try {
    s = eat::add_subtrip_shortcuts(u, v, t, lam, trip, n_conn, o.subtrip_len, sc, &err);
    if (s != EAT_OK) return set_err(s, err);
    const size_t total = (size_t)n_conn + sc.u.size();
    au.reserve(total);
    av.reserve(total);
    at.reserve(total);
    al.reserve(total);
    au.assign(u, u + n_conn);
    av.assign(v, v + n_conn);
    at.assign(t, t + n_conn);
    al.assign(lam, lam + n_conn);
    au.insert(au.end(), sc.u.begin(), sc.u.end());
    av.insert(av.end(), sc.v.begin(), sc.v.end());
    at.insert(at.end(), sc.t.begin(), sc.t.end());
    al.insert(al.end(), sc.lam.begin(), sc.lam.end());
  } catch (const std::bad_alloc &) {
    return set_err(EAT_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
  o.subtrip_len = 0;  // consumed here
  s = eat_layout_build(au.data(), av.data(), at.data(), al.data(), (int64_t)au.size(), n_vertices, &o, out);
  if (s != EAT_OK) return s;
  (*out)->n_trips = sc.n_trips;
  (*out)->n_shortcuts = (int64_t)sc.u.size();
  (*out)->subtrip_len = sc.subtrip_len;
  return EAT_OK;
}

extern "C" void eat_layout_free(eat_layout *layout) { delete layout; }

extern "C" eat_status eat_layout_info(const eat_layout *layout, eat_graph_info_t *out) {
  if (!layout || !out) return set_err(EAT_ERR_INVALID_ARGUMENT, "NULL argument");
  fill_info(*layout, out);
  return EAT_OK;
}

extern "C" eat_status eat_layout_view_get(const eat_layout *L, eat_layout_view *out) {
  if (!L || !out) return set_err(EAT_ERR_INVALID_ARGUMENT, "NULL argument");
  out->layout = L->kind;
  out->n_vertices = L->n_vertices;
  out->cluster_seconds = L->cluster_seconds;
  out->n_clusters = L->n_clusters;
  out->n_types = L->n_types;
  out->n_headers = L->n_headers;
  out->n_pool = (int64_t)L->pool.size() - eat::kPoolTail;
  out->vt = L->vt.data();
  out->order = L->order.data();
  out->ty = L->ty.data();
  out->ty_mask_hi = L->kind == EAT_LAYOUT_HYBRID ? L->mask_hi.data() : nullptr;
  out->hdr = L->kind == EAT_LAYOUT_HYBRID ? L->hdr.data() : nullptr;
  out->pool = L->pool.data();
  return EAT_OK;
}

// ---------------------------------------------------------------------------
// device graph
// ---------------------------------------------------------------------------
namespace {

// Device buffer sizes of one graph.
struct GraphBytes {
  size_t vt, ty, hdr, pool, side, tail, grid, desc, stats, total;
};

GraphBytes graph_bytes(const eat_layout &L, bool with_grid) {
  const bool hybrid = L.kind == EAT_LAYOUT_HYBRID;
  const size_t T = (size_t)std::max<int64_t>(L.n_types, 1);
  GraphBytes b{};
  b.vt = align_up(L.vt.size() * 4);
  b.ty = align_up(T * 32);
  b.hdr = hybrid ? align_up((size_t)(L.n_headers + 1) * 8) : 0;
  b.pool = align_up(std::max<size_t>(L.pool.size(), 1) * 4);
  b.side = with_grid ? align_up(T * 16) : 0;
  b.tail = with_grid ? align_up(T * 4) : 0;
  b.grid = with_grid ? align_up(T * (size_t)L.n_clusters * 16) : 0;
  b.desc = align_up(sizeof(GraphDev));
  b.stats = align_up(sizeof(eat_query_stats)) + align_up(4);
  b.total = b.vt + b.ty + b.hdr + b.pool + b.side + b.tail + b.grid + b.desc + b.stats;
  return b;
}

}  // namespace

extern "C" eat_status eat_graph_upload(const eat_layout *L, const eat_build_options *opt, void *stream,
                                       eat_graph **out) {
  if (!L || !out) return set_err(EAT_ERR_INVALID_ARGUMENT, "NULL argument");
  *out = nullptr;
  const int32_t header_grid = opt ? opt->header_grid : 0;
  if (header_grid != 0 && header_grid != -1) return set_err(EAT_ERR_INVALID_ARGUMENT, "header_grid must be 0 or -1");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
    return set_err(EAT_ERR_DEVICE, "no HIP device available");
  eat_graph *g = new (std::nothrow) eat_graph();
  if (!g) return set_err(EAT_ERR_OUT_OF_MEMORY, "host allocation failed");
  HIP_TRY(hipGetDevice(&g->device));
  fill_info(*L, &g->info);
  g->rank.assign((size_t)L->n_vertices, 0);
  for (int32_t r = 0; r < L->n_vertices; ++r) g->rank[(size_t)L->order[(size_t)r]] = r;

  const bool hybrid = L->kind == EAT_LAYOUT_HYBRID;
  const bool need_hi = hybrid && L->n_clusters > 32;
  const int64_t T = L->n_types;
  // grid entries address pool arrays with 30 bits and are indexed with 31
  bool with_grid = hybrid && header_grid == 0 && T > 0 && T * (int64_t)L->n_clusters < ((int64_t)1 << 31) &&
                   (int64_t)L->pool.size() < ((int64_t)1 << 30);
  GraphBytes b = graph_bytes(*L, with_grid);
  hipError_t e = hipMalloc(&g->d_buf, b.total);
  if (e != hipSuccess && with_grid) {  // the grid is an accelerator: go without it
    (void)hipGetLastError();
    with_grid = false;
    b = graph_bytes(*L, false);
    e = hipMalloc(&g->d_buf, b.total);
  }
  if (e != hipSuccess) {
    delete g;
    return set_err(EAT_ERR_OUT_OF_MEMORY, std::string("hipMalloc of the graph failed: ") + hipGetErrorString(e));
  }
  char *p = static_cast<char *>(g->d_buf);
  auto take = [&](size_t n) {
    char *q = p;
    p += n;
    return q;
  };
  g->desc.vt = reinterpret_cast<const int2 *>(take(b.vt));
  g->desc.ty = reinterpret_cast<const int4 *>(take(b.ty));
  g->desc.hdr = hybrid ? reinterpret_cast<const int2 *>(take(b.hdr)) : nullptr;
  g->desc.pool = reinterpret_cast<const int32_t *>(take(b.pool));
  g->desc.side = with_grid ? reinterpret_cast<const int4 *>(take(b.side)) : nullptr;
  g->desc.tail = with_grid ? reinterpret_cast<const int32_t *>(take(b.tail)) : nullptr;
  g->desc.grid = with_grid ? reinterpret_cast<const int4 *>(take(b.grid)) : nullptr;
  g->d_desc = reinterpret_cast<GraphDev *>(take(b.desc));
  g->d_stats = reinterpret_cast<eat_query_stats *>(take(align_up(sizeof(eat_query_stats))));
  g->d_failed = reinterpret_cast<int32_t *>(take(align_up(4)));
  g->desc.n_types = T;
  g->desc.n_vertices = L->n_vertices;
  g->desc.cluster_seconds = L->cluster_seconds;
  g->desc.n_clusters = L->n_clusters;
  g->desc.kind = L->kind;
  g->desc.horizon = (int32_t)std::min<int64_t>((int64_t)L->n_clusters * L->cluster_seconds, INT32_MAX);
  g->desc.inv_cw = 1.0f / (float)L->cluster_seconds;
  g->info.device_bytes = (int64_t)b.total;
  g->info.n_grid_entries = with_grid ? T * (int64_t)L->n_clusters : 0;

  const hipStream_t hs = static_cast<hipStream_t>(stream);
  // host staging of the type records; it lives until the stream has finished
  std::vector<int32_t> ty2, side, tail;
  auto up = [&](const void *dst, const void *src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(const_cast<void *>(dst), src, bytes, hipMemcpyHostToDevice, hs);
  };
  hipError_t ue = hipSuccess;
  if (ue == hipSuccess) ue = up(g->desc.vt, L->vt.data(), L->vt.size() * 4);
  if (ue == hipSuccess && T > 0) {
    // 32-byte type records; with the grid also the 16-byte side records and
    // the tail stop of every type
    try {
      ty2.resize((size_t)T * 8);
      if (with_grid) {
        side.resize((size_t)T * 4);
        tail.resize((size_t)T);
      }
    } catch (const std::bad_alloc &) {
      ue = hipErrorOutOfMemory;
    }
    if (ue == hipSuccess) {
      for (int64_t j = 0; j < T; ++j) {
        const int32_t *r = &L->ty[(size_t)(4 * j)];
        int32_t *o = &ty2[(size_t)(8 * j)];
        o[0] = r[0];
        o[1] = r[1];
        o[2] = r[2];
        o[3] = r[3];
        o[4] = L->vt[(size_t)2 * r[0]];
        o[5] = L->vt[(size_t)2 * r[0] + 1];
        o[6] = need_hi ? (int32_t)L->mask_hi[(size_t)j] : 0;
        o[7] = 0;
        if (with_grid) {
          int32_t *sd = &side[(size_t)(4 * j)];
          sd[0] = r[0];
          sd[1] = r[1];
          sd[2] = o[4];
          sd[3] = o[5];
        }
      }
      if (with_grid)
        for (int32_t u = 0; u < L->n_vertices; ++u) {
          const int32_t b0 = L->vt[(size_t)2 * u], n = L->vt[(size_t)2 * u + 1];
          for (int32_t j = b0; j < b0 + n; ++j) tail[(size_t)j] = u;
        }
      ue = up(g->desc.ty, ty2.data(), (size_t)T * 32);
      if (ue == hipSuccess && with_grid) ue = up(g->desc.side, side.data(), (size_t)T * 16);
      if (ue == hipSuccess && with_grid) ue = up(g->desc.tail, tail.data(), (size_t)T * 4);
    }
  }
  if (ue == hipSuccess && hybrid) {
    ue = up(g->desc.hdr, L->hdr.data(), (size_t)L->n_headers * 8);
    if (ue == hipSuccess) ue = hipMemsetAsync(const_cast<int2 *>(g->desc.hdr) + L->n_headers, 0, 8, hs);
  }
  if (ue == hipSuccess) ue = up(g->desc.pool, L->pool.data(), L->pool.size() * 4);
  if (ue == hipSuccess) ue = up(g->d_desc, &g->desc, sizeof(GraphDev));
  if (ue == hipSuccess) ue = hipMemsetAsync(g->d_failed, 0, sizeof(int32_t), hs);
  if (ue == hipSuccess && with_grid) ue = eat::launch_build_grid(g->desc, hs);
  if (ue == hipSuccess) ue = hipStreamSynchronize(hs);
  if (ue != hipSuccess) {
    (void)hipFree(g->d_buf);
    delete g;
    return hip_err(ue, "graph upload");
  }
  *out = g;
  return EAT_OK;
}

extern "C" eat_status eat_graph_build(const int32_t *u, const int32_t *v, const int32_t *t,
                                      const int32_t *lam, int64_t n_conn, int32_t n_vertices,
                                      const eat_build_options *opt, void *stream, eat_graph **out) {
  if (!out) return set_err(EAT_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  eat_layout *L = nullptr;
  eat_status s = eat_layout_build(u, v, t, lam, n_conn, n_vertices, opt, &L);
  if (s != EAT_OK) return s;
  s = eat_graph_upload(L, opt, stream, out);
  eat_layout_free(L);
  return s;
}

extern "C" eat_status eat_graph_build_trips(const int32_t *u, const int32_t *v, const int32_t *t,
                                            const int32_t *lam, const int32_t *trip, int64_t n_conn,
                                            int32_t n_vertices, const eat_build_options *opt, void *stream,
                                            eat_graph **out) {
  if (!out) return set_err(EAT_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  eat_layout *L = nullptr;
  eat_status s = eat_layout_build_trips(u, v, t, lam, trip, n_conn, n_vertices, opt, &L);
  if (s != EAT_OK) return s;
  s = eat_graph_upload(L, opt, stream, out);
  eat_layout_free(L);
  return s;
}

extern "C" void eat_graph_free(eat_graph *g) {
  if (!g) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(g->device);
  (void)hipDeviceSynchronize();
  (void)hipFree(g->d_buf);
  (void)hipSetDevice(cur);
  delete g;
}

extern "C" eat_status eat_graph_info(const eat_graph *g, eat_graph_info_t *out) {
  if (!g || !out) return set_err(EAT_ERR_INVALID_ARGUMENT, "NULL argument");
  *out = g->info;
  return EAT_OK;
}

extern "C" eat_status eat_graph_failures(const eat_graph *g, int32_t *count) {
  if (!g || !count) return set_err(EAT_ERR_INVALID_ARGUMENT, "NULL argument");
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != g->device) HIP_TRY(hipSetDevice(g->device));
  const hipError_t e = hipMemcpy(count, g->d_failed, sizeof(int32_t), hipMemcpyDeviceToHost);
  if (cur != g->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return hip_err(e, "reading the failure count");
  return EAT_OK;
}

// ---------------------------------------------------------------------------
// run options
// ---------------------------------------------------------------------------
namespace eat {

// LDS bytes: two frontier lists of (item, type begin, type count) and the
// expand list of (item, type begin, type count, arrival), fcap entries each,
// plus the arrival table or the stop bitmap.
static size_t lists_lds(int fcap) { return (size_t)fcap * 40; }
static size_t table_lds(int H, int fcap) { return (size_t)H * 8 + lists_lds(fcap); }

eat_status exec_kind(const eat_graph *const *g, int32_t n, int headers, int *kind) {
  if (headers < EAT_HEADERS_AUTO || headers > EAT_HEADERS_COMPACT)
    return set_err(EAT_ERR_INVALID_ARGUMENT, "unknown header form");
  const int layout = g[0]->info.layout;
  bool all_grid = true;
  for (int32_t i = 0; i < n; ++i) {
    if (g[i]->info.layout != layout)
      return set_err(EAT_ERR_UNSUPPORTED, "all graphs of one call must share a layout kind");
    all_grid = all_grid && g[i]->desc.grid != nullptr;
  }
  if (layout == EAT_LAYOUT_FLAT) {
    *kind = kKindFlat;
    return EAT_OK;
  }
  if (headers == EAT_HEADERS_GRID && !all_grid)
    return set_err(EAT_ERR_UNSUPPORTED, "the header grid was requested but a graph was built without one");
  *kind = (headers != EAT_HEADERS_COMPACT && all_grid) ? kKindGrid : kKindCompact;
  return EAT_OK;
}

eat_status make_plan(const eat_run_options *ro, int32_t max_v, int device, Plan *pl) {
  eat_run_options o{};
  if (ro) o = *ro;
  for (int r : o.reserved)
    if (r != 0) return set_err(EAT_ERR_INVALID_ARGUMENT, "reserved run options must be zero");
  if (o.mode < EAT_MODE_AUTO || o.mode > EAT_MODE_TOPOLOGY) return set_err(EAT_ERR_INVALID_ARGUMENT, "unknown mode");
  if (o.max_rounds < 0) return set_err(EAT_ERR_INVALID_ARGUMENT, "max_rounds must be >= 0");
  if (o.threads_per_vertex != 0 && !valid_tpv(o.threads_per_vertex))
    return set_err(EAT_ERR_INVALID_ARGUMENT, "threads_per_vertex must be 0 or a power of two up to 64");
  if (o.frontier_cap < 0) return set_err(EAT_ERR_INVALID_ARGUMENT, "frontier_cap must be >= 0");
  const bool table_auto = o.table_cap == 0;
  if (o.table_cap < -1 || (o.table_cap > 0 && ((o.table_cap & (o.table_cap - 1)) || o.table_cap < 64)))
    return set_err(EAT_ERR_INVALID_ARGUMENT, "table_cap must be 0, -1 or a power of two >= 64");
  // 0 = load-balanced expansion (one connection type per lane)
  pl->tpv = o.threads_per_vertex;
  if (o.types_per_lane < 0 || o.types_per_lane > 3)
    return set_err(EAT_ERR_INVALID_ARGUMENT, "types_per_lane must be 0..3");
  pl->ub = o.types_per_lane ? o.types_per_lane : 1;
  pl->mode = o.mode;
  if (o.headers < EAT_HEADERS_AUTO || o.headers > EAT_HEADERS_COMPACT)
    return set_err(EAT_ERR_INVALID_ARGUMENT, "unknown header form");
  pl->headers = o.headers;
  if (o.time_window < -1) return set_err(EAT_ERR_INVALID_ARGUMENT, "time_window must be >= -1");
  if (o.threads_per_query != 0 && o.threads_per_query != kBlock && o.threads_per_query != kBlockSmall &&
      o.threads_per_query != kBlockMid && o.threads_per_query != kBlockQuarter && o.threads_per_query != kBlockSixth)
    return set_err(EAT_ERR_INVALID_ARGUMENT, "threads_per_query must be 0, 256, 384, 512, 768 or 1024");
  pl->block = o.threads_per_query ? o.threads_per_query : kBlock;
  if (pl->block != kBlock && o.threads_per_vertex != 0)
    return set_err(EAT_ERR_INVALID_ARGUMENT, "threads_per_query 512 or 768 needs threads_per_vertex 0");
  if ((pl->block == kBlockMid || pl->block == kBlockQuarter || pl->block == kBlockSixth) && pl->ub != 1)
    return set_err(EAT_ERR_INVALID_ARGUMENT, "threads_per_query 256, 384 and 768 run one connection type per lane");
  pl->window = o.time_window == 0 ? 7200 : (o.time_window < 0 ? 0 : o.time_window);
  if (o.query_order < EAT_ORDER_AUTO || o.query_order > EAT_ORDER_BANDED)
    return set_err(EAT_ERR_INVALID_ARGUMENT, "unknown query order");
  pl->order = o.query_order;
  pl->max_rounds = o.max_rounds;
  pl->bm_words = (max_v + 31) / 32;
  const int qpc = queries_per_cu(pl->block);  // work-groups sharing a CU
  const bool small = qpc > 1;
  // default list capacity: the largest that still leaves room for a
  // 16,384-slot table (1024 threads) or an 8,192-slot one (512, 768 threads);
  // with four or six queries per CU, a 4,096- or 2,048-slot table
  int fcap = o.frontier_cap ? o.frontier_cap : (qpc >= 4 ? 128 : small ? 256 : 704);
  // a multiple of 64, at least 64: a sweep stages the active items of 64
  // consecutive items at once, which must fit an empty list
  fcap = (fcap + 63) / 64 * 64;
  DeviceLimits lim;
  eat_status s = device_limits(device, &lim);
  if (s != EAT_OK) return s;
  int H = 0;
  if (table_auto) {
    H = 64;
    while (H < 16384 && H < 2 * max_v) H <<= 1;
  } else if (o.table_cap > 0) {
    H = o.table_cap;
  }
  // a frontier never holds more items than there are stops (or table slots)
  const int items = std::max(64, (std::max(max_v, H) + 63) / 64 * 64);
  fcap = std::min(fcap, items);
  // work-groups that share a CU split its LDS
  const size_t budget = (small ? lim.lds / (size_t)qpc : lim.lds) - kStaticLds;
  // slab mode (no table, or a table that overflowed): one activity bit per
  // stop, in LDS while it fits, else in a region of HBM per work-group
  pl->bits_global = (size_t)pl->bm_words * 4 + lists_lds(fcap) > budget;
  if (pl->bits_global && small)
    return set_err(EAT_ERR_UNSUPPORTED, "a graph whose activity bitmap does not fit the LDS share of a "
                                        "smaller work-group runs 1024-thread queries (threads_per_query 0 or 1024)");
  pl->bits_stride = (pl->bm_words + 63) / 64 * 64;
  const size_t slab_lds = (pl->bits_global ? 0 : (size_t)pl->bm_words * 4) + lists_lds(fcap);
  auto need = [&](int h) { return std::max(table_lds(h, fcap), slab_lds); };
  while (table_auto && H >= 64 && need(H) > budget) H >>= 1;
  if (H < 64) H = 0;
  if (H && need(H) + kStaticLds > lim.lds)
    return set_err(EAT_ERR_UNSUPPORTED, "table_cap too large for the device's LDS");
  pl->table_cap = H;
  pl->ns_per_tick = lim.ns_per_tick;
  pl->table_bits = 0;
  while (H && (1 << pl->table_bits) < H) ++pl->table_bits;
  pl->fcap = fcap;
  pl->lds = H ? need(H) : slab_lds;
  if (pl->lds + kStaticLds > lim.lds)
    return set_err(EAT_ERR_UNSUPPORTED, "frontier lists too large for the device's LDS (" +
                                            std::to_string(pl->lds) + " bytes needed, " +
                                            std::to_string(lim.lds) + " available)");
  return EAT_OK;
}

bool query_before(const eat_graph *const *graphs, const QueryDev &a, const QueryDev &b) {
  const eat_graph *ga = graphs[(size_t)a.graph], *gb = graphs[(size_t)b.graph];
  if (ga->info.n_vertices != gb->info.n_vertices) return ga->info.n_vertices > gb->info.n_vertices;
  if (a.graph != b.graph) return a.graph < b.graph;
  const int32_t ra = ga->rank[(size_t)a.s], rb = gb->rank[(size_t)b.s];
  if (ra != rb) return ra < rb;
  return a.index < b.index;
}

int32_t bucket_offsets(int64_t n, int n_buckets, int32_t *off) {
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(n_buckets, std::max<int64_t>(n, 1)));
  for (int b = 0; b <= nb; ++b) off[b] = (int32_t)(n * b / nb);
  return nb;
}

void order_in_buckets(const eat_graph *const *graphs, QueryDev *qs, const int32_t *off, int32_t nb, int bands) {
  if (bands < 0) return;
  for (int32_t b = 0; b < nb; ++b) {
    QueryDev *q0 = qs + off[b];
    const int64_t n = off[b + 1] - off[b];
    std::sort(q0, q0 + n, [](const QueryDev &x, const QueryDev &y) {
      return x.ts != y.ts ? x.ts < y.ts : x.index < y.index;
    });
    for (int k = 0; k < bands; ++k)  // inside a band of departure times: the locality order
      std::sort(q0 + n * k / bands, q0 + n * (k + 1) / bands,
                [&](const QueryDev &x, const QueryDev &y) { return query_before(graphs, x, y); });
  }
}

int order_bands(int order, int32_t n_q, int64_t slots) {
  if (order == EAT_ORDER_LOCALITY) return -1;
  if (order == EAT_ORDER_LONGEST_FIRST) return 0;
  if (order == EAT_ORDER_BANDED) return 4;
  return (int64_t)n_q > slots ? 0 : -1;  // auto
}

void order_queries(const std::vector<const eat_graph *> &graphs, std::vector<QueryDev> &qs,
                   int n_buckets, std::vector<int32_t> &off, int bands) {
  const eat_graph *const *g = graphs.data();
  std::sort(qs.begin(), qs.end(), [&](const QueryDev &a, const QueryDev &b) { return query_before(g, a, b); });
  off.assign((size_t)std::max(1, n_buckets) + 1, 0);
  const int32_t nb = bucket_offsets((int64_t)qs.size(), n_buckets, off.data());
  off.resize((size_t)nb + 1);
  order_in_buckets(g, qs.data(), off.data(), nb, bands);
}

void apply_plan(const Plan &pl, RunArgs *a) {
  a->max_rounds = pl.max_rounds;
  a->window = pl.window;
  a->mode = pl.mode;
  a->fcap = pl.fcap;
  a->bm_words = pl.bm_words;
  a->bits_stride = pl.bits_stride;
  a->table_cap = pl.table_cap;
  a->table_bits = pl.table_bits;
  a->ns_per_tick = pl.ns_per_tick;
}

}  // namespace eat


// ---------------------------------------------------------------------------
// single query
// ---------------------------------------------------------------------------
// Goal-directed queries run the type-window kernels with one connection type
// per lane.
static eat_status goal_plan(Plan *pl) {
  if (pl->tpv != 0)
    return set_err(EAT_ERR_UNSUPPORTED, "goal-directed queries run with threads_per_vertex 0 (type windows)");
  pl->ub = 1;
  return EAT_OK;
}

// One query; target = -1: every stop, else a goal-directed query.
static eat_status query_impl(const eat_graph *g, int32_t s, int32_t ts, int32_t target, int32_t *arr,
                             void *stream, const eat_run_options *ro, eat_query_stats *stats) {
  if (!g) return set_err(EAT_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (!arr) return set_err(EAT_ERR_INVALID_ARGUMENT, "arr is NULL");
  if (s < 0 || s >= g->info.n_vertices) return set_err(EAT_ERR_INVALID_ARGUMENT, "source out of range");
  if (ts < 0) return set_err(EAT_ERR_INVALID_ARGUMENT, "ts must be >= 0");
  if (target < -1 || target >= g->info.n_vertices)
    return set_err(EAT_ERR_INVALID_ARGUMENT, "destination out of range");
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != g->device) return set_err(EAT_ERR_INVALID_ARGUMENT, "graph lives on another device than the current one");
  Plan pl;
  eat_status st = make_plan(ro, g->info.n_vertices, g->device, &pl);
  if (st != EAT_OK) return st;
  if (target >= 0 && (st = goal_plan(&pl)) != EAT_OK) return st;
  int kind = 0;
  st = eat::exec_kind(&g, 1, pl.headers, &kind);
  if (st != EAT_OK) return st;
  RunArgs a{};
  a.graphs = g->d_desc;
  a.queries = nullptr;
  a.single = QueryDev{0, s, ts, 0, arr};
  a.goal = target >= 0 ? 1 : 0;
  a.single_target = target;
  a.buckets = nullptr;
  a.n_buckets = 1;
  a.nq = 1;
  eat::apply_plan(pl, &a);
  a.work = nullptr;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  eat_graph *gm = const_cast<eat_graph *>(g);
  // activity bits that do not fit the LDS: a stream-ordered region of HBM,
  // freed after the launch in stream order
  if (pl.bits_global) {
    HIP_TRY(hipMallocAsync(reinterpret_cast<void **>(&a.bits_global), (size_t)pl.bits_stride * 4, hs));
  }
  auto launch = [&]() -> hipError_t {
    hipError_t e = eat::launch_relax(a, pl.tpv, pl.ub, kind, pl.block, 1, pl.lds, hs);
    if (a.bits_global) {
      const hipError_t f = hipFreeAsync(a.bits_global, hs);
      if (e == hipSuccess) e = f;
    }
    return e;
  };
  if (!stats) {
    a.stats = nullptr;
    a.n_failed = g->d_failed;  // read by eat_graph_failures
    hipError_t e = launch();
    if (e != hipSuccess) return hip_err(e, "relaxation launch");
    return EAT_OK;
  }
  std::lock_guard<std::mutex> lk(gm->mu);
  a.stats = gm->d_stats;
  a.n_failed = nullptr;
  hipError_t e = launch();
  if (e != hipSuccess) return hip_err(e, "relaxation launch");
  HIP_TRY(hipMemcpyAsync(stats, gm->d_stats, sizeof(eat_query_stats), hipMemcpyDeviceToHost, hs));
  HIP_TRY(hipStreamSynchronize(hs));
  if (stats->status != EAT_OK) return set_err(EAT_ERR_NOT_CONVERGED, "query hit its round limit");
  return EAT_OK;
}

extern "C" eat_status eat_query(const eat_graph *g, int32_t s, int32_t ts, int32_t *arr,
                                void *stream, const eat_run_options *ro, eat_query_stats *stats) {
  return query_impl(g, s, ts, -1, arr, stream, ro, stats);
}

extern "C" eat_status eat_query_goal(const eat_graph *g, int32_t s, int32_t ts, int32_t d, int32_t *arr,
                                     void *stream, const eat_run_options *ro, eat_query_stats *stats) {
  if (g && (d < 0 || d >= g->info.n_vertices)) return set_err(EAT_ERR_INVALID_ARGUMENT, "destination out of range");
  return query_impl(g, s, ts, d, arr, stream, ro, stats);
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
// q_dst (nullable): per query a destination, or -1 for every stop.
static eat_status batch_create(const eat_graph *const *graphs, int32_t n_graphs, const int32_t *q_graph,
                               const int32_t *q_src, const int32_t *q_ts, const int32_t *q_dst, int32_t n_q,
                               int32_t *const *arr, const eat_run_options *ro, eat_batch **out) {
  if (!out) return set_err(EAT_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (!graphs || n_graphs < 1) return set_err(EAT_ERR_INVALID_ARGUMENT, "need at least one graph");
  if (n_q < 0) return set_err(EAT_ERR_INVALID_ARGUMENT, "n_q must be >= 0");
  if (n_q > 0 && (!q_graph || !q_src || !q_ts || !arr))
    return set_err(EAT_ERR_INVALID_ARGUMENT, "NULL query array");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  int32_t max_v = 1;
  for (int32_t i = 0; i < n_graphs; ++i) {
    if (!graphs[i]) return set_err(EAT_ERR_INVALID_ARGUMENT, "graph " + std::to_string(i) + " is NULL");
    if (graphs[i]->device != dev)
      return set_err(EAT_ERR_INVALID_ARGUMENT, "graph " + std::to_string(i) + " lives on another device");
  }
  std::vector<QueryDev> qs((size_t)n_q);
  bool goal = false;
  for (int32_t i = 0; i < n_q; ++i) {
    const int32_t gi = q_graph[i];
    if (gi < 0 || gi >= n_graphs) return set_err(EAT_ERR_INVALID_ARGUMENT, "query " + std::to_string(i) + ": graph index out of range");
    const eat_graph *g = graphs[gi];
    if (q_src[i] < 0 || q_src[i] >= g->info.n_vertices)
      return set_err(EAT_ERR_INVALID_ARGUMENT, "query " + std::to_string(i) + ": source out of range");
    if (q_ts[i] < 0) return set_err(EAT_ERR_INVALID_ARGUMENT, "query " + std::to_string(i) + ": ts < 0");
    if (!arr[i]) return set_err(EAT_ERR_INVALID_ARGUMENT, "query " + std::to_string(i) + ": arr is NULL");
    const int32_t d = q_dst ? q_dst[i] : -1;
    if (d < -1 || d >= g->info.n_vertices)
      return set_err(EAT_ERR_INVALID_ARGUMENT, "query " + std::to_string(i) + ": destination out of range");
    qs[(size_t)i] = QueryDev{gi, q_src[i], q_ts[i], i, arr[i]};
    goal = goal || d >= 0;
    max_v = std::max(max_v, g->info.n_vertices);
  }
  // no options: the tuned record for this device, graph set and batch size,
  // else the defaults
  eat_run_options chosen{};
  if (ro) chosen = *ro;
  else if (!eat::tuned_options(dev, graphs, n_graphs, n_q, &chosen)) chosen = eat::default_batch_options(dev, n_q, max_v);
  if (goal && !ro && chosen.threads_per_vertex != 0) chosen = eat::default_batch_options(dev, n_q, max_v);
  Plan pl;
  eat_status st = make_plan(&chosen, max_v, dev, &pl);
  if (st != EAT_OK) return st;
  if (goal && (st = goal_plan(&pl)) != EAT_OK) return st;
  int kind = 0;
  st = eat::exec_kind(graphs, n_graphs, pl.headers, &kind);
  if (st != EAT_OK) return st;
  DeviceLimits lim;
  st = device_limits(dev, &lim);
  if (st != EAT_OK) return st;
  const int per_cu = std::max(1, eat::relax_blocks_per_cu(pl.tpv, pl.ub, kind, pl.block, pl.lds, goal));
  const int slots = lim.cus * per_cu;  // work-groups in flight
  std::vector<int32_t> boff;
  eat::order_queries(std::vector<const eat_graph *>(graphs, graphs + n_graphs), qs,
                     std::min(lim.xccs, eat::kMaxBuckets), boff, eat::order_bands(pl.order, n_q, slots));
  const int nb = (int)boff.size() - 1;

  eat_batch *b = new (std::nothrow) eat_batch();
  if (!b) return set_err(EAT_ERR_OUT_OF_MEMORY, "host allocation failed");
  b->device = dev;
  b->n_q = n_q;
  b->tpv = pl.tpv;
  b->ub = pl.ub;
  b->kind = kind;
  b->block = pl.block;
  b->lds = pl.lds;
  b->options = chosen;
  const size_t b_g = align_up((size_t)n_graphs * sizeof(GraphDev));
  const size_t b_q = align_up(std::max<size_t>((size_t)n_q, 1) * sizeof(QueryDev));
  const size_t b_s = align_up(std::max<size_t>((size_t)n_q, 1) * sizeof(eat_query_stats));
  const size_t b_c = align_up(eat::kCounterWords * sizeof(int32_t));
  const size_t b_b = align_up(boff.size() * sizeof(int32_t));
  const int grid = std::max(1, std::min<int>(n_q, slots));
  const size_t b_bits = pl.bits_global ? align_up((size_t)grid * (size_t)pl.bits_stride * 4) : 0;
  const size_t b_t = goal ? align_up((size_t)n_q * sizeof(int32_t)) : 0;  // destinations, in query order
  hipError_t e = hipMalloc(&b->d_buf, b_g + b_q + b_s + b_c + b_b + b_bits + b_t);
  if (e != hipSuccess) {
    delete b;
    return set_err(EAT_ERR_OUT_OF_MEMORY, "hipMalloc of the batch failed");
  }
  char *p = static_cast<char *>(b->d_buf);
  GraphDev *d_g = reinterpret_cast<GraphDev *>(p);
  QueryDev *d_q = reinterpret_cast<QueryDev *>(p + b_g);
  eat_query_stats *d_s = reinterpret_cast<eat_query_stats *>(p + b_g + b_q);
  int32_t *d_c = reinterpret_cast<int32_t *>(p + b_g + b_q + b_s);
  int32_t *d_b = reinterpret_cast<int32_t *>(p + b_g + b_q + b_s + b_c);
  std::vector<GraphDev> gd((size_t)n_graphs);
  for (int32_t i = 0; i < n_graphs; ++i) gd[(size_t)i] = graphs[i]->desc;
  e = hipMemcpy(d_g, gd.data(), gd.size() * sizeof(GraphDev), hipMemcpyHostToDevice);
  if (e == hipSuccess && n_q > 0) e = hipMemcpy(d_q, qs.data(), qs.size() * sizeof(QueryDev), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(d_s, 0, b_s + b_c);
  if (e == hipSuccess) e = hipMemcpy(d_b, boff.data(), boff.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  int32_t *d_t = goal ? reinterpret_cast<int32_t *>(p + b_g + b_q + b_s + b_c + b_b + b_bits) : nullptr;
  if (e == hipSuccess && goal) e = hipMemcpy(d_t, q_dst, (size_t)n_q * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipFree(b->d_buf);
    delete b;
    return hip_err(e, "batch upload");
  }
  b->grid = grid;
  RunArgs &a = b->args;
  a.graphs = d_g;
  a.queries = d_q;
  a.nq = n_q;
  eat::apply_plan(pl, &a);
  a.buckets = d_b;
  a.n_buckets = nb;
  a.work = d_c;
  a.stats = d_s;
  a.n_failed = d_c + 1;
  a.bits_global = pl.bits_global ? reinterpret_cast<uint32_t *>(p + b_g + b_q + b_s + b_c + b_b) : nullptr;
  a.goal = goal ? 1 : 0;
  a.targets = d_t;
  *out = b;
  return EAT_OK;
}

extern "C" eat_status eat_batch_create(const eat_graph *const *graphs, int32_t n_graphs,
                                       const int32_t *q_graph, const int32_t *q_src,
                                       const int32_t *q_ts, int32_t n_q, int32_t *const *arr,
                                       const eat_run_options *ro, eat_batch **out) {
  try {
    return batch_create(graphs, n_graphs, q_graph, q_src, q_ts, nullptr, n_q, arr, ro, out);
  } catch (const std::bad_alloc &) {  // nothing throws across the C ABI
    if (out) *out = nullptr;
    return set_err(EAT_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

extern "C" eat_status eat_batch_create_goal(const eat_graph *const *graphs, int32_t n_graphs,
                                            const int32_t *q_graph, const int32_t *q_src,
                                            const int32_t *q_ts, const int32_t *q_dst, int32_t n_q,
                                            int32_t *const *arr, const eat_run_options *ro, eat_batch **out) {
  if (n_q > 0 && !q_dst) {
    if (out) *out = nullptr;
    return set_err(EAT_ERR_INVALID_ARGUMENT, "q_dst is NULL");
  }
  try {
    return batch_create(graphs, n_graphs, q_graph, q_src, q_ts, q_dst, n_q, arr, ro, out);
  } catch (const std::bad_alloc &) {
    if (out) *out = nullptr;
    return set_err(EAT_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

extern "C" eat_status eat_batch_options(const eat_batch *b, eat_run_options *out) {
  if (!b || !out) return set_err(EAT_ERR_INVALID_ARGUMENT, "NULL argument");
  *out = b->options;
  return EAT_OK;
}

extern "C" eat_status eat_batch_run(eat_batch *b, void *stream) {
  if (!b) return set_err(EAT_ERR_INVALID_ARGUMENT, "batch is NULL");
  if (b->n_q == 0) return EAT_OK;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  hipError_t e = eat::launch_relax(b->args, b->tpv, b->ub, b->kind, b->block, b->grid, b->lds, hs);
  if (e != hipSuccess) return hip_err(e, "relaxation launch");
  HIP_TRY(hipEventRecord(b->done, hs));
  b->ran = true;
  return EAT_OK;
}

extern "C" eat_status eat_batch_wait(eat_batch *b, eat_query_stats *stats) {
  if (!b) return set_err(EAT_ERR_INVALID_ARGUMENT, "batch is NULL");
  if (!b->ran) {
    if (stats && b->n_q > 0) std::memset(stats, 0, sizeof(eat_query_stats) * (size_t)b->n_q);
    return EAT_OK;
  }
  HIP_TRY(hipEventSynchronize(b->done));
  int32_t failed = 0;
  HIP_TRY(hipMemcpy(&failed, b->args.work + 2, 4, hipMemcpyDeviceToHost));
  if (stats && b->n_q > 0)
    HIP_TRY(hipMemcpy(stats, b->args.stats, sizeof(eat_query_stats) * (size_t)b->n_q, hipMemcpyDeviceToHost));
  if (failed) return set_err(EAT_ERR_NOT_CONVERGED, std::to_string(failed) + " queries hit their round limit");
  return EAT_OK;
}

extern "C" void eat_batch_free(eat_batch *b) {
  if (!b) return;
  if (b->ran) (void)hipEventSynchronize(b->done);
  if (b->done) (void)hipEventDestroy(b->done);
  (void)hipFree(b->d_buf);
  delete b;
}

extern "C" eat_status eat_query_batch(const eat_graph *const *graphs, int32_t n_graphs,
                                      const int32_t *q_graph, const int32_t *q_src,
                                      const int32_t *q_ts, int32_t n_q, int32_t *const *arr,
                                      void *stream, const eat_run_options *ro,
                                      eat_query_stats *stats) {
  eat_batch *b = nullptr;
  eat_status s = eat_batch_create(graphs, n_graphs, q_graph, q_src, q_ts, n_q, arr, ro, &b);
  if (s != EAT_OK) return s;
  s = eat_batch_run(b, stream);
  if (s == EAT_OK) s = eat_batch_wait(b, stats);
  std::string keep = g_last_error;
  eat_batch_free(b);
  g_last_error = keep;
  return s;
}

// ---------------------------------------------------------------------------
// diagnostics
// ---------------------------------------------------------------------------
extern "C" eat_status eat_next_departure(const eat_graph *g, int32_t headers, const int32_t *type_ids,
                                         const int32_t *x, int32_t *out, int32_t n, void *stream) {
  if (!g) return set_err(EAT_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (n < 0) return set_err(EAT_ERR_INVALID_ARGUMENT, "n must be >= 0");
  if (n > 0 && (!type_ids || !x || !out)) return set_err(EAT_ERR_INVALID_ARGUMENT, "NULL array");
  int kind = 0;
  const eat_status st = eat::exec_kind(&g, 1, headers, &kind);
  if (st != EAT_OK) return st;
  hipError_t e = eat::launch_next_departure(g->d_desc, kind, type_ids, x, out, n,
                                            static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_err(e, "next-departure launch");
  return EAT_OK;
}
