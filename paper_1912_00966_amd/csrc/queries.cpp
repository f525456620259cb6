// queries.cpp -- C ABI of the query variants beside the single-source answer
// (Section I): parent connections (journeys) and profiles of a source over an
// interval of departure times.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "device.hpp"
#include "eat.h"
#include "internal.hpp"

using eat::hip_err;
using eat::set_err;

namespace eat {
hipError_t launch_parents(const GraphDev &g, int kind, const int32_t *arr, int32_t s, unsigned long long *key,
                          int32_t *par, hipStream_t stream);
hipError_t launch_departures(const GraphDev &g, int kind, int32_t s, int32_t lo, int32_t hi, int32_t cap,
                             int32_t *out, int32_t *info, hipStream_t stream);
hipError_t launch_profile_filter(int32_t *arr, const int32_t *later, int32_t k, int32_t V, int32_t s,
                                 hipStream_t stream);
}  // namespace eat

static eat_status check_graph(const eat_graph *g) {
  if (!g) return set_err(EAT_ERR_INVALID_ARGUMENT, "graph is NULL");
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != g->device) return set_err(EAT_ERR_INVALID_ARGUMENT, "graph lives on another device than the current one");
  return EAT_OK;
}

extern "C" eat_status eat_parents(const eat_graph *g, int32_t s, const int32_t *arr, int32_t *par, void *stream) {
  eat_status st = check_graph(g);
  if (st != EAT_OK) return st;
  if (!arr || !par) return set_err(EAT_ERR_INVALID_ARGUMENT, "arr or par is NULL");
  if (s < 0 || s >= g->info.n_vertices) return set_err(EAT_ERR_INVALID_ARGUMENT, "source out of range");
  int kind = 0;
  st = eat::exec_kind(&g, 1, EAT_HEADERS_AUTO, &kind);
  if (st != EAT_OK) return st;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  unsigned long long *key = nullptr;
  HIP_TRY(hipMallocAsync(reinterpret_cast<void **>(&key), (size_t)g->info.n_vertices * 8, hs));
  hipError_t e = eat::launch_parents(g->desc, kind, arr, s, key, par, hs);
  const hipError_t f = hipFreeAsync(key, hs);
  if (e == hipSuccess) e = f;
  if (e != hipSuccess) return hip_err(e, "parents launch");
  return EAT_OK;
}

extern "C" eat_status eat_profile(const eat_graph *g, int32_t s, int32_t t_lo, int32_t t_hi, int32_t cap,
                                  int32_t *dep, int32_t *n_dep, int32_t *arr, void *stream,
                                  const eat_run_options *ro) {
  eat_status st = check_graph(g);
  if (st != EAT_OK) return st;
  const int32_t V = g->info.n_vertices;
  if (!n_dep) return set_err(EAT_ERR_INVALID_ARGUMENT, "n_dep is NULL");
  if (s < 0 || s >= V) return set_err(EAT_ERR_INVALID_ARGUMENT, "source out of range");
  if (t_lo < 0 || t_hi < t_lo) return set_err(EAT_ERR_INVALID_ARGUMENT, "need 0 <= t_lo <= t_hi");
  if (cap < 0 || (cap > 0 && (!dep || !arr))) return set_err(EAT_ERR_INVALID_ARGUMENT, "cap < 0, or dep/arr NULL");
  int kind = 0;
  st = eat::exec_kind(&g, 1, ro ? ro->headers : EAT_HEADERS_AUTO, &kind);
  if (st != EAT_OK) return st;
  hipStream_t hs = static_cast<hipStream_t>(stream);
  // scratch: {count, next}, the departures, the row of the query after the interval
  const size_t b_info = eat::align_up(2 * sizeof(int32_t));
  const size_t b_dep = eat::align_up((size_t)std::max(cap, 1) * sizeof(int32_t));
  const size_t b_row = eat::align_up((size_t)V * sizeof(int32_t));
  char *buf = nullptr;
  HIP_TRY(hipMalloc(reinterpret_cast<void **>(&buf), b_info + b_dep + b_row));
  int32_t *d_info = reinterpret_cast<int32_t *>(buf);
  int32_t *d_dep = reinterpret_cast<int32_t *>(buf + b_info);
  int32_t *d_later = reinterpret_cast<int32_t *>(buf + b_info + b_dep);
  auto done = [&](eat_status r) {
    (void)hipStreamSynchronize(hs);
    (void)hipFree(buf);
    return r;
  };
  int32_t info[2] = {0, 0};
  hipError_t e = eat::launch_departures(g->desc, kind, s, t_lo, t_hi, cap, d_dep, d_info, hs);
  if (e == hipSuccess) e = hipMemcpyAsync(info, d_info, sizeof(info), hipMemcpyDeviceToHost, hs);
  if (e == hipSuccess) e = hipStreamSynchronize(hs);
  if (e != hipSuccess) return done(hip_err(e, "profile departures"));
  const int32_t k = info[0], next = info[1];
  *n_dep = k;
  if (k > cap) {
    if (cap == 0 && !arr) return done(EAT_OK);  // the count only
    return done(set_err(EAT_ERR_UNSUPPORTED, std::to_string(k) + " departures in the interval, cap is " +
                                                 std::to_string(cap)));
  }
  if (k == 0) return done(EAT_OK);
  std::vector<int32_t> h_dep((size_t)k);
  e = hipMemcpy(h_dep.data(), d_dep, (size_t)k * sizeof(int32_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return done(hip_err(e, "profile departures copy"));
  // one batch: a query per departure, and one at the first departure after t_hi
  const int32_t nq = k + (next != EAT_INF ? 1 : 0);
  std::vector<int32_t> qg((size_t)nq, 0), qs((size_t)nq, s), qt((size_t)nq);
  std::vector<int32_t *> rows((size_t)nq);
  for (int32_t i = 0; i < k; ++i) {
    qt[(size_t)i] = h_dep[(size_t)i];
    rows[(size_t)i] = arr + (int64_t)i * V;
  }
  if (nq > k) {
    qt[(size_t)k] = next;
    rows[(size_t)k] = d_later;
  }
  eat_batch *b = nullptr;
  st = eat_batch_create(&g, 1, qg.data(), qs.data(), qt.data(), nq, rows.data(), ro, &b);
  if (st != EAT_OK) return done(st);
  st = eat_batch_run(b, stream);
  if (st == EAT_OK) st = eat_batch_wait(b, nullptr);
  eat_batch_free(b);
  if (st != EAT_OK) return done(st);
  for (int32_t i = 0; i < k; ++i) dep[i] = h_dep[(size_t)i];
  e = eat::launch_profile_filter(arr, nq > k ? d_later : nullptr, k, V, s, hs);
  if (e != hipSuccess) return done(hip_err(e, "profile filter"));
  return done(EAT_OK);
}
