// journeys.hip -- the query variants of Section I beside the single-source
// answer: the journey (earliest arrival path) behind every arrival time, and
// the profile of a source over an interval of departure times.  Both run the
// relaxation's own lookup device functions (next departure of a connection
// type at or after a time, Sections II-B..II-D).
#include "relax.hpp"

namespace eat {
namespace {

// ---------------------------------------------------------------------------
// Parents.  The arrival arr[v] (v != s) of an EAT answer is realised by a
// connection (u, v, t, lam) with arr[u] <= t and t + lam == arr[v].  Within a
// connection type (u, v, lam) the only candidate is its first departure at or
// after arr[u]: a later one arrives later.  Each reached stop u checks its
// types; the realising one with the smallest (u, lam) wins one 64-bit atomic
// minimum on key[v] = u << 32 | lam.
// ---------------------------------------------------------------------------
template <int KIND>
__global__ void k_parents(GraphDev Gd, const int32_t *arr, int32_t s, unsigned long long *key) {
  const GraphG G = graph_g(Gd);
  gp<const int32_t> A = (gp<const int32_t>)arr;
  const int32_t V = G.n_vertices;
  for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < V; u += gridDim.x * blockDim.x) {
    const int32_t x = A[u];
    if (x == INF) continue;
    const int2 r = G.vt[u];
    for (int32_t j = r.x; j < r.x + r.y; ++j) {
      int4 rec;
      if constexpr (KIND == kKindGrid) rec = G.side[j];  // {v, lam, ..}
      else rec = G.ty[2 * (int64_t)j];                   // {v, lam, ..}
      const int32_t v = rec.x, lam = rec.y;
      const int32_t av = A[v];
      if (v == s || av == INF || (int64_t)x + lam > av) continue;  // no departure at or after x can realise av
      Ctr c;
      const int32_t tc = next_departure<KIND>(G, j, r.x, r.y, x, c);
      if (tc != INF && (int64_t)tc + lam == av)
        atomicMin(key + v, ((unsigned long long)(uint32_t)u << 32) | (uint32_t)lam);
    }
  }
}

__global__ void k_fill_u64(unsigned long long *p, int32_t n, unsigned long long x) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = x;
}

// par[3v .. 3v + 2] = (u, t, lam) of v's parent, or -1 three times.
__global__ void k_parents_finish(const int32_t *arr, const unsigned long long *key, int32_t V, int32_t *par) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x) {
    const unsigned long long k = key[v];
    int32_t pu = -1, pt = -1, pl = -1;
    if (k != ~0ull) {
      pu = (int32_t)(k >> 32);
      pl = (int32_t)(uint32_t)k;
      pt = arr[v] - pl;
    }
    par[3 * (int64_t)v] = pu;
    par[3 * (int64_t)v + 1] = pt;
    par[3 * (int64_t)v + 2] = pl;
  }
}

// ---------------------------------------------------------------------------
// Profiles.  The departures of s in [lo, hi], in increasing order: one wave
// walks them, each step taking the minimum over s's types of the next
// departure after the previous one.  out[0..cap) receives the first cap of
// them; info[0] = their count, info[1] = the first departure after hi (INF if
// none).
// ---------------------------------------------------------------------------
template <int KIND>
__global__ __launch_bounds__(64) void k_departures(GraphDev Gd, int32_t s, int32_t lo, int32_t hi, int32_t cap,
                                                   int32_t *out, int32_t *info) {
  const GraphG G = graph_g(Gd);
  const int2 r = G.vt[s];
  const int lane = __lane_id();
  int32_t x = lo, k = 0, next = INF;
  for (;;) {
    int32_t best = INF;
    for (int32_t j = r.x + lane; j < r.x + r.y; j += 64) {
      Ctr c;
      best = min(best, next_departure<KIND>(G, j, r.x, r.y, x, c));
    }
    for (int d = 32; d >= 1; d >>= 1) best = min(best, __shfl_xor(best, d));
    if (best == INF) break;
    if (best > hi) {
      next = best;
      break;
    }
    if (lane == 0 && k < cap) out[k] = best;
    ++k;
    x = best + 1;  // best <= hi < INF
  }
  if (lane == 0) {
    info[0] = k;
    info[1] = next;
  }
}

// Row i of the k x V profile matrix keeps arr[i][v] only where it beats row
// i + 1 (the last row: the query at the first departure after the interval,
// `later`, or nothing when there is none); each thread walks one column.
__global__ void k_profile_filter(int32_t *arr, const int32_t *later, int32_t k, int32_t V, int32_t s) {
  for (int32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < V; v += gridDim.x * blockDim.x) {
    int32_t a = arr[v];
    for (int32_t i = 0; i < k; ++i) {
      const int32_t b = i + 1 < k ? arr[(int64_t)(i + 1) * V + v] : (later ? later[v] : INF);
      arr[(int64_t)i * V + v] = (v != s && a < b) ? a : INF;
      a = b;
    }
  }
}

int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

}  // namespace

hipError_t launch_parents(const GraphDev &g, int kind, const int32_t *arr, int32_t s, unsigned long long *key,
                          int32_t *par, hipStream_t stream) {
  const int32_t V = g.n_vertices;
  if (V <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(V)), dim3(256), 0, stream, key, V, ~0ull);
  if (kind == kKindGrid)
    hipLaunchKernelGGL(k_parents<kKindGrid>, dim3(blocks_for(V)), dim3(256), 0, stream, g, arr, s, key);
  else if (kind == kKindCompact)
    hipLaunchKernelGGL(k_parents<kKindCompact>, dim3(blocks_for(V)), dim3(256), 0, stream, g, arr, s, key);
  else if (kind == kKindFlat)
    hipLaunchKernelGGL(k_parents<kKindFlat>, dim3(blocks_for(V)), dim3(256), 0, stream, g, arr, s, key);
  else
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_parents_finish, dim3(blocks_for(V)), dim3(256), 0, stream, arr, key, V, par);
  return hipGetLastError();
}

hipError_t launch_departures(const GraphDev &g, int kind, int32_t s, int32_t lo, int32_t hi, int32_t cap,
                             int32_t *out, int32_t *info, hipStream_t stream) {
  if (kind == kKindGrid)
    hipLaunchKernelGGL(k_departures<kKindGrid>, dim3(1), dim3(64), 0, stream, g, s, lo, hi, cap, out, info);
  else if (kind == kKindCompact)
    hipLaunchKernelGGL(k_departures<kKindCompact>, dim3(1), dim3(64), 0, stream, g, s, lo, hi, cap, out, info);
  else if (kind == kKindFlat)
    hipLaunchKernelGGL(k_departures<kKindFlat>, dim3(1), dim3(64), 0, stream, g, s, lo, hi, cap, out, info);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_profile_filter(int32_t *arr, const int32_t *later, int32_t k, int32_t V, int32_t s,
                                 hipStream_t stream) {
  if (k <= 0 || V <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_profile_filter, dim3(blocks_for(V)), dim3(256), 0, stream, arr, later, k, V, s);
  return hipGetLastError();
}

}  // namespace eat
