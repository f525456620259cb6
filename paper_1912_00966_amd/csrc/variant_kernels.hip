// variant_kernels.hip -- kernels of the paper's algorithm ladder (one launch per
// iteration, one work item per thread) and of the ESDG baseline (one launch
// per level).  They are comparison points for the production relaxation
// kernel; every one of them computes the same EAT answer.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "variants.hpp"

namespace eat {
namespace {

constexpr int32_t INF = EAT_INF;

// arr[] is read and lowered by other threads during an iteration: relaxed
// atomics at agent scope (no stale per-CU L1 line after an atomic minimum).
__device__ __forceinline__ int32_t ld(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Relax (Algorithm 3) of the connection (u, v, t, lam) with x = e[u]: if
// x <= t and t + lam < e[v], e[v] drops to t + lam by an atomic minimum
// (Section III-C) and v becomes active for the next iteration (nextactive,
// Section III-B).  True if e[v] dropped.
__device__ __forceinline__ bool relax(int32_t *arr, uint8_t *next, int32_t x, int32_t v, int32_t t, int32_t lam) {
  if (t == INF || x > t) return false;
  const int32_t cand = t + lam;
  if (cand >= ld(arr + v)) return false;
  const int32_t old = __hip_atomic_fetch_min(arr + v, cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (cand >= old) return false;
  next[v] = 1;
  return true;
}

// The change flag and the examined-work counter, one write per wave.
__device__ __forceinline__ void wave_report(bool changed, uint32_t examined, int32_t *flag,
                                            unsigned long long *count) {
  if (__ballot(changed) && __lane_id() == __ffsll((unsigned long long)__ballot(1)) - 1) *flag = 1;
  if (count) {
    unsigned long long c = examined;
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d);
    if (__lane_id() == __ffsll((unsigned long long)__ballot(1)) - 1) atomicAdd(count, c);
  }
}

// Algorithm 6 over the tuples p[0..n): the smallest term >= x, or INF.
__device__ __forceinline__ int32_t from_aps(const int4 *p, int32_t n, int32_t x, uint32_t &examined) {
  int32_t tc = INF;
  for (int32_t i = 0; i < n; ++i) {
    const int4 a = p[i];  // {start, end, difference}
    if (a.x < x && x <= a.y) {
      const int32_t k = (x - a.x + a.z - 1) / a.z;  // ceil((x - start) / difference)
      tc = min(tc, a.x + k * a.z);
    }
    if (x <= a.x) tc = min(tc, a.x);
  }
  examined += (uint32_t)n;
  return tc;
}

// Cluster-AP (Section II-D): the tuples of cluster x / width of type j, else
// the first departure of the next non-empty cluster.
__device__ __forceinline__ int32_t cluster_ap(const VariantDev &g, int32_t j, int32_t x, uint32_t &examined) {
  const int32_t K = g.n_clusters;
  int32_t k = x / g.cluster_seconds;
  if (k >= K) return INF;
  const int32_t *off = g.cloff + (int64_t)j * K;
  const int32_t b = off[k], e = off[k + 1];
  int32_t tc = from_aps(g.cap + b, e - b, x, examined);
  if (tc != INF) return tc;
  for (++k; k < K; ++k) {  // the tuples of a cluster are ordered by first term
    const int32_t bb = off[k];
    if (off[k + 1] > bb) {
      ++examined;
      return g.cap[bb].x;
    }
  }
  return INF;
}

__global__ void k_var_init(int32_t *arr, uint8_t *act, uint8_t *next, int32_t nv, int32_t s, int32_t ts) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += gridDim.x * blockDim.x) {
    arr[i] = i == s ? ts : INF;
    act[i] = i == s;
    next[i] = 0;
  }
}

__global__ void k_var_clear(uint8_t *p, int32_t n) {
  for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

// Algorithm 4: a thread per connection.
__global__ void k_var_connection(VariantDev g, int32_t *arr, const uint8_t *act, uint8_t *next, int32_t *flag,
                                 unsigned long long *count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ch = false;
  uint32_t ex = 0;
  if (i < g.n_conn) {
    const int32_t u = g.cu[i];
    if (act[u]) {
      ex = 1;
      ch = relax(arr, next, ld(arr + u), g.cv[i], g.ct[i], g.clam[i]);
    }
  }
  wave_report(ch, ex, flag, count);
}

// Algorithm 5: a thread per connection type.  Early termination (Section
// III-D): the first departure later than e[v], or e[u] later than the last.
// getConnection: linear search of the sorted departures (Section II-B); with
// progressions, Algorithm 6 over the type's tuples (Section II-C).
template <bool AP>
__global__ void k_var_type(VariantDev g, int32_t *arr, const uint8_t *act, uint8_t *next, int32_t *flag,
                           unsigned long long *count) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ch = false;
  uint32_t ex = 0;
  if (j < g.n_types) {
    const int32_t u = g.tu[j];
    if (act[u]) {
      const int32_t x = ld(arr + u), v = g.tv[j], lam = g.tlam[j];
      const int32_t av = ld(arr + v);
      if constexpr (AP) {
        const int32_t b = g.tapoff[j], e = g.tapoff[j + 1];
        if (e > b && av >= g.tap[b].x) {  // the first tuple's first term is the first departure
          const int32_t tc = from_aps(g.tap + b, e - b, x, ex);
          ch = relax(arr, next, x, v, tc, lam);
        }
      } else {
        const int32_t b = g.tdoff[j], e = g.tdoff[j + 1];
        if (e > b && g.dep[b] <= av && x <= g.dep[e - 1]) {
          int32_t q = b;
          while (g.dep[q] < x) ++q;  // x <= the last departure: stops inside
          ex = (uint32_t)(q - b + 1);
          ch = relax(arr, next, x, v, g.dep[q], lam);
        }
      }
    }
  }
  wave_report(ch, ex, flag, count);
}

// Section II-D: a thread per connection type, Cluster-AP lookup.
__global__ void k_var_cluster(VariantDev g, int32_t *arr, const uint8_t *act, uint8_t *next, int32_t *flag,
                              unsigned long long *count) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool ch = false;
  uint32_t ex = 0;
  if (j < g.n_types) {
    const int32_t u = g.tu[j];
    if (act[u]) {
      const int32_t x = ld(arr + u), v = g.tv[j];
      if (g.dep[g.tdoff[j]] <= ld(arr + v)) ch = relax(arr, next, x, v, cluster_ap(g, (int32_t)j, x, ex), g.tlam[j]);
    }
  }
  wave_report(ch, ex, flag, count);
}

// Sections II-E and II-F: W lanes per edge (u, v), lane i taking the edge's
// types i, i + W, ...; W = 1 is the edge version.
template <int W>
__global__ void k_var_edge(VariantDev g, int32_t *arr, const uint8_t *act, uint8_t *next, int32_t *flag,
                           unsigned long long *count) {
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t e = gid / W;
  const int32_t lane = (int32_t)(gid % W);
  bool ch = false;
  uint32_t ex = 0;
  if (e < g.n_edges) {
    const int32_t u = g.eu[e];
    if (act[u]) {
      const int32_t x = ld(arr + u);
      for (int32_t j = g.etoff[e] + lane; j < g.etoff[e + 1]; j += W) {
        const int32_t v = g.tv[j];
        if (g.dep[g.tdoff[j]] <= ld(arr + v)) ch |= relax(arr, next, x, v, cluster_ap(g, j, x, ex), g.tlam[j]);
      }
    }
  }
  wave_report(ch, ex, flag, count);
}

// ESDG (Section I-A): the connections of one level, each relaxed once with
// the test of Algorithm 1.
__global__ void k_esdg_level(VariantDev g, int64_t begin, int64_t end, int32_t *arr, unsigned long long *count) {
  const int64_t i = begin + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t ex = 0;
  if (i < end) {
    ex = 1;
    const int32_t x = ld(arr + g.lu[i]), t = g.lt[i];
    if (x <= t) {
      const int32_t cand = t + g.llam[i];
      if (cand < ld(arr + g.lv[i]))
        __hip_atomic_fetch_min(arr + g.lv[i], cand, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (count) {
    unsigned long long c = ex;
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d);
    if (__lane_id() == 0) atomicAdd(count, c);
  }
}

unsigned blocks(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, (n + per - 1) / per); }

}  // namespace

hipError_t launch_variant_init(int32_t *arr, uint8_t *active, uint8_t *next, int32_t nv, int32_t s, int32_t ts,
                               hipStream_t stream) {
  hipLaunchKernelGGL(k_var_init, dim3(std::min(blocks(nv, 256), 4096u)), dim3(256), 0, stream, arr, active, next, nv,
                     s, ts);
  return hipGetLastError();
}

hipError_t launch_variant_clear(uint8_t *p, int32_t n, hipStream_t stream) {
  hipLaunchKernelGGL(k_var_clear, dim3(std::min(blocks(n, 256), 4096u)), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

hipError_t launch_variant_iteration(const VariantDev &g, int variant, int warp_size, int32_t *arr,
                                    const uint8_t *active, uint8_t *next, int32_t *flag,
                                    unsigned long long *count, hipStream_t stream) {
  const dim3 B(256);
  switch (variant) {
    case EAT_VARIANT_CONNECTION:
      if (g.n_conn) hipLaunchKernelGGL(k_var_connection, dim3(blocks(g.n_conn, 256)), B, 0, stream, g, arr, active, next, flag, count);
      break;
    case EAT_VARIANT_CONNECTION_TYPE:
      if (g.n_types) hipLaunchKernelGGL(k_var_type<false>, dim3(blocks(g.n_types, 256)), B, 0, stream, g, arr, active, next, flag, count);
      break;
    case EAT_VARIANT_CONNECTION_TYPE_AP:
      if (g.n_types) hipLaunchKernelGGL(k_var_type<true>, dim3(blocks(g.n_types, 256)), B, 0, stream, g, arr, active, next, flag, count);
      break;
    case EAT_VARIANT_CLUSTER_AP:
      if (g.n_types) hipLaunchKernelGGL(k_var_cluster, dim3(blocks(g.n_types, 256)), B, 0, stream, g, arr, active, next, flag, count);
      break;
    case EAT_VARIANT_EDGE:
    case EAT_VARIANT_WARPS: {
      const int w = variant == EAT_VARIANT_EDGE ? 1 : warp_size;
      if (!g.n_edges) break;
      const unsigned nb = blocks(g.n_edges * w, 256);
      switch (w) {
        case 1: hipLaunchKernelGGL(k_var_edge<1>, dim3(nb), B, 0, stream, g, arr, active, next, flag, count); break;
        case 2: hipLaunchKernelGGL(k_var_edge<2>, dim3(nb), B, 0, stream, g, arr, active, next, flag, count); break;
        case 4: hipLaunchKernelGGL(k_var_edge<4>, dim3(nb), B, 0, stream, g, arr, active, next, flag, count); break;
        case 8: hipLaunchKernelGGL(k_var_edge<8>, dim3(nb), B, 0, stream, g, arr, active, next, flag, count); break;
        case 16: hipLaunchKernelGGL(k_var_edge<16>, dim3(nb), B, 0, stream, g, arr, active, next, flag, count); break;
        case 32: hipLaunchKernelGGL(k_var_edge<32>, dim3(nb), B, 0, stream, g, arr, active, next, flag, count); break;
        case 64: hipLaunchKernelGGL(k_var_edge<64>, dim3(nb), B, 0, stream, g, arr, active, next, flag, count); break;
        default: return hipErrorInvalidValue;
      }
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_esdg_level(const VariantDev &g, int64_t begin, int64_t end, int32_t *arr,
                             unsigned long long *count, hipStream_t stream) {
  if (end <= begin) return hipSuccess;
  hipLaunchKernelGGL(k_esdg_level, dim3(blocks(end - begin, 256)), dim3(256), 0, stream, g, begin, end, arr, count);
  return hipGetLastError();
}

}  // namespace eat
