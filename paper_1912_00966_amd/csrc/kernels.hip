// kernels.hip -- gfx950 kernels of the earliest-arrival-time relaxation.
//
// Design (one query per work-group):
//   The paper (Sections II, III, IV-C) runs one query at a time with one kernel
//   launch per relaxation round over all connection types and a host round
//   trip to test convergence.  Per query the useful work is small (a few
//   thousand type evaluations spread over tens of rounds), so on a 256-CU part
//   the cost is the chain of dependent rounds, not bandwidth.  Here a whole
//   query lives inside one work-group: rounds are separated by work-group
//   barriers (no grid barrier, no kernel launch, no host round trip), the
//   active set stays in LDS, and many queries run side by side, one per
//   work-group, pulled from a shared counter by a persistent grid.
//
// Per query:
//   arr[]      the caller's result slab in HBM (Algorithm 2 fills it with
//              infinity, arr[s] = ts); updated with atomic minimum (Algorithm
//              3, Section III-C).
//   bitmap     one bit per stop in LDS: "improved since it was last expanded"
//              (the active/nextactive flags of Section III-B).  Setting the bit
//              also de-duplicates pushes.
//   lists      two frontier lists in LDS (current / next round).  When the next
//              frontier does not fit, the next round sweeps the bitmap instead
//              (the topology-driven scan of the paper, at bit granularity).
//   Each active stop u is expanded by a group of TPV lanes (the virtual warps
//   of Section IV-B): lane i takes u's connection types i, i+TPV, ...  A type
//   (u, v, lam) gives the earliest departure t_c >= arr[u] (Section II-B) via
//   the cluster lookup of Section II-D and the progression closed form of
//   Algorithm 6; arr[v] drops to t_c + lam if that is earlier.
//
// The fixpoint is the unique EAT answer whatever the order of updates: an
// improved stop is always expanded again after its last improvement, with a
// value read after that improvement.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace eat {
namespace {

constexpr int32_t INF = EAT_INF;

// arr[] accesses: relaxed atomics at agent scope.  Loads bypass the per-CU
// vector L1, so a stop's value is never read from a stale L1 line after an
// atomic minimum (performed in L2) lowered it.
__device__ __forceinline__ int32_t ld_arr(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t min_arr(int32_t *p, int32_t v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_arr(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct Ctr {
  uint32_t act = 0, tev = 0, hdr = 0, pool = 0, imp = 0;
};

// ---------------------------------------------------------------------------
// Next departure of connection type j at or after x (Section II-B:
// t_c = min{t in C_{u,v,lam} : t >= x}); INF when there is none.
// ---------------------------------------------------------------------------
template <int KIND>
__device__ __forceinline__ int32_t next_departure(const GraphDev &G, const int4 r, int64_t j,
                                                  int32_t x, Ctr &c);

// Hybrid layout: hourly clusters (Section II-D) + one progression or a sorted
// array per cluster.  Cluster k = x / width.  If cluster k holds departures,
// the first one >= x inside it comes from the progression closed form
// t0 + ceil((x - t0) / h) * h (Algorithm 6) or a bisection of its array;
// otherwise -- cluster k empty, or all its departures earlier than x -- the
// answer is the first departure of the next non-empty cluster (Section II-D),
// which is the next header because only non-empty clusters have one.
template <>
__device__ __forceinline__ int32_t next_departure<EAT_LAYOUT_HYBRID>(const GraphDev &G, const int4 r,
                                                                     int64_t j, int32_t x, Ctr &c) {
  const uint32_t k = (uint32_t)x / (uint32_t)G.cluster_seconds;
  if (k >= (uint32_t)G.n_clusters) return INF;  // after the last departure of the timetable
  uint64_t m = (uint32_t)r.w;
  if (G.mask_hi) m |= (uint64_t)G.mask_hi[j] << 32;
  const uint64_t ahead = m >> k;  // bit 0: cluster k itself
  if (ahead == 0) return INF;     // no departure in cluster k or later
  const int32_t idx = r.z + __popcll(m & ((1ull << k) - 1ull));
  const int2 h = G.hdr[idx];
  c.hdr++;
  if (!(ahead & 1ull) || x <= h.x) return h.x;
  if (h.y >= 0) {  // one progression t0 + i*d, i < n
    const int32_t d = h.y & 0xffff, n = h.y >> 16;
    const int32_t i = (x - h.x - 1) / d + 1;  // ceil((x - t0) / d), x > t0
    if (i < n) return h.x + i * d;
  } else {  // sorted array p[1..n], p[1] = t0 < x
    const int32_t *p = G.pool + (~h.y);
    const int32_t n = p[0];
    int32_t lo = 2, hi = n + 1;
    c.pool++;
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      c.pool++;
      if (p[mid] < x) lo = mid + 1; else hi = mid;
    }
    if (lo <= n) {
      c.pool++;
      return p[lo];
    }
  }
  if ((ahead >> 1) == 0) return INF;
  c.hdr++;
  return G.hdr[idx + 1].x;
}

// Flat layout: one sorted array per type, bisection.
template <>
__device__ __forceinline__ int32_t next_departure<EAT_LAYOUT_FLAT>(const GraphDev &G, const int4 r,
                                                                   int64_t, int32_t x, Ctr &c) {
  const int32_t *p = G.pool + r.z;
  int32_t lo = 0, hi = r.w;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    c.pool++;
    if (p[mid] < x) lo = mid + 1; else hi = mid;
  }
  if (lo < r.w) {
    c.pool++;
    return p[lo];
  }
  return INF;
}

// ---------------------------------------------------------------------------
// Frontier push: wave64 ballot, one LDS atomic per wave, lane offsets by
// masked population count.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void push(bool want, int32_t v, int32_t *nxt, int32_t fcap, bool append,
                                     int32_t *sh_nn) {
  const uint64_t m = __ballot(want);
  if (m == 0) return;
  const int lane = __lane_id();
  const int leader = __ffsll((unsigned long long)m) - 1;
  int32_t base = 0;
  if (lane == leader) base = atomicAdd(sh_nn, (int32_t)__popcll(m));
  base = __shfl(base, leader);
  if (want && append) {
    const int32_t slot = base + (int32_t)__popcll(m & ((1ull << lane) - 1ull));
    if (slot < fcap) nxt[slot] = v;
  }
}

// Relax (Algorithm 3) the best connection of type j for a tail reached at x.
template <int KIND>
__device__ __forceinline__ void relax(const GraphDev &G, int32_t *arr, int64_t j, int32_t x,
                                      int32_t *nxt, uint32_t *bm, int32_t fcap, bool append,
                                      int32_t *sh_nn, Ctr &c) {
  const int4 r = G.ty[j];
  const int32_t v = r.x, lam = r.y;
  c.tev++;
  const int32_t av = ld_arr(arr + v);
  bool want = false;
  // Any departure of this type leaves at t_c >= x, so it arrives at >= x + lam:
  // skip the lookup when that cannot beat arr[v] (early termination, Section
  // III-D, in its strongest exact form).
  if (x < av - lam) {
    const int32_t tc = next_departure<KIND>(G, r, j, x, c);
    if (tc != INF) {
      const int32_t cand = tc + lam;
      if (cand < av) {
        const int32_t old = min_arr(arr + v, cand);
        if (cand < old) {
          c.imp++;
          const uint32_t bit = 1u << (v & 31);
          want = !(atomicOr(&bm[v >> 5], bit) & bit);
        }
      }
    }
  }
  push(want, v, nxt, fcap, append, sh_nn);
}

// Expand every stop of list[0..n): groups of TPV lanes, one stop per group.
template <int TPV, int KIND>
__device__ __forceinline__ void expand_list(const GraphDev &G, int32_t *arr, const int32_t *list,
                                            int32_t n, int32_t *nxt, uint32_t *bm, int32_t fcap,
                                            bool append, int32_t *sh_nn, Ctr &c) {
  constexpr int kGroups = kBlock / TPV;
  const int g = threadIdx.x / TPV, lane = threadIdx.x % TPV;
  for (int32_t base = 0; base < n; base += kGroups) {
    const int32_t i = base + g;
    if (i < n) {
      const int32_t u = list[i];
      const int32_t x = ld_arr(arr + u);
      const int32_t b = G.vt_off[u], e = G.vt_off[u + 1];
      if (lane == 0) c.act++;
      for (int32_t j = b + lane; j < e; j += TPV) relax<KIND>(G, arr, j, x, nxt, bm, fcap, append, sh_nn, c);
    }
  }
}

template <int TPV, int KIND>
__global__ __launch_bounds__(kBlock) void k_relax(RunArgs a) {
  extern __shared__ uint32_t lds[];
  __shared__ int32_t sh_q, sh_nn, sh_cnt;
  __shared__ unsigned long long sh_acc[5];

  const int tid = threadIdx.x;
  uint32_t *bm = lds;
  int32_t *list0 = reinterpret_cast<int32_t *>(lds + a.bm_words);
  int32_t *list1 = list0 + a.fcap;
  const bool batch = a.queries != nullptr;
  const bool topo = a.mode == EAT_MODE_TOPOLOGY;

  for (int iter = 0;; ++iter) {
    if (tid == 0)
      sh_q = batch ? __hip_atomic_fetch_add(a.work, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                   : (iter == 0 ? 0 : a.nq);
    if (tid < 5) sh_acc[tid] = 0ull;
    __syncthreads();
    const int32_t q = sh_q;
    if (q >= a.nq) {
      // The last work-group to leave re-arms the shared counters for the next
      // launch of the same batch, so a run is a single kernel launch.
      if (batch && tid == 0) {
        const int32_t left = __hip_atomic_fetch_add(a.work + 1, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (left == (int32_t)gridDim.x - 1) {
          const int32_t failed = __hip_atomic_exchange(a.work + 2, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(a.work + 3, failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(a.work + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(a.work, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      break;
    }
    const QueryDev Q = batch ? a.queries[q] : a.single;
    const GraphDev G = a.graphs[batch ? Q.graph : 0];
    const int32_t V = G.n_vertices;
    const int32_t VW = (V + 31) >> 5;
    int32_t *arr = Q.arr;
    const int32_t max_rounds = a.max_rounds > 0 ? a.max_rounds : V + 2;

    // ---- Initialize (Algorithm 2) -------------------------------------------
    if ((reinterpret_cast<uintptr_t>(arr) & 15u) == 0) {
      int4 *a4 = reinterpret_cast<int4 *>(arr);
      const int32_t n4 = V >> 2;
      const int4 inf4 = make_int4(INF, INF, INF, INF);
      for (int32_t i = tid; i < n4; i += kBlock) a4[i] = inf4;
      for (int32_t i = (n4 << 2) + tid; i < V; i += kBlock) arr[i] = INF;
    } else {
      for (int32_t i = tid; i < V; i += kBlock) arr[i] = INF;
    }
    for (int32_t i = tid; i < VW; i += kBlock) bm[i] = 0u;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the fill is in L2 before anyone reads arr
    __syncthreads();
    if (tid == 0) {
      st_arr(arr + Q.s, Q.ts);
      if (topo) bm[Q.s >> 5] = 1u << (Q.s & 31);
      else list0[0] = Q.s;
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();

    // ---- rounds until no arrival improves ------------------------------------
    int32_t *cur = list0, *nxt = list1;
    int32_t nf = topo ? 0 : 1;
    bool sweep = topo;
    int32_t rounds = 0, sweeps = 0, maxf = 1, status = EAT_OK;
    Ctr c;
    const int32_t chunk_words = a.fcap >> 5;  // a sweep stages at most fcap stops at a time
    for (;;) {
      if (rounds >= max_rounds) {
        status = EAT_ERR_NOT_CONVERGED;
        break;
      }
      if (tid == 0) sh_nn = 0;
      __syncthreads();
      if (!sweep) {
        expand_list<TPV, KIND>(G, arr, cur, nf, nxt, bm, a.fcap, !topo, &sh_nn, c);
      } else {
        ++sweeps;
        for (int32_t w0 = 0; w0 < VW; w0 += chunk_words) {
          if (tid == 0) sh_cnt = 0;
          __syncthreads();
          const int32_t w1 = min(w0 + chunk_words, VW);
          for (int32_t w = w0 + tid; w < w1; w += kBlock) {
            uint32_t bits = bm[w];
            if (bits) {
              bits = atomicExch(&bm[w], 0u);  // claim: these stops are expanded now
              int32_t pos = atomicAdd(&sh_cnt, (int32_t)__popc(bits));
              while (bits) {
                const int b = __ffs(bits) - 1;
                bits &= bits - 1u;
                cur[pos++] = (w << 5) + b;
              }
            }
          }
          __syncthreads();
          const int32_t cnt = sh_cnt;
          if (cnt) expand_list<TPV, KIND>(G, arr, cur, cnt, nxt, bm, a.fcap, !topo, &sh_nn, c);
          __syncthreads();
        }
      }
      __syncthreads();
      const int32_t nn = sh_nn;
      ++rounds;
      if (nn == 0) break;
      maxf = max(maxf, nn);
      const bool next_sweep = topo || nn > a.fcap;
      if (!next_sweep) {
        // the pushed stops become the current list: clear their bits so that the
        // next round's pushes are de-duplicated afresh
        for (int32_t i = tid; i < nn; i += kBlock) {
          const int32_t v = nxt[i];
          atomicAnd(&bm[v >> 5], ~(1u << (v & 31)));
        }
      }
      int32_t *tmp = cur;
      cur = nxt;
      nxt = tmp;
      nf = next_sweep ? 0 : nn;
      sweep = next_sweep;
      __syncthreads();
    }

    // ---- per-query statistics --------------------------------------------------
    if (a.stats || (status != EAT_OK && a.n_failed)) {
      atomicAdd(&sh_acc[0], (unsigned long long)c.act);
      atomicAdd(&sh_acc[1], (unsigned long long)c.tev);
      atomicAdd(&sh_acc[2], (unsigned long long)c.hdr);
      atomicAdd(&sh_acc[3], (unsigned long long)c.pool);
      atomicAdd(&sh_acc[4], (unsigned long long)c.imp);
      __syncthreads();
      if (tid == 0) {
        if (a.stats) {
          eat_query_stats *st = a.stats + Q.index;
          st->status = status;
          st->rounds = rounds;
          st->sweep_rounds = sweeps;
          st->max_frontier = maxf;
          st->activations = (int64_t)sh_acc[0];
          st->type_evals = (int64_t)sh_acc[1];
          st->header_loads = (int64_t)sh_acc[2];
          st->pool_loads = (int64_t)sh_acc[3];
          st->improvements = (int64_t)sh_acc[4];
        }
        if (status != EAT_OK && a.n_failed)
          __hip_atomic_fetch_add(a.n_failed, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
  }
}

__global__ void k_zero(int32_t *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

template <int KIND>
__global__ void k_next_departure(const GraphDev *gd, const int32_t *ids, const int32_t *xs,
                                 int32_t *out, int32_t n) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const GraphDev G = *gd;
  const int32_t j = ids[i], x = xs[i];
  if (j < 0 || (int64_t)j >= G.n_types || x < 0) {
    out[i] = -1;
    return;
  }
  Ctr c;
  out[i] = next_departure<KIND>(G, G.ty[j], j, x, c);
}

using RelaxFn = void (*)(RunArgs);

template <int KIND>
RelaxFn relax_fn(int tpv) {
  switch (tpv) {
    case 1: return k_relax<1, KIND>;
    case 2: return k_relax<2, KIND>;
    case 4: return k_relax<4, KIND>;
    case 8: return k_relax<8, KIND>;
    case 16: return k_relax<16, KIND>;
    case 32: return k_relax<32, KIND>;
    case 64: return k_relax<64, KIND>;
    default: return nullptr;
  }
}

RelaxFn pick(int tpv, int kind) {
  return kind == EAT_LAYOUT_FLAT ? relax_fn<EAT_LAYOUT_FLAT>(tpv) : relax_fn<EAT_LAYOUT_HYBRID>(tpv);
}

}  // namespace

hipError_t launch_relax(const RunArgs &a, int tpv, int kind, int grid, size_t lds_bytes,
                        hipStream_t stream) {
  RelaxFn f = pick(tpv, kind);
  if (!f) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(f),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(f, dim3(grid), dim3(kBlock), lds_bytes, stream, a);
  return hipGetLastError();
}

int relax_blocks_per_cu(int tpv, int kind, size_t lds_bytes) {
  RelaxFn f = pick(tpv, kind);
  if (!f) return 0;
  (void)hipFuncSetAttribute(reinterpret_cast<const void *>(f), hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)lds_bytes);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(f), kBlock,
                                                   lds_bytes) != hipSuccess)
    return 0;
  return nb;
}

hipError_t launch_zero(int32_t *p, int n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3((n + 255) / 256), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

hipError_t launch_next_departure(const GraphDev *g_dev, int kind, const int32_t *type_ids,
                                 const int32_t *x, int32_t *out, int32_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int grid = (n + 255) / 256;
  if (kind == EAT_LAYOUT_FLAT)
    hipLaunchKernelGGL(k_next_departure<EAT_LAYOUT_FLAT>, dim3(grid), dim3(256), 0, stream, g_dev,
                       type_ids, x, out, n);
  else
    hipLaunchKernelGGL(k_next_departure<EAT_LAYOUT_HYBRID>, dim3(grid), dim3(256), 0, stream, g_dev,
                       type_ids, x, out, n);
  return hipGetLastError();
}

}  // namespace eat
