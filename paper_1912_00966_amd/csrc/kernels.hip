// kernels.hip -- the small gfx950 kernels (next-departure probes, header-grid
// construction, zero fill) and the host-side launchers of every kernel.  The
// relaxation kernel itself is in relax.hpp.
#include "relax.hpp"

namespace eat {
namespace {

__global__ void k_zero(int32_t *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Fingerprint of every query's result slab (one work-group per query): the sum
// over stops i of a mix of (i, arr[i]), into out[q] (zeroed by the caller).
// Equal slabs give equal sums; the autotuner compares candidates with it.
__global__ void k_slab_hash(const QueryDev *qs, const GraphDev *graphs, int32_t nq, unsigned long long *out) {
  const int32_t q = blockIdx.x;
  if (q >= nq) return;
  const QueryDev Q = qs[q];
  const int32_t V = graphs[Q.graph].n_vertices;
  unsigned long long acc = 0;
  for (int32_t i = threadIdx.x; i < V; i += blockDim.x) {
    unsigned long long x = ((unsigned long long)(uint32_t)i << 32) | (uint32_t)Q.arr[i];
    x ^= x >> 31;
    x *= 0x9E3779B97F4A7C15ull;
    x ^= x >> 29;
    acc += x;
  }
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d);
  if (__lane_id() == 0) atomicAdd(out + Q.index, acc);
}

template <int KIND>
__global__ void k_next_departure(const GraphDev *gd, const int32_t *ids, const int32_t *xs,
                                 int32_t *out, int32_t n) {
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const GraphG G = graph_g(*gd);
  const int32_t j = ids[i], x = xs[i];
  if (j < 0 || (int64_t)j >= G.n_types || x < 0) {
    out[i] = -1;
    return;
  }
  int32_t b = 0, cnt = 0;
  if constexpr (KIND == kKindGrid) {
    const int2 r = G.vt[G.tail[j]];
    b = r.x;
    cnt = r.y;
  }
  Ctr c;
  out[i] = next_departure<KIND>(G, j, b, cnt, x, c);
}

// One thread per connection type: writes the type's n_clusters grid entries
// from its compact headers, from the last cluster down, carrying the first
// departure of the clusters after the current one.
//   progression {t0, (n << 16) | d, next, m = ceil(2^32 / d), 0 for d = 1}
//   empty       {next, (1 << 16) | 1, next, 0}: a one-term progression at next
//   array n<=5  {t0, 2 << 30 | o2 << 15 | o3, next, o4 << 15 | o5}: o_i = d_i - t0
//               (departure i of the cluster; 0 past n); an array holds at
//               least three departures (two always form a progression)
//   array n>5   {t0, ~off, next, n}: pool[off] = n, pool[off + 1 ..] = departures
// Offsets fit 15 bits because a cluster is narrower than 2^15 seconds; pool
// offsets are below 2^30 (checked on the host before the grid is built).
__global__ void k_build_grid(GraphDev Gd) {
  const GraphG G = graph_g(Gd);
  gp<int4> grid = (gp<int4>)const_cast<int4 *>(Gd.grid);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < G.n_types; j += stride) {
    const int4 r = G.ty[2 * j], r2 = G.ty[2 * j + 1];
    const uint64_t m = (uint64_t)(uint32_t)r.w | ((uint64_t)(uint32_t)r2.z << 32);
    const int2 rng = G.vt[G.tail[j]];
    const int64_t base = (int64_t)rng.x * G.n_clusters + (j - rng.x);
    int32_t idx = r.z + __popcll(m) - 1;  // header of the last non-empty cluster
    int32_t next = INF;
    for (int32_t k = G.n_clusters - 1; k >= 0; --k) {
      int4 e;
      if ((m >> k) & 1ull) {
        const int2 h = G.hdr[idx--];
        if (h.y >= 0) {
          // progression step d >= 2: m = ceil(2^32 / d) <= 2^31; d = 1 (or a
          // single term): 0
          const uint32_t d = (uint32_t)(h.y & 0xffff);
          const uint32_t mul = d >= 2 ? (uint32_t)((((uint64_t)1 << 32) + d - 1) / d) : 0u;
          e = make_int4(h.x, h.y, next, (int32_t)mul);
        } else {
          const int32_t off = ~h.y, n = G.pool[off];
          if (n <= 5) {
            const int32_t o2 = G.pool[off + 2] - h.x, o3 = G.pool[off + 3] - h.x;
            const int32_t o4 = n > 3 ? G.pool[off + 4] - h.x : 0, o5 = n > 4 ? G.pool[off + 5] - h.x : 0;
            e = make_int4(h.x, (int32_t)(0x80000000u | ((uint32_t)o2 << 15) | (uint32_t)o3), next,
                          (o4 << 15) | o5);
          } else {
            e = make_int4(h.x, h.y, next, n);
          }
        }
        next = h.x;
      } else {
        e = make_int4(next, (1 << 16) | 1, next, 0);
      }
      grid[base + (int64_t)k * rng.y] = e;
    }
  }
}

RelaxFn pick(int tpv, int ub, int kind, int block, bool goal) {
  switch (kind) {
    case kKindCompact: return relax_fn_compact(tpv, ub, block, goal);
    case kKindFlat: return relax_fn_flat(tpv, ub, block, goal);
    case kKindGrid: return relax_fn_grid(tpv, ub, block, goal);
    default: return nullptr;
  }
}

// Raises a kernel's dynamic-LDS limit when a launch needs more than any earlier
// launch of the same kernel in this process.
hipError_t allow_lds(RelaxFn f, size_t bytes) {
  static std::mutex mu;
  static std::map<const void *, size_t> granted;
  std::lock_guard<std::mutex> lk(mu);
  const void *key = reinterpret_cast<const void *>(f);
  auto it = granted.find(key);
  if (it != granted.end() && it->second >= bytes) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) granted[key] = bytes;
  return e;
}

}  // namespace

hipError_t launch_relax(const RunArgs &a, int tpv, int ub, int kind, int block, int grid, size_t lds_bytes,
                        hipStream_t stream) {
  RelaxFn f = pick(tpv, ub, kind, block, a.goal != 0);
  if (!f) return hipErrorInvalidValue;
  hipError_t e = allow_lds(f, lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(f, dim3(grid), dim3(block), lds_bytes, stream, a);
  return hipGetLastError();
}

int relax_blocks_per_cu(int tpv, int ub, int kind, int block, size_t lds_bytes, bool goal) {
  RelaxFn f = pick(tpv, ub, kind, block, goal);
  if (!f) return 0;
  if (allow_lds(f, lds_bytes) != hipSuccess) return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(f), block,
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
  if (kind == kKindFlat)
    hipLaunchKernelGGL(k_next_departure<kKindFlat>, dim3(grid), dim3(256), 0, stream, g_dev,
                       type_ids, x, out, n);
  else if (kind == kKindGrid)
    hipLaunchKernelGGL(k_next_departure<kKindGrid>, dim3(grid), dim3(256), 0, stream, g_dev,
                       type_ids, x, out, n);
  else if (kind == kKindCompact)
    hipLaunchKernelGGL(k_next_departure<kKindCompact>, dim3(grid), dim3(256), 0, stream, g_dev,
                       type_ids, x, out, n);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_slab_hash(const QueryDev *qs, const GraphDev *graphs, int32_t nq, unsigned long long *out,
                            hipStream_t stream) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slab_hash, dim3(nq), dim3(256), 0, stream, qs, graphs, nq, out);
  return hipGetLastError();
}

hipError_t launch_build_grid(const GraphDev &g, hipStream_t stream) {
  if (g.n_types <= 0) return hipSuccess;
  if (!g.grid || !g.tail || !g.hdr || !g.vt || !g.ty) return hipErrorInvalidValue;
  const int64_t blocks = std::min<int64_t>((g.n_types + 255) / 256, 65536);
  hipLaunchKernelGGL(k_build_grid, dim3((unsigned)blocks), dim3(256), 0, stream, g);
  return hipGetLastError();
}

}  // namespace eat
