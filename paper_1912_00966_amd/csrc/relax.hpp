// relax.hpp -- device code of the earliest-arrival-time relaxation (gfx950),
// shared by the kernel sources: the relaxation kernel k_relax and the lookup
// functions it uses.  Each relax_<form>.hip instantiates the kernel variants of
// one timetable form (header grid, compact headers, flat layout), so the three
// compile in parallel; kernels.hip holds the small kernels and the launchers.
#pragma once
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
//   arrivals   an open-addressing hash table in LDS of the stops the query has
//              touched: one 64-bit word per slot {arrival, idle flag, stop}.
//              The caller's result slab in HBM (Algorithm 2: infinity
//              everywhere, arr[s] = ts; the fill is issued in pieces while the
//              rounds run) receives the final values; if the table overflows,
//              the query runs again with its arrivals in the slab, updated with
//              global atomic minimum (Algorithm 3, Section III-C).
//   activity   the slot's flag (one LDS bit per stop in slab mode): "improved
//              since it was last expanded" (the active/nextactive flags of
//              Section III-B).  Setting it also de-duplicates pushes.
//   lists      two frontier lists in LDS (current / next round).  When the next
//              frontier does not fit, the next round sweeps the flags instead
//              (the topology-driven scan of the paper, 64 items at a time).
//   Each round takes the listed stops (those past the round's arrival window
//   wait for a later round) and numbers their connection types; the waves then
//   relax windows of 64 consecutive types, one type per lane, dealt to them in
//   turn (or, with TPV > 0, a group of TPV lanes per stop: the virtual warps
//   of Section IV-B).  A type
//   (u, v, lam) gives the earliest departure t_c >= arr[u] (Section II-B) via
//   the cluster lookup of Section II-D and the progression closed form of
//   Algorithm 6; arr[v] drops to t_c + lam if that is earlier.
//
// The fixpoint is the unique EAT answer whatever the order of updates: an
// improved stop is always expanded again after its last improvement, with a
// value read after that improvement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "device.hpp"

namespace eat {

using RelaxFn = void (*)(RunArgs);

namespace {

constexpr int32_t INF = EAT_INF;
constexpr int kClaim = 4;  // frontier entries a wave claims at a time (rounds of many types)
// A round's connection types, numbered in list order, are cut into windows of
// 64; a wave relaxes whole windows.  Rounds of up to kWin windows take this
// path; larger ones fall back to claims of kClaim entries.
constexpr int kWin = 128;
// Chunks of the slab fill a lane issues per step a wave waits for others.
constexpr int32_t kFillPerStep = 8;

// Pointers into device (global) memory.  The graph descriptor and the query
// records hold plain pointers; the kernels read through these so that every
// access compiles to a global (not flat) instruction: flat accesses also count
// against the LDS wait counter, which would make each on-chip probe wait for
// the outstanding global reads.
// (The host pass of this single-source file only parses device code; it sees
// plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gp = __attribute__((address_space(1))) T *;
#else
template <class T>
using gp = T *;
#endif

struct GraphG {
  gp<const int2> vt;
  gp<const int4> ty;
  gp<const int2> hdr;
  gp<const int32_t> pool;
  gp<const int4> side;
  gp<const int4> grid;
  gp<const int32_t> tail;
  int64_t n_types;
  int32_t n_vertices;
  int32_t cluster_seconds;
  int32_t n_clusters;
  int32_t horizon;
  float inv_cw;
};

__device__ __forceinline__ GraphG graph_g(const GraphDev &g) {
  GraphG o;
  o.vt = (gp<const int2>)g.vt;
  o.ty = (gp<const int4>)g.ty;
  o.hdr = (gp<const int2>)g.hdr;
  o.pool = (gp<const int32_t>)g.pool;
  o.side = (gp<const int4>)g.side;
  o.grid = (gp<const int4>)g.grid;
  o.tail = (gp<const int32_t>)g.tail;
  o.n_types = g.n_types;
  o.n_vertices = g.n_vertices;
  o.cluster_seconds = g.cluster_seconds;
  o.n_clusters = g.n_clusters;
  o.horizon = g.horizon;
  o.inv_cw = g.inv_cw;
  return o;
}

// arr[] accesses: relaxed atomics at agent scope.  Loads bypass the per-CU
// vector L1, so a stop's value is never read from a stale L1 line after an
// atomic minimum (performed in L2) lowered it.
__device__ __forceinline__ int32_t ld_arr(gp<const int32_t> p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t min_arr(gp<int32_t> p, int32_t v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_arr(gp<int32_t> p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct Ctr {
  uint32_t act = 0, tev = 0, hdr = 0, pool = 0, imp = 0;
};

// ---------------------------------------------------------------------------
// Next departure of connection type j at or after x (Section II-B:
// t_c = min{t in C_{u,v,lam} : t >= x}); INF when there is none.
// ---------------------------------------------------------------------------

// First of the sorted departures d[0..n) (n <= 16, read from 16-byte chunks)
// that is >= x, or INF.  Words past n are ignored.
__device__ __forceinline__ int32_t first_at_or_after(const int32_t *d, int32_t n, int32_t x) {
  int32_t best = INF;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int32_t t = d[i];
    best = (i < n && t >= x && t < best) ? t : best;
  }
  return best;
}

// A lookup is split into stages so that a lane can keep several lookups in
// flight: locate (needs the type record), fetch (header / departure chunks),
// finish (arithmetic on registers).
//
// Hybrid layout: hourly clusters (Section II-D) + one progression or a sorted
// array per cluster.  Cluster k = x / width.  If cluster k holds departures,
// the first one >= x inside it comes from the progression closed form
// t0 + ceil((x - t0) / h) * h (Algorithm 6) or from its sorted array;
// otherwise -- cluster k empty, or all its departures earlier than x -- the
// answer is the first departure of the next non-empty cluster (Section II-D),
// which is the next header because only non-empty clusters have one.  The
// next header is fetched together with the first; arrays of <= 7 departures
// (the common case) are read as two independent 16-byte chunks.
//
// Header grid (hybrid layout): the 16-byte entry of (type j, cluster k) sits at
// an address computed from j, k and the tail stop's type range [b, b + n), so
// it is read at the same time as the type's record instead of after it.  Empty
// clusters hold the next departure as a one-term progression, every entry
// carries the next cluster's first departure, and arrays of up to five
// departures carry departures 2..5 as offsets from the first: one read
// answers the lookup, except inside a longer array (one more read of its
// departures from the pool).
struct Look {
  int32_t idx;    // header index (hybrid)
  int32_t mode;   // 0: no departure >= x; 1: the first departure of header idx; 2: search in header idx
  bool has_next;  // another non-empty cluster follows cluster idx
  int2 h, hn;     // header idx and idx + 1 (hybrid)
  int32_t gidx;   // grid entry index (grid)
  int4 e;         // grid entry {t0, c, next, m}
  int4 c0, c1;    // first chunks of an array cluster (hybrid) or departures 0..7 (flat)
  int4 c2, c3;    // departures 8..15 (flat)
};

// Cluster index floor(x / width) of a time x < horizon (< 2^24, so x is exact
// in float): a float product is within one of it, and one step fixes that.
__device__ __forceinline__ int32_t cluster_of(const GraphG &G, int32_t x) {
  int32_t k = (int32_t)((float)x * G.inv_cw);
  k += ((k + 1) * G.cluster_seconds <= x) ? 1 : 0;
  k -= (k * G.cluster_seconds > x) ? 1 : 0;
  return k;
}

// Grid entry kinds by the top two bits of c: 0x progression (or an empty
// cluster), 10 an array of three to five departures held in the entry, 11 an
// array in the pool at ~c.
__device__ __forceinline__ bool grid_pool_array(int32_t c) { return (uint32_t)c >= 0xC0000000u; }

// Grid: entry of type j (tail stop's types [b, b + n)) in the cluster of x.
// Grids have fewer than 2^31 entries.
__device__ __forceinline__ void look_locate_grid(const GraphG &G, int64_t j, int32_t b, int32_t n, int32_t x,
                                                 Look &L) {
  L.mode = 0;  // x at or after the horizon: no departure
  L.gidx = 0;
  if (x < G.horizon) {
    L.mode = 2;
    L.gidx = b * G.n_clusters + cluster_of(G, x) * n + ((int32_t)j - b);
  }
}

template <int KIND>
__device__ __forceinline__ void look_locate(const GraphG &G, const int4 r, uint32_t mhi, int32_t x, Look &L) {
  if constexpr (KIND == EAT_LAYOUT_HYBRID) {
    L.mode = 0;
    L.idx = 0;
    L.has_next = false;
    if (x >= G.horizon) return;  // after the last departure of the timetable
    const uint32_t k = (uint32_t)cluster_of(G, x);
    const uint64_t m = (uint64_t)(uint32_t)r.w | ((uint64_t)mhi << 32);
    const uint64_t ahead = m >> k;  // bit 0: cluster k itself
    if (ahead == 0) return;         // no departure in cluster k or later
    L.idx = r.z + __popcll(m & ((1ull << k) - 1ull));
    L.mode = (ahead & 1ull) ? 2 : 1;
    L.has_next = (ahead >> 1) != 0;
  } else if constexpr (KIND == EAT_LAYOUT_FLAT) {
    L.mode = r.w > 0 ? 2 : 0;
  }
}

// Issues the memory reads of a located lookup (no use of their results).
template <int KIND>
__device__ __forceinline__ void look_fetch_headers(const GraphG &G, const int4 r, Look &L) {
  if constexpr (KIND == EAT_LAYOUT_HYBRID) {
    // header idx + 1 exists: the header array carries one padding entry
    L.h = G.hdr[L.idx];
    L.hn = G.hdr[L.idx + 1];
  } else if constexpr (KIND == kKindGrid) {
    if (L.mode != 0) L.e = G.grid[L.gidx];
  } else {
    if (L.mode != 0 && r.w <= 16) {
      gp<const int4> p4 = (gp<const int4>)(G.pool + r.z);
      L.c0 = p4[0];
      L.c1 = p4[1];
      L.c2 = p4[2];
      L.c3 = p4[3];
    }
  }
}

// Hybrid only: the chunks of an array cluster that x falls into (needs the header).
template <int KIND>
__device__ __forceinline__ void look_fetch_chunks(const GraphG &G, int32_t x, Look &L, Ctr &c) {
  if constexpr (KIND == EAT_LAYOUT_HYBRID) {
    if (L.mode == 2 && L.h.y < 0 && x > L.h.x) {
      gp<const int4> p4 = (gp<const int4>)(G.pool + (~L.h.y));
      L.c0 = p4[0];
      L.c1 = p4[1];
      c.pool += 8;
    }
  } else if constexpr (KIND == kKindGrid) {
    // arrays of more than five departures, x past the first: the departures
    if (L.mode == 2 && grid_pool_array(L.e.y) && x > L.e.x) {
      gp<const int4> p4 = (gp<const int4>)(G.pool + (~L.e.y));
      L.c0 = p4[0];
      L.c1 = p4[1];
      c.pool += 8;
    }
  }
}

// First departure >= x of the array cluster at pool[off] (pool[off] = n, then
// n sorted departures, the first < x); L.c0, L.c1 hold its first 8 words.
__device__ __forceinline__ int32_t array_next(const GraphG &G, int32_t off, int32_t x, const Look &L, Ctr &c) {
  const int32_t n = L.c0.x;
  int32_t t = INF;
  if (n <= 7) {
    const int32_t d7[7] = {L.c0.y, L.c0.z, L.c0.w, L.c1.x, L.c1.y, L.c1.z, L.c1.w};
#pragma unroll
    for (int i = 0; i < 7; ++i) t = (i < n && d7[i] >= x && d7[i] < t) ? d7[i] : t;
  } else {
    gp<const int32_t> p = G.pool + off;
    int32_t lo = 2, hi = n + 1;
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      c.pool++;
      if (p[mid] < x) lo = mid + 1; else hi = mid;
    }
    if (lo <= n) t = p[lo];
  }
  return t;
}

template <int KIND>
__device__ __forceinline__ int32_t look_finish(const GraphG &G, const int4 r, int32_t x, const Look &L, Ctr &c) {
  if (L.mode == 0) return INF;
  if constexpr (KIND == EAT_LAYOUT_HYBRID) {
    const int2 h = L.h;
    if (L.mode == 1 || x <= h.x) return h.x;
    if (h.y >= 0) {  // one progression t0 + i*d, i < n
      const int32_t d = h.y & 0xffff, n = h.y >> 16;
      const int32_t i = (x - h.x - 1) / d + 1;  // ceil((x - t0) / d), x > t0
      if (i < n) return h.x + i * d;
    } else {  // sorted array p[1..n], p[0] = n, p[1] = t0 < x
      const int32_t t = array_next(G, ~h.y, x, L, c);
      if (t != INF) return t;
    }
    if (!L.has_next) return INF;
    c.hdr++;
    return L.hn.x;
  } else if constexpr (KIND == kKindGrid) {
    const int4 e = L.e;
    if (x <= e.x) return e.x;  // also every empty cluster: e.x is the next departure
    if (e.y >= 0) {            // one progression t0 + i*d, i < n
      const int32_t d = e.y & 0xffff, n = e.y >> 16;
      // i = ceil((x - t0) / d) = floor((x - t0 - 1) / d) + 1 with x - t0 - 1 <
      // width < 2^15: the high half of the product with m = ceil(2^32 / d) is
      // that quotient exactly (m = 0 stands for d = 1)
      const uint32_t r = (uint32_t)(x - e.x - 1);
      const int32_t i = (int32_t)(e.w ? __umulhi(r, (uint32_t)e.w) : r) + 1;
      if (i < n) return e.x + i * d;
    } else if (grid_pool_array(e.y)) {  // sorted array in the pool (more than five departures)
      const int32_t t = array_next(G, ~e.y, x, L, c);
      if (t != INF) return t;
    } else {  // sorted array of three to five departures: offsets of departures
              // 2..5 from the first, 15 bits each (0 = no such departure)
      const int32_t r = x - e.x;  // 0 < r < width <= 32767
      const int32_t o2 = (e.y >> 15) & 0x7fff, o3 = e.y & 0x7fff;
      const int32_t o4 = (e.w >> 15) & 0x7fff, o5 = e.w & 0x7fff;
      if (r <= o2) return e.x + o2;
      if (r <= o3) return e.x + o3;
      if (o4 != 0 && r <= o4) return e.x + o4;
      if (o5 != 0 && r <= o5) return e.x + o5;
    }
    return e.z;  // first departure of a later cluster
  } else {
    const int32_t n = r.w;
    if (n <= 16) {
      const int32_t d[16] = {L.c0.x, L.c0.y, L.c0.z, L.c0.w, L.c1.x, L.c1.y, L.c1.z, L.c1.w,
                             L.c2.x, L.c2.y, L.c2.z, L.c2.w, L.c3.x, L.c3.y, L.c3.z, L.c3.w};
      return first_at_or_after(d, n, x);
    }
    // long arrays: bisection
    gp<const int32_t> p = G.pool + r.z;
    int32_t lo = 0, hi = n;
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      c.pool++;
      if (p[mid] < x) lo = mid + 1; else hi = mid;
    }
    if (lo < n) {
      c.pool++;
      return p[lo];
    }
    return INF;
  }
}

// Counts the words of a header fetch that a lookup actually needs.
template <int KIND>
__device__ __forceinline__ void count_fetch(const int4 r, const Look &L, Ctr &c) {
  if constexpr (KIND == EAT_LAYOUT_HYBRID) c.hdr += 1;  // +1 more if the next cluster is needed
  else if constexpr (KIND == kKindGrid) c.hdr += 1;    // one grid entry
  else if (L.mode != 0 && r.w <= 16) c.pool += 16;
}

// Next departure of connection type j at or after x (Section II-B:
// t_c = min{t in C_{u,v,lam} : t >= x}); INF when there is none.  [b, b + n)
// is the type range of j's tail stop (read by the grid form only).
template <int KIND>
__device__ __forceinline__ int32_t next_departure(const GraphG &G, int64_t j, int32_t b, int32_t n, int32_t x,
                                                  Ctr &c) {
  Look L;
  int4 r = make_int4(0, 0, 0, 0);
  if constexpr (KIND == kKindGrid) {
    look_locate_grid(G, j, b, n, x, L);
  } else {
    r = G.ty[2 * j];
    const uint32_t mhi = (KIND == EAT_LAYOUT_HYBRID && G.n_clusters > 32) ? (uint32_t)G.ty[2 * j + 1].z : 0u;
    look_locate<KIND>(G, r, mhi, x, L);
  }
  if (L.mode == 0) return INF;
  look_fetch_headers<KIND>(G, r, L);
  count_fetch<KIND>(r, L, c);
  look_fetch_chunks<KIND>(G, x, L, c);
  return look_finish<KIND>(G, r, x, L, c);
}

// ---------------------------------------------------------------------------
// Frontier lists.  An entry names an item (a table slot or a stop) and the
// item's stop's range of connection types, loaded by the lane that pushed it
// (cnt < 0: not known yet, the expansion loads it).
// ---------------------------------------------------------------------------
struct FList {
  int32_t *item;
  int32_t *beg;
  int32_t *cnt;
};

// The stops a round expands (type windows): {first type, type count,
// arrival time, offset of the first type in the round's type numbering} per
// entry, read by a wave in one 16-byte load.
using XList = int4 *;

// Pushes into the next round's list: the list's entry count is the low half
// of a 64-bit LDS word, one atomic per wave.  The smallest arrival a lane
// pushes is kept in a register and reduced once per round (wave_min).
struct ListPush {
  FList nxt;
  int32_t fcap;
  bool append;
  unsigned long long *cx;
  int32_t lmin;
  // wave64 ballot, one LDS atomic per wave, lane offsets by masked population count
  __device__ __forceinline__ void operator()(bool want, int32_t item, int32_t beg, int32_t cnt, int32_t val) {
    const uint64_t m = __ballot(want);
    if (m == 0) return;
    if (want) lmin = min(lmin, val);
    const int lane = __lane_id();
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = (uint32_t)atomicAdd(cx, (unsigned long long)__popcll(m));
    base = (uint32_t)__builtin_amdgcn_readlane((int32_t)base, leader);
    if (want && append) {
      const int32_t slot = (int32_t)base + (int32_t)__popcll(m & ((1ull << lane) - 1ull));
      if (slot < fcap) {
        nxt.item[slot] = item;
        nxt.beg[slot] = beg;
        nxt.cnt[slot] = cnt;
      }
    }
  }
};

// Minimum over the 64 lanes of a wave, every lane active: DPP steps inside
// rows of 16 lanes, then row broadcasts; lane 63 ends with the minimum.
__device__ __forceinline__ int32_t wave_min(int32_t v) {
  v = min(v, __builtin_amdgcn_update_dpp(INF, v, 0x111, 0xf, 0xf, false));  // row_shr:1
  v = min(v, __builtin_amdgcn_update_dpp(INF, v, 0x112, 0xf, 0xf, false));  // row_shr:2
  v = min(v, __builtin_amdgcn_update_dpp(INF, v, 0x114, 0xf, 0xf, false));  // row_shr:4
  v = min(v, __builtin_amdgcn_update_dpp(INF, v, 0x118, 0xf, 0xf, false));  // row_shr:8
  v = min(v, __builtin_amdgcn_update_dpp(INF, v, 0x142, 0xa, 0xf, false));  // row_bcast:15
  v = min(v, __builtin_amdgcn_update_dpp(INF, v, 0x143, 0xc, 0xf, false));  // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
}

// Inclusive prefix sum over the 64 lanes of a wave, every lane active: the
// same DPP steps, adding where wave_min takes the minimum.
__device__ __forceinline__ int32_t wave_incl_sum(int32_t v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
  return v;
}

__device__ __forceinline__ int32_t lds_ld(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// A value every lane of the wave holds alike (read after a barrier, or
// derived from such values), moved to a scalar register: loops and branches
// on it become scalar, and addresses built from it use scalar bases.
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------------------
// Where a query keeps its arrival times.  An "item" names one stop's entry.
// Each item carries an activity flag: set when the item's arrival improves
// (and it is pushed), cleared when the item is taken for expansion (the active
// / nextactive flags of Section III-B).  Both stores offer:
//   find(v, pos)              arrival of stop v (INF if none yet), pos = where
//   improve(v, pos, av, cand, item, c)
//                             lower v's arrival to cand < av (av, pos from
//                             find); true if the item was not active, i.e.
//                             the caller pushes it; item = v's item
//   value / stop / active / deactivate / reactivate   per item
//   claim_group(g, lane, act) a sweep stages every active item of items
//                             [64 g, 64 g + 64): clear their flags
//   full()                    the store overflowed (checked between rounds)
// ---------------------------------------------------------------------------

// Activity bits of the slab store: one per stop, in LDS (uint32_t *) or -- for
// a graph whose bitmap does not fit the LDS -- in the work-group's own region
// of HBM (gp<uint32_t>), updated by global atomics at agent scope (loads
// bypass the per-CU L1, which atomics do not update).
__device__ __forceinline__ uint32_t bits_or(uint32_t *b, int32_t w, uint32_t m) { return atomicOr(b + w, m); }
__device__ __forceinline__ void bits_and(uint32_t *b, int32_t w, uint32_t m) { atomicAnd(b + w, m); }
__device__ __forceinline__ uint32_t bits_ld(uint32_t *b, int32_t w) {
  return (uint32_t)__hip_atomic_load(reinterpret_cast<int32_t *>(b + w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void bits_st(uint32_t *b, int32_t w, uint32_t x) { b[w] = x; }

// (The host pass sees plain pointers for both forms: only the LDS form there.)
#if defined(__HIP_DEVICE_COMPILE__)
__device__ __forceinline__ uint32_t bits_or(gp<uint32_t> b, int32_t w, uint32_t m) {
  return __hip_atomic_fetch_or(b + w, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void bits_and(gp<uint32_t> b, int32_t w, uint32_t m) {
  __hip_atomic_fetch_and(b + w, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t bits_ld(gp<uint32_t> b, int32_t w) {
  return __hip_atomic_load(b + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void bits_st(gp<uint32_t> b, int32_t w, uint32_t x) {
  __hip_atomic_store(b + w, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
#endif

template <class P>
__device__ __forceinline__ bool mark_improved(P bits, int32_t it) {
  const uint32_t bit = 1u << (it & 31);
  return !(bits_or(bits, it >> 5, bit) & bit);
}

// In the caller's result slab (HBM), item = stop id; one activity bit per
// stop, in LDS or in HBM (P, see bits_or).
template <class P>
struct SlabStore {
  static constexpr bool kGoal = false;
  gp<int32_t> arr;
  P bits;
  int32_t n;
  __device__ __forceinline__ int32_t stop(int32_t item) const { return item; }
  __device__ __forceinline__ int32_t value(int32_t item) const { return ld_arr(arr + item); }
  __device__ __forceinline__ int32_t find(int32_t v, int32_t &pos) const {
    pos = v;
    return ld_arr(arr + v);
  }
  __device__ __forceinline__ bool improve(int32_t v, int32_t, int32_t, int32_t cand, int32_t &item, Ctr &c) const {
    item = v;
    if (cand < min_arr(arr + v, cand)) {
      c.imp++;
      return mark_improved(bits, v);
    }
    return false;
  }
  __device__ __forceinline__ bool active(int32_t item) const { return (bits_ld(bits, item >> 5) >> (item & 31)) & 1; }
  __device__ __forceinline__ void deactivate(int32_t item) const { bits_and(bits, item >> 5, ~(1u << (item & 31))); }
  __device__ __forceinline__ bool reactivate(int32_t item) const { return mark_improved(bits, item); }
  __device__ __forceinline__ void claim_group(int32_t g, int lane, bool) const {
    // items 64 g .. 64 g + 63 are words 2 g and 2 g + 1; no relaxation runs
    const int32_t first = (g << 6) + lane;
    if ((lane & 31) == 0 && first < n) bits_st(bits, first >> 5, 0u);
  }
  __device__ __forceinline__ bool full() const { return false; }
};

// In an on-chip open-addressing hash table (LDS) of the stops the query has
// touched, item = table slot; the result slab only receives the final values.
// A slot is one 64-bit word: arrival time in the high half, the idle flag
// (set = not active) and the stop id in the low half.  One 64-bit atomic
// minimum with {candidate, stop, flag clear} then lowers the arrival, makes the
// item active and tells whether it was idle.  An equal candidate never reaches
// an idle slot: within a relaxation phase flags only go from idle to active and
// arrivals only drop, and a candidate is tried only below the arrival find()
// read, so an arrival equal to it was set during the phase, flag clear.
constexpr uint32_t IDLE = 0x80000000u;
constexpr uint32_t NO_KEY = 0xffffffffu;  // low half of an empty slot (idle, no stop)
constexpr unsigned long long EMPTY_SLOT = ((unsigned long long)(uint32_t)INF << 32) | NO_KEY;
struct TableStore {
  static constexpr bool kGoal = false;
  unsigned long long *kv;
  int32_t *count;  // slots in use
  int32_t *over;   // set when a stop found no slot
  uint32_t mask;
  int32_t shift;
  int32_t limit;   // more slots in use than this (checked between rounds): overflow
  __device__ __forceinline__ uint32_t home(int32_t v) const { return ((uint32_t)v * 2654435761u) >> shift; }
  __device__ __forceinline__ int32_t *lo(int32_t p) const { return reinterpret_cast<int32_t *>(kv + p); }
  __device__ __forceinline__ int32_t *hi(int32_t p) const { return reinterpret_cast<int32_t *>(kv + p) + 1; }
  __device__ __forceinline__ unsigned long long entry(uint32_t p) const {
    return __hip_atomic_load(kv + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
  __device__ __forceinline__ int32_t stop(int32_t item) const { return (int32_t)((uint32_t)lds_ld(lo(item)) & ~IDLE); }
  __device__ __forceinline__ int32_t value(int32_t item) const { return lds_ld(hi(item)); }
  // pos = v's slot, or the empty slot where it would go (slots are never
  // freed, so a later insertion of v lands at pos or after it); -1 if full.
  // The home slot is read on its own: most lookups end there.
  __device__ __forceinline__ int32_t find(int32_t v, int32_t &pos) const {
    uint32_t p = home(v);
    unsigned long long e = entry(p);
    pos = (int32_t)p;
    uint32_t key = (uint32_t)e;
    for (uint32_t n = 1; (key & ~IDLE) != (uint32_t)v && key != NO_KEY; ++n) {
      if (n > mask) {
        pos = -1;
        return INF;
      }
      p = (p + 1u) & mask;
      e = entry(p);
      pos = (int32_t)p;
      key = (uint32_t)e;
    }
    return key == NO_KEY ? INF : (int32_t)(e >> 32);
  }
  // The common case is straight-line: a new stop takes the empty slot find()
  // returned with a compare-and-swap, a known one is lowered with an atomic
  // minimum; a wave issues both kinds together and waits once.  Only a lane
  // whose swap lost a race for its slot goes on probing (improve_probe).
  __device__ __forceinline__ bool improve(int32_t v, int32_t pos, int32_t av, int32_t cand, int32_t &item,
                                          Ctr &c) const {
    if (pos < 0) {
      __hip_atomic_store(over, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      return false;
    }
    const unsigned long long want = ((unsigned long long)(uint32_t)cand << 32) | (uint32_t)v;
    const bool fresh = av == INF;  // pos is an empty slot (every stored arrival is finite)
    const unsigned long long old = fresh ? atomicCAS(kv + pos, EMPTY_SLOT, want) : atomicMin(kv + pos, want);
    item = pos;
    if (fresh) {
      if (old == EMPTY_SLOT) {
        atomicAdd(count, 1);
        c.imp++;
        return true;
      }
      return improve_probe(v, (uint32_t)pos, (uint32_t)old, want, cand, item, c);
    }
    if (cand < (int32_t)(old >> 32)) {
      c.imp++;
      return ((uint32_t)old & IDLE) != 0u;
    }
    return false;
  }
  // After a lost swap at slot p (key = the stop now there): lower v's slot if
  // that is v, else probe on to v's slot or the next empty one.
  __device__ __forceinline__ bool improve_probe(int32_t v, uint32_t p, uint32_t key, unsigned long long want,
                                             int32_t cand, int32_t &item, Ctr &c) const {
    for (uint32_t n = 0; n <= mask; ++n) {
      if (key == NO_KEY) {
        const unsigned long long old = atomicCAS(kv + p, EMPTY_SLOT, want);
        if (old == EMPTY_SLOT) {
          atomicAdd(count, 1);
          item = (int32_t)p;
          c.imp++;
          return true;
        }
        key = (uint32_t)old;
      }
      if ((key & ~IDLE) == (uint32_t)v) {
        const unsigned long long old = atomicMin(kv + p, want);
        item = (int32_t)p;
        if (cand < (int32_t)(old >> 32)) {
          c.imp++;
          return ((uint32_t)old & IDLE) != 0u;
        }
        return false;
      }
      p = (p + 1u) & mask;
      key = (uint32_t)lds_ld(lo((int32_t)p));
    }
    __hip_atomic_store(over, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    return false;
  }
  __device__ __forceinline__ bool active(int32_t item) const { return !((uint32_t)lds_ld(lo(item)) & IDLE); }
  __device__ __forceinline__ void deactivate(int32_t item) const {
    atomicOr(reinterpret_cast<uint32_t *>(lo(item)), IDLE);
  }
  __device__ __forceinline__ bool reactivate(int32_t item) const {
    return (atomicAnd(reinterpret_cast<uint32_t *>(lo(item)), ~IDLE) & IDLE) != 0u;
  }
  __device__ __forceinline__ void claim_group(int32_t g, int lane, bool act) const {
    if (act) deactivate((g << 6) + lane);
  }
  __device__ __forceinline__ bool full() const { return lds_ld(count) > limit; }
};

// Goal-directed queries (one destination, Section I): a store that only keeps
// what can still lead to an earlier arrival at the target.  bound (LDS) is the
// earliest arrival at the target found so far.  Any journey through a stop
// reached at x arrives at the target later than x (lam >= 1), so a candidate
// >= bound is not written, a listed stop whose arrival is >= bound is dropped
// when taken, and the query ends once every listed stop is at or past bound:
// entry target of the result is then exact (every prefix of an optimal
// journey to the target arrives before bound, so none of it is pruned).  The
// target itself is never expanded: its types give arrivals after bound.
// Destination of query Q of a launch (-1: every stop).
__device__ __forceinline__ int32_t batch_target(const RunArgs &a, const QueryDev &Q) {
  return a.queries ? a.targets[Q.index] : a.single_target;
}

template <class Inner>
struct GoalStore : Inner {
  static constexpr bool kGoal = true;
  int32_t *bound;
  int32_t target;
  __device__ __forceinline__ int32_t goal_bound() const { return lds_ld(bound); }
  __device__ __forceinline__ bool improve(int32_t v, int32_t pos, int32_t av, int32_t cand, int32_t &item,
                                          Ctr &c) const {
    if (cand >= lds_ld(bound)) return false;
    if (v == target) {
      atomicMin(bound, cand);
      Inner::improve(v, pos, av, cand, item, c);
      return false;
    }
    return Inner::improve(v, pos, av, cand, item, c);
  }
};

// Relax (Algorithm 3) U connection types per lane, with their memory reads
// overlapped: all type records (and, for the grid, the grid entries, whose
// addresses need no record), then the (speculative) cluster headers, then the
// on-chip arrival lookups, then the rare array chunks, then the updates.
// Lane type u: j[u] of a tail stop with types [tb[u], tb[u] + tn[u]) reached
// at x[u]; ok[u] false = no type.
template <int KIND, int U, class Store, class Push>
__device__ __forceinline__ void relax_batch(const GraphG &G, const Store &S, const int64_t *j,
                                            const int32_t *tb, const int32_t *tn, const int32_t *x,
                                            const bool *ok, Push &P, Ctr &c) {
  int4 r[U], r2[U];
  Look L[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t jj = ok[u] ? j[u] : 0;  // type 0 always exists when any item does
    if constexpr (KIND == kKindGrid) {
      r[u] = G.side[jj];  // {v, lam, first type of v, type count of v}
      look_locate_grid(G, jj, tb[u], tn[u], x[u], L[u]);
      if (!ok[u]) L[u].mode = 0;
      look_fetch_headers<KIND>(G, r[u], L[u]);
    } else {
      r[u] = G.ty[2 * jj];
      r2[u] = G.ty[2 * jj + 1];
    }
  }
  if constexpr (KIND != kKindGrid) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      look_locate<KIND>(G, r[u], KIND == EAT_LAYOUT_HYBRID ? (uint32_t)r2[u].z : 0u, x[u], L[u]);
      if (!ok[u]) L[u].mode = 0;
      look_fetch_headers<KIND>(G, r[u], L[u]);
    }
  }
  int32_t av[U], pos[U];
  bool live[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    pos[u] = -1;
    av[u] = ok[u] ? S.find(r[u].x, pos[u]) : INF;
    // any departure leaves at t_c >= x, so it arrives at >= x + lam: skip the
    // type when that cannot beat arr[v] (early termination, Section III-D)
    live[u] = ok[u] && x[u] < av[u] - r[u].y && L[u].mode != 0;
    if (ok[u]) c.tev++;
    if (live[u]) {
      count_fetch<KIND>(r[u], L[u], c);
      look_fetch_chunks<KIND>(G, x[u], L[u], c);
    }
  }
  bool want[U];
  int32_t item[U], val[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    want[u] = false;
    item[u] = 0;
    val[u] = INF;
    if (live[u]) {
      const int32_t tc = look_finish<KIND>(G, r[u], x[u], L[u], c);
      if (tc != INF) {
        const int32_t cand = tc + r[u].y;
        if (cand < av[u]) {
          want[u] = S.improve(r[u].x, pos[u], av[u], cand, item[u], c);
          val[u] = cand;
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if constexpr (KIND == kKindGrid) P(want[u], item[u], r[u].z, r[u].w, val[u]);
    else P(want[u], item[u], r2[u].x, r2[u].y, val[u]);
  }
}

// One connection type per lane.
template <int KIND, class Store, class Push>
__device__ __forceinline__ void relax(const GraphG &G, const Store &S, int64_t j, int32_t b, int32_t n, int32_t x,
                                      Push &P, Ctr &c) {
  const bool ok = true;
  relax_batch<KIND, 1>(G, S, &j, &b, &n, &x, &ok, P, c);
}

struct Shared {
  int32_t q, cnt, count, over, reached;
  int32_t bound;                // goal-directed queries: best arrival at the target so far
  int32_t nmin[3];              // smallest arrival pushed in round r: nmin[r % 3]
  int32_t cur[3];               // wave-claim cursor of round r: cur[r % 3]
  int32_t wcur, resume;         // sweep: next group to claim, first group of the next chunk
  int32_t first, start;         // sweep: the chunk's first group, its first list entry
  unsigned long long cx[3];     // round r: low half entries pushed to the next list
  unsigned long long xt[3];     // round r (per sweep chunk): low half X entries, high half their types
  unsigned long long acc[5];
  // windows of 64 types: bit i of wstart[w] is set if an X entry's types start
  // at type 64 w + i; wentry[w] is the X entry holding type 64 w.  A wave
  // clears the bits of each window it relaxes, so they are zero between rounds.
  unsigned long long wstart[kWin];
  int32_t wentry[kWin];
  // the infinity fill of the result slab still to issue: 16-byte chunks
  // [fill_next, fill_n4) of fill_p (table queries; see fill_idle)
  int4 *fill_p;
  int32_t fill_n4, fill_next;
};
static_assert(sizeof(Shared) <= kStaticLds, "the plan reserves kStaticLds bytes of LDS for Shared");

__device__ __forceinline__ uint64_t lanes_below(int lane) { return (1ull << lane) - 1ull; }

typedef int v4i __attribute__((ext_vector_type(4)));

// The slab's infinity fill of a table query is issued in pieces by waves that
// would otherwise wait at the end of a round: a wave's reads wait for every
// store it issued before them (one in-order counter), so a fill issued all at
// once up front would hold up the query's first reads.  k chunks of 16 bytes
// per lane, nontemporal (the slab's lines are not read again).
__device__ __forceinline__ void fill_issue(Shared &sh, int32_t k) {
  const int32_t n4 = sh.fill_n4;
  if (lds_ld(&sh.fill_next) >= n4) return;
  const int lane = __lane_id();
  int32_t base = 0;
  if (lane == 0) base = atomicAdd(&sh.fill_next, 64 * k);
  base = __builtin_amdgcn_readlane(base, 0);
  gp<v4i> a4 = (gp<v4i>)sh.fill_p;
  const v4i inf4 = {INF, INF, INF, INF};
  for (int32_t j = 0; j < k; ++j) {
    const int32_t i = base + 64 * j + lane;
    if (i < n4) __builtin_nontemporal_store(inf4, a4 + i);
  }
}

// The rest of the deferred fill, by the whole work-group (after a barrier
// that ended the rounds, so fill_next is final).
template <int B>
__device__ __forceinline__ void fill_rest(Shared &sh) {
  const int32_t n4 = sh.fill_n4;
  gp<v4i> a4 = (gp<v4i>)sh.fill_p;
  const v4i inf4 = {INF, INF, INF, INF};
  for (int32_t i = sh.fill_next + (int32_t)threadIdx.x; i < n4; i += B) __builtin_nontemporal_store(inf4, a4 + i);
}

// Expand the entries of list[0..n) whose arrival is below thr; the others
// are deferred: they go to the next list unexpanded, still active (made
// active again after a sweep, which staged them), so a later round expands
// them.  An expanded entry is made idle (with `clear`; a sweep has done it
// already) before its connection types are relaxed, so an improvement that
// lands later pushes it again.
// TPV == 0: the take pass lists the expanded entries in X, numbering their
//   connection types consecutively; the windows of 64 types are dealt to the
//   waves U at a time (wave w: windows wU .. wU + U - 1, then the U windows
//   U waves further on, ...), one step per U windows, so a round of T types
//   costs every wave at most ceil(T / (64 U waves)) steps whatever its stops'
//   degrees.
//   A round of more than kWin windows falls back to wave claims: each wave
//   takes 4 * U entries at a time from a cursor and spreads their types over
//   its lanes.
// TPV > 0: virtual warps (Section IV-B) -- groups of TPV lanes, one stop per
//   group, lane i of a group takes the stop's types i, i + TPV, ...
template <int TPV, int KIND, int U, int B, class Store>
__device__ __forceinline__ void expand_list(const GraphG &G, const Store &S, const FList &cur, int32_t n,
                                            bool clear, int32_t thr, ListPush &P, const XList X, Shared &sh,
                                            int r3, Ctr &c) {
  // Takes entry e (e < n), reading its arrival x: true if it is expanded
  // this round (with its type range in beg, cnt); defer = pushed to the next
  // list instead.  No relaxation runs during the take.
  auto take = [&](int32_t e, int32_t &item, int32_t &beg, int32_t &cnt, int32_t &x, bool &defer) -> bool {
    item = cur.item[e];
    beg = cur.beg[e];
    cnt = cur.cnt[e];
    x = S.value(item);
    if constexpr (Store::kGoal) {
      if (x >= S.goal_bound()) {  // cannot lead to an earlier arrival at the target
        defer = false;
        if (clear) S.deactivate(item);
        return false;
      }
    }
    defer = thr != INF && x >= thr;
    if (defer) {
      // list mode: still active; after a sweep, active again unless an
      // improvement of this round has made it so (and pushed it) already
      if (!clear) defer = S.reactivate(item);
      return false;
    }
    if (clear) S.deactivate(item);
    if (cnt < 0) {  // staged by a sweep: load the stop's type range
      const int2 r = G.vt[S.stop(item)];
      beg = r.x;
      cnt = r.y;
    }
    c.act++;
    return true;
  };
  const int lane = __lane_id();
  if constexpr (TPV == 0) {
    unsigned long long *const xt = &sh.xt[r3];
    // Take pass: every thread takes list entries.  Deferred ones go to the
    // next list (one atomic per wave); expanded ones with connection types go
    // to X with the offset of their first type (one more atomic per wave books
    // the X entries and the types together, so X order is type order), and
    // mark their window starts.
    for (int32_t e0 = 0; e0 < n; e0 += B) {
      const int32_t e = e0 + (int32_t)threadIdx.x;
      bool defer = false, go = false;
      int32_t item = 0, beg = 0, cnt = 0, x = INF;
      if (e < n) go = take(e, item, beg, cnt, x, defer);
      go = go && cnt > 0;  // a stop without connection types has nothing to relax
      const uint64_t md = __ballot(defer), mg = __ballot(go);
      if (md) {
        if (defer) P.lmin = min(P.lmin, x);
        const int leader = __ffsll((unsigned long long)md) - 1;
        uint32_t lo = 0;
        if (lane == leader) lo = (uint32_t)atomicAdd(P.cx, (unsigned long long)__popcll(md));
        lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)lo, leader);
        if (defer && P.append) {
          const int32_t slot = (int32_t)lo + (int32_t)__popcll(md & lanes_below(lane));
          if (slot < P.fcap) {
            P.nxt.item[slot] = item;
            P.nxt.beg[slot] = beg;
            P.nxt.cnt[slot] = cnt;
          }
        }
      }
      if (mg) {  // every lane active: the scan reads all of them
        const int32_t mine = go ? cnt : 0;
        const int32_t incl = wave_incl_sum(mine);
        const int32_t tot = __builtin_amdgcn_readlane(incl, 63);
        const int leader = __ffsll((unsigned long long)mg) - 1;
        unsigned long long old = 0;
        if (lane == leader)
          old = atomicAdd(xt, (unsigned long long)__popcll(mg) | ((unsigned long long)(uint32_t)tot << 32));
        const int32_t xb = __builtin_amdgcn_readlane((int32_t)(uint32_t)old, leader);
        const int32_t tb = __builtin_amdgcn_readlane((int32_t)(uint32_t)(old >> 32), leader);
        if (go) {
          const int32_t slot = xb + (int32_t)__popcll(mg & lanes_below(lane));
          const int32_t toff = tb + incl - mine;
          X[slot] = make_int4(beg, cnt, x, toff);
          if ((toff >> 6) < kWin) atomicOr(&sh.wstart[toff >> 6], 1ull << (toff & 63));
          // the windows whose first type is one of this entry's
          for (int32_t w = (toff + 63) >> 6; w < kWin && (w << 6) < toff + cnt; ++w) sh.wentry[w] = slot;
        }
      }
    }
    __syncthreads();  // X and the windows complete
    const unsigned long long xv = __hip_atomic_load(xt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const int32_t nx = uniform((int32_t)(uint32_t)xv), T = uniform((int32_t)(uint32_t)(xv >> 32));
    const int32_t nw = (T + 63) >> 6;
    constexpr int kWaves = B / 64;
    const int32_t wave = uniform((int32_t)(threadIdx.x >> 6));
    if (nw <= kWin) {
      // Windows: lane i of window w relaxes type k = 64 w + i, of the X entry
      // that holds it: wentry[w] plus the entries starting in (64 w, k].
      for (int32_t w0 = wave * U; w0 < nw; w0 += kWaves * U) {
        int64_t jj[U];
        int32_t tb[U], tn[U], xx[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int32_t w = w0 + u;
          const int32_t wc = w < nw ? w : nw - 1;
          const unsigned long long starts = sh.wstart[wc];
          const int32_t first = sh.wentry[wc];
          const unsigned long long upto = lane == 63 ? ~0ull : (2ull << lane) - 1ull;
          int32_t ei = first + (int32_t)__popcll(starts & ~1ull & upto);
          const int32_t k = (w << 6) + lane;
          ok[u] = w < nw && k < T && ei >= 0 && ei < nx;
          const int4 t = X[ok[u] ? ei : 0];
          const int32_t d = k - t.w;  // the type's place in its stop's range
          ok[u] = ok[u] && d >= 0 && d < t.y;
          tb[u] = ok[u] ? t.x : 0;
          tn[u] = ok[u] ? t.y : 0;
          jj[u] = ok[u] ? (int64_t)t.x + d : 0;
          xx[u] = ok[u] ? t.z : 0;
        }
        // the windows' start bits have been read by every lane: clear them
        if (lane == 0) {
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (w0 + u < nw) sh.wstart[w0 + u] = 0ull;
        }
        relax_batch<KIND, U>(G, S, jj, tb, tn, xx, ok, P, c);
      }
      // a wave with fewer steps than wave 0 issues part of the fill meanwhile
      constexpr int32_t kPer = kWaves * U;
      const int32_t most = (nw + kPer - 1) / kPer;
      const int32_t mine = nw > wave * U ? (nw - 1 - wave * U) / kPer + 1 : 0;
      if (most > mine) fill_issue(sh, min(kFillPerStep * (most - mine), 2 * kFillPerStep));
      return;
    }
    // More than kWin windows: no wave reads the start bits; clear the ones set.
    for (int32_t i = (int32_t)threadIdx.x; i < kWin; i += B) sh.wstart[i] = 0ull;
    // Wave claims: wave w first takes entries [w kC, w kC + kC) of X, then
    // further groups of kC from a shared cursor (fetched one claim ahead), and
    // spreads their connection types over its 64 lanes (a prefix sum of their
    // counts in scalar registers), U types per lane in flight, until X is used
    // up.  No block-wide scan and no barrier inside.
    int32_t *const cursor = &sh.cur[r3];
    constexpr int kC = kClaim * U;
    int32_t base = wave * kC;
    while (base < nx) {
      int32_t ahead = 0;
      if (lane == 0) ahead = atomicAdd(cursor, kC);
      int32_t beg = 0, cnt = 0, x = 0;
      if (lane < kC && base + lane < nx) {
        const int4 t = X[base + lane];
        beg = t.x;
        cnt = t.y;
        x = t.z;
      }
      int32_t sb[kC], sn[kC], sx[kC], eo[kC];  // wave-uniform
      int32_t total = 0;
#pragma unroll
      for (int i = 0; i < kC; ++i) {
        sb[i] = __builtin_amdgcn_readlane(beg, i);
        sn[i] = __builtin_amdgcn_readlane(cnt, i);
        sx[i] = __builtin_amdgcn_readlane(x, i);
        eo[i] = total;
        total += sn[i];
      }
      // wave-uniform trip count
      for (int32_t k0 = 0; k0 < total; k0 += 64 * U) {
        int64_t jj[U];
        int32_t tb[U], tn[U], xx[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int32_t k = k0 + lane + 64 * u;
          ok[u] = k < total;
          // the last entry whose offset is <= k
          int32_t bi = sb[0], oi = 0, xi = sx[0], ni = sn[0];
#pragma unroll
          for (int t = 1; t < kC; ++t) {
            const bool ge = eo[t] <= k;
            bi = ge ? sb[t] : bi;
            oi = ge ? eo[t] : oi;
            xi = ge ? sx[t] : xi;
            ni = ge ? sn[t] : ni;
          }
          tb[u] = ok[u] ? bi : 0;
          tn[u] = ok[u] ? ni : 0;
          jj[u] = ok[u] ? (int64_t)bi + (k - oi) : 0;
          xx[u] = ok[u] ? xi : 0;
        }
        relax_batch<KIND, U>(G, S, jj, tb, tn, xx, ok, P, c);
      }
      base = kWaves * kC + __builtin_amdgcn_readlane(ahead, 0);
    }
  } else {
    constexpr int kGroups = B / TPV;
    const int g = threadIdx.x / TPV, gl = threadIdx.x % TPV;
    // take the entries (defer, make idle, load unknown type ranges) before
    // any relaxation pushes
    for (int32_t e0 = 0; e0 < n; e0 += B) {
      const int32_t e = e0 + (int32_t)threadIdx.x;
      bool defer = false;
      int32_t item = 0, beg = 0, cnt = 0, x = INF;
      if (e < n) {
        if (take(e, item, beg, cnt, x, defer)) {
          cur.beg[e] = beg;
          cur.cnt[e] = cnt;
        } else {
          cur.item[e] = -1;  // not expanded this round
        }
      }
      P(defer, item, beg, cnt, x);
    }
    __syncthreads();
    for (int32_t base = 0; base < n; base += kGroups) {
      const int32_t i = base + g;
      if (i < n && cur.item[i] >= 0) {
        const int32_t x = S.value(cur.item[i]);
        const int32_t b = cur.beg[i], cn = cur.cnt[i], e = b + cn;
        for (int32_t j = b + gl; j < e; j += TPV) relax<KIND>(G, S, j, b, cn, x, P, c);
      }
    }
  }
}

struct QState {
  int32_t rounds = 0, sweeps = 0, maxf = 1, status = EAT_OK;
};

// Relaxation rounds until no arrival improves (the iteration of Algorithms 4
// and 5, with the activity flags of Section III-B).  On entry the first item
// is list0 entry 0 and active (frontier mode), or only active (topology mode);
// every other item is idle.  Returns false if the store overflowed.
template <int TPV, int KIND, int U, int B, class Store>
__device__ __forceinline__ bool run_rounds(const RunArgs &a, const GraphG &G, const Store &S, int32_t n_items,
                           const FList &list0, const FList &list1, const XList X, bool topo,
                           int32_t max_rounds, int32_t x0, Shared &sh, QState &qs, Ctr &c) {
  const int tid = threadIdx.x;
  const int lane = __lane_id();
  const int32_t ngroups = (n_items + 63) >> 6;
  FList cur = list0, nxt = list1;
  int32_t nf = topo ? 0 : 1;
  bool sweep = topo;
  int32_t rounds = 0;
  int32_t base = x0;  // smallest arrival pushed for the round ("before round 0": the first item)
  if (tid < 3) {
    sh.cx[tid] = 0ull;
    sh.xt[tid] = 0ull;
    sh.cur[tid] = 0;
    sh.nmin[tid] = tid == 2 ? x0 : INF;  // "pushed before round 0": the first item
  }
  __syncthreads();
  for (;;) {
    if (rounds >= max_rounds) {
      qs.status = EAT_ERR_NOT_CONVERGED;
      break;
    }
    const int r3 = rounds % 3;
    // the counters of round rounds + 1 were last read at the end of round
    // rounds - 2, before the barrier that ended round rounds - 1: safe to reset
    if (tid == 0) {
      sh.cx[(rounds + 1) % 3] = 0ull;
      sh.xt[(rounds + 1) % 3] = 0ull;
      sh.nmin[(rounds + 1) % 3] = INF;
      sh.cur[(rounds + 1) % 3] = 0;
    }
    // this round expands the items below the smallest arrival pushed for it
    // plus the window (that item itself always qualifies)
    const int32_t thr = (a.window <= 0 || base >= INF - a.window) ? INF : base + a.window;
    ListPush P{nxt, a.fcap, !topo, &sh.cx[r3], INF};
    if (!sweep) {
      expand_list<TPV, KIND, U, B>(G, S, cur, nf, true, thr, P, X, sh, r3, c);
    } else {
      ++qs.sweeps;
      // Chunks of up to fcap items: each wave claims groups of 64 items from
      // a shared cursor and stages a group's active items only if all of them
      // fit (no relaxation runs while staging); the next chunk resumes at the
      // first group that did not fit.  The chunk's first group always fits: it
      // owns list entries [64 - its count, 64), the others are booked from 64
      // on, so every chunk stages it and the sweep ends after at most one
      // chunk per group, whatever the order in which the waves book.
      if (tid == 0) sh.wcur = 0;
      for (;;) {
        if (tid == 0) {
          sh.cnt = 64;
          sh.start = 64;
          sh.first = sh.wcur;
          sh.cur[r3] = 0;
          sh.xt[r3] = 0ull;  // X entries of the chunk
          sh.resume = ngroups;
        }
        __syncthreads();
        // The chunk's first group, from before the barrier.  (Not the cursor
        // itself: a wave that reaches its claims first moves it, and a wave
        // that read it later could leave the sweep while the others stage a
        // chunk, so that the waves' barriers would no longer pair up.)
        const int32_t g0 = uniform(sh.first);
        if (g0 >= ngroups) break;
        for (;;) {
          int32_t g = 0;
          if (lane == 0) g = atomicAdd(&sh.wcur, 1);
          g = __builtin_amdgcn_readlane(g, 0);
          if (g >= ngroups) break;
          const int32_t it = (g << 6) + lane;
          const bool act = it < n_items && S.active(it);
          const uint64_t m = __ballot(act);
          if (!m) continue;
          const int32_t pc = (int32_t)__popcll(m);
          int32_t pos = 0;
          if (g == g0) {
            pos = 64 - pc;
            if (lane == 0) sh.start = pos;
          } else if (lane == 0) {
            pos = lds_ld(&sh.cnt);
            bool fits = false;
            while (pos + pc <= a.fcap) {
              const int32_t seen = atomicCAS(&sh.cnt, pos, pos + pc);
              if (seen == pos) {
                fits = true;
                break;
              }
              pos = seen;
            }
            if (!fits) {  // the chunk is full: this group starts the next one
              atomicMin(&sh.resume, g);
              pos = -1;
            }
          }
          pos = __builtin_amdgcn_readlane(pos, 0);
          if (pos < 0) break;
          S.claim_group(g, lane, act);  // staged: these items are expanded now
          if (act) {
            const int32_t slot = pos + (int32_t)__popcll(m & lanes_below(lane));
            cur.item[slot] = it;
            cur.cnt[slot] = -1;
          }
        }
        __syncthreads();
        const int32_t cnt = uniform(sh.cnt), st = uniform(sh.start);
        if (tid == 0) sh.wcur = min(sh.wcur, sh.resume);  // read by all after the next barrier
        if (cnt > st) {
          const FList chunk{cur.item + st, cur.beg + st, cur.cnt + st};
          expand_list<TPV, KIND, U, B>(G, S, chunk, cnt - st, false, thr, P, X, sh, r3, c);
        }
        __syncthreads();
      }
    }
    // the smallest arrival pushed in the round, one atomic per wave
    const int32_t wm = wave_min(P.lmin);
    if (lane == 0 && wm != INF) atomicMin(&sh.nmin[r3], wm);
    __syncthreads();  // all pushes of the round are in
    // independent reads, one LDS round trip
    const int32_t over = uniform(lds_ld(&sh.over));
    const bool full = uniform(S.full() ? 1 : 0) != 0;
    const int32_t nnv = uniform(lds_ld(reinterpret_cast<int32_t *>(&sh.cx[r3])));
    base = uniform(lds_ld(&sh.nmin[r3]));
    if (over != 0 || full) {
      qs.rounds += rounds + 1;
      return false;
    }
    ++rounds;
    if (nnv == 0) break;
    if constexpr (Store::kGoal) {
      // every stop of the next round is at or past the target's arrival.  No
      // thread changes bound before every thread has passed the next round's
      // first barrier, so all threads read the same value here.
      if (base >= S.goal_bound()) break;
    }
    qs.maxf = max(qs.maxf, nnv);
    const bool next_sweep = topo || nnv > a.fcap;  // an overflowed list: its flags still name every item
    FList tmp = cur;
    cur = nxt;
    nxt = tmp;
    nf = next_sweep ? 0 : nnv;
    sweep = next_sweep;
  }
  qs.rounds += rounds;
  return true;
}

// A query with its arrivals in the result slab (no table, or the table
// overflowed; the slab still holds infinity): activity bits `bits` (LDS or
// HBM, cleared here), frontier lists at l in LDS.
template <int TPV, int KIND, int U, int B, bool GOAL, class P>
__device__ __forceinline__ void slab_query(const RunArgs &a, const GraphG &G, gp<int32_t> arr, const QueryDev &Q,
                                           P bits, int32_t *l, const XList X, bool topo, int32_t max_rounds,
                                           Shared &sh, QState &qs, Ctr &c) {
  const int tid = threadIdx.x;
  const int32_t V = G.n_vertices;
  const int32_t F = a.fcap;
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  SlabStore<P> S;
  S.arr = arr;
  S.bits = bits;
  S.n = V;
  const int32_t VW = (V + 31) >> 5;
  const FList l0{l, l + F, l + 2 * F}, l1{l + 3 * F, l + 4 * F, l + 5 * F};
  for (int32_t i = tid; i < VW; i += B) bits_st(bits, i, 0u);
  if (tid == 0) {
    sh.over = 0;
    sh.fill_n4 = 0;  // the fill is complete: the slab now holds the arrivals
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (tid == 0) {
    st_arr(arr + Q.s, Q.ts);
    if constexpr (GOAL) sh.bound = batch_target(a, Q) == Q.s ? Q.ts : INF;  // a fresh start after a table overflow too
    bits_st(bits, Q.s >> 5, 1u << (Q.s & 31));
    l0.item[0] = Q.s;
    l0.cnt[0] = -1;
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if constexpr (GOAL) {
    GoalStore<SlabStore<P>> GS;
    static_cast<SlabStore<P> &>(GS) = S;
    GS.bound = &sh.bound;
    GS.target = batch_target(a, Q);
    run_rounds<TPV, KIND, U, B>(a, G, GS, V, l0, l1, X, topo, max_rounds, Q.ts, sh, qs, c);
  } else {
    run_rounds<TPV, KIND, U, B>(a, G, S, V, l0, l1, X, topo, max_rounds, Q.ts, sh, qs, c);
  }
  // reached stops
  int32_t mine = 0;
  for (int32_t i = tid; i < V; i += B) mine += ld_arr(arr + i) != INF;
  if (mine) atomicAdd(&sh.reached, mine);
}

// 768-thread work-groups share a CU two at a time, 384-thread ones four and
// 256-thread ones six at a time: 24 waves, 6 per SIMD, which needs at most
// 80 VGPRs: asked of the compiler here.
template <int TPV, int KIND, int U, int B, bool GOAL>
__global__ __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(
    B == kBlockMid || B == kBlockQuarter || B == kBlockSixth ? 6 : 1))) void k_relax(RunArgs a) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ Shared sh;

  const int tid = threadIdx.x;
  const bool batch = a.queries != nullptr;
  const bool topo = a.mode == EAT_MODE_TOPOLOGY;
  const int32_t F = a.fcap;

  for (int iter = 0;; ++iter) {
    if (tid == 0) {
      int32_t q = a.nq;
      if (batch) {
        const int32_t nb = a.n_buckets;
        int32_t b = (int32_t)(blockIdx.x % (uint32_t)nb);
        for (int32_t k = 0; k < nb; ++k, b = (b + 1 == nb) ? 0 : b + 1) {
          const int32_t lo = a.buckets[b], cnt = a.buckets[b + 1] - lo;
          int32_t *cursor = a.work + 4 + b;
          if (__hip_atomic_load(cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= cnt) continue;
          const int32_t i = __hip_atomic_fetch_add(cursor, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (i < cnt) {
            q = lo + i;
            break;
          }
        }
      } else if (iter == 0) {
        q = 0;
      }
      sh.q = q;
    }
    if (tid < 5) sh.acc[tid] = 0ull;
    if (tid < kWin) sh.wstart[tid] = 0ull;
    if (tid == 0) {
      sh.count = 0;
      sh.over = 0;
      sh.reached = 0;
    }
    __syncthreads();
    const int32_t q = uniform(sh.q);
    if (q >= a.nq) {
      // The last work-group to leave re-arms the shared counters for the next
      // launch of the same batch, so a run is a single kernel launch.
      if (batch && tid == 0) {
        const int32_t left = __hip_atomic_fetch_add(a.work, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (left == (int32_t)gridDim.x - 1) {
          const int32_t failed = __hip_atomic_exchange(a.work + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(a.work + 2, failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          for (int32_t b = 0; b < a.n_buckets; ++b)
            __hip_atomic_store(a.work + 4 + b, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(a.work, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      break;
    }
    const uint64_t t_start = wall_clock64();
    const QueryDev Q = batch ? a.queries[q] : a.single;
    const GraphG G = graph_g(a.graphs[batch ? Q.graph : 0]);
    const int32_t V = G.n_vertices;
    gp<int32_t> arr = (gp<int32_t>)Q.arr;
    const int32_t max_rounds = a.max_rounds > 0 ? a.max_rounds : (a.window > 0 ? 8 * V + 64 : V + 2);
    QState qs;
    Ctr c;

    // ---- Initialize (Algorithm 2): the slab gets infinity everywhere, with
    // nontemporal stores (streamed past the caches, so the slab does not evict
    // the graph's lines that the relaxation reads).  A table query's fill is
    // issued while its rounds run (fill_issue), the rest after them; a slab
    // query needs it first.
    const bool aligned = (reinterpret_cast<uintptr_t>(arr) & 15u) == 0;
    if (aligned && a.table_cap > 0) {
      for (int32_t i = ((V >> 2) << 2) + tid; i < V; i += B) arr[i] = INF;
      if (tid == 0) {
        sh.fill_p = reinterpret_cast<int4 *>(arr);
        sh.fill_n4 = V >> 2;
        sh.fill_next = 0;
      }
    } else {
      if (aligned) {
        gp<v4i> a4 = (gp<v4i>)arr;
        const int32_t n4 = V >> 2;
        const v4i inf4 = {INF, INF, INF, INF};
        for (int32_t i = tid; i < n4; i += B) __builtin_nontemporal_store(inf4, a4 + i);
        for (int32_t i = (n4 << 2) + tid; i < V; i += B) arr[i] = INF;
      } else {
        for (int32_t i = tid; i < V; i += B) arr[i] = INF;
      }
      if (tid == 0) {
        sh.fill_p = nullptr;
        sh.fill_n4 = 0;
        sh.fill_next = 0;
      }
    }

    bool done = false;
    // LDS: X (F x 16 bytes) | table slots or slab bits | two lists (item, beg, cnt) x F
    const XList X = reinterpret_cast<int4 *>(lds);
    uint32_t *const store = lds + 4 * F;
    if (a.table_cap > 0) {
      // ---- arrivals in the on-chip table ----------------------------------------
      const int32_t H = a.table_cap;
      TableStore T;
      T.kv = reinterpret_cast<unsigned long long *>(store);
      T.count = &sh.count;
      T.over = &sh.over;
      T.mask = (uint32_t)H - 1u;
      T.shift = 32 - a.table_bits;
      T.limit = H - H / 4;
      int32_t *l = reinterpret_cast<int32_t *>(T.kv + H);
      const FList l0{l, l + F, l + 2 * F}, l1{l + 3 * F, l + 4 * F, l + 5 * F};
      for (int32_t i = tid; i < H; i += B) T.kv[i] = EMPTY_SLOT;
      __syncthreads();
      if (tid == 0) {
        const uint32_t p = T.home(Q.s);  // empty table: the home slot is free
        T.kv[p] = ((unsigned long long)(uint32_t)Q.ts << 32) | (uint32_t)Q.s;  // active
        sh.count = 1;
        if constexpr (GOAL) sh.bound = batch_target(a, Q) == Q.s ? Q.ts : INF;
        l0.item[0] = (int32_t)p;
        l0.cnt[0] = -1;
      }
      __syncthreads();
      bool ok;
      if constexpr (GOAL) {
        GoalStore<TableStore> GS;
        static_cast<TableStore &>(GS) = T;
        GS.bound = &sh.bound;
        GS.target = batch_target(a, Q);
        ok = run_rounds<TPV, KIND, U, B>(a, G, GS, H, l0, l1, X, topo, max_rounds, Q.ts, sh, qs, c);
      } else {
        ok = run_rounds<TPV, KIND, U, B>(a, G, T, H, l0, l1, X, topo, max_rounds, Q.ts, sh, qs, c);
      }
      fill_rest<B>(sh);  // before the final values, or before slab mode after an overflow
      if (ok) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the infinity fill has landed
        __syncthreads();
        for (int32_t p = tid; p < H; p += B) {
          const unsigned long long e = T.kv[p];
          const uint32_t key = (uint32_t)e;
          // nontemporal like the fill: the reached stops' lines are not read again
          if (key != NO_KEY) __builtin_nontemporal_store((int32_t)(e >> 32), arr + (key & ~IDLE));
        }
        if (tid == 0) sh.reached = sh.count;
        done = true;
      }
    }
    if (!done) {
      // ---- arrivals in the result slab (no table, or the table overflowed) ----------
      // An overflowed table attempt never wrote the slab: it holds infinity once
      // the fill issued above has landed (slab_query waits for it).
      // The bitmap in HBM (it does not fit the LDS) is compiled into the
      // 1024-thread kernels only; the host runs such graphs with those.
      bool in_hbm = false;
      if constexpr (B == kBlock) {
        if (a.bits_global) {  // this work-group's region of HBM
          gp<uint32_t> bits = (gp<uint32_t>)(a.bits_global + (size_t)blockIdx.x * (size_t)a.bits_stride);
          slab_query<TPV, KIND, U, B, GOAL>(a, G, arr, Q, bits, reinterpret_cast<int32_t *>(store), X, topo, max_rounds,
                                      sh, qs, c);
          in_hbm = true;
        }
      }
      if (!in_hbm)
        slab_query<TPV, KIND, U, B, GOAL>(a, G, arr, Q, store, reinterpret_cast<int32_t *>(store + ((V + 31) >> 5)), X,
                                    topo, max_rounds, sh, qs, c);
    }

    // ---- per-query statistics --------------------------------------------------
    if (a.stats || (qs.status != EAT_OK && a.n_failed)) {
      // wave sums first, then one LDS atomic per wave and counter
      uint32_t v5[5] = {c.act, c.tev, c.hdr, c.pool, c.imp};
#pragma unroll
      for (int k = 0; k < 5; ++k) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) v5[k] += __shfl_xor(v5[k], d);
      }
      if (__lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < 5; ++k) atomicAdd(&sh.acc[k], (unsigned long long)v5[k]);
      }
      __syncthreads();
      if (tid == 0) {
        if (a.stats) {
          eat_query_stats *st = a.stats + Q.index;
          st->status = qs.status;
          st->rounds = qs.rounds;
          st->sweep_rounds = qs.sweeps;
          st->max_frontier = qs.maxf;
          st->reached = sh.reached;
          st->spilled = done ? 0 : (a.table_cap > 0 ? 1 : 0);
          st->activations = (int64_t)sh.acc[0];
          st->type_evals = (int64_t)sh.acc[1];
          st->header_loads = (int64_t)sh.acc[2];
          st->pool_loads = (int64_t)sh.acc[3];
          st->improvements = (int64_t)sh.acc[4];
          st->elapsed_ns = (int64_t)((wall_clock64() - t_start) * (uint64_t)a.ns_per_tick >> 10);
        }
        if (qs.status != EAT_OK && a.n_failed)
          __hip_atomic_fetch_add(a.n_failed, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (a.done) {
      // every thread's slab (and thread 0's statistics) writes reach system
      // scope before the query's completion word does
      __threadfence_system();
      __syncthreads();
      if (tid == 0) __hip_atomic_store(a.done + Q.index, a.epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __syncthreads();
  }
}


// TPV = 0: type windows with ub connection types in flight per lane
// (1..3); TPV > 0: virtual warps of TPV lanes.  Goal-directed queries (goal)
// run the type-window kernels with one type per lane.
template <int KIND>
RelaxFn relax_fn(int tpv, int ub, int block, bool goal) {
  if (goal) {
    if (tpv != 0 || ub != 1) return nullptr;
    return block == kBlockSmall   ? k_relax<0, KIND, 1, kBlockSmall, true>
         : block == kBlockMid     ? k_relax<0, KIND, 1, kBlockMid, true>
         : block == kBlockQuarter ? k_relax<0, KIND, 1, kBlockQuarter, true>
         : block == kBlockSixth   ? k_relax<0, KIND, 1, kBlockSixth, true>
         : block == kBlock        ? k_relax<0, KIND, 1, kBlock, true> : nullptr;
  }
  if (block == kBlockQuarter || block == kBlockSixth) {  // wave claims, one type per lane (80 VGPRs)
    if (tpv != 0 || ub != 1) return nullptr;
    return block == kBlockQuarter ? k_relax<0, KIND, 1, kBlockQuarter, false> : k_relax<0, KIND, 1, kBlockSixth, false>;
  }
  if (block == kBlockSmall) {  // wave claims only
    if (tpv != 0) return nullptr;
    return ub == 1 ? k_relax<0, KIND, 1, kBlockSmall, false>
                   : ub == 3 ? k_relax<0, KIND, 3, kBlockSmall, false> : k_relax<0, KIND, 2, kBlockSmall, false>;
  }
  if (block == kBlockMid) {  // wave claims, one type per lane: U > 1 would spill at 80 VGPRs
    if (tpv != 0 || ub != 1) return nullptr;
    return k_relax<0, KIND, 1, kBlockMid, false>;
  }
  if (block != kBlock) return nullptr;
  switch (tpv) {
    case 0: return ub == 1 ? k_relax<0, KIND, 1, kBlock, false>
                           : ub == 3 ? k_relax<0, KIND, 3, kBlock, false> : k_relax<0, KIND, 2, kBlock, false>;
    case 1: return k_relax<1, KIND, 1, kBlock, false>;
    case 2: return k_relax<2, KIND, 1, kBlock, false>;
    case 4: return k_relax<4, KIND, 1, kBlock, false>;
    case 8: return k_relax<8, KIND, 1, kBlock, false>;
    case 16: return k_relax<16, KIND, 1, kBlock, false>;
    case 32: return k_relax<32, KIND, 1, kBlock, false>;
    case 64: return k_relax<64, KIND, 1, kBlock, false>;
    default: return nullptr;
  }
}

}  // namespace

// Kernel variant of one timetable form (defined in relax_<form>.hip).
RelaxFn relax_fn_compact(int tpv, int ub, int block, bool goal);
RelaxFn relax_fn_flat(int tpv, int ub, int block, bool goal);
RelaxFn relax_fn_grid(int tpv, int ub, int block, bool goal);

}  // namespace eat
