// variants.hpp -- the paper's own ladder of GPU algorithms, as a comparison
// harness beside the production kernel: connection (Algorithm 4), connection
// type (Algorithm 5), connection type over arithmetic-progression tuples
// (Algorithms 5 and 6), Cluster-AP (Section II-D), edge (Section II-E) and
// (virtual) warps per edge (Sections II-F, IV-B), each a topology-driven
// iteration of one kernel launch over all its work items with the
// active / nextactive flags of Section III-B; and the edge-scan-dependency
// graph (ESDG) algorithm of Section I-A, level by level.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "eat.h"

namespace eat {

// Device arrays of a variant graph.
struct VariantDev {
  // connections in type order (connection version)
  const int32_t *cu, *cv, *ct, *clam;
  // connection types: tail, head, duration, departures dep[tdoff[j] .. tdoff[j+1]) sorted
  const int32_t *tu, *tv, *tlam, *tdoff, *dep;
  // greedy progression cover of each type's departures: tap[tapoff[j] .. tapoff[j+1])
  // = {first, last, difference, 0}, increasing first terms
  const int32_t *tapoff;
  const int4 *tap;
  // per (type j, cluster k): cap[cloff[j * n_clusters + k] .. cloff[j * n_clusters + k + 1])
  const int32_t *cloff;
  const int4 *cap;
  // edges (u, v): their types are etoff[e] .. etoff[e+1]
  const int32_t *eu, *etoff;
  // ESDG: connections ordered by level, level l = [loff[l], loff[l+1])
  const int32_t *lu, *lv, *lt, *llam;
  int64_t n_conn, n_types, n_edges;
  int32_t n_vertices, n_clusters, cluster_seconds, n_levels;
};

// Host arrays (built by build_variants).
struct VariantHost {
  int32_t n_vertices = 0, n_clusters = 1, cluster_seconds = 3600, n_levels = 0;
  int64_t n_esdg_edges = 0;
  std::vector<int32_t> cu, cv, ct, clam;
  std::vector<int32_t> tu, tv, tlam, tdoff, dep;
  std::vector<int32_t> tapoff, cloff;
  std::vector<int32_t> tap, cap;  // 4 words per tuple
  std::vector<int32_t> eu, etoff;
  std::vector<int32_t> lu, lv, lt, llam, loff;
};

// Greedy cover of sorted distinct d[0..n) by arithmetic progressions (the
// technique of Section I-A): repeatedly take the smallest uncovered value a and
// the progression from a, made only of values of d, that covers the most
// uncovered values (then the longest, then the smallest difference); appends
// {first, last, difference, 0} per progression (difference 0: one term).
void greedy_ap_cover(const int32_t *d, int64_t n, std::vector<int32_t> &out);

// ESDG level of each of the C connections (cu, cv, ct, clam) over nv stops
// (Section I-A); n_edges receives the number of dependency edges.
void esdg_levels(const int32_t *cu, const int32_t *cv, const int32_t *ct, const int32_t *clam, int64_t C,
                 int32_t nv, std::vector<int32_t> &level, int64_t &n_edges);

eat_status build_variants(const int32_t *u, const int32_t *v, const int32_t *t, const int32_t *lam, int64_t n,
                          int32_t nv, const eat_variant_build_options &opt, VariantHost &out, std::string *err);

// Launchers (variant_kernels.hip).
hipError_t launch_variant_init(int32_t *arr, uint8_t *active, uint8_t *next, int32_t nv, int32_t s, int32_t ts,
                               hipStream_t stream);
// One iteration of `variant` reading `active`, writing `next` (cleared by the
// caller) and arr; *flag |= 1 if an arrival improved; *count += examined
// departures / tuples when count is not NULL.
hipError_t launch_variant_iteration(const VariantDev &g, int variant, int warp_size, int32_t *arr,
                                    const uint8_t *active, uint8_t *next, int32_t *flag,
                                    unsigned long long *count, hipStream_t stream);
hipError_t launch_variant_clear(uint8_t *p, int32_t n, hipStream_t stream);
// ESDG: relax the connections of level l.
hipError_t launch_esdg_level(const VariantDev &g, int64_t begin, int64_t end, int32_t *arr,
                             unsigned long long *count, hipStream_t stream);

}  // namespace eat
