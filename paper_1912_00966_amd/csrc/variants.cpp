// variants.cpp -- host preprocessing and C ABI of the paper's algorithm ladder
// (connection, connection type, connection type + progressions, Cluster-AP,
// edge, warps) and of the ESDG baseline; the kernels are in variant_kernels.hip.
#include "variants.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>

#include "internal.hpp"
#include "layout.hpp"

using eat::hip_err;
using eat::set_err;

struct eat_variant_graph {
  int device = 0;
  eat_variant_info info{};
  eat::VariantDev desc{};
  std::vector<int64_t> loff;  // ESDG level offsets (host: launch sizes)
  void *d_buf = nullptr;
};

namespace eat {
namespace {

template <class F>
void parallel_range(int nthreads, int64_t n, F &&f) {
  if (n <= 0) return;
  const int64_t nt = std::max<int64_t>(1, std::min<int64_t>(nthreads, n));
  std::vector<std::thread> th;
  for (int64_t i = 0; i < nt; ++i) th.emplace_back([&, i] { f(n * i / nt, n * (i + 1) / nt); });
  for (auto &x : th) x.join();
}

// The progression from d[a] with difference dd: its terms (all values of d)
// by index, visited in order; returns (terms, uncovered terms).
template <class Visit>
void walk_ap(const int32_t *d, int64_t n, int64_t a, int32_t dd, Visit &&visit) {
  visit(a);
  if (dd <= 0) return;
  int64_t p = a;
  int64_t next = (int64_t)d[a] + dd;
  for (;;) {
    const int32_t *q = std::lower_bound(d + p + 1, d + n, next);
    if (q == d + n || *q != next) return;
    p = q - d;
    visit(p);
    next += dd;
  }
}

}  // namespace

// ESDG levels (Section I-A).  Connections are the ESDG's vertices; c = (u, v,
// t, lam) -> c' = (v, w, t', lam') when t' >= t + lam and no connection of the
// edge (v, w) leaving at or after t + lam arrives before t' + lam'.  level(c')
// is the longest path to c' from a connection without incoming edges.  Every
// edge goes to a later departure (lam >= 1), so one pass in departure order
// settles each level before it is propagated.
void esdg_levels(const int32_t *cu, const int32_t *cv, const int32_t *ct, const int32_t *clam, int64_t C,
                 int32_t nv, std::vector<int32_t> &level, int64_t &n_edges) {
  // connections grouped by edge (u, v), each edge's by departure, then arrival
  std::vector<int64_t> byedge((size_t)C);
  std::iota(byedge.begin(), byedge.end(), 0);
  std::sort(byedge.begin(), byedge.end(), [&](int64_t x, int64_t y) {
    if (cu[x] != cu[y]) return cu[x] < cu[y];
    if (cv[x] != cv[y]) return cv[x] < cv[y];
    if (ct[x] != ct[y]) return ct[x] < ct[y];
    const int32_t ax = ct[x] + clam[x], ay = ct[y] + clam[y];
    return ax != ay ? ax < ay : x < y;
  });
  std::vector<int32_t> edep((size_t)C), earr((size_t)C), sufmin((size_t)C);
  std::vector<int64_t> amin((size_t)C), eoff;
  std::vector<int64_t> first_edge((size_t)nv + 1, 0);
  for (int64_t i = 0; i < C; ++i) {
    const int64_t c = byedge[(size_t)i];
    edep[(size_t)i] = ct[c];
    earr[(size_t)i] = ct[c] + clam[c];
    if (i == 0 || cu[c] != cu[byedge[(size_t)i - 1]] || cv[c] != cv[byedge[(size_t)i - 1]]) {
      eoff.push_back(i);
      first_edge[(size_t)cu[c] + 1]++;
    }
  }
  const int64_t E = (int64_t)eoff.size();
  eoff.push_back(C);
  for (int32_t a = 0; a < nv; ++a) first_edge[(size_t)a + 1] += first_edge[(size_t)a];
  // per edge: suffix minimum of the arrival and the first index achieving it
  for (int64_t e = 0; e < E; ++e) {
    const int64_t b = eoff[(size_t)e], k = eoff[(size_t)e + 1];
    for (int64_t i = k - 1; i >= b; --i) {
      if (i == k - 1 || earr[(size_t)i] <= sufmin[(size_t)i + 1]) {
        sufmin[(size_t)i] = earr[(size_t)i];
        amin[(size_t)i] = i;
      } else {
        sufmin[(size_t)i] = sufmin[(size_t)i + 1];
        amin[(size_t)i] = amin[(size_t)i + 1];
      }
    }
  }
  // connections in departure order
  std::vector<int64_t> order((size_t)C);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return ct[x] < ct[y]; });
  level.assign((size_t)C, 0);
  n_edges = 0;
  for (int64_t c : order) {
    const int32_t v = cv[c];
    const int32_t x = ct[c] + clam[c];
    const int32_t lc = level[(size_t)c] + 1;
    for (int64_t e = first_edge[(size_t)v]; e < first_edge[(size_t)v + 1]; ++e) {
      const int64_t b = eoff[(size_t)e], end = eoff[(size_t)e + 1];
      const int64_t p = std::lower_bound(edep.begin() + b, edep.begin() + end, x) - edep.begin();
      if (p == end) continue;
      const int32_t A = sufmin[(size_t)p];
      // every connection of the edge from p on that arrives at A
      for (int64_t q = amin[(size_t)p]; q < end && earr[(size_t)q] == A;) {
        int32_t &l = level[(size_t)byedge[(size_t)q]];
        l = std::max(l, lc);
        ++n_edges;
        q = (q + 1 < end && sufmin[(size_t)q + 1] == A) ? amin[(size_t)q + 1] : end;
      }
    }
  }
}

void greedy_ap_cover(const int32_t *d, int64_t n, std::vector<int32_t> &out) {
  std::vector<char> cov((size_t)n, 0);
  int64_t covered = 0, a = 0;
  while (covered < n) {
    while (cov[(size_t)a]) ++a;
    int64_t best_unc = 1, best_len = 1;
    int32_t best_d = 0;
    for (int64_t j = a + 1; j < n; ++j) {
      const int32_t dd = d[j] - d[a];
      int64_t len = 0, unc = 0;
      walk_ap(d, n, a, dd, [&](int64_t i) {
        ++len;
        unc += !cov[(size_t)i];
      });
      if (unc > best_unc || (unc == best_unc && len > best_len)) {  // ties: the smaller difference
        best_unc = unc;
        best_len = len;
        best_d = dd;
      }
    }
    int64_t last = a;
    walk_ap(d, n, a, best_d, [&](int64_t i) {
      if (!cov[(size_t)i]) {
        cov[(size_t)i] = 1;
        ++covered;
      }
      last = i;
    });
    out.push_back(d[a]);
    out.push_back(d[last]);
    out.push_back(best_d);
    out.push_back(0);
  }
}

eat_status build_variants(const int32_t *u, const int32_t *v, const int32_t *t, const int32_t *lam, int64_t n,
                          int32_t nv, const eat_variant_build_options &opt, VariantHost &H, std::string *err) {
  for (int r : opt.reserved)
    if (r != 0) {
      *err = "reserved build options must be zero";
      return EAT_ERR_INVALID_ARGUMENT;
    }
  const int32_t cw = opt.cluster_seconds ? opt.cluster_seconds : 3600;
  if (cw < 1 || cw > 86400) {
    *err = "cluster_seconds must be 1..86400";
    return EAT_ERR_INVALID_ARGUMENT;
  }
  eat_build_options bo{};
  bo.layout = EAT_LAYOUT_FLAT;
  bo.n_threads = opt.n_threads;
  eat_layout L;
  eat_status st = build_layout(u, v, t, lam, n, nv, bo, L, err);
  if (st != EAT_OK) return st;
  const unsigned hw = std::thread::hardware_concurrency();
  const int nth = std::max(1, std::min(opt.n_threads > 0 ? opt.n_threads : (hw ? (int)hw : 4), 64));
  const int64_t T = L.n_types, C = L.n_conn;
  if (C > INT32_MAX || T > INT32_MAX) {
    *err = "more than 2^31-1 connections";
    return EAT_ERR_UNSUPPORTED;
  }
  try {
    H.n_vertices = nv;
    H.cluster_seconds = cw;
    // types, their departures, and the connections in type order
    H.tu.resize((size_t)T);
    H.tv.resize((size_t)T);
    H.tlam.resize((size_t)T);
    H.tdoff.assign((size_t)T + 1, 0);
    int32_t max_dep = 0;
    for (int32_t a = 0; a < nv; ++a)
      for (int32_t j = L.vt[(size_t)2 * a]; j < L.vt[(size_t)2 * a] + L.vt[(size_t)2 * a + 1]; ++j) {
        H.tu[(size_t)j] = a;
        H.tv[(size_t)j] = L.ty[(size_t)4 * j];
        H.tlam[(size_t)j] = L.ty[(size_t)4 * j + 1];
        H.tdoff[(size_t)j + 1] = L.ty[(size_t)4 * j + 3];
      }
    for (int64_t j = 0; j < T; ++j) H.tdoff[(size_t)j + 1] += H.tdoff[(size_t)j];
    H.dep.resize((size_t)C);
    H.cu.resize((size_t)C);
    H.cv.resize((size_t)C);
    H.ct.resize((size_t)C);
    H.clam.resize((size_t)C);
    for (int64_t j = 0; j < T; ++j) {
      const int32_t off = L.ty[(size_t)4 * j + 2];
      for (int32_t q = H.tdoff[(size_t)j]; q < H.tdoff[(size_t)j + 1]; ++q) {
        const int32_t d = L.pool[(size_t)(off + (q - H.tdoff[(size_t)j]))];
        H.dep[(size_t)q] = d;
        H.cu[(size_t)q] = H.tu[(size_t)j];
        H.cv[(size_t)q] = H.tv[(size_t)j];
        H.ct[(size_t)q] = d;
        H.clam[(size_t)q] = H.tlam[(size_t)j];
        max_dep = std::max(max_dep, d);
      }
    }
    L = eat_layout();  // free the layout
    H.n_clusters = max_dep / cw + 1;
    if ((int64_t)H.n_clusters * T >= INT32_MAX) {
      *err = "types x clusters exceeds 2^31-1: widen cluster_seconds";
      return EAT_ERR_UNSUPPORTED;
    }
    // edges: the types of one tail with one head (types are ordered by (v, lam))
    H.etoff.push_back(0);
    for (int64_t j = 0; j < T; ++j) {
      if (j == 0 || H.tu[(size_t)j] != H.tu[(size_t)j - 1] || H.tv[(size_t)j] != H.tv[(size_t)j - 1]) {
        if (j > 0) H.etoff.push_back((int32_t)j);
        H.eu.push_back(H.tu[(size_t)j]);
      }
    }
    if (T > 0) H.etoff.push_back((int32_t)T);
    // progression covers: whole types, and (type, cluster) parts, per thread
    // in contiguous type ranges, then concatenated
    std::vector<std::vector<int32_t>> tparts((size_t)nth), cparts((size_t)nth);
    std::vector<std::vector<int32_t>> tcnt((size_t)nth), ccnt((size_t)nth);
    std::vector<int64_t> split((size_t)nth + 1);
    for (int i = 0; i <= nth; ++i) split[(size_t)i] = T * i / nth;
    const int32_t K = H.n_clusters;
    parallel_range(nth, nth, [&](int64_t b, int64_t e) {
      for (int64_t th = b; th < e; ++th) {
        auto &tp = tparts[(size_t)th], &cp = cparts[(size_t)th];
        auto &tc = tcnt[(size_t)th], &cc = ccnt[(size_t)th];
        for (int64_t j = split[(size_t)th]; j < split[(size_t)th + 1]; ++j) {
          const int32_t *d = H.dep.data() + H.tdoff[(size_t)j];
          const int64_t m = H.tdoff[(size_t)j + 1] - H.tdoff[(size_t)j];
          const size_t before = tp.size();
          greedy_ap_cover(d, m, tp);
          tc.push_back((int32_t)((tp.size() - before) / 4));
          int64_t i = 0;
          for (int32_t k = 0; k < K; ++k) {
            int64_t i2 = i;
            while (i2 < m && d[i2] / cw == k) ++i2;
            const size_t cb = cp.size();
            if (i2 > i) greedy_ap_cover(d + i, i2 - i, cp);
            cc.push_back((int32_t)((cp.size() - cb) / 4));
            i = i2;
          }
        }
      }
    });
    H.tapoff.assign((size_t)T + 1, 0);
    H.cloff.assign((size_t)T * K + 1, 0);
    int64_t jt = 0, jc = 0;
    for (int th = 0; th < nth; ++th) {
      H.tap.insert(H.tap.end(), tparts[(size_t)th].begin(), tparts[(size_t)th].end());
      H.cap.insert(H.cap.end(), cparts[(size_t)th].begin(), cparts[(size_t)th].end());
      for (int32_t c : tcnt[(size_t)th]) {
        H.tapoff[(size_t)jt + 1] = H.tapoff[(size_t)jt] + c;
        ++jt;
      }
      for (int32_t c : ccnt[(size_t)th]) {
        H.cloff[(size_t)jc + 1] = H.cloff[(size_t)jc] + c;
        ++jc;
      }
      std::vector<int32_t>().swap(tparts[(size_t)th]);
      std::vector<int32_t>().swap(cparts[(size_t)th]);
    }
    if ((int64_t)H.tap.size() / 4 >= INT32_MAX || (int64_t)H.cap.size() / 4 >= INT32_MAX) {
      *err = "too many progression tuples";
      return EAT_ERR_UNSUPPORTED;
    }
    // ESDG
    if (opt.esdg) {
      std::vector<int32_t> level;
      esdg_levels(H.cu.data(), H.cv.data(), H.ct.data(), H.clam.data(), C, nv, level, H.n_esdg_edges);
      int32_t nl = 0;
      for (int32_t l : level) nl = std::max(nl, l + 1);
      H.n_levels = C > 0 ? nl : 0;
      std::vector<int64_t> cnt((size_t)H.n_levels + 1, 0);
      for (int32_t l : level) cnt[(size_t)l + 1]++;
      for (int32_t l = 0; l < H.n_levels; ++l) cnt[(size_t)l + 1] += cnt[(size_t)l];
      H.loff.assign(cnt.begin(), cnt.end());
      H.lu.resize((size_t)C);
      H.lv.resize((size_t)C);
      H.lt.resize((size_t)C);
      H.llam.resize((size_t)C);
      std::vector<int64_t> at(cnt.begin(), cnt.end() - 1);
      for (int64_t c = 0; c < C; ++c) {
        const int64_t p = at[(size_t)level[(size_t)c]]++;
        H.lu[(size_t)p] = H.cu[(size_t)c];
        H.lv[(size_t)p] = H.cv[(size_t)c];
        H.lt[(size_t)p] = H.ct[(size_t)c];
        H.llam[(size_t)p] = H.clam[(size_t)c];
      }
    }
  } catch (const std::bad_alloc &) {
    *err = "host allocation failed";
    return EAT_ERR_OUT_OF_MEMORY;
  }
  return EAT_OK;
}

}  // namespace eat

extern "C" eat_status eat_variant_graph_build(const int32_t *u, const int32_t *v, const int32_t *t,
                                              const int32_t *lam, int64_t n_conn, int32_t n_vertices,
                                              const eat_variant_build_options *opt, eat_variant_graph **out) {
  if (!out) return set_err(EAT_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  eat_variant_build_options o{};
  if (opt) o = *opt;
  eat::VariantHost H;
  std::string err;
  eat_status st = eat::build_variants(u, v, t, lam, n_conn, n_vertices, o, H, &err);
  if (st != EAT_OK) return set_err(st, err);
  auto *g = new (std::nothrow) eat_variant_graph();
  if (!g) return set_err(EAT_ERR_OUT_OF_MEMORY, "host allocation failed");
  HIP_TRY(hipGetDevice(&g->device));
  // one device buffer for every array
  struct Part {
    const void *src;
    size_t bytes;
    size_t off;
  };
  std::vector<Part> parts;
  size_t total = 0;
  auto add = [&](const void *p, size_t bytes) {
    parts.push_back({p, bytes, total});
    total += eat::align_up(std::max<size_t>(bytes, 4));
    return parts.size() - 1;
  };
  auto vec = [&](const std::vector<int32_t> &x) { return add(x.data(), x.size() * 4); };
  const size_t i_cu = vec(H.cu), i_cv = vec(H.cv), i_ct = vec(H.ct), i_cl = vec(H.clam);
  const size_t i_tu = vec(H.tu), i_tv = vec(H.tv), i_tl = vec(H.tlam), i_td = vec(H.tdoff), i_dep = vec(H.dep);
  const size_t i_tao = vec(H.tapoff), i_ta = vec(H.tap), i_clo = vec(H.cloff), i_ca = vec(H.cap);
  const size_t i_eu = vec(H.eu), i_eo = vec(H.etoff);
  const size_t i_lu = vec(H.lu), i_lv = vec(H.lv), i_lt = vec(H.lt), i_ll = vec(H.llam);
  hipError_t e = hipMalloc(&g->d_buf, total);
  if (e != hipSuccess) {
    delete g;
    return set_err(EAT_ERR_OUT_OF_MEMORY, "hipMalloc of the variant graph failed");
  }
  char *base = static_cast<char *>(g->d_buf);
  for (const Part &p : parts)
    if (e == hipSuccess && p.bytes) e = hipMemcpy(base + p.off, p.src, p.bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(g->d_buf);
    delete g;
    return hip_err(e, "variant graph upload");
  }
  auto P = [&](size_t i) { return reinterpret_cast<const int32_t *>(base + parts[i].off); };
  eat::VariantDev &d = g->desc;
  d.cu = P(i_cu), d.cv = P(i_cv), d.ct = P(i_ct), d.clam = P(i_cl);
  d.tu = P(i_tu), d.tv = P(i_tv), d.tlam = P(i_tl), d.tdoff = P(i_td), d.dep = P(i_dep);
  d.tapoff = P(i_tao), d.tap = reinterpret_cast<const int4 *>(P(i_ta));
  d.cloff = P(i_clo), d.cap = reinterpret_cast<const int4 *>(P(i_ca));
  d.eu = P(i_eu), d.etoff = P(i_eo);
  d.lu = P(i_lu), d.lv = P(i_lv), d.lt = P(i_lt), d.llam = P(i_ll);
  d.n_conn = (int64_t)H.cu.size();
  d.n_types = (int64_t)H.tu.size();
  d.n_edges = (int64_t)H.eu.size();
  d.n_vertices = H.n_vertices;
  d.n_clusters = H.n_clusters;
  d.cluster_seconds = H.cluster_seconds;
  d.n_levels = H.n_levels;
  g->loff.assign(H.loff.begin(), H.loff.end());
  eat_variant_info &in = g->info;
  in.n_vertices = H.n_vertices;
  in.n_clusters = H.n_clusters;
  in.n_levels = H.n_levels;
  in.n_conn = d.n_conn;
  in.n_types = d.n_types;
  in.n_edges = d.n_edges;
  in.n_type_aps = (int64_t)H.tap.size() / 4;
  in.n_cluster_aps = (int64_t)H.cap.size() / 4;
  in.n_esdg_edges = H.n_esdg_edges;
  in.device_bytes = (int64_t)total;
  *out = g;
  return EAT_OK;
}

extern "C" eat_status eat_ap_cover(const int32_t *d, int64_t n, int32_t *out, int64_t cap, int64_t *n_out) {
  if (n < 0 || cap < 0 || !n_out || (n > 0 && !d) || (cap > 0 && !out))
    return set_err(EAT_ERR_INVALID_ARGUMENT, "bad size or NULL array");
  for (int64_t i = 1; i < n; ++i)
    if (d[i] <= d[i - 1]) return set_err(EAT_ERR_INVALID_ARGUMENT, "values must be strictly increasing");
  std::vector<int32_t> v;
  try {
    eat::greedy_ap_cover(d, n, v);
  } catch (const std::bad_alloc &) {
    return set_err(EAT_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
  const int64_t k = (int64_t)v.size() / 4;
  *n_out = k;
  if (k > cap) return cap == 0 && !out ? EAT_OK : set_err(EAT_ERR_UNSUPPORTED, "cap too small");
  for (int64_t i = 0; i < k; ++i) {
    out[3 * i] = v[(size_t)(4 * i)];
    out[3 * i + 1] = v[(size_t)(4 * i + 1)];
    out[3 * i + 2] = v[(size_t)(4 * i + 2)];
  }
  return EAT_OK;
}

extern "C" eat_status eat_esdg_levels(const int32_t *u, const int32_t *v, const int32_t *t, const int32_t *lam,
                                      int64_t n_conn, int32_t n_vertices, int32_t *level, int32_t *n_levels,
                                      int64_t *n_edges) {
  if (n_conn < 0 || n_vertices < 0 || (n_conn > 0 && (!u || !v || !t || !lam || !level)))
    return set_err(EAT_ERR_INVALID_ARGUMENT, "bad size or NULL array");
  for (int64_t i = 0; i < n_conn; ++i)
    if (u[i] < 0 || u[i] >= n_vertices || v[i] < 0 || v[i] >= n_vertices || t[i] < 0 || lam[i] < 1 ||
        (int64_t)t[i] + lam[i] > (int64_t)EAT_INF - 1)
      return set_err(EAT_ERR_INVALID_ARGUMENT, "connection " + std::to_string(i) + " out of range");
  std::vector<int32_t> lv;
  int64_t ne = 0;
  try {
    eat::esdg_levels(u, v, t, lam, n_conn, n_vertices, lv, ne);
  } catch (const std::bad_alloc &) {
    return set_err(EAT_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
  int32_t nl = 0;
  for (int64_t i = 0; i < n_conn; ++i) {
    level[i] = lv[(size_t)i];
    nl = std::max(nl, lv[(size_t)i] + 1);
  }
  if (n_levels) *n_levels = nl;
  if (n_edges) *n_edges = ne;
  return EAT_OK;
}

extern "C" eat_status eat_variant_graph_info(const eat_variant_graph *g, eat_variant_info *out) {
  if (!g || !out) return set_err(EAT_ERR_INVALID_ARGUMENT, "NULL argument");
  *out = g->info;
  return EAT_OK;
}

extern "C" void eat_variant_graph_free(eat_variant_graph *g) {
  if (!g) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(g->d_buf);
  delete g;
}

extern "C" eat_status eat_variant_query(const eat_variant_graph *g, int32_t s, int32_t ts, int32_t *arr,
                                        void *stream, const eat_variant_options *opt, eat_variant_stats *stats) {
  if (!g) return set_err(EAT_ERR_INVALID_ARGUMENT, "graph is NULL");
  if (!arr) return set_err(EAT_ERR_INVALID_ARGUMENT, "arr is NULL");
  const int32_t V = g->info.n_vertices;
  if (s < 0 || s >= V) return set_err(EAT_ERR_INVALID_ARGUMENT, "source out of range");
  if (ts < 0) return set_err(EAT_ERR_INVALID_ARGUMENT, "ts must be >= 0");
  eat_variant_options o{};
  if (opt) o = *opt;
  for (int r : o.reserved)
    if (r != 0) return set_err(EAT_ERR_INVALID_ARGUMENT, "reserved options must be zero");
  if (o.variant < EAT_VARIANT_CONNECTION || o.variant > EAT_VARIANT_ESDG)
    return set_err(EAT_ERR_INVALID_ARGUMENT, "unknown variant");
  const int ws = o.warp_size ? o.warp_size : 32;
  if (ws < 1 || ws > 64 || (ws & (ws - 1))) return set_err(EAT_ERR_INVALID_ARGUMENT, "warp_size must be 1, 2, .., 64");
  if (o.check_every < 0 || o.max_iterations < 0) return set_err(EAT_ERR_INVALID_ARGUMENT, "negative option");
  if (o.variant == EAT_VARIANT_ESDG && g->info.n_levels == 0 && g->info.n_conn > 0)
    return set_err(EAT_ERR_UNSUPPORTED, "the graph was built without the ESDG");
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != g->device) return set_err(EAT_ERR_INVALID_ARGUMENT, "graph lives on another device than the current one");
  hipStream_t hs = static_cast<hipStream_t>(stream);
  // scratch: change flag and counter | active | next
  const size_t b_f = 256, b_a = eat::align_up((size_t)V);
  char *buf = nullptr;
  HIP_TRY(hipMalloc(reinterpret_cast<void **>(&buf), b_f + 2 * b_a));
  int32_t *flag = reinterpret_cast<int32_t *>(buf);
  unsigned long long *count = o.count ? reinterpret_cast<unsigned long long *>(buf + 8) : nullptr;
  uint8_t *act = reinterpret_cast<uint8_t *>(buf + b_f), *nxt = act + b_a;
  auto finish = [&](eat_status r) {
    (void)hipStreamSynchronize(hs);
    (void)hipFree(buf);
    return r;
  };
  eat_variant_stats st{};
  hipError_t e = hipMemsetAsync(buf, 0, b_f, hs);
  if (e == hipSuccess) e = eat::launch_variant_init(arr, act, nxt, V, s, ts, hs);
  if (e != hipSuccess) return finish(hip_err(e, "variant init"));
  if (o.variant == EAT_VARIANT_ESDG) {
    // Section I-A: the levels in increasing order, the connections of one
    // level in parallel; one pass is exact
    for (int32_t l = 0; l < g->info.n_levels && e == hipSuccess; ++l)
      e = eat::launch_esdg_level(g->desc, g->loff[(size_t)l], g->loff[(size_t)l + 1], arr, count, hs);
    st.iterations = g->info.n_levels;
  } else {
    const int32_t every = o.check_every ? o.check_every : 1;
    const int32_t limit = o.max_iterations ? o.max_iterations : V + 2;
    st.status = EAT_ERR_NOT_CONVERGED;
    int32_t it = 0;
    while (it < limit && e == hipSuccess) {
      // iterations it .. it + every - 1, then one read of the change flag
      // (set by any of them; cleared after the read)
      const int32_t n = std::min(every, limit - it);
      for (int32_t k = 0; k < n && e == hipSuccess; ++k) {
        e = eat::launch_variant_iteration(g->desc, o.variant, ws, arr, act, nxt, flag, count, hs);
        std::swap(act, nxt);
        if (e == hipSuccess) e = eat::launch_variant_clear(nxt, V, hs);
      }
      it += n;
      int32_t changed = 0;
      if (e == hipSuccess) e = hipMemcpyAsync(&changed, flag, 4, hipMemcpyDeviceToHost, hs);
      if (e == hipSuccess) e = hipMemsetAsync(flag, 0, 4, hs);
      if (e == hipSuccess) e = hipStreamSynchronize(hs);
      ++st.host_checks;
      if (e == hipSuccess && !changed) {
        st.status = EAT_OK;
        break;
      }
    }
    st.iterations = it;
  }
  if (e == hipSuccess && count) e = hipMemcpyAsync(&st.examined, count, 8, hipMemcpyDeviceToHost, hs);
  if (e == hipSuccess) e = hipStreamSynchronize(hs);
  if (e != hipSuccess) return finish(hip_err(e, "variant iterations"));
  if (stats) *stats = st;
  if (st.status != EAT_OK) return finish(set_err(EAT_ERR_NOT_CONVERGED, "iteration limit reached"));
  return finish(EAT_OK);
}
