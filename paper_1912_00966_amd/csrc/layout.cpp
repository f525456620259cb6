// layout.cpp -- host preprocessing of a connection list into the device layout.
//
// Section III-A builds a three-level hierarchy: connection types (Section
// II-B: connections with the same tail u, head v and duration lam), per type
// the clusters of departures that fall in the same hour (Section II-D), and per
// cluster the arithmetic-progression tuples that cover its departures (Section
// II-C).  Here:
//   * one active stop's types are contiguous (vt: first type and count per
//     stop) and ordered by (v, lam), which also keeps the types of one edge
//     (u, v) of Section II-E adjacent; the stops' blocks follow a breadth-first
//     order of the stop graph, so stops close in the graph sit close in memory;
//   * only non-empty clusters get a header; a 64-bit occupancy mask per type
//     plus a population count finds the header of any cluster in O(1);
//   * a cluster whose sorted departures form one progression is stored as that
//     progression (first term, difference, count); any other cluster keeps its
//     sorted departures in a pool.  The greedy multi-progression cover of the
//     paper would cover the second kind with several tuples; the lookup result
//     is the same either way (the earliest departure >= x), only its cost
//     differs.
// The flat layout keeps one sorted departure array per type instead.
#include "layout.hpp"

#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>

namespace eat {
namespace {

struct Rec {  // one connection inside its tail's bucket
  int32_t v, lam, t;
};

inline bool rec_less(const Rec &a, const Rec &b) {
  if (a.v != b.v) return a.v < b.v;
  if (a.lam != b.lam) return a.lam < b.lam;
  return a.t < b.t;
}
inline bool same_type(const Rec &a, const Rec &b) { return a.v == b.v && a.lam == b.lam; }

// Pool entries start on 16-byte boundaries (the device reads them in int4
// chunks); the gaps hold infinity.
inline int64_t pad4(int64_t words) { return (words + 3) & ~int64_t(3); }

int resolve_threads(int32_t req) {
  unsigned hw = std::thread::hardware_concurrency();
  int n = req > 0 ? req : (hw ? (int)hw : 4);
  return std::max(1, std::min(n, 64));
}

template <class F>
void parallel_for_chunks(int nthreads, int64_t n, F &&f) {
  if (n <= 0) return;
  int64_t nt = std::min<int64_t>(nthreads, n);
  if (nt <= 1) {
    f(0, (int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve((size_t)nt);
  for (int64_t i = 0; i < nt; ++i) {
    int64_t b = n * i / nt, e = n * (i + 1) / nt;
    th.emplace_back([&, i, b, e] { f((int)i, b, e); });
  }
  for (auto &x : th) x.join();
}

// Per-cluster statistics of one type's sorted, distinct departures d[0..n).
// Calls emit(cluster, is_progression, first, difference, count, begin) for every
// non-empty cluster, in increasing cluster order; begin indexes d.
template <class Emit>
void for_each_cluster(const Rec *d, int64_t n, int32_t cw, Emit &&emit) {
  int64_t i = 0;
  while (i < n) {
    int32_t k = d[i].t / cw;
    int64_t j = i + 1;
    while (j < n && d[j].t / cw == k) ++j;
    int64_t cnt = j - i;
    bool ap = true;
    int32_t h = 1;
    if (cnt >= 2) {
      h = d[i + 1].t - d[i].t;
      for (int64_t q = i + 2; q < j && ap; ++q) ap = (d[q].t - d[q - 1].t) == h;
    }
    emit(k, ap, d[i].t, h, cnt, i);
    i = j;
  }
}

// Stop order for the layout: breadth-first over the stop graph (edges in both
// directions), each connected component started from a pseudo-peripheral stop
// (the last stop reached by a first sweep).  Stops that are close in the
// graph get close positions, so one query's stops share cache lines, and a
// contiguous range of positions is a connected region.
std::vector<int32_t> locality_order(int32_t nv, const std::vector<int64_t> &out_off,
                                    const std::vector<int32_t> &out_v) {
  std::vector<int64_t> nb_off((size_t)nv + 1, 0);
  for (int32_t u = 0; u < nv; ++u) {
    nb_off[(size_t)u + 1] += out_off[(size_t)u + 1] - out_off[(size_t)u];
    for (int64_t k = out_off[(size_t)u]; k < out_off[(size_t)u + 1]; ++k) nb_off[(size_t)out_v[(size_t)k] + 1]++;
  }
  for (int32_t u = 0; u < nv; ++u) nb_off[(size_t)u + 1] += nb_off[(size_t)u];
  std::vector<int32_t> nb((size_t)nb_off[(size_t)nv]);
  std::vector<int64_t> fill(nb_off.begin(), nb_off.end() - 1);
  for (int32_t u = 0; u < nv; ++u)
    for (int64_t k = out_off[(size_t)u]; k < out_off[(size_t)u + 1]; ++k) {
      const int32_t v = out_v[(size_t)k];
      nb[(size_t)fill[(size_t)u]++] = v;
      nb[(size_t)fill[(size_t)v]++] = u;
    }
  std::vector<int32_t> order;
  order.reserve((size_t)nv);
  std::vector<int32_t> seen((size_t)nv, -1);  // component stamp of the first sweep
  std::vector<char> placed((size_t)nv, 0);
  std::vector<int32_t> queue((size_t)nv);
  for (int32_t start = 0; start < nv; ++start) {
    if (placed[(size_t)start]) continue;
    // first sweep: the last stop reached is far from `start`
    size_t qh = 0, qt = 0;
    queue[qt++] = start;
    seen[(size_t)start] = start;
    int32_t last = start;
    while (qh < qt) {
      const int32_t u = queue[qh++];
      last = u;
      for (int64_t k = nb_off[(size_t)u]; k < nb_off[(size_t)u + 1]; ++k) {
        const int32_t v = nb[(size_t)k];
        if (seen[(size_t)v] != start) {
          seen[(size_t)v] = start;
          queue[qt++] = v;
        }
      }
    }
    // second sweep from there fixes the order of the component
    qh = qt = 0;
    queue[qt++] = last;
    placed[(size_t)last] = 1;
    while (qh < qt) {
      const int32_t u = queue[qh++];
      order.push_back(u);
      for (int64_t k = nb_off[(size_t)u]; k < nb_off[(size_t)u + 1]; ++k) {
        const int32_t v = nb[(size_t)k];
        if (!placed[(size_t)v]) {
          placed[(size_t)v] = 1;
          queue[qt++] = v;
        }
      }
    }
  }
  return order;
}

}  // namespace

eat_status build_layout(const int32_t *u, const int32_t *v, const int32_t *t,
                        const int32_t *lam, int64_t n, int32_t nv,
                        const eat_build_options &opt, eat_layout &L, std::string *err) {
  auto fail = [&](eat_status s, const std::string &m) {
    if (err) *err = m;
    return s;
  };
  if (nv < 1) return fail(EAT_ERR_INVALID_ARGUMENT, "n_vertices must be >= 1");
  if (n < 0) return fail(EAT_ERR_INVALID_ARGUMENT, "n_conn must be >= 0");
  if (n > 0 && (!u || !v || !t || !lam)) return fail(EAT_ERR_INVALID_ARGUMENT, "null connection array");
  if (opt.layout != EAT_LAYOUT_HYBRID && opt.layout != EAT_LAYOUT_FLAT)
    return fail(EAT_ERR_INVALID_ARGUMENT, "unknown layout kind");
  int32_t cw = opt.cluster_seconds == 0 ? 3600 : opt.cluster_seconds;
  if (cw < 1 || cw > 32767) return fail(EAT_ERR_INVALID_ARGUMENT, "cluster_seconds must be in 1..32767");
  if (opt.header_grid != 0 && opt.header_grid != -1)
    return fail(EAT_ERR_INVALID_ARGUMENT, "header_grid must be 0 or -1");
  for (int r : opt.reserved)
    if (r != 0) return fail(EAT_ERR_INVALID_ARGUMENT, "reserved build options must be zero");
  if (opt.subtrip_len != 0)
    return fail(EAT_ERR_INVALID_ARGUMENT, "subtrip_len applies to the *_build_trips functions only");
  const int nth = resolve_threads(opt.n_threads);

  L = eat_layout();
  L.kind = opt.layout;
  L.n_vertices = nv;
  L.cluster_seconds = cw;
  L.n_conn_input = n;

  // ---- 1. validate; count connections per tail (self-loops dropped) ----------
  std::vector<std::vector<int64_t>> part_cnt((size_t)nth);
  std::vector<int64_t> bad((size_t)nth, -1), loops((size_t)nth, 0);
  std::vector<int32_t> tmax((size_t)nth, 0);
  std::vector<int64_t> chunk_b((size_t)nth + 1, 0);
  {
    int64_t nt = std::max<int64_t>(1, std::min<int64_t>(nth, n));
    for (int64_t i = 0; i <= nt; ++i) chunk_b[(size_t)i] = n * i / nt;
    for (int64_t i = nt + 1; i <= nth; ++i) chunk_b[(size_t)i] = n;
  }
  parallel_for_chunks(nth, nth, [&](int, int64_t cb, int64_t ce) {
    for (int64_t c = cb; c < ce; ++c) {
      auto &cnt = part_cnt[(size_t)c];
      cnt.assign((size_t)nv, 0);
      for (int64_t i = chunk_b[(size_t)c]; i < chunk_b[(size_t)c + 1]; ++i) {
        int32_t a = u[i], b = v[i], tt = t[i], l = lam[i];
        if (a < 0 || a >= nv || b < 0 || b >= nv || tt < 0 || l < 1 ||
            (int64_t)tt + (int64_t)l > (int64_t)EAT_INF - 1) {
          bad[(size_t)c] = i;
          break;
        }
        if (a == b) {
          ++loops[(size_t)c];
          continue;
        }
        ++cnt[(size_t)a];
        tmax[(size_t)c] = std::max(tmax[(size_t)c], tt);
      }
    }
  });
  for (int c = 0; c < nth; ++c)
    if (bad[(size_t)c] >= 0)
      return fail(EAT_ERR_INVALID_ARGUMENT,
                  "connection " + std::to_string(bad[(size_t)c]) +
                      " is invalid (need 0<=u,v<n_vertices, t>=0, lam>=1, t+lam<=INT32_MAX-1)");
  for (int c = 0; c < nth; ++c) {
    L.n_self_loops += loops[(size_t)c];
    L.max_departure = std::max(L.max_departure, tmax[(size_t)c]);
  }
  L.n_clusters = L.max_departure / cw + 1;
  if (L.kind == EAT_LAYOUT_HYBRID && L.n_clusters > 64)
    return fail(EAT_ERR_UNSUPPORTED,
                "hybrid layout holds at most 64 clusters per type; raise cluster_seconds or use the flat layout");

  // ---- 2. bucket by tail (stable counting sort, chunk-parallel) -------------
  std::vector<int64_t> boff((size_t)nv + 1, 0);
  for (int32_t a = 0; a < nv; ++a) {
    int64_t s = 0;
    for (int c = 0; c < nth; ++c) s += part_cnt[(size_t)c][(size_t)a];
    boff[(size_t)a + 1] = boff[(size_t)a] + s;
  }
  const int64_t m = boff[(size_t)nv];
  std::vector<Rec> rec((size_t)std::max<int64_t>(m, 1));
  {
    // each chunk writes after the chunks before it inside every bucket
    std::vector<int64_t> run((size_t)nv);
    for (int c = 0; c < nth; ++c) {
      auto &cnt = part_cnt[(size_t)c];
      for (int32_t a = 0; a < nv; ++a) {
        int64_t base = (c == 0) ? boff[(size_t)a] : run[(size_t)a];
        run[(size_t)a] = base + cnt[(size_t)a];
        cnt[(size_t)a] = base;  // becomes this chunk's write cursor
      }
    }
    parallel_for_chunks(nth, nth, [&](int, int64_t cb, int64_t ce) {
      for (int64_t c = cb; c < ce; ++c) {
        auto &cur = part_cnt[(size_t)c];
        for (int64_t i = chunk_b[(size_t)c]; i < chunk_b[(size_t)c + 1]; ++i) {
          if (u[i] == v[i]) continue;
          rec[(size_t)cur[(size_t)u[i]]++] = Rec{v[i], lam[i], t[i]};
        }
      }
    });
    part_cnt.clear();
    part_cnt.shrink_to_fit();
  }

  // ---- 3. per tail: sort by (v, lam, t), drop duplicates, count --------------
  // Work split over tails with balanced connection counts.
  std::vector<int32_t> split((size_t)nth + 1, nv);
  split[0] = 0;
  for (int i = 1; i < nth; ++i) {
    int64_t target = m * i / nth;
    split[(size_t)i] = (int32_t)(std::lower_bound(boff.begin(), boff.end(), target) - boff.begin());
    split[(size_t)i] = std::min(std::max(split[(size_t)i], split[(size_t)i - 1]), nv);
  }
  std::vector<int64_t> blen((size_t)nv, 0);  // bucket length after dedupe
  std::vector<int64_t> n_ty_u((size_t)nv + 1, 0), n_hd_u((size_t)nv + 1, 0), n_pl_u((size_t)nv + 1, 0);
  std::vector<int64_t> edges_c((size_t)nth, 0), ap_c((size_t)nth, 0), arr_c((size_t)nth, 0);
  const bool hybrid = L.kind == EAT_LAYOUT_HYBRID;
  parallel_for_chunks(nth, nth, [&](int, int64_t cb, int64_t ce) {
    for (int64_t c = cb; c < ce; ++c) {
      for (int32_t a = split[(size_t)c]; a < split[(size_t)c + 1]; ++a) {
        Rec *b = rec.data() + boff[(size_t)a];
        int64_t len = boff[(size_t)a + 1] - boff[(size_t)a];
        std::sort(b, b + len, rec_less);
        int64_t w = 0;
        for (int64_t i = 0; i < len; ++i)
          if (w == 0 || rec_less(b[w - 1], b[i])) b[w++] = b[i];
        blen[(size_t)a] = w;
        int64_t nty = 0, nhd = 0, npl = 0, ned = 0;
        int64_t i = 0;
        while (i < w) {
          int64_t j = i + 1;
          while (j < w && same_type(b[i], b[j])) ++j;
          ++nty;
          if (i == 0 || b[i].v != b[i - 1].v) ++ned;
          if (hybrid) {
            for_each_cluster(b + i, j - i, cw, [&](int32_t, bool ap, int32_t, int32_t, int64_t cnt, int64_t) {
              ++nhd;
              if (ap) ++ap_c[(size_t)c];
              else {
                ++arr_c[(size_t)c];
                npl += pad4(1 + cnt);
              }
            });
          } else {
            npl += pad4(j - i);
          }
          i = j;
        }
        n_ty_u[(size_t)a + 1] = nty;
        n_hd_u[(size_t)a + 1] = nhd;
        n_pl_u[(size_t)a + 1] = npl;
        edges_c[(size_t)c] += ned;
      }
    }
  });
  // ---- 3b. layout order of the stops ------------------------------------------
  {
    std::vector<int64_t> out_off((size_t)nv + 1, 0);
    for (int32_t a = 0; a < nv; ++a) {
      const Rec *b = rec.data() + boff[(size_t)a];
      int64_t ne = 0;
      for (int64_t i = 0; i < blen[(size_t)a]; ++i) ne += (i == 0 || b[i].v != b[i - 1].v);
      out_off[(size_t)a + 1] = out_off[(size_t)a] + ne;
    }
    std::vector<int32_t> out_v((size_t)out_off[(size_t)nv]);
    for (int32_t a = 0; a < nv; ++a) {
      const Rec *b = rec.data() + boff[(size_t)a];
      int64_t k = out_off[(size_t)a];
      for (int64_t i = 0; i < blen[(size_t)a]; ++i)
        if (i == 0 || b[i].v != b[i - 1].v) out_v[(size_t)k++] = b[i].v;
    }
    L.order = locality_order(nv, out_off, out_v);
  }
  // offsets of every stop's block, in layout order
  std::vector<int64_t> ty_at((size_t)nv), hd_at((size_t)nv), pl_at((size_t)nv);
  {
    int64_t t0 = 0, h0 = 0, p0 = 0;
    for (int32_t r = 0; r < nv; ++r) {
      const int32_t a = L.order[(size_t)r];
      ty_at[(size_t)a] = t0;
      hd_at[(size_t)a] = h0;
      pl_at[(size_t)a] = p0;
      t0 += n_ty_u[(size_t)a + 1];
      h0 += n_hd_u[(size_t)a + 1];
      p0 += n_pl_u[(size_t)a + 1];
    }
    L.n_types = t0;
    L.n_headers = h0;
  }
  int64_t npool = 0;
  for (int32_t a = 0; a < nv; ++a) npool += n_pl_u[(size_t)a + 1];
  for (int c = 0; c < nth; ++c) {
    L.n_edges += edges_c[(size_t)c];
    L.n_ap += ap_c[(size_t)c];
    L.n_array += arr_c[(size_t)c];
  }
  for (int32_t a = 0; a < nv; ++a) L.n_conn += blen[(size_t)a];
  L.n_duplicates = m - L.n_conn;
  const int64_t lim = (int64_t)INT32_MAX - 1;
  if (L.n_types > lim || L.n_headers > lim || npool > lim)
    return fail(EAT_ERR_UNSUPPORTED, "more than 2^31-1 types, cluster headers or pool words");

  // ---- 4. fill the arrays ----------------------------------------------------
  try {
    L.vt.assign((size_t)nv * 2, 0);
    L.ty.assign((size_t)(4 * std::max<int64_t>(L.n_types, 1)), 0);
    if (hybrid) {
      L.mask_hi.assign((size_t)std::max<int64_t>(L.n_types, 1), 0u);
      L.hdr.assign((size_t)(2 * std::max<int64_t>(L.n_headers, 1)), 0);
    }
    // kPoolTail words of infinity after the last entry keep the fixed-size
    // chunk reads of the lookup inside the array
    L.pool.assign((size_t)(npool + kPoolTail), EAT_INF);
  } catch (const std::bad_alloc &) {
    return fail(EAT_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
  for (int32_t a = 0; a < nv; ++a) {
    L.vt[(size_t)2 * a] = (int32_t)ty_at[(size_t)a];
    L.vt[(size_t)2 * a + 1] = (int32_t)n_ty_u[(size_t)a + 1];
  }
  std::vector<int32_t> maxdeg((size_t)nth, 0);
  parallel_for_chunks(nth, nth, [&](int, int64_t cb, int64_t ce) {
    for (int64_t c = cb; c < ce; ++c) {
      for (int32_t a = split[(size_t)c]; a < split[(size_t)c + 1]; ++a) {
        const Rec *b = rec.data() + boff[(size_t)a];
        int64_t w = blen[(size_t)a];
        int64_t ti = ty_at[(size_t)a], hi = hd_at[(size_t)a], pi = pl_at[(size_t)a];
        maxdeg[(size_t)c] = std::max<int32_t>(maxdeg[(size_t)c], (int32_t)n_ty_u[(size_t)a + 1]);
        int64_t i = 0;
        while (i < w) {
          int64_t j = i + 1;
          while (j < w && same_type(b[i], b[j])) ++j;
          int32_t *r = &L.ty[(size_t)(4 * ti)];
          r[0] = b[i].v;
          r[1] = b[i].lam;
          if (hybrid) {
            uint64_t mask = 0;
            r[2] = (int32_t)hi;
            for_each_cluster(b + i, j - i, cw,
                             [&](int32_t k, bool ap, int32_t t0, int32_t h, int64_t cnt, int64_t beg) {
                               mask |= 1ull << k;
                               L.hdr[(size_t)(2 * hi)] = t0;
                               if (ap) {
                                 L.hdr[(size_t)(2 * hi + 1)] = (int32_t)((cnt << 16) | (cnt >= 2 ? h : 1));
                               } else {
                                 L.hdr[(size_t)(2 * hi + 1)] = ~(int32_t)pi;
                                 L.pool[(size_t)pi] = (int32_t)cnt;
                                 for (int64_t q = 0; q < cnt; ++q) L.pool[(size_t)(pi + 1 + q)] = b[i + beg + q].t;
                                 pi += pad4(1 + cnt);
                               }
                               ++hi;
                             });
            r[3] = (int32_t)(uint32_t)(mask & 0xffffffffu);
            L.mask_hi[(size_t)ti] = (uint32_t)(mask >> 32);
          } else {
            r[2] = (int32_t)pi;
            r[3] = (int32_t)(j - i);
            for (int64_t q = i; q < j; ++q) L.pool[(size_t)(pi + (q - i))] = b[q].t;
            pi += pad4(j - i);
          }
          ++ti;
          i = j;
        }
      }
    }
  });
  for (int c = 0; c < nth; ++c) L.max_types_per_vertex = std::max(L.max_types_per_vertex, maxdeg[(size_t)c]);
  if (!hybrid) L.n_headers = 0;
  return EAT_OK;
}

}  // namespace eat
