/*
 * journeys.c -- reference answers for the query variants that Section I names
 * beside the single-source EAT problem: the journey behind an arrival time,
 * and the profile of a source over an interval of departure times.  The
 * goal-directed variant (one destination d) needs no code of its own: its
 * answer is entry d of the single-source answer.
 * Test infrastructure only (see oracle.h).
 *
 * Parents.  An arrival arr[v] < INF, v != s, of an EAT answer is realised by
 * at least one connection (u, v, t, lam) with arr[u] <= t and t + lam ==
 * arr[v] (the witness condition of the certificate).  The parent of v is the
 * realising connection with the smallest tail u, then the smallest duration
 * lam; its departure is then arr[v] - lam.  Since lam >= 1, a parent's tail
 * has an earlier arrival than v, so following parents from any reached stop
 * ends at s and, read backwards, is a time-respecting path (a journey)
 * arriving at arr[v].
 *
 * Profiles.  Fix s and an interval [t_lo, t_hi].  Among all journeys that
 * leave s (take their first connection) at or after t_lo, a pair (dep, arr)
 * at stop v is Pareto-optimal when no journey to v leaves no earlier and
 * arrives no later with one of the two strictly better.  The profile of v is
 * the set of Pareto-optimal pairs with dep <= t_hi.  Every dep is the
 * departure time of a connection leaving s.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

int oracle_parents(int64_t n, const int32_t *u, const int32_t *v, const int32_t *t,
                   const int32_t *lam, int32_t nv, int32_t s, const int32_t *arr,
                   int32_t *par_u, int32_t *par_t, int32_t *par_lam) {
  int rc = oracle_validate(n, u, v, t, lam, nv);
  if (rc != ORACLE_OK) return rc;
  if (!arr || !par_u || !par_t || !par_lam || s < 0 || s >= nv) return ORACLE_EINVAL;
  for (int32_t x = 0; x < nv; ++x) par_u[x] = par_t[x] = par_lam[x] = -1;
  for (int64_t i = 0; i < n; ++i) {
    const int32_t a = arr[u[i]], w = v[i];
    if (w == s || a > t[i] || t[i] + lam[i] != arr[w]) continue; /* does not realise arr[w] */
    if (par_u[w] < 0 || u[i] < par_u[w] || (u[i] == par_u[w] && lam[i] < par_lam[w])) {
      par_u[w] = u[i];
      par_lam[w] = lam[i];
      par_t[w] = t[i];
    }
  }
  for (int32_t x = 0; x < nv; ++x)
    if (x != s && arr[x] != ORACLE_INF && par_u[x] < 0) return ORACLE_EINVAL; /* not an EAT answer */
  return ORACLE_OK;
}

/* Sorted distinct departure times of the connections leaving s inside
 * [lo, hi], into out (cap entries); returns their count (it may exceed cap). */
static int64_t departures_of(int64_t n, const int32_t *u, const int32_t *t, int32_t s, int32_t lo,
                             int32_t hi, int32_t *out, int64_t cap) {
  int32_t *all = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  if (!all) return -1;
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i)
    if (u[i] == s && t[i] >= lo && t[i] <= hi) all[m++] = t[i];
  /* insertion sort: the departures of one stop are few */
  for (int64_t i = 1; i < m; ++i) {
    const int32_t x = all[i];
    int64_t j = i;
    while (j > 0 && all[j - 1] > x) {
      all[j] = all[j - 1];
      --j;
    }
    all[j] = x;
  }
  int64_t k = 0;
  for (int64_t i = 0; i < m; ++i) {
    if (i > 0 && all[i] == all[i - 1]) continue;
    if (k < cap) out[k] = all[i];
    ++k;
  }
  free(all);
  return k;
}

/* The scan-based profile: one connection scan per departure time d_i of s in
 * [t_lo, t_hi], and one more at the first departure after t_hi (if any).
 * EAT(s, d_i)[v] is the best arrival over journeys leaving at or after d_i;
 * it is realised by a journey leaving exactly at d_i when it beats
 * EAT(s, d_{i+1})[v] (journeys leaving later all arrive no earlier than that),
 * and then (d_i, EAT(s, d_i)[v]) is Pareto-optimal; otherwise a journey
 * leaving later does as well and the pair is dominated.  (u, t) is the raw
 * connection list the scan h was built from (its departures of s). */
int oracle_profile(int64_t n, const int32_t *u, const int32_t *t, const oracle_csa *h, int32_t nv,
                   int32_t s, int32_t t_lo, int32_t t_hi, int32_t cap, int32_t *dep, int32_t *n_dep,
                   int32_t *arr) {
  if (!h || !n_dep || (n > 0 && (!u || !t)) || s < 0 || s >= nv || t_lo < 0 || t_hi < t_lo || cap < 0)
    return ORACLE_EINVAL;
  if (cap > 0 && (!dep || !arr)) return ORACLE_EINVAL;
  int32_t *d = (int32_t *)malloc((size_t)(cap > 0 ? cap : 1) * sizeof(int32_t));
  if (!d) return ORACLE_ENOMEM;
  const int64_t k = departures_of(n, u, t, s, t_lo, t_hi, d, cap);
  if (k < 0) {
    free(d);
    return ORACLE_ENOMEM;
  }
  *n_dep = (int32_t)k;
  if (k > cap) {
    free(d);
    return ORACLE_ELIMIT;
  }
  /* the first departure of s after t_hi */
  int32_t next = ORACLE_INF;
  for (int64_t i = 0; i < n; ++i)
    if (u[i] == s && t[i] > t_hi && t[i] < next) next = t[i];
  int32_t *later = (int32_t *)malloc((size_t)(nv > 0 ? nv : 1) * sizeof(int32_t));
  if (!later) {
    free(d);
    return ORACLE_ENOMEM;
  }
  int rc = ORACLE_OK;
  if (next != ORACLE_INF) rc = oracle_csa_query(h, s, next, later);
  else for (int32_t x = 0; x < nv; ++x) later[x] = ORACLE_INF;
  for (int64_t i = 0; i < k && rc == ORACLE_OK; ++i) {
    dep[i] = d[i];
    rc = oracle_csa_query(h, s, d[i], arr + i * (int64_t)nv);
  }
  /* first row down: row i is compared with row i + 1 before that row is
   * filtered in its turn (the last row with the scan after t_hi) */
  for (int64_t i = 0; i < k && rc == ORACLE_OK; ++i) {
    int32_t *row = arr + i * (int64_t)nv;
    const int32_t *after = (i + 1 < k) ? arr + (i + 1) * (int64_t)nv : later;
    for (int32_t x = 0; x < nv; ++x)
      if (x == s || !(row[x] < after[x])) row[x] = ORACLE_INF;
  }
  free(d);
  free(later);
  return rc;
}

/* ---- the profile straight from its definition ------------------------------- */

typedef struct {
  int64_t n;
  const int32_t *u, *v, *t, *lam;
  int32_t nv;
  int32_t *best;       /* best[x * nd + j]: earliest arrival at x of a journey leaving at dd[j] */
  const int32_t *dd;   /* every departure time of s at or after t_lo, sorted, distinct */
  int64_t nd;
  int64_t paths, max_paths;
} pdfs_ctx;

static int64_t index_of(const int32_t *a, int64_t n, int32_t x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

/* At stop `at` at time `now` on a journey that left s at dd[j]. */
static int pdfs(pdfs_ctx *c, int32_t at, int32_t now, int64_t j) {
  for (int64_t i = 0; i < c->n; ++i) {
    if (c->u[i] != at || c->t[i] < now) continue;
    if (++c->paths > c->max_paths) return ORACLE_ELIMIT;
    const int32_t a = c->t[i] + c->lam[i];
    int32_t *b = c->best + (int64_t)c->v[i] * c->nd + j;
    if (a < *b) *b = a;
    const int rc = pdfs(c, c->v[i], a, j);
    if (rc != ORACLE_OK) return rc;
  }
  return ORACLE_OK;
}

/* Enumerates every journey that leaves s at or after t_lo (its first
 * connection leaves s at some departure time dd[j] >= t_lo), records the
 * earliest arrival per (stop, dd[j]), and keeps (dd[j], a) when dd[j] <= t_hi
 * and no journey to the same stop leaving strictly later arrives at a or
 * earlier.  Output in the layout of oracle_profile.  Exponential: tiny inputs. */
int oracle_brute_profile(int64_t n, const int32_t *u, const int32_t *v, const int32_t *t,
                         const int32_t *lam, int32_t nv, int32_t s, int32_t t_lo, int32_t t_hi,
                         int64_t max_paths, int32_t cap, int32_t *dep, int32_t *n_dep, int32_t *arr) {
  int rc = oracle_validate(n, u, v, t, lam, nv);
  if (rc != ORACLE_OK) return rc;
  if (!n_dep || s < 0 || s >= nv || t_lo < 0 || t_hi < t_lo || cap < 0) return ORACLE_EINVAL;
  if (cap > 0 && (!dep || !arr)) return ORACLE_EINVAL;
  int32_t *dd = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  if (!dd) return ORACLE_ENOMEM;
  const int64_t nd = departures_of(n, u, t, s, t_lo, ORACLE_INF, dd, n);
  int64_t k = 0; /* departures inside [t_lo, t_hi] */
  while (k < nd && dd[k] <= t_hi) ++k;
  *n_dep = (int32_t)k;
  if (k > cap) {
    free(dd);
    return ORACLE_ELIMIT;
  }
  int32_t *best = (int32_t *)malloc((size_t)(nv > 0 ? nv : 1) * (size_t)(nd > 0 ? nd : 1) * sizeof(int32_t));
  if (!best) {
    free(dd);
    return ORACLE_ENOMEM;
  }
  for (int64_t i = 0; i < (int64_t)nv * nd; ++i) best[i] = ORACLE_INF;
  pdfs_ctx c = {n, u, v, t, lam, nv, best, dd, nd, 0, max_paths};
  /* the first connection of a journey: any connection leaving s at >= t_lo */
  for (int64_t i = 0; i < n && rc == ORACLE_OK; ++i) {
    if (u[i] != s || t[i] < t_lo) continue;
    if (++c.paths > c.max_paths) {
      rc = ORACLE_ELIMIT;
      break;
    }
    const int64_t j = index_of(dd, nd, t[i]);
    const int32_t a = t[i] + lam[i];
    int32_t *b = best + (int64_t)v[i] * nd + j;
    if (a < *b) *b = a;
    rc = pdfs(&c, v[i], a, j);
  }
  for (int64_t j = 0; j < k && rc == ORACLE_OK; ++j) {
    dep[j] = dd[j];
    for (int32_t x = 0; x < nv; ++x) {
      const int32_t a = best[(int64_t)x * nd + j];
      int dominated = (x == s || a == ORACLE_INF);
      for (int64_t j2 = j + 1; j2 < nd && !dominated; ++j2)
        if (best[(int64_t)x * nd + j2] <= a) dominated = 1;
      arr[j * (int64_t)nv + x] = dominated ? ORACLE_INF : a;
    }
  }
  free(dd);
  free(best);
  return rc;
}
