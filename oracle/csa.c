/*
 * csa.c -- the Connection-Scan Algorithm (Algorithm 1, Section I-A) as the
 * reference answer for every EAT query.  Test infrastructure only (see oracle.h).
 *
 * Algorithm 1: set e[] to infinity except e[s] = ts; visit the connections in
 * non-decreasing order of departure time; a connection (u, v, t, lam) with
 * e[u] <= t and t + lam < e[v] sets e[v] = t + lam.  One pass is exact because
 * every connection that could extend a path to u departs no earlier than the
 * path's arrival at u, which (lam >= 1) is later than that connection's own
 * departure, so it is visited afterwards.
 *
 * The scan starts at the first connection with t >= ts.  Every connection
 * before it has t < ts <= e[x] for every vertex x whose entry is finite, so the
 * relaxation test fails for all of them and skipping them changes nothing.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

struct oracle_csa {
  int64_t n;
  int32_t nv;
  int32_t *u, *v, *t, *lam; /* ordered by t */
};

int oracle_validate(int64_t n, const int32_t *u, const int32_t *v,
                    const int32_t *t, const int32_t *lam, int32_t nv) {
  if (n < 0 || nv < 0) return ORACLE_EINVAL;
  if (n > 0 && (!u || !v || !t || !lam)) return ORACLE_EINVAL;
  for (int64_t i = 0; i < n; ++i) {
    if (u[i] < 0 || u[i] >= nv || v[i] < 0 || v[i] >= nv) return ORACLE_EINVAL;
    if (t[i] < 0 || lam[i] < 1) return ORACLE_EINVAL;
    if ((int64_t)t[i] + (int64_t)lam[i] > (int64_t)ORACLE_INF - 1) return ORACLE_EINVAL;
  }
  return ORACLE_OK;
}

/* Order of the scan: the indices 0..n-1 sorted by departure time, ties kept
 * in input order (a stable least-significant-digit radix sort on the two
 * 16-bit halves of t).  Any order by t gives the same answer (lam >= 1). */
static int order_by_departure(int64_t n, const int32_t *t, uint32_t *out) {
  uint32_t *tmp = (uint32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
  size_t *count = (size_t *)malloc(65537 * sizeof(size_t));
  if (!tmp || !count) {
    free(tmp);
    free(count);
    return ORACLE_ENOMEM;
  }
  for (int64_t i = 0; i < n; ++i) tmp[i] = (uint32_t)i;
  uint32_t *src = tmp, *dst = out;
  for (int pass = 0; pass < 2; ++pass) {
    const int shift = 16 * pass;
    memset(count, 0, 65537 * sizeof(size_t));
    for (int64_t i = 0; i < n; ++i) count[(((uint32_t)t[src[i]] >> shift) & 0xffffu) + 1]++;
    for (int d = 0; d < 65536; ++d) count[d + 1] += count[d];
    for (int64_t i = 0; i < n; ++i) dst[count[((uint32_t)t[src[i]] >> shift) & 0xffffu]++] = src[i];
    uint32_t *sw = src;
    src = dst;
    dst = sw;
  }
  /* after two passes the sorted indices are back in tmp: copy them out */
  memcpy(out, src, (size_t)n * sizeof(uint32_t));
  free(tmp);
  free(count);
  return ORACLE_OK;
}

oracle_csa *oracle_csa_new(int64_t n, const int32_t *u, const int32_t *v,
                           const int32_t *t, const int32_t *lam, int32_t nv) {
  if (oracle_validate(n, u, v, t, lam, nv) != ORACLE_OK) return NULL;
  if (n > (int64_t)UINT32_MAX) return NULL;
  oracle_csa *h = (oracle_csa *)calloc(1, sizeof(*h));
  if (!h) return NULL;
  h->n = n;
  h->nv = nv;
  size_t bytes = (size_t)(n > 0 ? n : 1) * sizeof(int32_t);
  h->u = (int32_t *)malloc(bytes);
  h->v = (int32_t *)malloc(bytes);
  h->t = (int32_t *)malloc(bytes);
  h->lam = (int32_t *)malloc(bytes);
  uint32_t *idx = (uint32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
  if (!h->u || !h->v || !h->t || !h->lam || !idx || order_by_departure(n, t, idx) != ORACLE_OK) {
    free(idx);
    oracle_csa_free(h);
    return NULL;
  }
  for (int64_t k = 0; k < n; ++k) {
    int64_t i = (int64_t)idx[k];
    h->u[k] = u[i];
    h->v[k] = v[i];
    h->t[k] = t[i];
    h->lam[k] = lam[i];
  }
  free(idx);
  return h;
}

void oracle_csa_free(oracle_csa *h) {
  if (!h) return;
  free(h->u);
  free(h->v);
  free(h->t);
  free(h->lam);
  free(h);
}

int oracle_csa_query(const oracle_csa *h, int32_t s, int32_t ts, int32_t *arr) {
  if (!h || !arr || s < 0 || s >= h->nv || ts < 0) return ORACLE_EINVAL;
  /* Initialisation of Algorithm 1 */
  for (int32_t x = 0; x < h->nv; ++x) arr[x] = ORACLE_INF;
  arr[s] = ts;
  /* first connection departing at or after ts (binary search on the order) */
  int64_t lo = 0, hi = h->n;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (h->t[mid] < ts) lo = mid + 1; else hi = mid;
  }
  /* the scan: relax each connection in departure order */
  for (int64_t i = lo; i < h->n; ++i) {
    int32_t tu = arr[h->u[i]];
    int32_t a = h->t[i] + h->lam[i];
    if (tu <= h->t[i] && a < arr[h->v[i]]) arr[h->v[i]] = a;
  }
  return ORACLE_OK;
}

int oracle_csa_query_many(const oracle_csa *h, int32_t nq, const int32_t *s,
                          const int32_t *ts, int32_t *arr) {
  if (!h || nq < 0 || (nq > 0 && (!s || !ts || !arr))) return ORACLE_EINVAL;
  for (int32_t q = 0; q < nq; ++q) {
    int rc = oracle_csa_query(h, s[q], ts[q], arr + (int64_t)q * h->nv);
    if (rc != ORACLE_OK) return rc;
  }
  return ORACLE_OK;
}
