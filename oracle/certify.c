/*
 * certify.c -- an O(|C| + |V|) check that an arrival array is the EAT answer,
 * and the per-type "next departure" of Section II-B written as its definition.
 * Test infrastructure only (see oracle.h).
 */
#include "oracle.h"

#include <stdlib.h>

int oracle_certify(int64_t n, const int32_t *u, const int32_t *v,
                   const int32_t *t, const int32_t *lam, int32_t nv,
                   int32_t s, int32_t ts, const int32_t *arr,
                   int32_t *bad_vertex) {
  if (oracle_validate(n, u, v, t, lam, nv) != ORACLE_OK) return -1;
  if (!arr || s < 0 || s >= nv || ts < 0) return -1;
  if (bad_vertex) *bad_vertex = -1;
  /* (1) the source is reached at the query time */
  if (arr[s] != ts) {
    if (bad_vertex) *bad_vertex = s;
    return 1;
  }
  /* (2) closure: no connection that can be boarded improves its head */
  for (int64_t i = 0; i < n; ++i) {
    if (arr[u[i]] <= t[i] && arr[v[i]] > t[i] + lam[i]) {
      if (bad_vertex) *bad_vertex = v[i];
      return 2;
    }
  }
  /* (3) witness: every finite entry other than the source is the arrival of a
   * connection that can be boarded */
  char *seen = (char *)calloc((size_t)nv + 1, 1);
  if (!seen) return -1;
  for (int64_t i = 0; i < n; ++i)
    if (arr[u[i]] <= t[i] && t[i] + lam[i] == arr[v[i]]) seen[v[i]] = 1;
  int rc = 0;
  for (int32_t x = 0; x < nv; ++x) {
    if (x == s || arr[x] == ORACLE_INF) continue;
    if (!seen[x]) {
      if (bad_vertex) *bad_vertex = x;
      rc = 3;
      break;
    }
  }
  free(seen);
  return rc;
}

int32_t oracle_next_departure(int64_t n, const int32_t *d, int32_t x) {
  /* t_c = min { t in the type : t >= x } (Section II-B) */
  int32_t best = ORACLE_INF;
  for (int64_t i = 0; i < n; ++i)
    if (d[i] >= x && d[i] < best) best = d[i];
  return best;
}
