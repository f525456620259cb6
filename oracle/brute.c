/*
 * brute.c -- the EAT answer computed straight from its definition (Section I:
 * a time-respecting path leaves each intermediate stop no earlier than it
 * arrived there; the query asks for the earliest arrival over paths that leave
 * s at or after ts).  Two independent brute forces for tiny inputs.
 * Test infrastructure only (see oracle.h).
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

/* ---- 1. enumerate every time-respecting connection sequence ----------------- */

typedef struct {
  int64_t n;
  const int32_t *u, *v, *t, *lam;
  int32_t *arr;
  int64_t paths, max_paths;
} dfs_ctx;

/* We stand at stop `at` at time `now`; every connection leaving `at` no earlier
 * than `now` extends the current path by one more connection. */
static int dfs(dfs_ctx *c, int32_t at, int32_t now) {
  for (int64_t i = 0; i < c->n; ++i) {
    if (c->u[i] != at || c->t[i] < now) continue;
    if (++c->paths > c->max_paths) return ORACLE_ELIMIT;
    int32_t a = c->t[i] + c->lam[i];
    if (a < c->arr[c->v[i]]) c->arr[c->v[i]] = a;
    int rc = dfs(c, c->v[i], a); /* time strictly grows (lam >= 1): finite depth */
    if (rc != ORACLE_OK) return rc;
  }
  return ORACLE_OK;
}

int oracle_brute_paths(int64_t n, const int32_t *u, const int32_t *v,
                       const int32_t *t, const int32_t *lam, int32_t nv,
                       int32_t s, int32_t ts, int64_t max_paths, int32_t *arr) {
  int rc = oracle_validate(n, u, v, t, lam, nv);
  if (rc != ORACLE_OK) return rc;
  if (!arr || s < 0 || s >= nv || ts < 0) return ORACLE_EINVAL;
  for (int32_t x = 0; x < nv; ++x) arr[x] = ORACLE_INF;
  arr[s] = ts; /* the empty path */
  dfs_ctx c = {n, u, v, t, lam, arr, 0, max_paths};
  rc = dfs(&c, s, ts);
  arr[s] = ts; /* a path that returns to s arrives after ts */
  return rc;
}

/* ---- 2. closure over reachable (stop, time) states -------------------------- */

int oracle_brute_states(int64_t n, const int32_t *u, const int32_t *v,
                        const int32_t *t, const int32_t *lam, int32_t nv,
                        int32_t s, int32_t ts, int32_t *arr) {
  int rc = oracle_validate(n, u, v, t, lam, nv);
  if (rc != ORACLE_OK) return rc;
  if (!arr || s < 0 || s >= nv || ts < 0) return ORACLE_EINVAL;
  /* state k: "present at stop sv[k] at time st[k]"; at most one per connection
   * arrival plus the start state */
  int64_t cap = n + 1;
  int32_t *sv = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
  int32_t *st = (int32_t *)malloc((size_t)cap * sizeof(int32_t));
  char *used = (char *)calloc((size_t)(n > 0 ? n : 1), 1); /* connection already produced its state */
  if (!sv || !st || !used) {
    free(sv);
    free(st);
    free(used);
    return ORACLE_ENOMEM;
  }
  int64_t ns = 0;
  sv[ns] = s;
  st[ns] = ts;
  ++ns;
  int grew = 1;
  while (grew) {
    grew = 0;
    for (int64_t i = 0; i < n; ++i) {
      if (used[i]) continue;
      /* is some known state at u[i] early enough to board connection i? */
      for (int64_t k = 0; k < ns; ++k) {
        if (sv[k] == u[i] && st[k] <= t[i]) {
          used[i] = 1;
          sv[ns] = v[i];
          st[ns] = t[i] + lam[i];
          ++ns;
          grew = 1;
          break;
        }
      }
    }
  }
  for (int32_t x = 0; x < nv; ++x) arr[x] = ORACLE_INF;
  for (int64_t k = 0; k < ns; ++k)
    if (st[k] < arr[sv[k]]) arr[sv[k]] = st[k];
  free(sv);
  free(st);
  free(used);
  return ORACLE_OK;
}
