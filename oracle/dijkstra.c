/*
 * dijkstra.c -- the EAT answer by Dijkstra's label-setting search on the two
 * classical transit models the paper's introduction names: the time-expanded
 * model and the time-dependent model (Section I; Bui-Xuan, Ferreira and
 * Jarry's foremost journeys).  Independent of the connection scan in csa.c:
 * different data structures, different visiting order.
 * Test infrastructure only (see oracle.h).
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

/* ---- a binary min-heap of (key, id) pairs ----------------------------------- */

typedef struct {
  int64_t key;
  int64_t id;
} heap_item;

typedef struct {
  heap_item *a;
  int64_t n, cap;
} heap;

static int heap_push(heap *h, int64_t key, int64_t id) {
  if (h->n == h->cap) {
    int64_t nc = h->cap ? 2 * h->cap : 64;
    heap_item *na = (heap_item *)realloc(h->a, (size_t)nc * sizeof(heap_item));
    if (!na) return ORACLE_ENOMEM;
    h->a = na;
    h->cap = nc;
  }
  int64_t i = h->n++;
  h->a[i].key = key;
  h->a[i].id = id;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h->a[p].key <= h->a[i].key) break;
    heap_item tmp = h->a[p];
    h->a[p] = h->a[i];
    h->a[i] = tmp;
    i = p;
  }
  return ORACLE_OK;
}

static heap_item heap_pop(heap *h) {
  heap_item top = h->a[0];
  h->a[0] = h->a[--h->n];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, m = i;
    if (l < h->n && h->a[l].key < h->a[m].key) m = l;
    if (r < h->n && h->a[r].key < h->a[m].key) m = r;
    if (m == i) break;
    heap_item tmp = h->a[m];
    h->a[m] = h->a[i];
    h->a[i] = tmp;
    i = m;
  }
  return top;
}

/* ---- time-expanded model ----------------------------------------------------- */

/* event = (stop, time) packed so that sorting orders by stop, then time */
static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}
static int64_t pack_event(int32_t stop, int32_t time) {
  return ((int64_t)stop << 32) | (int64_t)(uint32_t)time;
}

/* index of event (stop, time) in the sorted unique event list */
static int64_t find_event(const int64_t *ev, int64_t nev, int64_t key) {
  int64_t lo = 0, hi = nev;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (ev[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo; /* the key is always present */
}

int oracle_te_dijkstra(int64_t n, const int32_t *u, const int32_t *v,
                       const int32_t *t, const int32_t *lam, int32_t nv,
                       int32_t s, int32_t ts, int32_t *arr) {
  int rc = oracle_validate(n, u, v, t, lam, nv);
  if (rc != ORACLE_OK) return rc;
  if (!arr || s < 0 || s >= nv || ts < 0) return ORACLE_EINVAL;

  /* nodes: every departure event, every arrival event, and the query start */
  int64_t nev = 2 * n + 1;
  int64_t *ev = (int64_t *)malloc((size_t)nev * sizeof(int64_t));
  if (!ev) return ORACLE_ENOMEM;
  for (int64_t i = 0; i < n; ++i) {
    ev[2 * i] = pack_event(u[i], t[i]);
    ev[2 * i + 1] = pack_event(v[i], t[i] + lam[i]);
  }
  ev[2 * n] = pack_event(s, ts);
  qsort(ev, (size_t)nev, sizeof(int64_t), cmp_i64);
  int64_t m = 0;
  for (int64_t i = 0; i < nev; ++i)
    if (m == 0 || ev[i] != ev[m - 1]) ev[m++] = ev[i];
  nev = m;

  /* connection arcs in CSR form by tail node */
  int64_t *off = (int64_t *)calloc((size_t)nev + 1, sizeof(int64_t));
  int64_t *head = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  int64_t *tail = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  int32_t *wt = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int64_t *fill = (int64_t *)malloc((size_t)nev * sizeof(int64_t));
  int64_t *dist = (int64_t *)malloc((size_t)nev * sizeof(int64_t));
  heap hp = {NULL, 0, 0};
  if (!off || !head || !tail || !wt || !fill || !dist) {
    rc = ORACLE_ENOMEM;
    goto done;
  }
  for (int64_t i = 0; i < n; ++i) {
    tail[i] = find_event(ev, nev, pack_event(u[i], t[i]));
    off[tail[i] + 1]++;
  }
  for (int64_t k = 0; k < nev; ++k) off[k + 1] += off[k];
  memcpy(fill, off, (size_t)nev * sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i) {
    int64_t slot = fill[tail[i]]++;
    head[slot] = find_event(ev, nev, pack_event(v[i], t[i] + lam[i]));
    wt[slot] = lam[i];
  }

  /* Dijkstra from the start event; arc weights are elapsed seconds */
  for (int64_t k = 0; k < nev; ++k) dist[k] = INT64_MAX;
  int64_t src = find_event(ev, nev, pack_event(s, ts));
  dist[src] = 0;
  if ((rc = heap_push(&hp, 0, src)) != ORACLE_OK) goto done;
  while (hp.n > 0) {
    heap_item it = heap_pop(&hp);
    int64_t k = it.id;
    if (it.key != dist[k]) continue; /* stale entry */
    /* waiting arc to the next event of the same stop */
    if (k + 1 < nev && (ev[k + 1] >> 32) == (ev[k] >> 32)) {
      int64_t w = (int64_t)(uint32_t)ev[k + 1] - (int64_t)(uint32_t)ev[k];
      if (dist[k] + w < dist[k + 1]) {
        dist[k + 1] = dist[k] + w;
        if ((rc = heap_push(&hp, dist[k + 1], k + 1)) != ORACLE_OK) goto done;
      }
    }
    /* connection arcs boarding at this event */
    for (int64_t a = off[k]; a < off[k + 1]; ++a) {
      int64_t h2 = head[a];
      if (dist[k] + wt[a] < dist[h2]) {
        dist[h2] = dist[k] + wt[a];
        if ((rc = heap_push(&hp, dist[h2], h2)) != ORACLE_OK) goto done;
      }
    }
  }
  /* earliest arrival at a stop = time of its earliest reached event */
  for (int32_t x = 0; x < nv; ++x) arr[x] = ORACLE_INF;
  for (int64_t k = 0; k < nev; ++k) {
    if (dist[k] == INT64_MAX) continue;
    int32_t stop = (int32_t)(ev[k] >> 32);
    int64_t when = (int64_t)ts + dist[k];
    if (when < arr[stop]) arr[stop] = (int32_t)when;
  }
  rc = ORACLE_OK;
done:
  free(ev);
  free(off);
  free(head);
  free(tail);
  free(wt);
  free(fill);
  free(dist);
  free(hp.a);
  return rc;
}

/* ---- time-dependent model ---------------------------------------------------- */

int oracle_td_dijkstra(int64_t n, const int32_t *u, const int32_t *v,
                       const int32_t *t, const int32_t *lam, int32_t nv,
                       int32_t s, int32_t ts, int32_t *arr) {
  int rc = oracle_validate(n, u, v, t, lam, nv);
  if (rc != ORACLE_OK) return rc;
  if (!arr || s < 0 || s >= nv || ts < 0) return ORACLE_EINVAL;
  /* outgoing connections of every stop (CSR by u, any order inside) */
  int64_t *off = (int64_t *)calloc((size_t)nv + 1, sizeof(int64_t));
  int64_t *idx = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  int64_t *fill = (int64_t *)malloc((size_t)nv * sizeof(int64_t) + 1);
  char *settled = (char *)calloc((size_t)nv + 1, 1);
  heap hp = {NULL, 0, 0};
  if (!off || !idx || !fill || !settled) {
    rc = ORACLE_ENOMEM;
    goto done;
  }
  for (int64_t i = 0; i < n; ++i) off[u[i] + 1]++;
  for (int32_t x = 0; x < nv; ++x) off[x + 1] += off[x];
  memcpy(fill, off, (size_t)nv * sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i) idx[fill[u[i]]++] = i;

  for (int32_t x = 0; x < nv; ++x) arr[x] = ORACLE_INF;
  arr[s] = ts;
  if ((rc = heap_push(&hp, ts, s)) != ORACLE_OK) goto done;
  while (hp.n > 0) {
    heap_item it = heap_pop(&hp);
    int32_t x = (int32_t)it.id;
    if (settled[x] || it.key != arr[x]) continue;
    settled[x] = 1;
    /* arriving at x at arr[x]: any connection leaving x no earlier can be taken */
    for (int64_t k = off[x]; k < off[x + 1]; ++k) {
      int64_t i = idx[k];
      if (t[i] < arr[x]) continue;
      int32_t a = t[i] + lam[i];
      if (a < arr[v[i]]) {
        arr[v[i]] = a;
        if ((rc = heap_push(&hp, a, v[i])) != ORACLE_OK) goto done;
      }
    }
  }
  rc = ORACLE_OK;
done:
  free(off);
  free(idx);
  free(fill);
  free(settled);
  free(hp.a);
  return rc;
}
