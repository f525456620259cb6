/*
 * oracle.h -- CPU reference implementations for the earliest-arrival-time (EAT)
 * problem of Haryan, Ramakrishna, Nasre and Reddy, "GPU Algorithm for Earliest
 * Arrival Time Problem in Public Transport Networks" (arXiv 1912.00966).
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  The GPU library never links,
 * includes or calls anything here, and nothing here includes a header of the GPU
 * library.
 *
 * Conventions shared by every function (Section I-A, "Preliminaries"):
 *   - a connection (u, v, t, lam) leaves stop u at second t and reaches stop v at
 *     t + lam; vertices are 0 .. nv-1;
 *   - a query is (s, ts); the answer arr[] holds, for each vertex, the earliest
 *     arrival time over time-respecting paths that leave s at or after ts
 *     (Section I, the EAT problem statement), arr[s] = ts, and ORACLE_INF for
 *     vertices no such path reaches;
 *   - inputs must satisfy t >= 0, lam >= 1 and t + lam <= ORACLE_INF - 1;
 *     functions return ORACLE_EINVAL otherwise.  lam >= 1 is the reading under
 *     which a single time-ordered scan is exact (with lam = 0 the scan would
 *     depend on the order of equal departure times).
 * All buffers are owned by the caller; nothing is retained after a call except
 * inside the opaque handle of the connection-scan oracle.
 */
#ifndef EAT_ORACLE_H
#define EAT_ORACLE_H
#include <stdint.h>

#define ORACLE_INF INT32_MAX
#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_ENOMEM 2
#define ORACLE_ELIMIT 3

#ifdef __cplusplus
extern "C" {
#endif

/* Checks every connection against the conventions above. */
int oracle_validate(int64_t n, const int32_t *u, const int32_t *v,
                    const int32_t *t, const int32_t *lam, int32_t nv);

/* ---- Connection-Scan Algorithm (Algorithm 1, Section I-A) ------------------ */
typedef struct oracle_csa oracle_csa;
/* Copies the connections and orders them by non-decreasing departure time.
 * Returns NULL on invalid input or allocation failure. */
oracle_csa *oracle_csa_new(int64_t n, const int32_t *u, const int32_t *v,
                           const int32_t *t, const int32_t *lam, int32_t nv);
void oracle_csa_free(oracle_csa *h);
/* arr must hold nv int32. */
int oracle_csa_query(const oracle_csa *h, int32_t s, int32_t ts, int32_t *arr);
/* Runs nq queries one after another; arr is nq x nv, row-major. */
int oracle_csa_query_many(const oracle_csa *h, int32_t nq, const int32_t *s,
                          const int32_t *ts, int32_t *arr);

/* ---- Brute force from the definition (Section I) ---------------------------- */
/* Depth-first enumeration of every time-respecting connection sequence that
 * starts at s no earlier than ts.  Exponential: tiny inputs only.  Gives up with
 * ORACLE_ELIMIT after max_paths sequences. */
int oracle_brute_paths(int64_t n, const int32_t *u, const int32_t *v,
                       const int32_t *t, const int32_t *lam, int32_t nv,
                       int32_t s, int32_t ts, int64_t max_paths, int32_t *arr);
/* Closure over reachable (vertex, time) states: start from (s, ts); a state
 * (x, tau) and a connection leaving x at t >= tau yield (v, t + lam).  Iterates
 * until no new state appears.  Polynomial, small inputs. */
int oracle_brute_states(int64_t n, const int32_t *u, const int32_t *v,
                        const int32_t *t, const int32_t *lam, int32_t nv,
                        int32_t s, int32_t ts, int32_t *arr);

/* ---- Dijkstra on the time-expanded model (Section I, related-work models) ---- */
/* One node per (stop, event time); waiting arcs join consecutive events of a
 * stop, connection arcs join (u, t) to (v, t + lam).  Label-setting search with
 * a binary heap from the event (s, ts). */
int oracle_te_dijkstra(int64_t n, const int32_t *u, const int32_t *v,
                       const int32_t *t, const int32_t *lam, int32_t nv,
                       int32_t s, int32_t ts, int32_t *arr);
/* ---- Dijkstra on the time-dependent model ----------------------------------- */
/* One node per stop; the label of a stop is its arrival time; when a stop is
 * settled every connection leaving it at or after the label is relaxed. */
int oracle_td_dijkstra(int64_t n, const int32_t *u, const int32_t *v,
                       const int32_t *t, const int32_t *lam, int32_t nv,
                       int32_t s, int32_t ts, int32_t *arr);

/* ---- Certificate ------------------------------------------------------------ */
/* Checks arr[] against the EAT definition without recomputing it:
 *   (1) arr[s] == ts;
 *   (2) closure: every connection with arr[u] <= t has arr[v] <= t + lam;
 *   (3) witness: every v != s with arr[v] < INF has an incoming connection with
 *       arr[u] <= t and t + lam == arr[v].
 * (2) bounds arr from above by every path's arrival; (3) gives each finite
 * entry a chain of strictly earlier entries ending at s (lam >= 1), i.e. a real
 * path, which bounds arr from below.  Returns 0 when arr is the EAT answer, else
 * the number (1, 2 or 3) of the first failed condition; *bad_vertex receives a
 * vertex where it failed (nullable). */
int oracle_certify(int64_t n, const int32_t *u, const int32_t *v,
                   const int32_t *t, const int32_t *lam, int32_t nv,
                   int32_t s, int32_t ts, const int32_t *arr,
                   int32_t *bad_vertex);

/* ---- Journeys and profiles (Section I: the query variants) ------------------- */
/* Parent connection of every stop for an EAT answer arr of the query from s:
 * for v != s with arr[v] < INF, among the connections (u, v, t, lam) with
 * arr[u] <= t and t + lam == arr[v], the one with the smallest u, then the
 * smallest lam: par_u[v] = u, par_t[v] = t, par_lam[v] = lam (-1 for s and for
 * unreached stops).  ORACLE_EINVAL if some reached v != s has no such
 * connection (arr is then not an EAT answer). */
int oracle_parents(int64_t n, const int32_t *u, const int32_t *v, const int32_t *t,
                   const int32_t *lam, int32_t nv, int32_t s, const int32_t *arr,
                   int32_t *par_u, int32_t *par_t, int32_t *par_lam);
/* Profile of s over departures in [t_lo, t_hi]: *n_dep = the number k of
 * distinct departure times of connections leaving s inside the interval;
 * dep[0..k) receives them in increasing order and arr (k x nv, row-major)
 * receives in row i, for every stop x, the arrival of the Pareto-optimal
 * journey to x that leaves s at dep[i] (optimal among all journeys leaving s
 * at or after t_lo), or ORACLE_INF if there is none (always for x = s).
 * ORACLE_ELIMIT (nothing written but *n_dep) when k > cap.  Computed with one
 * connection scan per departure (h: the scan of the same connections, whose
 * raw u and t are passed too). */
int oracle_profile(int64_t n, const int32_t *u, const int32_t *t, const oracle_csa *h, int32_t nv,
                   int32_t s, int32_t t_lo, int32_t t_hi, int32_t cap, int32_t *dep, int32_t *n_dep,
                   int32_t *arr);
/* The same profile by enumerating every journey from s (tiny inputs; gives up
 * with ORACLE_ELIMIT after max_paths connection sequences). */
int oracle_brute_profile(int64_t n, const int32_t *u, const int32_t *v, const int32_t *t,
                         const int32_t *lam, int32_t nv, int32_t s, int32_t t_lo, int32_t t_hi,
                         int64_t max_paths, int32_t cap, int32_t *dep, int32_t *n_dep, int32_t *arr);

/* ---- Next departure of one connection type (Section II-B) ------------------- */
/* min { d[i] : d[i] >= x } over n departures in any order, or ORACLE_INF. */
int32_t oracle_next_departure(int64_t n, const int32_t *d, int32_t x);

#ifdef __cplusplus
}
#endif
#endif
