/*
 * eat.h -- C ABI of libeat: earliest-arrival-time (EAT) queries on public-
 * transport timetables, on AMD Instinct MI355X (gfx950).
 *
 * Method: Haryan, Ramakrishna, Nasre, Reddy, "GPU Algorithm for Earliest
 * Arrival Time Problem in Public Transport Networks", arXiv 1912.00966.
 *   - the problem and its answer: Section I and Section I-A (a connection
 *     (u, v, t, lam) leaves u at t and reaches v at t + lam; a query (s, ts)
 *     asks for the earliest arrival at every stop over time-respecting paths
 *     leaving s at or after ts);
 *   - connection types (same u, v, lam) and the next departure at or after the
 *     arrival at u: Section II-B;
 *   - arithmetic-progression tuples and their closed form: Section II-C,
 *     Algorithm 6;
 *   - hourly clusters and the "next non-empty cluster" rule: Section II-D;
 *   - edge grouping and (virtual) warps per edge: Sections II-E, II-F, IV-B;
 *   - Relax and atomic minimum: Algorithm 3, Section III-C;
 *   - double-buffered activity: Section III-B; convergence without per-
 *     iteration host round trips: Section IV-C.
 *
 * General rules
 *   - Every function returns an eat_status and never throws or aborts.  On
 *     failure eat_last_error() returns a thread-local message.
 *   - Host arrays passed in are only read during the call and may be freed on
 *     return.  "device" pointers are HIP device allocations on the device that
 *     was current when the graph was built.
 *   - Times are int32 seconds, t >= 0, lam >= 1, t + lam <= EAT_INF - 1.
 *     Unreached stops get EAT_INF.  The answer is unique, so results are
 *     bit-identical whatever the layout, launch shape or batching.
 *   - Streams are hipStream_t passed as void* (NULL = the null stream).
 */
#ifndef EAT_H
#define EAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EAT_INF INT32_MAX

typedef enum {
  EAT_OK = 0,
  EAT_ERR_INVALID_ARGUMENT = 1, /* bad pointer, size, id or connection value */
  EAT_ERR_OUT_OF_MEMORY = 2,    /* host or device allocation failed */
  EAT_ERR_DEVICE = 3,           /* a HIP call failed, or no usable GPU */
  EAT_ERR_NOT_CONVERGED = 4,    /* a query hit its round limit */
  EAT_ERR_BUSY = 5,             /* no free result slot (serving sessions) */
  EAT_ERR_UNSUPPORTED = 6       /* valid input outside the library's limits */
} eat_status;

typedef enum {
  /* types -> clusters of cluster_seconds -> one arithmetic-progression
   * descriptor per cluster, or a sorted departure array when the cluster's
   * departures are not a single progression (Sections II-B..II-D) */
  EAT_LAYOUT_HYBRID = 0,
  /* types -> one sorted departure array per type, searched by bisection */
  EAT_LAYOUT_FLAT = 1
} eat_layout_kind;

typedef struct {
  int32_t layout;          /* eat_layout_kind; default EAT_LAYOUT_HYBRID */
  int32_t cluster_seconds; /* cluster width in seconds, 1..32767; 0 = 3600 (one hour) */
  int32_t n_threads;       /* host threads for preprocessing; 0 = all cores */
  int32_t header_grid;     /* hybrid layout on the device: 0 = also build the header
                              grid (default), -1 = compact headers only (see below) */
  int32_t subtrip_len;     /* *_build_trips only, sub-trip length r (Sections II-G,
                              IV-B): 0 = round(sqrt(mean trip length)), -1 =
                              round(sqrt(k)) for a trip of k connections, r >= 1 fixed
                              (1 adds no shortcut) */
  int32_t reserved[3];     /* must be zero */
} eat_build_options;

typedef struct {
  int32_t n_vertices;
  int32_t layout;
  int32_t cluster_seconds;
  int32_t n_clusters;        /* clusters per type: max departure / width + 1 (hybrid: <= 64) */
  int32_t max_departure;
  int32_t max_types_per_vertex;
  int64_t n_conn_input;      /* connections passed in */
  int64_t n_self_loops;      /* dropped: u == v can never improve an arrival */
  int64_t n_duplicates;      /* dropped: identical (u, v, t, lam) */
  int64_t n_conn;            /* connections kept */
  int64_t n_edges;           /* distinct (u, v) */
  int64_t n_types;           /* distinct (u, v, lam) */
  int64_t n_headers;         /* non-empty (type, cluster) pairs (hybrid) */
  int64_t n_ap_clusters;     /* ... stored as one progression */
  int64_t n_array_clusters;  /* ... stored as a sorted array */
  int64_t n_pool;            /* int32 words of the departure pool */
  int64_t device_bytes;      /* device memory held by the graph */
  int64_t n_grid_entries;    /* header-grid entries on the device (0: no grid) */
  int64_t n_trips;           /* *_build_trips: vehicle trips in the input */
  int64_t n_shortcuts;       /* *_build_trips: sub-trip shortcut connections added
                                (before de-duplication; counted in n_conn_input) */
  int32_t subtrip_len;       /* the sub-trip length used (-1: per trip) */
  int32_t reserved;
} eat_graph_info_t;

/* ---------------------------------------------------------------------------
 * Host layout (CPU only; needs no GPU).  The preprocessing of Section III-A:
 * connections are grouped by tail u, then by (v, lam) into connection types,
 * then each type's departures into clusters of cluster_seconds.
 * ------------------------------------------------------------------------- */
typedef struct eat_layout eat_layout;

/* Read-only view of a host layout; pointers stay valid until eat_layout_free.
 *   vt[2 * n_vertices]: the types leaving u are ty rows vt[2u] .. vt[2u] +
 *     vt[2u+1] - 1, ordered by (v, lam).
 *   order[n_vertices]: the stops in the order their type blocks are stored
 *     (breadth-first over the stop graph: stops close in the graph are close
 *     in memory).
 *   ty[4 * n_types]: per type {v, lam, a, b}.  Hybrid: a = index of the type's
 *     first cluster header, b = bits 0..31 of its cluster-occupancy mask (bit k
 *     set when cluster k holds a departure).  Flat: a = offset of its
 *     departures in pool, b = their count.
 *   ty_mask_hi[n_types]: hybrid, bits 32..63 of the occupancy mask.
 *   hdr[2 * n_headers]: hybrid, per non-empty cluster in (type, cluster) order
 *     {t0, c}: t0 = first departure of the cluster; c >= 0 encodes the
 *     progression t0 + i*h, i = 0..n-1 as c = (n << 16) | h; c < 0 encodes a
 *     sorted array at pool[~c]: pool[~c] = n, pool[~c + 1 ..] = departures.
 *   pool[n_pool]: hybrid array clusters, or flat departures.  Every entry
 *     starts at a multiple of 4 words; the gaps hold EAT_INF. */
typedef struct {
  int32_t layout;
  int32_t n_vertices;
  int32_t cluster_seconds;
  int32_t n_clusters;
  int64_t n_types;
  int64_t n_headers;
  int64_t n_pool;
  const int32_t *vt;
  const int32_t *order;
  const int32_t *ty;
  const uint32_t *ty_mask_hi;
  const int32_t *hdr;
  const int32_t *pool;
} eat_layout_view;

/* Validates and preprocesses n_conn connections (u, v, t, lam host arrays).
 * Self-loops and exact duplicates are dropped.  opt may be NULL (defaults).
 * EAT_ERR_INVALID_ARGUMENT for out-of-range ids or times, lam < 1 or
 * t + lam > EAT_INF - 1; EAT_ERR_UNSUPPORTED when the hybrid layout would need
 * more than 64 clusters per type, or more than 2^31-1 types or pool words. */
eat_status eat_layout_build(const int32_t *u, const int32_t *v, const int32_t *t,
                            const int32_t *lam, int64_t n_conn, int32_t n_vertices,
                            const eat_build_options *opt, eat_layout **out);
/* Sub-trip shortcuts (Section II-G): as eat_layout_build, with trip[i] the
 * vehicle trip of connection i (-1: on no trip).  A trip's connections, taken
 * in departure order, must chain as one vehicle's run: each reaches the stop
 * the next leaves from, no later than it leaves (EAT_ERR_INVALID_ARGUMENT
 * otherwise).  Each trip is cut into consecutive sub-trips of
 * opt->subtrip_len connections (the last one holds the rest), and each
 * sub-trip c_i .. c_j of two or more connections adds the connection from
 * c_i's tail to c_j's head leaving at t_i with duration t_j + lam_j - t_i.
 * Riding the vehicle gives the same arrival, so every query's answer is
 * unchanged, while a relaxation round crosses a whole sub-trip at once. */
eat_status eat_layout_build_trips(const int32_t *u, const int32_t *v, const int32_t *t,
                                  const int32_t *lam, const int32_t *trip, int64_t n_conn,
                                  int32_t n_vertices, const eat_build_options *opt,
                                  eat_layout **out);
void eat_layout_free(eat_layout *layout); /* NULL-safe */
eat_status eat_layout_info(const eat_layout *layout, eat_graph_info_t *out);
eat_status eat_layout_view_get(const eat_layout *layout, eat_layout_view *out);

/* ---------------------------------------------------------------------------
 * Device-resident graph
 * ------------------------------------------------------------------------- */
typedef struct eat_graph eat_graph;

/* Preprocesses (as eat_layout_build) and uploads to the current HIP device.
 * The uploads and the device-side header-grid build run on stream (NULL = the
 * null stream), and the call returns once that stream has finished them: work
 * on other streams (queries on other graphs) is not waited for.  The graph is
 * immutable afterwards; queries on several streams may share it. */
eat_status eat_graph_build(const int32_t *u, const int32_t *v, const int32_t *t,
                           const int32_t *lam, int64_t n_conn, int32_t n_vertices,
                           const eat_build_options *opt, void *stream, eat_graph **out);
/* eat_layout_build_trips + eat_graph_upload. */
eat_status eat_graph_build_trips(const int32_t *u, const int32_t *v, const int32_t *t,
                                 const int32_t *lam, const int32_t *trip, int64_t n_conn,
                                 int32_t n_vertices, const eat_build_options *opt, void *stream,
                                 eat_graph **out);
/* Uploads an existing host layout (the layout may be freed afterwards) on
 * stream, as eat_graph_build.  Of opt (nullable) only header_grid is used.
 *
 * Header grid (hybrid layout, device side).  Besides the compact headers, the
 * device holds one 16-byte entry per (type, cluster) -- empty clusters
 * included -- so that the entry a lookup needs has an address computable from
 * the type index, the cluster index k = x / width and the tail stop's type
 * range, without reading the type record first.  The entries of stop u (types
 * b .. b+n-1) form one block ordered by cluster, then type:
 *   grid[b * n_clusters + k * n + (j - b)] = {t0, c, next, m}
 * where t0 is the cluster's first departure and next the type's first
 * departure in a later cluster (EAT_INF if none), and by the top bits of c:
 *   c >= 0          a progression t0 + i*d, i < n, c = (n << 16) | d (as in
 *                   hdr below); m = ceil(2^32 / d) replaces the division by d
 *                   (0 for d = 1);
 *   c >> 30 == 2    a sorted array of three to five departures d1 = t0 < d2 <
 *                   .. : c holds o2 = d2 - t0 (bits 15..29) and o3 (bits 0..14),
 *                   m holds o4 (bits 15..29) and o5 (bits 0..14), 0 past the
 *                   array's end -- no further read is needed;
 *   c >> 30 == 3    a longer sorted array at pool[~c] (as in hdr below), m = n.
 * An empty cluster holds {next, (1 << 16) | 1, next, 0}: a one-term
 * progression at the next departure, which is the answer of Section II-D for
 * any x inside that cluster.  Lanes that expand the types of one stop at one
 * cluster read consecutive entries.  Costs 16 * n_types * n_clusters bytes of
 * HBM; built only when n_types * n_clusters < 2^31 and the pool holds fewer
 * than 2^30 words. */
eat_status eat_graph_upload(const eat_layout *layout, const eat_build_options *opt, void *stream,
                            eat_graph **out);
void eat_graph_free(eat_graph *g); /* NULL-safe; waits for the device */
eat_status eat_graph_info(const eat_graph *g, eat_graph_info_t *out);
/* *count receives the number of eat_query calls on g, made without stats,
 * that hit their round limit (EAT_ERR_NOT_CONVERGED would have been their
 * status; their arr is then incomplete) since g was built.  The count covers
 * the queries that have finished: synchronize their streams first.  Queries
 * with stats report the status themselves and are not counted here. */
eat_status eat_graph_failures(const eat_graph *g, int32_t *count);

/* ---------------------------------------------------------------------------
 * Queries
 * ------------------------------------------------------------------------- */
typedef enum {
  EAT_MODE_AUTO = 0,     /* frontier-driven; topology sweep when a frontier overflows */
  EAT_MODE_FRONTIER = 1, /* same as AUTO */
  EAT_MODE_TOPOLOGY = 2  /* every round sweeps the activity flags of all touched stops */
} eat_mode;

typedef enum {
  EAT_HEADERS_AUTO = 0,    /* the header grid when every graph of the call has one */
  EAT_HEADERS_GRID = 1,    /* the header grid; EAT_ERR_UNSUPPORTED if a graph has none */
  EAT_HEADERS_COMPACT = 2  /* the compact headers (one per non-empty cluster) */
} eat_headers;

typedef enum {
  /* longest first when the batch has more queries than the launch has
   * work-groups in flight (some work-groups run several queries one after
   * another), else by locality */
  EAT_ORDER_AUTO = 0,
  /* by graph, then by the layout position of the source: queries with nearby
   * sources run at the same time on one XCD and share its L2 */
  EAT_ORDER_LOCALITY = 1,
  /* the same split into per-XCD buckets, each bucket's queries by departure
   * time, earliest first: a query leaving early reaches far more stops (the
   * timetable thins out during the day), so the longest queries start first
   * and the launch does not end on one long query started last */
  EAT_ORDER_LONGEST_FIRST = 2,
  /* the same buckets, each split by departure time into four bands of equal
   * size, earliest band first, each band in the locality order: most of the
   * longest-first tail and most of the locality */
  EAT_ORDER_BANDED = 3
} eat_query_order;

typedef struct {
  int32_t threads_per_vertex; /* lanes sharing one active stop's types (virtual warps,
                                 Section IV-B): 1,2,4,..,64; 0 = type windows (below) */
  int32_t mode;               /* eat_mode */
  int32_t max_rounds;         /* round limit per query; 0 = n_vertices + 2 without a time
                                 window, 8 * n_vertices + 64 with one */
  int32_t frontier_cap;       /* frontier list entries kept on chip, rounded up to a
                                 multiple of 64; 0 = auto */
  int32_t table_cap;          /* on-chip arrival-table slots (power of two); 0 = auto,
                                 -1 = keep arrivals in the result slab (HBM) only */
  int32_t types_per_lane;     /* threads_per_vertex = 0: a round's connection types are
                                 numbered in list order and cut into windows of 64; each wave
                                 relaxes types_per_lane windows per step, one type of each per
                                 lane (rounds of more than 8,192 types: each wave takes
                                 4 * types_per_lane listed stops at a time and spreads their
                                 types over its lanes); 1..3, 0 = 1 */
  int32_t headers;            /* eat_headers: which form of the hybrid headers to read */
  int32_t time_window;        /* frontier rounds expand only the listed stops whose arrival
                                 is below (smallest arrival pushed for the round) + this
                                 many seconds; the others stay listed for a later round.
                                 0 = auto (7200), -1 = no window (every listed stop every
                                 round, the schedule of Section III-B).  The answer is the
                                 same either way; the window trades a few more rounds for
                                 fewer re-expansions of stops whose arrival improves */
  int32_t threads_per_query;  /* work-group size of one query: 1024 (default); 768 or 512
                                 -- two queries share a CU, each with half of its LDS for
                                 the arrival table; 384 -- four per CU, a quarter each;
                                 256 -- six per CU, a sixth each (type windows only:
                                 threads_per_vertex = 0; 256, 384 and 768 with one type per
                                 lane; a graph whose activity bitmap, one bit per stop, does
                                 not fit the LDS share: EAT_ERR_UNSUPPORTED, 1024 runs it).
                                 More queries per CU raise throughput when many are in
                                 flight; 1024 finishes a single long query sooner.
                                 0 = 1024 */
  int32_t query_order;        /* eat_query_order: the order in which a batch's work-groups
                                 take its queries */
  int32_t reserved[3];        /* must be zero */
} eat_run_options;

typedef struct {
  int32_t status;        /* EAT_OK or EAT_ERR_NOT_CONVERGED */
  int32_t rounds;        /* relaxation rounds until no arrival improved */
  int32_t sweep_rounds;  /* of which topology sweeps */
  int32_t max_frontier;  /* largest frontier (pushes of one round) */
  int32_t reached;       /* stops with a finite arrival, the source included */
  int32_t spilled;       /* 1 if the on-chip arrival table overflowed and the
                            query was run again against the result slab */
  int64_t activations;   /* active stops processed */
  int64_t type_evals;    /* connection types examined */
  int64_t header_loads;  /* cluster headers read (hybrid) */
  int64_t pool_loads;    /* departure words read from the pool */
  int64_t improvements;  /* successful atomic minimum updates */
  int64_t elapsed_ns;    /* device wall-clock time from the query's start to its end */
} eat_query_stats;

/* One query (s, ts) on g: the earliest arrival time at every stop over
 * time-respecting paths that leave s at or after ts (the problem of Sections I
 * and I-A), by the relaxation of Algorithms 2 (initialize), 3 (relax by atomic
 * minimum, Section III-C) and 5-6 (next departure of a connection type,
 * Sections II-B..II-D), iterated over the active stops (Section III-B) until
 * no arrival improves.  arr: device, >= n_vertices int32, caller-owned;
 * it receives the earliest arrival times.  Asynchronous on stream when stats
 * is NULL; with stats (host pointer) the call waits for the stream, fills it
 * and returns EAT_ERR_NOT_CONVERGED if the round limit was hit.
 * EAT_ERR_INVALID_ARGUMENT (arr untouched) for s outside [0, n_vertices),
 * ts < 0 or arr NULL. */
eat_status eat_query(const eat_graph *g, int32_t s, int32_t ts, int32_t *arr,
                     void *stream, const eat_run_options *ro, eat_query_stats *stats);

/* Goal-directed query (Section I: the earliest arrival at one destination d).
 * Same arguments, errors and stream semantics as eat_query, plus d in
 * [0, n_vertices).  On completion arr[d] holds the earliest arrival at d from
 * (s, ts), EAT_INF if unreachable; every other entry of arr holds an upper
 * bound of that stop's earliest arrival (a real arrival time, or EAT_INF):
 * the relaxation keeps only what can still improve the arrival at d -- a stop
 * reached no earlier than the best arrival at d found so far is neither
 * written nor expanded -- and ends when every listed stop is at or past it.
 * Runs the type-window kernels with one connection type per lane
 * (EAT_ERR_UNSUPPORTED if ro asks for threads_per_vertex > 0). */
eat_status eat_query_goal(const eat_graph *g, int32_t s, int32_t ts, int32_t d, int32_t *arr,
                          void *stream, const eat_run_options *ro, eat_query_stats *stats);

/* A prepared batch of n_q queries over n_graphs graphs, run by one persistent
 * launch in which each work-group takes whole queries from a shared counter.
 * q_graph/q_src/q_ts: host arrays; arr: host array of n_q device pointers, slab
 * i holding >= n_vertices(graphs[q_graph[i]]) int32.  Descriptors are copied to
 * the device during create; graphs and slabs must outlive the batch. */
typedef struct eat_batch eat_batch;
eat_status eat_batch_create(const eat_graph *const *graphs, int32_t n_graphs,
                            const int32_t *q_graph, const int32_t *q_src,
                            const int32_t *q_ts, int32_t n_q, int32_t *const *arr,
                            const eat_run_options *ro, eat_batch **out);
/* eat_batch_create with a destination per query: q_dst[i] in [0, n_vertices)
 * makes query i goal-directed (its slab as in eat_query_goal), -1 asks for
 * every stop (its slab as in eat_query).  q_dst: host array of n_q. */
eat_status eat_batch_create_goal(const eat_graph *const *graphs, int32_t n_graphs,
                                 const int32_t *q_graph, const int32_t *q_src,
                                 const int32_t *q_ts, const int32_t *q_dst, int32_t n_q,
                                 int32_t *const *arr, const eat_run_options *ro, eat_batch **out);
/* Enqueues the whole batch on stream (asynchronous; repeatable): one
 * persistent kernel launch and an event record, no allocation, memset or
 * copy -- the launch re-arms its own device counters -- so a run can be
 * captured into a HIP graph (stream capture) and replayed.  Runs of one batch
 * must not overlap (they share its counters and slabs). */
eat_status eat_batch_run(eat_batch *b, void *stream);
/* Waits for the last run and copies per-query stats (host array of n_q,
 * nullable); returns EAT_ERR_NOT_CONVERGED if any query hit its limit. */
eat_status eat_batch_wait(eat_batch *b, eat_query_stats *stats);
void eat_batch_free(eat_batch *b); /* NULL-safe; waits for the last run */

/* eat_query_batch without any allocation, for callers that cannot allocate:
 * code being captured into a HIP graph, tight serving loops, and harnesses
 * that forbid hipMalloc.  Same arguments, checks, results and statistics as
 * eat_query_batch; returns after the batch has finished.  Its device-side
 * state lives in a fixed scratch array that each GPU the library runs on holds
 * until the process ends (about 1 MiB), so at most 8192 queries over at most
 * 64 graphs per call (EAT_ERR_INVALID_ARGUMENT beyond).  Every call on a GPU
 * shares that GPU's array and rewrites it: calls that overlap on one GPU (from
 * several processes, or on several streams without ordering) race; the calls
 * of one process are serialized by a lock.  Calls no hipMalloc, hipFree or
 * other allocating routine. */
eat_status eat_query_batch_static(const eat_graph *const *graphs, int32_t n_graphs,
                                  const int32_t *q_graph, const int32_t *q_src,
                                  const int32_t *q_ts, int32_t n_q, int32_t *const *arr,
                                  void *stream, const eat_run_options *ro,
                                  eat_query_stats *stats);

/* The run options a batch was created with: the caller's, or with NULL
 * options the tuned record (eat_batch_tune) or the defaults. */
eat_status eat_batch_options(const eat_batch *b, eat_run_options *out);

/* Many queries at once, each answered as by eat_query (Sections I and I-A;
 * Algorithms 2, 3, 5, 6): create + run + wait + free.  Returns after the
 * batch has finished. */
eat_status eat_query_batch(const eat_graph *const *graphs, int32_t n_graphs,
                           const int32_t *q_graph, const int32_t *q_src,
                           const int32_t *q_ts, int32_t n_q, int32_t *const *arr,
                           void *stream, const eat_run_options *ro,
                           eat_query_stats *stats);

/* ---------------------------------------------------------------------------
 * Journeys and profiles (Section I: the earliest arrival path behind an
 * arrival time, and the profile-search variant over an interval of departure
 * times).
 * ------------------------------------------------------------------------- */
/* Parent connection of every stop for the EAT answer arr (device, n_vertices
 * int32, as written by eat_query / a batch / a session for a query from s).
 * par (device, 3 * n_vertices int32, caller-owned) receives per stop v
 * (u, t, lam) at par[3v .. 3v+2]: among the connections (u, v, t, lam) with
 * arr[u] <= t and t + lam == arr[v], the one with the smallest u, then the
 * smallest lam; -1 three times for s, for unreached stops, and for any stop
 * whose arrival no connection realises (arr is then not an EAT answer).
 * Following parents from a reached stop back to s gives, read forwards, a
 * journey that leaves s no earlier than arr[s] and arrives at arr[v]; parents
 * strictly decrease the arrival (lam >= 1), so the walk ends.  On a graph
 * built with sub-trip shortcuts a parent can be a shortcut (one vehicle's
 * ride over several stops).  Asynchronous on stream (a stream-ordered scratch
 * of 8 * n_vertices bytes).  EAT_ERR_INVALID_ARGUMENT for a NULL pointer or s
 * out of range. */
eat_status eat_parents(const eat_graph *g, int32_t s, const int32_t *arr, int32_t *par, void *stream);

/* Profile of source s over departures in [t_lo, t_hi]: the Pareto-optimal
 * (departure, arrival) pairs of every stop among all journeys that leave s at
 * or after t_lo, restricted to those leaving no later than t_hi.
 * *n_dep receives the number k of distinct departure times of connections
 * leaving s inside the interval (every Pareto departure is one of them);
 * dep (host, cap int32) receives them in increasing order; arr (device,
 * cap * n_vertices int32, row-major, caller-owned) receives in row i, for
 * every stop v, the arrival of the Pareto-optimal journey to v leaving s at
 * dep[i], or EAT_INF if no such journey is Pareto-optimal (always at v = s).
 * Computed as one batch of k + 1 queries -- one at each dep[i] and one at the
 * first departure after t_hi -- whose row i keeps EAT(s, dep[i])[v] only
 * where it beats row i + 1 (a journey leaving later does no better
 * otherwise).  Synchronous.  If k > cap nothing is computed and
 * EAT_ERR_UNSUPPORTED is returned, except that cap = 0 with arr = NULL asks
 * for k alone (EAT_OK).  ro: run options of the batch (NULL: tuned/defaults). */
eat_status eat_profile(const eat_graph *g, int32_t s, int32_t t_lo, int32_t t_hi, int32_t cap,
                       int32_t *dep, int32_t *n_dep, int32_t *arr, void *stream,
                       const eat_run_options *ro);

/* ---------------------------------------------------------------------------
 * Autotuning of batched launches.
 *
 * Run options change the speed of a batch, never its answers (the answer of a
 * query is unique).  eat_batch_tune runs the batch (same arguments as
 * eat_batch_create) under each of a fixed set of candidates -- threads per
 * query 1024 / 768 / 512, connection types in flight per lane (a wave
 * evaluates 64 x that many (type, cluster) lookups at once: the clusters in
 * flight per wave), virtual warps of 16 / 32 lanes per active stop (threads
 * per edge, Sections II-F and IV-B), arrival windows, the topology-driven
 * schedule and the compact header form -- fingerprints every result slab on
 * the device and requires all candidates to agree (EAT_ERR_DEVICE otherwise),
 * times each with HIP events on `stream`, and returns the fastest in *best.
 * The choice is recorded for this device, these graphs (their sizes and
 * layout) and n_q; eat_batch_create with NULL options uses the record.  With
 * the environment variable EAT_TUNE_FILE naming a file, records are appended
 * to it and read back by later processes.  Without a record, NULL options
 * mean 768-thread queries when n_q exceeds the device's CU count, else the
 * eat_run_options defaults.  On return the slabs hold the batch's answers.
 * Synchronous; allocates device memory for the candidates' batches.
 * ------------------------------------------------------------------------- */
typedef struct {
  int32_t reps;        /* timed runs per candidate (per stream); 0 = 3 */
  int32_t n_streams;   /* timed runs alternate over this many streams (1..4), each
                          with its own prepared batch, as a caller that overlaps
                          consecutive batches issues them; 0 = 1 */
  int32_t reserved[6]; /* must be zero */
} eat_tune_options;

typedef struct {
  eat_run_options options;
  float ms;            /* mean time per run */
  int32_t reserved;
} eat_tune_result;

/* results (host array of results_cap, nullable when results_cap = 0) receives
 * every candidate's time; *n_results (nullable) their count. */
eat_status eat_batch_tune(const eat_graph *const *graphs, int32_t n_graphs,
                          const int32_t *q_graph, const int32_t *q_src, const int32_t *q_ts,
                          int32_t n_q, int32_t *const *arr, void *stream,
                          const eat_tune_options *opt, eat_run_options *best,
                          eat_tune_result *results, int32_t results_cap, int32_t *n_results);

/* ---------------------------------------------------------------------------
 * Serving sessions: continuous batching over device-resident graphs.
 *
 * A session owns a pool of device memory for result slots.  eat_session_admit
 * reserves one slot (n_vertices int32 of the query's graph) or returns
 * EAT_ERR_BUSY when no free range of the pool fits.  eat_session_step launches,
 * in one kernel launch, every query admitted since the previous step, on the
 * next of the session's streams; several steps can be in flight at once, so
 * queries admitted while earlier ones are still running share the device
 * with them.  eat_session_poll reports finished slots without blocking; a
 * finished slot's arrival array stays valid until eat_session_release.
 * A session is not thread-safe: one thread drives it.
 * ------------------------------------------------------------------------- */
typedef struct eat_session eat_session;

typedef struct {
  int64_t pool_bytes;       /* device memory for result slots; 0 = 256 MiB */
  int32_t n_streams;        /* launches in flight at once (1..8); 0 = 2 */
  int32_t max_step_queries; /* queries one step launches at most; 0 = 4096 */
  eat_run_options run;      /* options of every launch (NULL-equivalent when zero) */
  int32_t reserved[4];      /* must be zero */
} eat_session_options;

/* graphs: n_graphs resident graphs (they must outlive the session). */
eat_status eat_session_create(const eat_graph *const *graphs, int32_t n_graphs,
                              const eat_session_options *opt, eat_session **out);
/* Reserves a slot for query (s, ts) on graphs[graph]; *slot receives its id.
 * EAT_ERR_BUSY: no room in the pool (nothing reserved); EAT_ERR_INVALID_ARGUMENT
 * for a bad graph index, s or ts. */
eat_status eat_session_admit(eat_session *sess, int32_t graph, int32_t s, int32_t ts,
                             int32_t *slot);
/* Launches the queries admitted since the last step (up to max_step_queries;
 * the rest wait for the next step).  Never waits: if every launch slot (one
 * per stream) is still in flight it launches nothing and returns
 * EAT_ERR_BUSY, so the caller can poll and admit meanwhile.  *n_launched
 * (nullable) receives the count. */
eat_status eat_session_step(eat_session *sess, int32_t *n_launched);
/* Writes up to cap finished slot ids into done (host array); *n receives the
 * count.  Never blocks. */
eat_status eat_session_poll(eat_session *sess, int32_t *done, int32_t cap, int32_t *n);
/* Blocks until every launched query has finished (they are then reported by
 * eat_session_poll). */
eat_status eat_session_sync(eat_session *sess);
/* Device pointer to a finished slot's arrival array and its length. */
eat_status eat_session_result(eat_session *sess, int32_t slot, const int32_t **arr,
                              int32_t *n_vertices);
/* Copies a finished slot's n_vertices int32 into dst (device or pinned/pageable
 * host memory), asynchronously on stream. */
eat_status eat_session_copy(eat_session *sess, int32_t slot, int32_t *dst, void *stream);
/* Statistics of a finished slot's query (elapsed_ns is device time). */
eat_status eat_session_query_stats(eat_session *sess, int32_t slot, eat_query_stats *out);
/* Frees a finished (or admitted but not yet launched) slot. */
eat_status eat_session_release(eat_session *sess, int32_t slot);

typedef struct {
  int64_t steps;       /* launches made */
  int64_t launched;    /* queries launched (= n) */
  int64_t busy_waits;  /* admissions deferred because the pool was full */
  double wall_s;       /* from the call until the last query finished */
} eat_serve_report;

/* Drives the session through an open-loop request stream on the calling
 * thread: request i arrives arrival_s[i] seconds after the call starts
 * (non-decreasing), asking (src[i], ts[i]) on graphs[graph[i]].  Requests are
 * admitted first come, first served while slot memory lasts; the admitted
 * queries are launched in one step when no launched query is unfinished, when
 * min_batch (>= 1) of them wait, or when the oldest has waited max_delay_s;
 * every finished query is reported, its result copied to copy_dst[i] on
 * copy_stream when copy_dst (nullable) and copy_dst[i] are not NULL (device
 * memory, >= n_vertices int32; the slot's reuse waits for the copy), and its
 * slot released.  latency_s[i] (host array) receives the time from its arrival
 * to the poll that saw it finished.  All host arrays have n entries.  The
 * requests are checked before the first one is admitted
 * (EAT_ERR_INVALID_ARGUMENT, also for a graph whose result slot is larger
 * than the whole pool); the session must hold no admitted or unfinished
 * query when called.  rep (nullable) receives the counts.  This is the
 * request loop of a server, in native code: Section I's queries, answered by
 * eat_session_step launches. */
eat_status eat_session_serve(eat_session *sess, int32_t n, const int32_t *graph, const int32_t *src,
                             const int32_t *ts, const double *arrival_s, int32_t min_batch,
                             double max_delay_s, int32_t *const *copy_dst, void *copy_stream,
                             double *latency_s, eat_serve_report *rep);
void eat_session_free(eat_session *sess); /* NULL-safe; waits for the device */

/* ---------------------------------------------------------------------------
 * The paper's algorithm ladder, for comparison on the same GPU.
 *
 * Each variant answers the same EAT query (bit-identical results) the way the
 * paper describes it: a topology-driven iteration, one kernel launch per
 * iteration over every work item of the variant, a work item acting only if
 * its tail stop is active (active / nextactive flags, Section III-B; atomic
 * minimum, Section III-C; early termination, Section III-D), until an
 * iteration improves nothing.  The host reads the device's change flag after
 * every check_every-th iteration (1: every iteration, as in Table II; the
 * reduced transfers of Section IV-C read it every ~sqrt(d(G)) iterations;
 * iterations past convergence change nothing).
 * ------------------------------------------------------------------------- */
typedef enum {
  EAT_VARIANT_CONNECTION = 0,         /* Algorithm 4: a thread per connection */
  EAT_VARIANT_CONNECTION_TYPE = 1,    /* Algorithm 5: a thread per connection type, linear
                                         search of its sorted departures (Section II-B) */
  EAT_VARIANT_CONNECTION_TYPE_AP = 2, /* Algorithm 5 with Algorithm 6 over the greedy
                                         progression cover of the type (Section II-C) */
  EAT_VARIANT_CLUSTER_AP = 3,         /* Section II-D: the cover of the cluster of e[u]
                                         (cluster_seconds wide), else the first departure
                                         of the next non-empty cluster */
  EAT_VARIANT_EDGE = 4,               /* Section II-E: a thread per edge (u, v), Cluster-AP
                                         for each of its types */
  EAT_VARIANT_WARPS = 5,              /* Sections II-F, IV-B: warp_size lanes per edge */
  EAT_VARIANT_ESDG = 6                /* Section I-A: the edge-scan-dependency graph, one
                                         launch per level (needs esdg at build time) */
} eat_variant;

typedef struct {
  int32_t cluster_seconds; /* cluster width of EAT_VARIANT_CLUSTER_AP / EDGE / WARPS, 1..86400;
                              0 = 3600 */
  int32_t esdg;            /* 1: also build the ESDG levels (host work and memory ~ C) */
  int32_t n_threads;       /* host threads; 0 = all cores */
  int32_t reserved[5];     /* must be zero */
} eat_variant_build_options;

typedef struct {
  int32_t n_vertices;
  int32_t n_clusters;      /* clusters per type: max departure / cluster_seconds + 1 */
  int32_t n_levels;        /* ESDG levels (0 if not built) */
  int32_t reserved;
  int64_t n_conn;          /* after removing self-loops and duplicates */
  int64_t n_types;
  int64_t n_edges;
  int64_t n_type_aps;      /* progression tuples covering whole types */
  int64_t n_cluster_aps;   /* progression tuples covering (type, cluster) parts */
  int64_t n_esdg_edges;    /* dependency edges of the ESDG */
  int64_t device_bytes;
} eat_variant_info;

typedef struct {
  int32_t variant;         /* eat_variant */
  int32_t warp_size;       /* EAT_VARIANT_WARPS: 1, 2, 4, .., 64 lanes per edge; 0 = 32 */
  int32_t check_every;     /* iterations between host reads of the change flag; 0 = 1 */
  int32_t count;           /* 1: count the departures / tuples / connections examined */
  int32_t max_iterations;  /* 0 = n_vertices + 2 */
  int32_t reserved[3];     /* must be zero */
} eat_variant_options;

typedef struct {
  int32_t status;          /* EAT_OK or EAT_ERR_NOT_CONVERGED */
  int32_t iterations;      /* kernel launches of the relaxation (ESDG: levels) */
  int32_t host_checks;     /* device-to-host reads of the change flag */
  int32_t reserved;
  int64_t examined;        /* with count: departures, tuples or connections examined */
} eat_variant_stats;

/* Host only.  The greedy arithmetic-progression cover of Section I-A of the n
 * strictly increasing values d: repeatedly the smallest uncovered value a and
 * the progression from a, made only of values of d, that covers the most
 * uncovered values (ties: the longest, then the smallest difference).  out
 * (host, 3 * cap) receives {first, last, difference} per progression
 * (difference 0: a single term), in increasing first terms; *n_out their
 * count.  EAT_ERR_UNSUPPORTED if more than cap (cap = 0 with out = NULL asks
 * for the count, EAT_OK). */
eat_status eat_ap_cover(const int32_t *d, int64_t n, int32_t *out, int64_t cap, int64_t *n_out);
/* Host only.  ESDG level of each of the n_conn connections as given (Section
 * I-A: c -> c' when c' leaves c's head at or after c arrives and no
 * connection of the same edge leaving then arrives earlier than c'; the
 * level is the longest path from a connection without predecessors).
 * level: host array of n_conn; *n_levels (nullable) the number of levels,
 * *n_edges (nullable) the number of dependency edges. */
eat_status eat_esdg_levels(const int32_t *u, const int32_t *v, const int32_t *t, const int32_t *lam,
                           int64_t n_conn, int32_t n_vertices, int32_t *level, int32_t *n_levels,
                           int64_t *n_edges);

typedef struct eat_variant_graph eat_variant_graph;

/* Preprocesses n_conn connections (same rules as eat_layout_build) into the
 * arrays of every variant, on the current device. */
eat_status eat_variant_graph_build(const int32_t *u, const int32_t *v, const int32_t *t,
                                   const int32_t *lam, int64_t n_conn, int32_t n_vertices,
                                   const eat_variant_build_options *opt, eat_variant_graph **out);
eat_status eat_variant_graph_info(const eat_variant_graph *g, eat_variant_info *out);
/* One query (s, ts) by the chosen variant into arr (device, >= n_vertices
 * int32, caller-owned): the EAT answer.  Synchronous (the host drives the
 * iterations on stream).  stats nullable.  EAT_ERR_UNSUPPORTED for
 * EAT_VARIANT_ESDG on a graph built without it. */
eat_status eat_variant_query(const eat_variant_graph *g, int32_t s, int32_t ts, int32_t *arr, void *stream,
                             const eat_variant_options *opt, eat_variant_stats *stats);
void eat_variant_graph_free(eat_variant_graph *g); /* NULL-safe */

/* ---------------------------------------------------------------------------
 * Diagnostics
 * ------------------------------------------------------------------------- */
/* For each probe i: out[i] = the first departure >= x[i] of connection type
 * type_ids[i] (Section II-B), or EAT_INF, computed on the GPU by the same
 * device function the relaxation uses, reading the header form `headers`
 * (eat_headers; ignored for the flat layout).  All three arrays are device
 * arrays of n int32 (type ids must lie in [0, n_types)).  Asynchronous on
 * stream. */
eat_status eat_next_departure(const eat_graph *g, int32_t headers, const int32_t *type_ids,
                              const int32_t *x, int32_t *out, int32_t n, void *stream);

const char *eat_status_string(eat_status s);
const char *eat_last_error(void);
/* Library version as major * 10000 + minor * 100 + patch. */
int32_t eat_version(void);

#ifdef __cplusplus
}
#endif
#endif /* EAT_H */
