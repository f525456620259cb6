"""Benchmark: earliest-arrival-time (EAT) queries per second on one MI355X.

Default workload -- batched EAT over several graphs: 4,096 (s, ts) queries
spread over eight synthetic cities of 2k, 5k, 10k, 20k, 50k, 100k, 200k and
500k stops (about 208M connections in all), answered by one persistent launch
of the relaxation kernel per step into per-query int32 result slabs.  Graphs,
query descriptors and slabs are resident in HBM before the timed region; steps
alternate over a few streams, each with its own prepared batch and slabs.

Printed (one JSON line):
  value         batched queries/s over the timed steps
  plain         the same queries as one single-query launch each, one after another
  roofline      the relaxation kernel: algorithmic relaxation bytes per launch
                (per-unit model below) / mean launch time from HIP events on the
                launch stream, against the 8 TB/s HBM peak and a measured copy;
                the slab fill is reported beside it, not in it
  cpu_baseline  the oracle (connection scan) over every query, on the host cores
  served        continuous batching over the 10k/50k/500k cities at two Poisson rates
Every answer of every stream's batch, and of the plain run, is compared element
by element with the oracle's.

    python bench.py [--steps K] [--warmup W] [--workload mixed|city-50k|city-1k|region-500k]
    python bench.py --serve            (full serving report, its own JSON line)
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

# Algorithmic bytes per unit of relaxation work (what the method must move,
# counted by the kernel's own device-side counters):
#   activation   16  the stop's type range 8, its arrival 4, its frontier entry 4
#   type eval    40  type record 20, cluster header 12, arr[v] 4, array probes 4
#   improvement   8  atomic minimum (read-modify-write)
# and per query, reported separately (Algorithm 2's initialisation and the
# result): 4 * V (slab filled with infinity) + 4 * reached (final values).
BYTES_ACTIVATION, BYTES_TYPE_EVAL, BYTES_IMPROVEMENT = 16, 40, 8


def algorithmic_bytes(stats, n_vertices):
    """(relaxation bytes, fill bytes) of the queries in `stats`; n_vertices[i]
    is the stop count of query i's graph."""
    relax = fill = 0
    for st, V in zip(stats, n_vertices):
        relax += (BYTES_ACTIVATION * st["activations"] + BYTES_TYPE_EVAL * st["type_evals"]
                  + BYTES_IMPROVEMENT * st["improvements"])
        fill += 4 * V + 4 * st["reached"]
    return relax, fill


MODES = {"auto": 0, "topology": 2}  # eat_mode values
HEADERS = {"auto": 0, "grid": 1, "compact": 2}  # eat_headers values
# Overlapping consecutive batches pays when a batch is shorter than its slowest
# query (few queries per CU), and for the mixed batch, whose launch ends on a
# tail of long queries that the next launch fills.  Four streams use the
# runtime's four hardware queues.  Measured on MI355X.
DEFAULT_STREAMS = {"city-1k": 4, "city-50k": 4, "region-500k": 2, "mixed": 4}
# Threads per query: 768 puts two queries of 12 waves on a CU (more queries in
# flight, the heavy ones still with many waves), 1024 finishes one long query
# sooner and keeps the whole LDS for its table (region-500k).
DEFAULT_THREADS = {"city-1k": 1024, "city-50k": 768, "region-500k": 1024, "mixed": 768}


def launch_key(o):
    """The effective launch options of a batch (eat_batch_options), as text."""
    return ",".join(str(x) for x in (o["threads_per_query"] or 1024, o["types_per_lane"] or 1,
                                     o["threads_per_vertex"], o["time_window"] or 7200, o["mode"], o["headers"],
                                     o["table_cap"], o["frontier_cap"], o["query_order"]))


def profile_traffic_for(args, options):
    """HBM bytes per launch from the committed rocprofv3 summary of this
    workload (profiles/k_relax_<workload>[-topology].md), only while the kernel
    source and the launch options are the profiled ones."""
    if args.layout != "hybrid":
        return None
    name = f"k_relax_{args.workload}" + ("-topology" if args.mode == "topology" else "") + ".md"
    return profiled_traffic(os.path.join(ROOT, "profiles", name), launch_key(options))


# The sources whose code the relaxation kernel's traffic depends on.
KERNEL_SOURCES = ("relax.hpp", "relax_grid.hip", "kernels.hip", "device.hpp")


def kernel_source_digest():
    """SHA-256 of the kernel sources with their comments and blank lines
    removed: a change of code changes it, a change of comments does not."""
    import hashlib
    import re
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        text = open(os.path.join(ROOT, "paper_1912_00966_amd", "csrc", name), encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())
        h.update(code.encode())
    return h.hexdigest()


def profiled_traffic(path, key):
    """Bytes per launch measured by the rocprofv3 counter runs recorded in
    `path`, or None when the kernel sources or the launch options (key) differ
    from the profiled ones."""
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        line = line.strip().lstrip("-* ").strip()
        if ":" in line and line.startswith(("traffic_bytes_per_launch", "kernel_source_sha256", "launch_key")):
            k, v = line.split(":", 1)
            fields[k.strip().strip("`")] = v.strip().strip("` ")
    digest = kernel_source_digest()
    if fields.get("kernel_source_sha256") != digest or "traffic_bytes_per_launch" not in fields:
        return None
    if fields.get("launch_key") != key:
        return None
    return int(fields["traffic_bytes_per_launch"])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Threads for the oracle: the cores this process may use, at most 16 (a
    GPU's share of the host's cores on an 8-GPU node)."""
    return max(1, min(len(os.sched_getaffinity(0)), 16))


def _explicit_options(args):
    """True when a launch option was given on the command line."""
    return not (args.layout == "hybrid" and args.table == 0 and args.headers == "auto" and args.window == 0
                and args.tpv == 0 and args.types_per_lane == 0 and args.threads == 0 and args.fcap == 0
                and args.mode == "auto" and args.order == 0)


def _opts(args):
    threads = args.threads or DEFAULT_THREADS.get(args.workload, 1024)
    if args.tpv:
        threads = 1024  # virtual warps run in 1024-thread work-groups
    return {"threads_per_vertex": args.tpv, "types_per_lane": args.types_per_lane,
            "time_window": args.window, "table_cap": args.table, "mode": MODES[args.mode],
            "headers": HEADERS[args.headers], "threads_per_query": threads, "frontier_cap": args.fcap,
            "query_order": args.order}


def calibrate_copy(torch, mib, log):
    """Device-to-device copy of `mib` MiB: a kernel of known traffic (it also
    scales the profiler's byte counters) and the measured copy bandwidth
    (bytes read + written per second, best of three)."""
    n = mib * 2**20 // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    best = None
    for _ in range(3):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    gbs = 2 * n * 4 / (best / 1e3) / 1e9
    log(f"[bench] calibration copy: {mib} MiB read + {mib} MiB written, {gbs:.0f} GB/s")
    del src, dst
    torch.cuda.synchronize()
    return gbs


def build_workload(args, log):
    """(timetables, q_graph, q_src, q_ts, name) of the chosen workload."""
    from paper_1912_00966_amd import synth

    t0 = time.time()
    if args.workload == "mixed":
        tts, qsets = synth.mixed_batch(reading=args.reading)
        qg = np.concatenate([np.full(len(qs), i, np.int32) for i, qs in enumerate(qsets)])
        qs_ = np.concatenate([qs.s for qs in qsets])
        qt = np.concatenate([qs.ts for qs in qsets])
        perm = np.random.default_rng(4).permutation(len(qg))  # interleave the graphs
        qg, qs_, qt = qg[perm], qs_[perm], qt[perm]
        name = f"mixed batch: 8 cities of 2k..500k stops, 512 queries each ({args.reading} reading)"
    else:
        tt, q = synth.workload(args.workload, reading=args.reading)
        tts = [tt]
        qg, qs_, qt = np.zeros(len(q), np.int32), q.s, q.ts
        name = f"{args.workload} ({args.reading} reading)"
    log(f"[bench] {name}: {len(tts)} graphs, sum C={sum(t.n_conn for t in tts)}, Q={len(qg)} "
        f"generated in {time.time() - t0:.1f}s")
    return tts, qg.astype(np.int32), qs_.astype(np.int32), qt.astype(np.int32), name


class Slabs:
    """One device buffer holding a result slab per query (query k's slab holds
    V(graph of k) int32 at a 256-byte aligned offset); the slabs of one graph's
    queries are laid out one after another, in query order."""

    def __init__(self, torch, sizes, group):
        self.sizes = np.asarray(sizes, dtype=np.int64)
        words = (self.sizes + 63) // 64 * 64
        order = np.argsort(np.asarray(group), kind="stable")
        self.off = np.empty(len(words), np.int64)
        self.off[order] = np.concatenate([[0], np.cumsum(words[order])[:-1]])
        self.buf = torch.full((int(words.sum()),), -7, dtype=torch.int32, device="cuda")
        self.views = [self.buf[int(o):int(o) + int(n)] for o, n in zip(self.off, self.sizes)]

    def host(self, ks):
        """Host copies of the slabs of queries ks (one device-to-host copy)."""
        lo = int(min(self.off[k] for k in ks))
        hi = int(max(self.off[k] + self.sizes[k] for k in ks))
        h = self.buf[lo:hi].cpu().numpy()
        return [h[int(self.off[k]) - lo:int(self.off[k] + self.sizes[k]) - lo] for k in ks]


def time_steps(torch, batches, streams, steps, graphs=None):
    """K steps alternating over the streams; returns (wall seconds, per-launch ms)."""
    S = len(batches)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for i in range(steps):
        st = streams[i % S]
        starts[i].record(st)
        if graphs is not None:
            with torch.cuda.stream(st):
                graphs[i % S].replay()
        else:
            batches[i % S].run(st)
        ends[i].record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    return wall, [a.elapsed_time(b) for a, b in zip(starts, ends)]


def run_batched(args, log):
    import torch

    import oracle
    from paper_1912_00966_amd import eat

    copy_gbs = calibrate_copy(torch, args.copy_mib, log)
    tts, qg, qs_, qt, wname = build_workload(args, log)
    layout = eat.EAT_LAYOUT_HYBRID if args.layout == "hybrid" else eat.EAT_LAYOUT_FLAT
    t0 = time.time()
    graphs = [eat.graph_from_timetable(t, layout=layout) for t in tts]
    prep_s = time.time() - t0
    log(f"[bench] preprocess+upload {prep_s:.1f}s, device "
        f"{sum(g.info.device_bytes for g in graphs) / 2**30:.2f} GiB")
    Q = len(qg)
    Vq = np.array([graphs[int(gi)].n_vertices for gi in qg], np.int64)
    S = args.streams or DEFAULT_STREAMS.get(args.workload, 1)
    tuned = None
    if args.no_tune or _explicit_options(args):
        opts = _opts(args)
    else:
        # the library's autotuner picks the launch options for this device,
        # these graphs and this batch size (every candidate's slabs must agree);
        # batches created without options then use its record
        tslab = Slabs(torch, Vq, qg)
        t0 = time.time()
        best, results = eat.eat_batch_tune(graphs, qg, qs_, qt, tslab.views, reps=3, n_streams=S)
        del tslab
        torch.cuda.synchronize()
        tuned = {"best": best, "candidates": [[o["threads_per_query"], o["types_per_lane"], o["threads_per_vertex"],
                                               o["time_window"], o["mode"], o["headers"], o["query_order"],
                                               round(ms, 4)] for o, ms in results],
                 "candidate_fields": ["threads_per_query", "types_per_lane", "threads_per_vertex", "time_window",
                                      "mode", "headers", "query_order", "ms_per_run"],
                 "tune_s": round(time.time() - t0, 2)}
        log(f"[bench] autotuned in {tuned['tune_s']}s: {best}")
        opts = None
    slabs = [Slabs(torch, Vq, qg) for _ in range(S)]
    batches = [eat.Batch(graphs, qg, qs_, qt, sl.views, options=opts) for sl in slabs]
    # the current stream and S - 1 more (with the runtime's 4 hardware queues,
    # streams beyond that share queues)
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(S - 1)]
    # every stream's batch runs at least once before the timed steps (its first
    # run pays one-time costs: the slabs' first touch, the stream's queue)
    for w in range(max(args.warmup, S)):
        batches[w % S].run(streams[w % S])
    torch.cuda.synchronize()
    batches[0].run(streams[0])
    stats = batches[0].wait(stats=True)
    torch.cuda.synchronize()
    if args.dump_stats:
        with open(args.dump_stats, "w") as f:
            json.dump([dict(st, graph=int(qg[i]), s=int(qs_[i]), ts=int(qt[i])) for i, st in enumerate(stats)], f)
    hip_graphs = None
    if args.graph:
        # each stream's batch run captured once into a HIP graph, replayed in the timed steps
        hip_graphs = []
        cap = torch.cuda.Stream()
        for k in range(S):
            gr = torch.cuda.CUDAGraph()
            cap.wait_stream(torch.cuda.current_stream())
            with torch.cuda.graph(gr, stream=cap):
                batches[k].run(cap)
            hip_graphs.append(gr)
        torch.cuda.synchronize()

    # ---- timed region: K batched steps ------------------------------------------------
    wall, launch_ms = time_steps(torch, batches, streams, args.steps, hip_graphs)
    ms_per_step = wall * 1e3 / args.steps
    value = Q / (ms_per_step / 1e3)
    # The same steps on one stream: each launch runs alone, so HIP events on its
    # stream give the kernel's own duration (what a profiler that serializes
    # dispatches reports, and what the roofline divides by).
    one_stream = None
    if S > 1:
        w1, launch_ms = time_steps(torch, batches[:1], streams[:1], args.steps)
        one_stream = round(Q / (w1 / args.steps), 1)
    kernel_ms = float(np.mean(launch_ms))
    log(f"[bench] {value:.0f} queries/s ({ms_per_step:.4f} ms per step on {S} streams), "
        f"launch {kernel_ms:.4f} ms")

    # ---- plain path: one launch per query, one query after another ---------------------
    plain = None
    plain_slabs = None
    if not args.no_plain:
        plain_slabs = Slabs(torch, Vq, qg)
        st0 = streams[0]
        for i in range(min(Q, 8)):
            eat.eat_query(graphs[int(qg[i])], int(qs_[i]), int(qt[i]), plain_slabs.views[i], stream=st0,
                          options=opts)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for i in range(Q):
            eat.eat_query(graphs[int(qg[i])], int(qs_[i]), int(qt[i]), plain_slabs.views[i], stream=st0,
                          options=opts)
        torch.cuda.synchronize()
        p_s = time.perf_counter() - p0
        plain = {"value": round(Q / p_s, 1), "unit": "queries/s", "ms_per_query": round(p_s * 1e3 / Q, 4)}
        log(f"[bench] plain: {plain['value']:.0f} queries/s")

    # ---- CPU oracle on the host, and the check of every answer --------------------------
    cpu = None
    bit_exact = None
    checked = 0
    if not (args.no_cpu and args.no_verify):
        from concurrent.futures import ThreadPoolExecutor
        n_thr = host_threads()
        prep = scan_s = 0.0
        bit_exact = True
        with ThreadPoolExecutor(n_thr) as ex:
            for gi, t in enumerate(tts):
                ks = np.flatnonzero(qg == gi)
                c0 = time.perf_counter()
                csa = oracle.Csa(t.u, t.v, t.t, t.lam, t.n_vertices)
                c1 = time.perf_counter()
                exp = list(ex.map(lambda k: csa.query(int(qs_[k]), int(qt[k])), ks))
                c2 = time.perf_counter()
                prep += c1 - c0
                scan_s += c2 - c1
                csa.close()
                if not args.no_verify:
                    sets = slabs + ([plain_slabs] if plain_slabs is not None else [])
                    for c in range(0, len(ks), 128):
                        chunk = list(ks[c:c + 128])
                        for sl in sets:
                            for k, got in zip(chunk, sl.host(chunk)):
                                ok = np.array_equal(got, exp[int(np.searchsorted(ks, k))])
                                if not ok:
                                    log(f"[bench] MISMATCH query {k} (graph {gi}, s={qs_[k]}, ts={qt[k]})")
                                bit_exact &= bool(ok)
                    checked += len(ks)
                del exp
                log(f"[bench] oracle graph {gi} ({t.n_vertices} stops): {len(ks)} queries, "
                    f"{c2 - c1:.2f}s on {n_thr} threads")
        if not args.no_cpu:
            cpu = {"value": round(Q / scan_s, 2), "unit": "queries/s", "cores": n_thr, "kind": "oracle",
                   "sample": f"every one of the {Q} queries of the timed batch (no sampling): the "
                             f"connection scan, one query per thread at a time over {n_thr} threads, "
                             f"graph after graph; the scan's sort by departure time is excluded",
                   "cpu_model": cpu_model(), "host_cores_visible": os.cpu_count(),
                   "sort_s": round(prep, 2)}
        if args.no_verify:
            bit_exact = None
        else:
            log(f"[bench] verify vs oracle: {checked} queries x {len(slabs)} streams"
                f"{' + plain' if plain_slabs is not None else ''}: {'bit-exact' if bit_exact else 'MISMATCH'}")

    # ---- roofline of the relaxation kernel ---------------------------------------------
    relax_b, fill_b = algorithmic_bytes(stats, Vq)
    achieved = relax_b / (kernel_ms / 1e3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profile_traffic_for(args, batches[0].options()),
                "kernel": "k_relax", "kernel_ms": round(kernel_ms, 4),
                "relax_bytes_per_launch": int(relax_b), "fill_bytes_per_launch": int(fill_b),
                "frac_with_fill": round((relax_b + fill_b) / (kernel_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                "copy_gbs": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                # launches overlap on several streams: relaxation bytes of all steps over the wall time
                "sustained_gbs": round(relax_b / (ms_per_step / 1e3) / 1e9, 1)}

    served = None
    if args.workload == "mixed" and not args.no_serve:
        served = serving_record(args, log, rates=[float(r) for r in args.served_rates.split(",")],
                                requests=args.served_requests, checks=args.served_checks)

    per_q = {k: round(float(np.mean([s[k] for s in stats])), 2) for k in
             ("rounds", "activations", "type_evals", "header_loads", "pool_loads", "improvements",
              "reached", "spilled")}
    per_q["elapsed_us_p50"] = round(float(np.median([s["elapsed_ns"] for s in stats]) / 1e3), 2)
    per_q["elapsed_us_max"] = round(float(np.max([s["elapsed_ns"] for s in stats]) / 1e3), 2)
    out = {
        "metric": "EAT queries/sec & relax-kernel HBM GB/s (% peak), batched vs plain, bit-exact",
        "value": round(value, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": wname, "graphs": [t.n_vertices for t in tts],
                   "connections": int(sum(t.n_conn for t in tts)), "queries_per_step": Q,
                   "layout": args.layout, "mode": args.mode, "streams": S,
                   "threads_per_query": batches[0].options()["threads_per_query"],
                   "launch_options": batches[0].options(), "hip_graph": bool(args.graph),
                   "digests": [t.digest() for t in tts]},
        "bit_exact": bit_exact,
        "checked_answers": checked * (len(slabs) + (1 if plain_slabs is not None else 0)),
        "one_stream": one_stream,
        "plain": plain,
        "batched_vs_plain": round(value / plain["value"], 1) if plain else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "served": served,
        "autotune": tuned,
        "per_query_mean": per_q,
        "preprocess_s": round(prep_s, 3),
    }
    print(json.dumps(out), flush=True)


def serving_record(args, log, rates, requests, checks):
    """Continuous batching over the resident 10k/50k/500k-stop cities at the
    given Poisson rates: sustained queries/s and p50/p99 latency per rate;
    `checks` served answers per graph and rate compared with the oracle (the
    connection scan on the 10k and 50k cities, the certificate on the 500k
    city), and a few with the same query run alone."""
    import torch
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from paper_1912_00966_amd import eat, serve, synth

    native = args.serve_loop == "native"
    t0 = time.time()
    tts = synth.serving_cities(reading=args.reading)
    graphs = [eat.graph_from_timetable(t) for t in tts]
    log(f"[serve] cities {[t.n_vertices for t in tts]} ready in {time.time() - t0:.0f}s")
    sess = eat.Session(graphs, pool_bytes=1 << 30, n_streams=args.served_streams)
    n_thr = host_threads()
    csa = {}
    rows = []
    exact = True
    for rate in rates:
        reqs = serve.poisson_requests(rate, requests, [g.n_vertices for g in graphs], seed=599)
        want = set()
        seen = {gi: 0 for gi in range(len(graphs))}
        for r in reqs[::7]:
            if seen[r.graph] < checks:
                want.add(r.id)
                seen[r.graph] += 1
        # the checked answers are copied on a side stream into buffers made
        # beforehand, so that checking never stalls the serving loop (the
        # session orders a slot's reuse after such a copy)
        side = torch.cuda.Stream()
        bufs = {r.id: torch.empty(graphs[r.graph].n_vertices, dtype=torch.int32, device="cuda")
                for r in reqs if r.id in want}
        torch.cuda.synchronize()
        if native:
            order = sorted(reqs, key=lambda r: r.arrival)
            lat, nrep = sess.serve([r.graph for r in order], [r.s for r in order], [r.ts for r in order],
                                   [r.arrival for r in order], min_batch=64, max_delay_s=50e-6,
                                   copy_dst=[bufs.get(r.id) for r in order], copy_stream=side)
            span = nrep["wall_s"] - (order[0].arrival if order else 0.0)
            rep = serve.ServeReport(n=len(order), wall_s=nrep["wall_s"], qps=len(order) / span,
                                    latency_s=lat, steps=nrep["steps"],
                                    mean_step_queries=nrep["launched"] / max(1, nrep["steps"]),
                                    busy_waits=nrep["busy_waits"])
        else:
            def keep(r, slot):
                if r.id in want:
                    sess.result(slot, out=bufs[r.id], stream=side)

            rep = serve.serve(sess, reqs, on_done=keep, min_batch=64, max_delay_s=50e-6)
        side.synchronize()
        got = {i: b.cpu().numpy() for i, b in bufs.items() if i in want}
        with ThreadPoolExecutor(n_thr) as ex:
            for gi, t in enumerate(tts):
                mine = [reqs[i] for i in sorted(got) if reqs[i].graph == gi]
                if t.n_vertices <= 100_000:
                    if gi not in csa:
                        csa[gi] = oracle.Csa(t.u, t.v, t.t, t.lam, t.n_vertices)
                    exp = list(ex.map(lambda r: csa[gi].query(r.s, r.ts), mine))
                    exact &= all(np.array_equal(got[r.id], e) for r, e in zip(mine, exp))
                else:
                    rc = list(ex.map(lambda r: oracle.certify(t.u, t.v, t.t, t.lam, t.n_vertices, r.s, r.ts,
                                                              got[r.id]), mine))
                    exact &= all(x == 0 for x in rc)
                for r in mine[:4]:
                    exact &= bool(np.array_equal(got[r.id], graphs[gi].query(r.s, r.ts).cpu().numpy()))
        row = {"offered_qps": rate, "sustained_qps": round(rep.qps, 1), "p50_ms": round(rep.percentile_ms(50), 4),
               "p99_ms": round(rep.percentile_ms(99), 4), "requests": rep.n,
               "mean_step_queries": round(rep.mean_step_queries, 2), "checked": len(got)}
        log(f"[serve] {row}")
        rows.append(row)
    sess.free()
    return {"graphs": [t.n_vertices for t in tts], "rates": rows, "bit_exact": bool(exact),
            "streams": args.served_streams, "loop": "eat_session_serve (native)" if native else "serve.py",
            "check": "connection scan on the 10k and 50k cities, certificate on the 500k city, "
                     "a few also against the query alone"}


def run_ablation(args, log):
    """The paper's algorithm ladder on one city (--ablation): mean ms per single
    query of each variant (connection, connection type, connection type with
    progressions, Cluster-AP, edge, warps, ESDG), with the change flag read
    every iteration and every ~sqrt(iterations) (the reduced transfers of
    Section IV-C), the share of connections each examines, the cluster-width
    and virtual-warp sweeps, the production kernel (one launch per query, and
    batched), and the serial connection scan -- every answer checked against
    the oracle.  Prints its own JSON line."""
    import torch

    import oracle
    from paper_1912_00966_amd import eat, synth

    name = args.workload if args.workload != "mixed" else "city-50k"
    tt, q = synth.workload(name, reading=args.reading)
    nq = min(args.ablation_queries, len(q))
    s_, ts_ = q.s[:nq], q.ts[:nq]
    t0 = time.time()
    csa = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices)
    exp = [csa.query(int(s_[i]), int(ts_[i])) for i in range(nq)]
    c0 = time.perf_counter()
    for i in range(nq):
        csa.query(int(s_[i]), int(ts_[i]))
    serial_ms = (time.perf_counter() - c0) * 1e3 / nq
    log(f"[ablation] {name}: {tt.n_conn} connections, {nq} queries, serial scan {serial_ms:.3f} ms/query")
    out = torch.empty(tt.n_vertices, dtype=torch.int32, device="cuda")
    exact = True

    def timed(run):
        """(mean ms per query, last stats); every answer compared."""
        nonlocal exact
        run(0)  # warm-up
        torch.cuda.synchronize()
        a = time.perf_counter()
        st = None
        for i in range(nq):
            st = run(i)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - a) * 1e3 / nq
        for i in range(nq):
            run(i)
            exact &= bool(np.array_equal(out.cpu().numpy(), exp[i]))
        return ms, st

    rows = []
    vg = eat.VariantGraph(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, esdg=True)
    log(f"[ablation] variant arrays built in {time.time() - t0:.0f}s: {vg.info}")
    C = vg.info["n_conn"]
    for v in range(7):
        ws = 32 if v == eat.EAT_VARIANT_WARPS else 0
        # iterations of this variant (for the sqrt check interval) and its work
        its, ex = [], []
        for i in range(nq):
            _, st = vg.query(int(s_[i]), int(ts_[i]), v, out=out, warp_size=ws, count=True)
            its.append(st["iterations"])
            ex.append(st["examined"])
        every_r = max(1, int(round(np.sqrt(np.mean(its)))))
        for every in ((1,) if v == eat.EAT_VARIANT_ESDG else (1, every_r)):
            ms, _ = timed(lambda i: vg.query(int(s_[i]), int(ts_[i]), v, out=out, warp_size=ws,
                                             check_every=every)[1])
            rows.append({"variant": eat.VARIANT_NAMES[v], "warp_size": ws, "check_every": every,
                         "ms_per_query": round(ms, 4), "speedup_vs_serial": round(serial_ms / ms, 2),
                         "iterations_mean": round(float(np.mean(its)), 1),
                         "examined_frac": round(float(np.mean(ex)) / max(C, 1), 5)})
            log(f"[ablation] {rows[-1]}")
    warps = []
    for ws in (1, 2, 4, 8, 16, 32, 64):
        ms, _ = timed(lambda i: vg.query(int(s_[i]), int(ts_[i]), eat.EAT_VARIANT_WARPS, out=out, warp_size=ws)[1])
        warps.append({"warp_size": ws, "ms_per_query": round(ms, 4)})
    log(f"[ablation] virtual warps: {warps}")
    vg.free()
    # the production kernel, one launch per query and batched
    g = eat.graph_from_timetable(tt)
    ms_plain, _ = timed(lambda i: eat.eat_query(g, int(s_[i]), int(ts_[i]), out))
    tpv = []
    for t_ in (0, 1, 4, 16, 64):
        ms, _ = timed(lambda i: eat.eat_query(g, int(s_[i]), int(ts_[i]), out, options={"threads_per_vertex": t_}))
        tpv.append({"threads_per_vertex": t_, "ms_per_query": round(ms, 4)})
    slab = torch.empty((nq, tt.n_vertices), dtype=torch.int32, device="cuda")
    b = eat.Batch([g], np.zeros(nq, np.int32), s_, ts_, [slab[i] for i in range(nq)])
    b.run()
    b.wait()
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(5):
        b.run()
    b.wait()
    batched_qps = 5 * nq / (time.perf_counter() - a)
    exact &= all(np.array_equal(r, e) for r, e in zip(slab.cpu().numpy(), exp))
    # cluster widths (Section IV-B): Cluster-AP variant and the production kernel
    widths = []
    for cw in (3600, 1800, 900, 300):
        vg = eat.VariantGraph(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices, cluster_seconds=cw)
        ms_v, _ = timed(lambda i: vg.query(int(s_[i]), int(ts_[i]), eat.EAT_VARIANT_CLUSTER_AP, out=out)[1])
        vg.free()
        ms_k = None
        if int(tt.t.max()) // cw < 64:  # the hybrid layout's occupancy mask holds 64 clusters
            gw = eat.graph_from_timetable(tt, cluster_seconds=cw)
            ms_k, _ = timed(lambda i: eat.eat_query(gw, int(s_[i]), int(ts_[i]), out))
            gw.free()
        widths.append({"cluster_seconds": cw, "cluster_ap_ms": round(ms_v, 4),
                       "kernel_ms": None if ms_k is None else round(ms_k, 4)})
        log(f"[ablation] width {widths[-1]}")
    # query variants (Section I): goal-directed batches, journeys, profiles
    qv = query_variants_record(tt, s_, ts_, exp, g, out)
    exact &= qv.pop("bit_exact")
    log(f"[ablation] query variants {qv}")
    # sub-trip shortcuts (Sections II-G, IV-B) on a city served by bus lines
    sc = shortcuts_record(log)
    exact &= sc.pop("bit_exact")
    print(json.dumps({"metric": "paper algorithm ladder: ms per EAT query (one query at a time)",
                      "workload": f"{name} ({args.reading} reading)", "queries": nq, "connections": int(C),
                      "serial_scan_ms": round(serial_ms, 4), "variants": rows, "virtual_warps": warps,
                      "kernel": {"ms_per_query": round(ms_plain, 4), "speedup_vs_serial": round(serial_ms / ms_plain, 2),
                                 "threads_per_vertex": tpv, "batched_qps": round(batched_qps, 1)},
                      "cluster_widths": widths, "query_variants": qv, "shortcuts": sc, "bit_exact": bool(exact),
                      "device": torch.cuda.get_device_name()}), flush=True)


def query_variants_record(tt, s_, ts_, exp, g, out):
    """Goal-directed batch (destination: the reached stop of median arrival)
    against the same batch answering every stop; eat_parents and eat_profile
    timings; every result against the oracle."""
    import torch

    import oracle
    from paper_1912_00966_amd import eat

    nq, V = len(s_), tt.n_vertices
    INF = oracle.INF
    d = np.empty(nq, np.int32)
    for i in range(nq):
        r = np.flatnonzero(exp[i] != INF)
        d[i] = r[np.argsort(exp[i][r])[len(r) // 2]]
    slab = torch.empty((nq, V), dtype=torch.int32, device="cuda")
    views = [slab[i] for i in range(nq)]
    rec, exact = {}, True
    for name, kw in (("full", {}), ("goal", {"q_dst": d})):
        b = eat.Batch([g], np.zeros(nq, np.int32), s_, ts_, views, **kw)
        b.run()
        st = b.wait(stats=True)
        got = slab.cpu().numpy()
        if name == "goal":
            exact &= all(got[i][d[i]] == exp[i][d[i]] for i in range(nq))
        else:
            exact &= bool(np.array_equal(got, np.stack(exp)))
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(5):
            b.run()
        b.wait()
        rec[name] = {"qps": round(5 * nq / (time.perf_counter() - a), 1),
                     "rounds_mean": round(float(np.mean([x["rounds"] for x in st])), 2),
                     "type_evals_mean": round(float(np.mean([x["type_evals"] for x in st])), 1)}
        b.free()
    # journeys: parents of one answer
    par = torch.empty((V, 3), dtype=torch.int32, device="cuda")
    eat.eat_query(g, int(s_[0]), int(ts_[0]), out)
    g.parents(int(s_[0]), out, out=par)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(10):
        g.parents(int(s_[0]), out, out=par)
    torch.cuda.synchronize()
    rec["parents_ms"] = round((time.perf_counter() - a) * 100, 4)
    pu, pt, pl = oracle.parents(tt.u, tt.v, tt.t, tt.lam, V, int(s_[0]), out.cpu().numpy())
    exact &= bool(np.array_equal(par.cpu().numpy(), np.stack([pu, pt, pl], 1)))
    # profile of one source over two hours of the morning
    a = time.perf_counter()
    dep, parr = g.profile(int(s_[0]), 6 * 3600, 8 * 3600)
    rec["profile_ms"] = round((time.perf_counter() - a) * 1e3, 3)
    rec["profile_departures"] = int(len(dep))
    csa = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, V)
    dep_o, arr_o = csa.profile(int(s_[0]), 6 * 3600, 8 * 3600)
    exact &= bool(np.array_equal(dep, dep_o) and np.array_equal(parr.cpu().numpy(), arr_o))
    rec["bit_exact"] = bool(exact)
    return rec


def shortcuts_record(log):
    """The 10,000-stop city served by bus lines, 256 queries in one launch,
    without and with sub-trip shortcuts (sqrt of the mean trip length):
    rounds, queries/s, every answer against the oracle on the original
    connections."""
    import torch

    import oracle
    from paper_1912_00966_amd import eat, synth

    tt = synth.lines_city(10_000)
    q = synth.queries(tt.n_vertices, 256, 10601)
    exp = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, tt.n_vertices).query_many(q.s, q.ts)
    slab = torch.empty((len(q), tt.n_vertices), dtype=torch.int32, device="cuda")
    rec, exact = {}, True
    for name, rule in (("plain", None), ("shortcuts", 0)):
        g = eat.graph_from_timetable(tt, subtrip_len=rule)
        b = eat.Batch([g], np.zeros(len(q), np.int32), q.s, q.ts, [slab[i] for i in range(len(q))])
        b.run()
        st = b.wait(stats=True)
        exact &= bool(np.array_equal(slab.cpu().numpy(), exp))
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(10):
            b.run()
        b.wait()
        rec[name] = {"connections": int(g.info.n_conn), "qps": round(10 * len(q) / (time.perf_counter() - a), 1),
                     "rounds_mean": round(float(np.mean([x["rounds"] for x in st])), 2),
                     "rounds_max": int(max(x["rounds"] for x in st))}
        b.free()
        g.free()
    log(f"[ablation] shortcuts {rec}")
    rec["bit_exact"] = bool(exact)
    return rec


def run_serving(args, log):
    """Open-loop serving report over all rates (--serve)."""
    import torch

    from paper_1912_00966_amd import eat  # noqa: F401  (loads the library first)

    rates = [float(r) for r in args.rates.split(",")]
    rec = serving_record(args, log, rates, args.requests, args.serve_checks)
    print(json.dumps({"metric": "served EAT queries/s and latency (Poisson arrivals)", "unit": "queries/s",
                      "device": torch.cuda.get_device_name(), **rec}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="mixed",
                    help="mixed (eight cities, 4,096 queries; default), city-1k, city-50k, region-500k")
    ap.add_argument("--layout", default="hybrid", choices=["hybrid", "flat"])
    ap.add_argument("--reading", default="S", choices=["S", "F"])
    ap.add_argument("--tpv", type=int, default=0, help="threads per active stop (0 = type windows)")
    ap.add_argument("--window", type=int, default=0,
                    help="arrival window of a round in seconds (0 = auto, -1 = none)")
    ap.add_argument("--types-per-lane", type=int, default=0,
                    help="type windows: connection types in flight per lane (0 = auto)")
    ap.add_argument("--table", type=int, default=0,
                    help="on-chip arrival-table slots (0 = auto, -1 = arrivals in HBM only)")
    ap.add_argument("--mode", default="auto", choices=sorted(MODES),
                    help="relaxation schedule: frontier rounds (auto) or topology sweeps")
    ap.add_argument("--headers", default="auto", choices=sorted(HEADERS),
                    help="hybrid layout on the device: header grid (auto when built) or compact headers")
    ap.add_argument("--streams", type=int, default=0,
                    help="streams the timed steps alternate between (each with its own prepared "
                         "batch); 0 = per workload (%s)" % ", ".join(f"{k} {v}" for k, v in DEFAULT_STREAMS.items()))
    ap.add_argument("--threads", type=int, default=0, choices=(0, 256, 384, 512, 768, 1024),
                    help="threads per query (work-group size); 0 = per workload (%s)"
                         % ", ".join(f"{k} {v}" for k, v in DEFAULT_THREADS.items()))
    ap.add_argument("--fcap", type=int, default=0, help="frontier list entries (0 = default)")
    ap.add_argument("--order", type=int, default=0, choices=(0, 1, 2, 3),
                    help="query order of a batch: 0 auto, 1 locality, 2 longest first, 3 banded")
    ap.add_argument("--graph", action="store_true",
                    help="capture each stream's batch run into a HIP graph and replay it in the timed steps")
    ap.add_argument("--copy-mib", type=int, default=1024,
                    help="size of the calibration copy (measured copy bandwidth; scales profiler counters)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-launch-per-query comparison")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner: per-workload default launch options (with no option flags, the "
                         "library's autotuner picks them)")
    ap.add_argument("--no-serve", action="store_true", help="mixed workload: skip the served record")
    ap.add_argument("--served-rates", default="10000,50000", help="served record: Poisson rates (queries/s)")
    ap.add_argument("--served-requests", type=int, default=20000, help="served record: requests per rate")
    ap.add_argument("--serve-loop", default="native", choices=["native", "python"],
                    help="serving: the request loop in native code (eat_session_serve) or serve.py")
    ap.add_argument("--served-streams", type=int, default=4,
                    help="serving: launches in flight at once (session streams)")
    ap.add_argument("--served-checks", type=int, default=64,
                    help="served record: answers per graph and rate checked against the oracle")
    ap.add_argument("--dump-stats", default="", metavar="PATH",
                    help="write the per-query statistics of one launch as JSON")
    ap.add_argument("--serve", action="store_true",
                    help="full serving report: Poisson arrivals over the resident 10k/50k/500k-stop "
                         "cities at every rate of --rates (prints its own JSON line)")
    ap.add_argument("--ablation", action="store_true",
                    help="the paper's algorithm ladder, cluster widths and virtual warps on one city "
                         "(--workload city-1k or city-50k; prints its own JSON line)")
    ap.add_argument("--ablation-queries", type=int, default=64)
    ap.add_argument("--rates", default="1000,2000,5000,10000,20000,50000")
    ap.add_argument("--requests", type=int, default=20000, help="requests per rate (--serve)")
    ap.add_argument("--serve-checks", type=int, default=200,
                    help="--serve: answers per graph and rate checked against the oracle")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: queries are independent, so several GPUs would each "
              "run this same single-GPU batch on their own share of the queries; run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    if args.serve:
        return run_serving(args, log)
    if args.ablation:
        return run_ablation(args, log)
    return run_batched(args, log)


if __name__ == "__main__":
    main()
