"""Benchmark: earliest-arrival-time queries per second on one MI355X.

A step answers one batch of queries (256 random (s, ts) pairs on the 50,000-stop
synthetic city, about 12M connections) with one launch of the batched
relaxation kernel; results land in device-resident int32 slabs.  The batch and
the graph are prepared before the timed region (inputs resident in HBM).

Printed (one JSON line): queries/s of the batched path, the plain path (one
launch per query, queries one after another) beside it, the relaxation
kernel's algorithmic bytes against the HBM roofline, and the CPU oracle
(connection scan) timed on the host.  Every answer of the last timed step is
compared bit-exactly with the oracle.

    python bench.py [--steps K] [--warmup W] [--workload city-50k] [--layout hybrid]
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


def algorithmic_bytes(stats, n_vertices, slab_only=False, grid=False):
    """HBM bytes the relaxation must move per launch, from its operation counts.

    per query      : 4 * V (result slab written with infinity) + 4 * reached
                     (final arrival times scattered from the on-chip table)
    per activation : 8 (the stop's type range, vt_off[u] and vt_off[u+1])
    per type eval  : 16 (type record)
    per header     : 8 (compact cluster header; a second one only when the
                     next cluster is needed), or 12 (header-grid entry: the
                     cluster's header and the next cluster's first departure)
    per pool word  : 4 (array-cluster chunks, flat departures)
    A query whose arrivals live in the slab (table overflow, or no table) also
    moves 4 (arr[u]) per activation, 4 (arr[v]) per type eval and 8 (atomic
    minimum) per improvement.
    """
    total = 0
    for st in stats:
        total += 4 * n_vertices + 8 * st["activations"] + 16 * st["type_evals"]
        total += (12 if grid else 8) * st["header_loads"] + 4 * st["pool_loads"]
        if slab_only or st["spilled"]:
            total += 4 * st["activations"] + 4 * st["type_evals"] + 8 * st["improvements"]
        else:
            total += 4 * st["reached"]
    return total


MODES = {"auto": 0, "topology": 2}  # eat_mode values
# Overlapping consecutive batches pays when a batch is shorter than its slowest
# query (few queries per CU); a batch that fills the chip for its whole launch
# only loses L2 locality to it.  Measured on MI355X.
DEFAULT_STREAMS = {"city-1k": 4, "city-50k": 4, "region-500k": 2, "mixed": 2}
# Threads per query: 768 puts two queries of 12 waves on a CU (more queries in
# flight, the heavy ones still with many waves), 1024 finishes one long query
# sooner and keeps the whole LDS for its table (region-500k).
DEFAULT_THREADS = {"city-1k": 1024, "city-50k": 768, "region-500k": 1024, "mixed": 768}
HEADERS = {"auto": 0, "grid": 1, "compact": 2}  # eat_headers values


def profile_traffic_for(args):
    """HBM bytes per launch from the committed rocprofv3 summary of this
    workload (profiles/k_relax_<workload>[-topology].md), for the default
    launch options only, and only while the kernel source is the profiled one."""
    defaults = (args.layout == "hybrid" and args.table == 0 and args.headers == "auto" and args.window == 0
                and args.tpv == 0 and args.types_per_lane == 0 and args.threads == 0 and args.fcap == 0)
    if not defaults:
        return None
    name = f"k_relax_{args.workload}" + ("-topology" if args.mode == "topology" else "") + ".md"
    return profiled_traffic(os.path.join(ROOT, "profiles", name),
                            os.path.join(ROOT, "paper_1912_00966_amd", "csrc", "kernels.hip"))


def profiled_traffic(path, kernel_source):
    """Bytes per launch measured by the rocprofv3 counter runs recorded in
    `path`, or None when the kernel source changed since they were taken."""
    import hashlib
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        line = line.strip().lstrip("-* ").strip()
        if ":" in line and line.startswith(("traffic_bytes_per_launch", "kernel_source_sha256")):
            k, v = line.split(":", 1)
            fields[k.strip().strip("`")] = v.strip().strip("` ")
    digest = hashlib.sha256(open(kernel_source, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256") != digest or "traffic_bytes_per_launch" not in fields:
        return None
    return int(fields["traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="city-50k",
                    help="city-1k, city-50k, region-500k (one graph), or mixed (eight graphs, 4,096 queries)")
    ap.add_argument("--layout", default="hybrid", choices=["hybrid", "flat"])
    ap.add_argument("--reading", default="S", choices=["S", "F"])
    ap.add_argument("--tpv", type=int, default=0, help="threads per active stop (0 = auto)")
    ap.add_argument("--window", type=int, default=0,
                    help="arrival window of a round in seconds (0 = auto, -1 = none)")
    ap.add_argument("--types-per-lane", type=int, default=0,
                    help="load-balanced expansion: connection types in flight per lane (0 = auto)")
    ap.add_argument("--table", type=int, default=0,
                    help="on-chip arrival-table slots (0 = auto, -1 = arrivals in HBM only)")
    ap.add_argument("--mode", default="auto", choices=sorted(MODES),
                    help="relaxation schedule: frontier rounds (auto) or topology sweeps")
    ap.add_argument("--headers", default="auto", choices=sorted(HEADERS),
                    help="hybrid layout on the device: header grid (auto when built) or compact headers")
    ap.add_argument("--streams", type=int, default=0,
                    help="streams the timed steps alternate between (each with its own prepared "
                         "batch), so one launch's tail overlaps the next launch; 0 = per workload "
                         "(%s)" % ", ".join(f"{k} {v}" for k, v in DEFAULT_STREAMS.items()))
    ap.add_argument("--threads", type=int, default=0, choices=(0, 512, 768, 1024),
                    help="threads per query (work-group size); 0 = per workload (%s)"
                         % ", ".join(f"{k} {v}" for k, v in DEFAULT_THREADS.items()))
    ap.add_argument("--fcap", type=int, default=0, help="frontier list entries (0 = default)")
    ap.add_argument("--graph", action="store_true",
                    help="capture each stream's batch run into a HIP graph and replay it in the timed steps")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-launch-per-query comparison")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--dump-stats", default="", metavar="PATH",
                    help="write the per-query statistics of the last timed launch as JSON")
    ap.add_argument("--serve", action="store_true",
                    help="serving mode: Poisson arrivals over resident 10k/50k/500k-stop cities, "
                         "p50/p99 latency and sustained queries/s per rate (prints its own JSON line)")
    ap.add_argument("--rates", default="1000,2000,5000,10000,20000,50000")
    ap.add_argument("--requests", type=int, default=20000, help="requests per rate (serving mode)")
    ap.add_argument("--serve-sizes", default="10000,50000,500000")
    ap.add_argument("--serve-checks", type=int, default=200,
                    help="serving: answers per rate and graph (<= 100k stops) checked against the oracle")
    ap.add_argument("--serve-certs", type=int, default=8,
                    help="serving: answers per rate and graph (> 100k stops) certified")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the timed region, run one device-to-device copy of MIB MiB "
                         "(a kernel of known traffic, to scale profiler byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: queries are independent, so several GPUs would each "
              "run this same single-GPU batch on their own share of the queries; run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1912_00966_amd import eat, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log = lambda m: print(m, file=sys.stderr, flush=True)
    if args.calibrate_copy:
        n = args.calibrate_copy * 2**20 // 4
        src = torch.ones(n, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {args.calibrate_copy} MiB read + {args.calibrate_copy} MiB written")
        del src, dst
    if args.serve:
        return run_serving(args, log)
    if args.workload == "mixed":
        return run_mixed(args, log)

    t0 = time.time()
    tt, q = synth.workload(args.workload, reading=args.reading)
    log(f"[bench] {tt.name}: V={tt.n_vertices} E={tt.n_edges} C={tt.n_conn} Q={len(q)} "
        f"digest={tt.digest()} ({time.time() - t0:.1f}s)")
    layout = eat.EAT_LAYOUT_HYBRID if args.layout == "hybrid" else eat.EAT_LAYOUT_FLAT
    t0 = time.time()
    g = eat.graph_from_timetable(tt, layout=layout)
    prep_s = time.time() - t0
    info = g.info
    log(f"[bench] preprocess+upload {prep_s:.2f}s: T={info.n_types} K={info.n_headers} "
        f"ap={info.n_ap_clusters} array={info.n_array_clusters} device={info.device_bytes / 2**20:.1f} MiB")

    V, Q = tt.n_vertices, len(q)
    opts = _opts(args)
    grid = args.layout == "hybrid" and args.headers != "compact" and info.n_grid_entries > 0
    # One prepared batch (own result slabs and device counters) per stream:
    # step i runs on stream i % S, so a launch's tail overlaps the next
    # launch's start (the steps are independent batches of the same queries).
    S = args.streams or DEFAULT_STREAMS.get(args.workload, 1)
    slabs = [torch.empty((Q, V), dtype=torch.int32, device=dev) for _ in range(S)]
    batches = [eat.Batch([g], np.zeros(Q, np.int32), q.s, q.ts, [sl[i] for i in range(Q)], options=opts)
               for sl in slabs]
    # the current stream and S - 1 more: with the runtime's 4 hardware queues,
    # 4 new streams besides the current one share queues (1.36M q/s against
    # 2.4M with this set on city-50k)
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(S - 1)]
    slab, batch, stream = slabs[0], batches[0], streams[0]

    for w in range(max(args.warmup, 1)):
        batches[w % S].run(streams[w % S])
    torch.cuda.synchronize()
    batch.run(stream)
    stats = batch.wait(stats=True)
    torch.cuda.synchronize()
    if args.dump_stats:
        with open(args.dump_stats, "w") as f:
            json.dump([dict(st, s=int(q.s[i]), ts=int(q.ts[i])) for i, st in enumerate(stats)], f)

    # With --graph each stream's batch run is captured once into a HIP graph
    # and the timed steps replay the graphs (same kernel, no per-step launch
    # call through the library).
    graphs = None
    if args.graph:
        graphs = []
        cap = torch.cuda.Stream()  # capture needs a stream other than the default one
        for k in range(S):
            gr = torch.cuda.CUDAGraph()
            cap.wait_stream(torch.cuda.current_stream())
            with torch.cuda.graph(gr, stream=cap):
                batches[k].run(cap)
            graphs.append(gr)
        torch.cuda.synchronize()

    # ---- timed region: K batched steps ------------------------------------------------
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for i in range(args.steps):
        st_ = streams[i % S]
        starts[i].record(st_)
        if graphs is not None:
            with torch.cuda.stream(st_):
                graphs[i % S].replay()
        else:
            batches[i % S].run(st_)
        ends[i].record(st_)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_per_step = wall * 1e3 / args.steps
    value = Q / (ms_per_step / 1e3)
    # The same steps on one stream: each launch runs alone, so HIP events on
    # its stream give the kernel's own duration (what the roofline divides by,
    # and what a profiler that serializes dispatches reports).
    one_stream = None
    launch_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    if S > 1:
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for i in range(args.steps):
            starts[i].record(stream)
            batch.run(stream)
            ends[i].record(stream)
        torch.cuda.synchronize()
        one_stream = round(Q / ((time.perf_counter() - w0) / args.steps), 1)
        launch_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    kernel_ms = float(np.mean(launch_ms))

    bit_exact = None
    if not args.no_verify:
        import oracle
        exp = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, V).query_many(q.s, q.ts)
        bit_exact = all(bool(np.array_equal(sl.cpu().numpy(), exp)) for sl in slabs)
        log(f"[bench] verify vs oracle: {'bit-exact' if bit_exact else 'MISMATCH'}")

    # ---- plain path: one launch per query, one query after another ---------------------
    plain = None
    if not args.no_plain:
        for i in range(min(Q, 8)):
            eat.eat_query(g, int(q.s[i]), int(q.ts[i]), slab[i], stream=stream, options=opts)
        torch.cuda.synchronize()
        p0 = time.perf_counter()
        for i in range(Q):
            eat.eat_query(g, int(q.s[i]), int(q.ts[i]), slab[i], stream=stream, options=opts)
        torch.cuda.synchronize()
        p_s = time.perf_counter() - p0
        plain = {"value": Q / p_s, "unit": "queries/s", "ms_per_query": p_s * 1e3 / Q}
        if not args.no_verify:
            plain["bit_exact"] = bool(np.array_equal(slab.cpu().numpy(), exp))

    # ---- roofline of the relaxation kernel ---------------------------------------------
    bytes_per_launch = algorithmic_bytes(stats, V, slab_only=args.table == -1, grid=grid)
    achieved = bytes_per_launch / (kernel_ms / 1e3) / 1e9
    traffic = profile_traffic_for(args)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_relax", "kernel_ms": round(kernel_ms, 4),
                "algorithmic_bytes_per_launch": int(bytes_per_launch),
                # launches overlap on several streams: bytes of all steps over the wall time
                "sustained_gbs": round(bytes_per_launch / (ms_per_step / 1e3) / 1e9, 1)}

    # ---- CPU oracle on the host ----------------------------------------------------------
    cpu = None
    if not args.no_cpu:
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        c = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, V)
        c0 = time.perf_counter()
        c.query_many(q.s, q.ts)
        one_s = time.perf_counter() - c0
        # the same queries spread over the host cores this process may use (each
        # query is one native call that releases the interpreter lock)
        n_thr = max(1, min(len(os.sched_getaffinity(0)), 16))
        with ThreadPoolExecutor(n_thr) as ex:
            c0 = time.perf_counter()
            list(ex.map(lambda i: c.query(q.s[i], q.ts[i]), range(Q)))
            all_s = time.perf_counter() - c0
        cpu = {"value": round(Q / all_s, 2), "unit": "queries/s", "cores": n_thr, "kind": "oracle",
               "sample": f"all {Q} queries of the timed batch, connection scan, one query per "
                         f"thread at a time over {n_thr} threads ({os.cpu_count()} host cores visible)",
               "single_thread": round(Q / one_s, 2)}

    per_q = {k: float(np.mean([s[k] for s in stats])) for k in
             ("rounds", "activations", "type_evals", "header_loads", "pool_loads", "improvements",
              "reached", "spilled")}
    per_q["elapsed_us_p50"] = float(np.median([s["elapsed_ns"] for s in stats]) / 1e3)
    per_q["elapsed_us_max"] = float(np.max([s["elapsed_ns"] for s in stats]) / 1e3)
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
        "config": {"workload": f"{args.workload} ({args.reading} reading)", "stops": V,
                   "connections": tt.n_conn, "queries_per_step": Q, "layout": args.layout,
                   "headers": ("grid" if grid else "compact") if args.layout == "hybrid" else None,
                   "mode": args.mode, "time_window": args.window, "streams": S,
                   "threads_per_query": opts["threads_per_query"], "hip_graph": bool(args.graph),
                   "graphs": 1, "digest": tt.digest()},
        "bit_exact": bit_exact,
        "one_stream": one_stream,
        "plain": plain,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "per_query_mean": per_q,
        "preprocess_s": round(prep_s, 3),
    }
    print(json.dumps(out), flush=True)


def _opts(args):
    threads = args.threads or DEFAULT_THREADS.get(args.workload, 1024)
    if args.tpv:
        threads = 1024  # virtual warps run in 1024-thread work-groups
    return {"threads_per_vertex": args.tpv, "types_per_lane": args.types_per_lane,
            "time_window": args.window, "table_cap": args.table, "mode": MODES[args.mode],
            "headers": HEADERS[args.headers], "threads_per_query": threads, "frontier_cap": args.fcap}


def run_mixed(args, log):
    """Batched mode over eight cities of 2k..500k stops: 4,096 queries (512 per
    graph, interleaved) in one launch, against the same queries as 4,096
    sequential single-query launches."""
    import torch

    import oracle
    from paper_1912_00966_amd import eat, synth

    t0 = time.time()
    tts, qsets = synth.mixed_batch(reading=args.reading)
    graphs = [eat.graph_from_timetable(t) for t in tts]
    log(f"[bench] mixed: {len(tts)} graphs, sum C={sum(t.n_conn for t in tts)} built in {time.time() - t0:.0f}s")
    qg = np.concatenate([np.full(len(qs), i, np.int32) for i, qs in enumerate(qsets)])
    qs_ = np.concatenate([qs.s for qs in qsets])
    qt = np.concatenate([qs.ts for qs in qsets])
    perm = np.random.default_rng(4).permutation(len(qg))
    qg, qs_, qt = qg[perm], qs_[perm], qt[perm]
    Q = len(qg)
    S = args.streams or DEFAULT_STREAMS["mixed"]
    outsets = [[torch.empty(graphs[gi].n_vertices, dtype=torch.int32, device="cuda") for gi in qg]
               for _ in range(S)]
    batches = [eat.Batch(graphs, qg, qs_, qt, o, options=_opts(args)) for o in outsets]
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(S - 1)]
    outs, batch, stream = outsets[0], batches[0], streams[0]
    for w in range(max(args.warmup, 1)):
        batches[w % S].run(streams[w % S])
    torch.cuda.synchronize()
    batch.run(stream)
    stats = batch.wait(stats=True)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    wall0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(streams[i % S])
        batches[i % S].run(streams[i % S])
        ends[i].record(streams[i % S])
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_per_step = wall * 1e3 / args.steps
    launch_ms = [a.elapsed_time(b) for a, b in zip(starts, ends)]
    # the same steps on one stream: each launch alone gives the kernel's own
    # duration (what the roofline divides by, and what a profiler reports)
    one_stream = None
    if S > 1:
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for i in range(args.steps):
            starts[i].record(stream)
            batch.run(stream)
            ends[i].record(stream)
        torch.cuda.synchronize()
        one_stream = round(Q / ((time.perf_counter() - w0) / args.steps), 1)
        launch_ms = [a.elapsed_time(b) for a, b in zip(starts, ends)]
    kernel_ms = float(np.mean(launch_ms))
    # the same queries, one launch each
    plain = None
    if not args.no_plain:
        p0 = time.perf_counter()
        for i in range(Q):
            eat.eat_query(graphs[int(qg[i])], int(qs_[i]), int(qt[i]), outs[i], stream=stream,
                          options=_opts(args))
        torch.cuda.synchronize()
        p_s = time.perf_counter() - p0
        plain = {"value": round(Q / p_s, 1), "unit": "queries/s", "ms_per_query": round(p_s * 1e3 / Q, 4)}
    # checks: every answer on the graphs up to 10k stops against the scan, a
    # sample of the others against the certificate
    checked = certified = 0
    exact = True
    if not args.no_verify:
        csa = {}
        per_graph = {gi: 0 for gi in range(len(graphs))}
        for k in range(Q):
            gi = int(qg[k])
            t = tts[gi]
            if t.n_vertices <= 10_000:
                if gi not in csa:
                    csa[gi] = oracle.Csa(t.u, t.v, t.t, t.lam, t.n_vertices)
                exact &= bool(np.array_equal(outs[k].cpu().numpy(), csa[gi].query(qs_[k], qt[k])))
                checked += 1
            elif per_graph[gi] < 4:
                got = outs[k].cpu().numpy()
                exact &= oracle.certify(t.u, t.v, t.t, t.lam, t.n_vertices, qs_[k], qt[k], got) == 0
                per_graph[gi] += 1
                certified += 1
        log(f"[bench] mixed: {checked} answers vs the scan, {certified} certified: "
            f"{'bit-exact' if exact else 'MISMATCH'}")
    V = {gi: g.n_vertices for gi, g in enumerate(graphs)}
    grid = args.headers != "compact" and all(g.info.n_grid_entries > 0 for g in graphs)
    total = 0
    for k, st in enumerate(stats):
        total += algorithmic_bytes([st], V[int(qg[k])], slab_only=args.table == -1, grid=grid)
    achieved = total / (kernel_ms / 1e3) / 1e9
    out = {
        "metric": "EAT queries/sec, batched (8 graphs, one launch) vs plain",
        "value": round(Q / (ms_per_step / 1e3), 1), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"mixed batch ({args.reading} reading)",
                   "graphs": [t.n_vertices for t in tts], "queries_per_step": Q,
                   "connections": int(sum(t.n_conn for t in tts)), "time_window": args.window,
                   "streams": S, "threads_per_query": _opts(args)["threads_per_query"]},
        "bit_exact": exact if not args.no_verify else None, "one_stream": one_stream, "checked_vs_scan": checked,
        "certified": certified, "plain": plain,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profile_traffic_for(args),
                     "kernel": "k_relax",
                     "kernel_ms": round(kernel_ms, 4), "algorithmic_bytes_per_launch": int(total),
                     "sustained_gbs": round(total / (ms_per_step / 1e3) / 1e9, 1)},
        "per_query_mean": {k: float(np.mean([st[k] for st in stats]))
                           for k in ("rounds", "activations", "type_evals", "reached", "spilled")},
    }
    print(json.dumps(out), flush=True)


def run_serving(args, log):
    """Open-loop serving benchmark: continuous batching over resident graphs."""
    import torch

    import oracle
    from paper_1912_00966_amd import eat, serve, synth

    sizes = [int(x) for x in args.serve_sizes.split(",")]
    tts, graphs = [], []
    for i, n in enumerate(sizes):
        t0 = time.time()
        tt = synth.scaled_city(n, seed=501 + i)
        g = eat.graph_from_timetable(tt)
        log(f"[serve] graph {i}: {tt.name} V={tt.n_vertices} C={tt.n_conn} built in {time.time() - t0:.1f}s")
        tts.append(tt)
        graphs.append(g)
    sess = eat.Session(graphs, pool_bytes=1 << 30, n_streams=2)
    out = {"metric": "served EAT queries/s and latency (Poisson arrivals)", "unit": "queries/s",
           "graphs": [{"stops": t.n_vertices, "connections": t.n_conn} for t in tts], "rates": []}
    csa = {}
    for rate in [float(r) for r in args.rates.split(",")]:
        reqs = serve.poisson_requests(rate, args.requests, [g.n_vertices for g in graphs], seed=599)
        check_ids = set(range(0, len(reqs), max(1, len(reqs) // 32)))
        kept = {}

        def on_done(r, slot):
            if r.id in check_ids:
                kept[r.id] = sess.result(slot).cpu().numpy()

        rep = serve.serve(sess, reqs, on_done=on_done, min_batch=64, max_delay_s=50e-6)
        # spot checks of the timed run: served == alone on the GPU
        ok_alone = all(np.array_equal(kept[i], graphs[reqs[i].graph].query(reqs[i].s, reqs[i].ts).cpu().numpy())
                       for i in kept)
        # checking run (untimed, same arrivals and batching): every result of a
        # sample is copied out as it completes and checked against the oracle --
        # the connection scan on the smaller graphs, the certificate (source,
        # closure, witness) on graphs above 100k stops
        per_graph = {gi: (args.serve_checks if graphs[gi].n_vertices <= 100_000 else args.serve_certs)
                     for gi in range(len(graphs))}
        want, seen = set(), {gi: 0 for gi in per_graph}
        for r in reqs:
            if seen[r.graph] < per_graph[r.graph]:
                want.add(r.id)
                seen[r.graph] += 1
        got = {}

        def keep_all(r, slot):
            if r.id in want:
                got[r.id] = sess.result(slot).cpu().numpy()

        serve.serve(sess, reqs, on_done=keep_all, min_batch=64, max_delay_s=50e-6)
        n_csa = n_cert = 0
        ok_oracle = True
        for i in sorted(got):
            r = reqs[i]
            t = tts[r.graph]
            if graphs[r.graph].n_vertices <= 100_000:
                if r.graph not in csa:
                    csa[r.graph] = oracle.Csa(t.u, t.v, t.t, t.lam, t.n_vertices)
                ok_oracle &= bool(np.array_equal(got[i], csa[r.graph].query(r.s, r.ts)))
                n_csa += 1
            else:
                ok_oracle &= oracle.certify(t.u, t.v, t.t, t.lam, t.n_vertices, r.s, r.ts, got[i]) == 0
                n_cert += 1
        row = {"offered_qps": rate, **rep.as_dict(), "checked_vs_alone": len(kept),
               "bit_exact_vs_alone": bool(ok_alone), "checked_vs_oracle_scan": n_csa,
               "certified": n_cert, "bit_exact_vs_oracle": bool(ok_oracle)}
        log(f"[serve] {row}")
        out["rates"].append(row)
    sess.free()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
