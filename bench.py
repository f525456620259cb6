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


def algorithmic_bytes(stats, n_vertices):
    """Bytes the relaxation must move per query, from its operation counts.

    per query      : 4 * V (result slab written with infinity) + 4 (source)
    per activation : 4 (arr[u]) + 8 (vt_off[u], vt_off[u+1])
    per type eval  : 16 (type record) + 4 (arr[v])
    per header     : 8 (cluster header)
    per pool word  : 4
    per improvement: 8 (atomic minimum: read + write of arr[v])
    """
    total = 0
    for st in stats:
        total += 4 * n_vertices + 4
        total += 12 * st["activations"] + 20 * st["type_evals"] + 8 * st["header_loads"]
        total += 4 * st["pool_loads"] + 8 * st["improvements"]
    return total


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="city-50k")
    ap.add_argument("--layout", default="hybrid", choices=["hybrid", "flat"])
    ap.add_argument("--reading", default="S", choices=["S", "F"])
    ap.add_argument("--tpv", type=int, default=0, help="threads per active stop (0 = auto)")
    ap.add_argument("--table", type=int, default=0,
                    help="on-chip arrival-table slots (0 = auto, -1 = arrivals in HBM only)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-launch-per-query comparison")
    ap.add_argument("--no-verify", action="store_true")
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

    if args.calibrate_copy:
        n = args.calibrate_copy * 2**20 // 4
        src = torch.ones(n, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {args.calibrate_copy} MiB read + {args.calibrate_copy} MiB written")
        del src, dst

    V, Q = tt.n_vertices, len(q)
    slab = torch.empty((Q, V), dtype=torch.int32, device=dev)
    opts = {"threads_per_vertex": args.tpv, "table_cap": args.table}
    batch = eat.Batch([g], np.zeros(Q, np.int32), q.s, q.ts, [slab[i] for i in range(Q)], options=opts)
    stream = torch.cuda.current_stream()

    for _ in range(max(args.warmup, 1)):
        batch.run(stream)
    stats = batch.wait(stats=True)
    torch.cuda.synchronize()

    # ---- timed region: K batched steps ------------------------------------------------
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        batch.run(stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    launch_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    ms_per_step = wall * 1e3 / args.steps
    value = Q / (ms_per_step / 1e3)
    kernel_ms = float(np.mean(launch_ms))

    bit_exact = None
    if not args.no_verify:
        import oracle
        got = slab.cpu().numpy()
        exp = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, V).query_many(q.s, q.ts)
        bit_exact = bool(np.array_equal(got, exp))
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
    bytes_per_launch = algorithmic_bytes(stats, V)
    achieved = bytes_per_launch / (kernel_ms / 1e3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_relax", "kernel_ms": round(kernel_ms, 4),
                "algorithmic_bytes_per_launch": int(bytes_per_launch)}

    # ---- CPU oracle on the host ----------------------------------------------------------
    cpu = None
    if not args.no_cpu:
        import oracle
        c = oracle.Csa(tt.u, tt.v, tt.t, tt.lam, V)
        c0 = time.perf_counter()
        c.query_many(q.s, q.ts)
        c_s = time.perf_counter() - c0
        cpu = {"value": round(Q / c_s, 2), "unit": "queries/s", "cores": 1, "kind": "oracle",
               "sample": f"all {Q} queries of the timed batch, connection scan, one thread "
                         f"({os.cpu_count()} host cores visible)"}

    per_q = {k: float(np.mean([s[k] for s in stats])) for k in
             ("rounds", "activations", "type_evals", "header_loads", "pool_loads", "improvements")}
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
                   "graphs": 1, "digest": tt.digest()},
        "bit_exact": bit_exact,
        "plain": plain,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "per_query_mean": per_q,
        "preprocess_s": round(prep_s, 3),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
