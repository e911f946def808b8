"""Benchmark of one evolving-graph query on one MI355X.

A step is one query of the method over a window of snapshots (intersection and
union bound solves, unstable-vertex compaction, concurrent multi-snapshot
relaxation, writeback of values[V][L]) on a versioned graph already resident
in HBM.  Default workload: R-MAT scale 20 (1,048,576 vertices, 16,777,216
samples, weights uniform [1, 100]), 64 snapshots made by batches of 10k
deletions + 10k additions, SSSP from a seeded source with base out-degree > 0,
window [0, 64).

value = effective snapshot-edge rate = sum over the window's snapshots of
their edge counts / seconds per query (the same numerator for every method,
so work avoided is not counted as work done).

Prints one JSON line.  Options: --steps K --warmup W --gpus 1 --algo sssp
--config mid --no-cpu-baseline --no-roofline --no-plain --no-heavy.  Besides
the dominant kernel's roofline, the line reports the relaxer's on the headline
workload and on the same graph with 100k + 100k updates per snapshot, where
about half the vertices are unstable and the relaxation dominates.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def snapshot_edge_counts(ex, K):
    """Edges per snapshot from the versioned graph's masks."""
    m = ex["mask"]
    counts = np.zeros(K, dtype=np.int64)
    for t in range(K):
        w, b = divmod(t, 64)
        counts[t] = int(((m[:, w] >> np.uint64(b)) & np.uint64(1)).sum())
    return counts


def counter_traffic(kernel, workload):
    """HBM traffic per dispatch of `kernel` on `workload` ("<config> <algo> window [b,e)") from the committed
    rocprofv3 counter summaries, or (None, reason) when there is none or the kernel's sources changed since
    the counters were taken."""
    import glob
    import hashlib
    import re
    for path in glob.glob(os.path.join(ROOT, "profiles", "counters_*.md")):
        m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
        if not m:
            continue
        blk = json.loads(m.group(1))
        if blk.get("timing_name") != kernel or blk.get("workload") != workload:
            continue
        h = hashlib.sha256()
        for f in blk["sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
        if h.hexdigest() != blk["sources_sha256"]:
            return None, f"{os.path.basename(path)}: kernel sources changed since the counters were taken"
        return blk["traffic_bytes_per_dispatch"], os.path.basename(path)
    return None, "no counter summary for this kernel"


def algorithmic_bytes(kernel, st, L, V):
    """Bytes a kernel's work must move at minimum, from the query's counters.

    Bound-solve expansion: per edge visit the edge's (col, w) pair and one
    4-byte value read; per improving update one 4-byte atomic write; per
    frontier vertex its 16-byte item (edge offset, row position, vertex) and
    its value.  A pull iteration visits every all-present in-edge (source,
    weight, the source's value: the same 12 bytes) and writes each improved
    vertex once.  Relaxer: per edge visit one record (dst, w, lane mask), per
    (edge, snapshot) evaluation one 4-byte destination read.  Writeback: the
    V x L output, two 4-byte reads per vertex and the unstable rows.
    """
    if kernel == "solve_expand_cap_all":
        return 12 * st["edges_cap"] + 4 * st["updates_cap"] + 16 * st["items_cap"]
    if kernel == "solve_expand_cap":
        return 12 * st["edges_cap"] + 4 * st["updates_cap"] + 20 * st["items_cap"]
    if kernel == "solve_expand_cup":
        return 12 * st["edges_cup"] + 4 * st["updates_cup"] + 20 * st["items_cup"]
    if kernel == "relax":
        rec = 16 if L <= 64 else 24
        return rec * st["edge_visits_relax"] + 4 * st["lane_relaxations"]
    if kernel == "writeback":
        return 4 * V * L + 8 * V + 4 * L * st["n_unstable"]
    return None


def percentiles(x):
    x = np.asarray(x, dtype=np.float64)
    return {"p50": float(np.percentile(x, 50)), "p90": float(np.percentile(x, 90)),
            "p99": float(np.percentile(x, 99)), "max": float(x.max()), "mean": float(x.mean())}


def bench_served(args):
    """Serving: R-MAT scale 24 ring of 128 snapshots, one append of 100k + 100k updates per second, Poisson
    arrivals at each rate of --qps for --duration seconds; every query takes the newest len snapshots, len uniform
    in [16, 128], algorithm uniform over the four, source random with base out-degree > 0.  The same arrival trace
    and the same appends are replayed against the continuous-batching server and the plain one-at-a-time server,
    each on a freshly built graph.  Latency = arrival to compact result complete on the device."""
    import threading

    import torch

    import paper_2502_10579_amd as evq
    import synth

    torch.cuda.set_device(0)
    K = 128
    qps_list = [float(x) for x in args.qps.split(",")]
    T = args.duration
    n_app = int(T) + 1
    t0 = time.time()
    inst = synth.rmat_instance(seed=args.seed, **dict(synth.CONFIGS["served"], K=K + n_app))
    log(f"[served] generated: base {len(inst.base)} edges, {K + n_app} batches ({time.time() - t0:.1f}s)")
    V = inst.num_vertices
    src_pool = synth.pick_sources(inst, 4096, seed=args.seed)
    levels = []
    for qps in qps_list:
        rng = np.random.default_rng(int(qps * 1000) + args.seed)
        arr = np.cumsum(rng.exponential(1.0 / qps, size=int(qps * T * 2) + 16))
        arr = arr[arr < T]
        qs = [(int(rng.integers(0, 4)), int(src_pool[int(rng.integers(0, len(src_pool)))]), int(rng.integers(16, 129)))
              for _ in range(len(arr))]
        lev = {"qps": qps, "queries": len(qs)}
        for mode in ("batch", "plain"):
            g = evq.Graph(V, inst.base, inst.dels[:K], inst.adds[:K])
            with evq.Server(g, mode=mode, max_groups=args.max_groups, max_batch=args.max_batch,
                            queue_hi=args.queue_hi) as srv:
                # warm-up: the worker pool's buffers and the kernels' first launches
                for i in range(16):
                    srv.submit(i % 4, int(src_pool[i]), 128)
                got = 0
                while got < 16:
                    for c in srv.poll(64, 1000):
                        got += 1
                        if c["result"] is not None:
                            c["result"].free()
                torch.cuda.synchronize()
                app_ms = []
                start = time.perf_counter()

                def appender():
                    for k in range(0 if args.no_appends else n_app - 1):
                        dt = start + (k + 1) * 1.0 - time.perf_counter()
                        if dt > 0:
                            time.sleep(dt)
                        ta = time.perf_counter()
                        g.append(inst.dels[K + k], inst.adds[K + k])
                        app_ms.append((time.perf_counter() - ta) * 1000.0)

                def submitter():
                    for t_arr, (a, s_, L) in zip(arr, qs):
                        dt = start + t_arr - time.perf_counter()
                        if dt > 0:
                            time.sleep(dt)
                        srv.submit(a, s_, L)

                th = [threading.Thread(target=appender), threading.Thread(target=submitter)]
                for t in th:
                    t.start()
                comps = []
                while len(comps) < len(qs):
                    for c in srv.poll(256, 50):
                        comps.append({k: c[k] for k in ("t_arrival_ms", "t_admit_ms", "t_bounds_ms", "t_done_ms",
                                                        "status", "group_size")})
                        if c["result"] is not None:
                            c["result"].free()
                for t in th:
                    t.join()
                torch.cuda.synchronize()
            g.close()
            lat = [c["t_done_ms"] - c["t_arrival_ms"] for c in comps]
            wait = [c["t_admit_ms"] - c["t_arrival_ms"] for c in comps]
            span = (max(c["t_done_ms"] for c in comps) - min(c["t_arrival_ms"] for c in comps)) / 1000.0
            bnd = [c["t_bounds_ms"] - c["t_admit_ms"] for c in comps]
            tail = [c["t_done_ms"] - c["t_bounds_ms"] for c in comps]
            lev[mode] = {"latency_ms": percentiles(lat), "admission_wait_ms": percentiles(wait),
                         "bounds_ms": percentiles(bnd), "after_bounds_ms": percentiles(tail),
                         "mean_group_size": float(np.mean([c["group_size"] for c in comps])),
                         "completed_per_s": len(comps) / span, "failed": sum(1 for c in comps if c["status"]),
                         "append_ms": percentiles(app_ms) if app_ms else None}
            log(f"[served] qps {qps:g} {mode}: {len(comps)} queries, p50 {lev[mode]['latency_ms']['p50']:.1f} ms, "
                f"p99 {lev[mode]['latency_ms']['p99']:.1f} ms, {lev[mode]['completed_per_s']:.1f}/s, "
                f"wait p50 {lev[mode]['admission_wait_ms']['p50']:.1f}, bounds p50 {lev[mode]['bounds_ms']['p50']:.1f}, "
                f"after p50 {lev[mode]['after_bounds_ms']['p50']:.1f} ms, group {lev[mode]['mean_group_size']:.1f}, "
                f"appends {lev[mode]['append_ms']['p50'] if app_ms else 0:.0f} ms")
        levels.append(lev)
    top = levels[-1]
    res = {
        "metric": "served query latency p99 (ms)",
        "value": top["batch"]["latency_ms"]["p99"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": sum(l["queries"] for l in levels),
        "warmup": 16,
        "ms_per_step": top["batch"]["latency_ms"]["mean"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"served: R-MAT scale 24 ({V} vertices, {inst.meta['n_samples']} samples, "
                               f"w in [1,100]), ring of {K} snapshots of 100k+100k updates, 1 append/s, "
                               f"Poisson arrivals {args.qps} q/s for {T:g} s, newest len in [16,128], "
                               f"algorithm uniform over 4"},
        "levels": levels,
    }
    print(json.dumps(res), flush=True)


def bench_sweep(args):
    """Sensitivity (the paper's Fig. 12 analogue): R-MAT scale 20 (16,777,216 samples, w in [1,100]), SSSP
    from a seeded source over the whole window, with K = 32 / 64 / 128 snapshots of 10k+10k updates and, at
    K = 64, batches of 5k / 25k / 50k / 100k updates of each kind (0.03% - 0.6% of the edges per snapshot).
    Per point: |U|, reduced-subgraph edges, and the method against the plain concurrent and the sequential
    per-snapshot evaluations (all three checked equal on the device)."""
    import torch

    import paper_2502_10579_amd as evq
    import synth

    torch.cuda.set_device(0)
    points = [(32, 10000), (64, 10000), (128, 10000), (64, 5000), (64, 25000), (64, 50000), (64, 100000)]
    rows = []
    for K, nb in points:
        inst = synth.rmat_instance(20, 16777216, K, nb, nb, 1, 100, seed=args.seed)
        src = synth.pick_sources(inst, 1, seed=args.seed)[0]
        g = evq.Graph.from_instance(inst)
        ex = g.export()
        snap_edges = int(snapshot_edge_counts(ex, K).sum())
        del ex
        out = torch.empty((inst.num_vertices, K), dtype=torch.int32, device="cuda")
        ref = torch.empty_like(out)
        res = {}
        for name, fn in (("method", g.query), ("plain", g.query_plain), ("sequential", g.query_sequential)):
            # warm-up (the method's second full-window query builds the reverse CSR of the pull step)
            for _ in range(2 if name == "method" else 1):
                fn(0, src, 0, K, out=out if name == "method" else ref)
            torch.cuda.synchronize()
            reps = 5 if name == "method" else 2
            t = time.perf_counter()
            for _ in range(reps):
                fn(0, src, 0, K, out=out if name == "method" else ref)
            torch.cuda.synchronize()
            res[name] = (time.perf_counter() - t) * 1000.0 / reps
            if name != "method":
                res[name + "_identical"] = bool(torch.equal(out, ref))
        # the same query with sub-window splitting on (more than 35% unstable: two halves, recursively)
        with evq.tuning(split_frac=0.35):
            g.query(0, src, 0, K, out=ref)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(3):
                g.query(0, src, 0, K, out=ref)
            torch.cuda.synchronize()
            res["split"] = (time.perf_counter() - t) * 1000.0 / 3
            _, st = g.query(0, src, 0, K, out=ref, stats=True)
        res["split_identical"] = bool(torch.equal(out, ref))
        _, st0 = g.query(0, src, 0, K, out=out, stats=True)
        row = {"K": K, "batch": nb, "union_edges": g.info["num_edges"], "n_unstable": st0["n_unstable"],
               "unstable_frac": st0["n_unstable"] / inst.num_vertices, "reduced_edges": st0["n_relax_edges"],
               "seed_edges": st0["n_seed_edges"], "subwindows": st["subwindows"],
               "unstable_after_split": st["n_unstable"], "method_ms": round(res["method"], 3),
               "method_split_ms": round(res["split"], 3),
               "plain_ms": round(res["plain"], 3), "sequential_ms": round(res["sequential"], 3),
               "speedup_vs_plain": round(res["plain"] / res["method"], 2),
               "speedup_vs_sequential": round(res["sequential"] / res["method"], 2),
               "identical": res["plain_identical"] and res["sequential_identical"] and res["split_identical"],
               "snapshot_edges_per_s": snap_edges / (res["method"] / 1000.0)}
        log(f"[sweep] {json.dumps(row)}")
        rows.append(row)
        g.close()
        del out, ref
    res = {
        "metric": "snapshot-edge relaxations/s",
        "value": rows[1]["snapshot_edges_per_s"],
        "unit": "snapshot-edges/s",
        "n_gpus": 1,
        "steps": 5,
        "warmup": 1,
        "ms_per_step": rows[1]["method_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "sensitivity: R-MAT scale 20 (16777216 samples, w in [1,100]), SSSP over the "
                               "whole window; K in {32,64,128} at 10k+10k updates, batch in {5k,25k,50k,100k} "
                               "at K=64"},
        "points": rows,
    }
    print(json.dumps(res), flush=True)


def bench_batched(args):
    """Batching: R-MAT scale 22, K = 128 snapshots of 20k + 20k updates, 256 queries (algorithm uniform over the
    four, source random with base out-degree > 0, start uniform in [0, 100], length uniform in [25, 100] clamped
    to the last snapshot) answered by one evq_query_batch call, against the same queries one at a time."""
    import torch

    import paper_2502_10579_amd as evq
    import synth

    torch.cuda.set_device(0)
    t0 = time.time()
    inst = synth.config_instance("batched", seed=args.seed)
    qs = synth.batch_queries(inst, 256, seed=args.seed)
    log(f"[batched] generated ({time.time() - t0:.1f}s)")
    g = evq.Graph.from_instance(inst)
    ex = g.export()
    counts = snapshot_edge_counts(ex, inst.K)
    del ex
    snap_edges = int(sum(counts[b:b + L].sum() for (_, _, b, L) in qs))
    V = inst.num_vertices
    out = torch.empty(V * 128, dtype=torch.int32, device="cuda")
    for (a, s_, b, L) in qs[:8]:
        g.query(a, s_, b, L, out=out[:V * L].view(V, L))
    for _ in range(2):  # full-window warm-up: the second builds the reverse CSR of the pull step
        g.query(qs[0][0], qs[0][1], 0, inst.K, out=out[:V * inst.K].view(V, inst.K))
    torch.cuda.synchronize()
    t = time.perf_counter()
    for (a, s_, b, L) in qs:
        g.query(a, s_, b, L, out=out[:V * L].view(V, L))
    torch.cuda.synchronize()
    one_ms = (time.perf_counter() - t) * 1000.0
    log(f"[batched] one at a time: {one_ms:.1f} ms for {len(qs)} queries")
    if args.no_autotune:
        cfg, tune_ms = evq.batch_config(), None
    else:
        cfg, tune_ms = g.autotune_batch(qs)
    log(f"[batched] execution choices: {cfg} (autotune best {tune_ms} ms)")
    rows = {}
    for lanes in (1, 2):
        evq.set_batch_config(lanes=lanes, chunk=cfg["chunk"], blocks=cfg["blocks"])
        for r in g.query_batch(qs):
            r.free()
        torch.cuda.synchronize()
        best = None
        for _ in range(max(1, args.steps)):
            t = time.perf_counter()
            res = g.query_batch(qs)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t) * 1000.0
            best = ms if best is None else min(best, ms)
            for r in res:
                r.free()
        rows[lanes] = best
        log(f"[batched] batch lanes={lanes}: {best:.1f} ms for {len(qs)} queries")
    evq.set_batch_config(**cfg)
    ms = min(rows[1], rows[2])
    res = {
        "metric": "snapshot-edge relaxations/s",
        "value": snap_edges / (ms / 1000.0),
        "unit": "snapshot-edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "batched: R-MAT scale 22 (4194304 vertices, 67108864 samples, w in [1,100]), "
                               "K=128 snapshots of 20k+20k updates, 256 queries (algorithm uniform, start in "
                               "[0,100], length in [25,100] clamped), compact results"},
        "queries_per_s": len(qs) / (ms / 1000.0),
        "batch_config": cfg,
        "batch_ms": ms,
        "batch_shared_solves_ms": rows[1],
        "batch_one_solve_per_query_ms": rows[2],
        "one_at_a_time_ms": one_ms,
        "speedup_vs_one_at_a_time": one_ms / ms,
    }
    g.close()
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="mid")
    ap.add_argument("--algo", default="sssp")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-heavy", action="store_true", help="mid: skip the heavy-churn relaxer leg")
    ap.add_argument("--no-autotune", action="store_true", help="batched: keep the current execution choices")
    ap.add_argument("--qps", default="4,16,64", help="served: arrival rates")
    ap.add_argument("--duration", type=float, default=6.0, help="served: seconds of arrivals per rate")
    ap.add_argument("--max-groups", type=int, default=0, help="served: group solves at once (0: server default)")
    ap.add_argument("--queue-hi", type=int, default=0,
                    help="served: waiting queries from which groups start beside running ones (0: server default)")
    ap.add_argument("--max-batch", type=int, default=0, help="served: queries per group (0: server default)")
    ap.add_argument("--no-appends", action="store_true", help="served: no appends during the run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (this build has no "
              f"multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    if args.config == "served":
        return bench_served(args)
    if args.config == "batched":
        return bench_batched(args)
    if args.config == "sweep":
        return bench_sweep(args)

    import torch

    import paper_2502_10579_amd as evq
    import synth

    torch.cuda.set_device(0)
    t0 = time.time()
    inst = synth.config_instance(args.config, seed=args.seed)
    log(f"[bench] generated {args.config}: base {len(inst.base)} edges, K={inst.K} ({time.time() - t0:.1f}s)")
    source = synth.pick_sources(inst, 1, seed=args.seed)[0]
    K = inst.K
    b, L = 0, K
    algo = evq.ALGOS[args.algo]

    g = evq.Graph.from_instance(inst)
    info = g.info
    log(f"[bench] built versioned graph: {info['num_edges']} edges ({info['num_partial']} partial), "
        f"{info['build_ms']:.1f} ms")
    ex = g.export()
    counts = snapshot_edge_counts(ex, K)
    snap_edges = int(counts[b:b + L].sum())
    del ex

    out = torch.empty((inst.num_vertices, L), dtype=torch.int32, device="cuda")
    for _ in range(args.warmup):
        g.query(algo, source, b, L, out=out)
    torch.cuda.synchronize()
    # every query bracketed by HIP events on the stream it runs on (torch's current stream, which the
    # binding passes to the library): per-query device time, median and p99 beside the wall-clock mean
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t = time.perf_counter()
    for e0, e1 in evs:
        e0.record()
        g.query(algo, source, b, L, out=out)
        e1.record()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1000.0 / args.steps
    ev_ms = [e0.elapsed_time(e1) for e0, e1 in evs]
    q_ev = {"p50": float(np.median(ev_ms)), "p99": float(np.percentile(ev_ms, 99)), "mean": float(np.mean(ev_ms)),
            "min": float(np.min(ev_ms))}
    log(f"[bench] method: {ms:.3f} ms/query over {args.steps} steps (wall); HIP events p50 {q_ev['p50']:.3f} "
        f"p99 {q_ev['p99']:.3f} ms")

    # The paper's Fig. 11 split: QRS generation (both bound solves, then the unstable set and the reduced
    # subgraph) against the whole query.  The bound solves alone (evq_query_bounds, uninstrumented, HIP events)
    # give its lower part; the kernel-time share below adds the reduction kernels.
    rc_buf = torch.empty(inst.num_vertices, dtype=torch.int32, device="cuda")
    ru_buf = torch.empty_like(rc_buf)
    bev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for e0, e1 in bev:
        e0.record()
        evq._check(evq.lib.evq_query_bounds(g._h, algo, source, b, L, evq._ptr(rc_buf), evq._ptr(ru_buf),
                                            evq._stream(None)))
        e1.record()
    torch.cuda.synchronize()
    bounds_ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in bev]))
    del rc_buf, ru_buf

    _, st = g.query(algo, source, b, L, out=out, stats=True)
    log(f"[bench] stats: {json.dumps({k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()})}")

    plain_ms = None
    seq_ms = None
    push_ms = None
    if not args.no_plain:
        outp = torch.empty_like(out)
        g.query_plain(algo, source, b, L, out=outp)
        torch.cuda.synchronize()
        t = time.perf_counter()
        n_plain = max(1, min(args.steps, 5))
        for _ in range(n_plain):
            g.query_plain(algo, source, b, L, out=outp)
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - t) * 1000.0 / n_plain
        same = bool(torch.equal(out, outp))
        log(f"[bench] plain concurrent evaluation: {plain_ms:.3f} ms/query, identical={same}")
        g.query_sequential(algo, source, b, L, out=outp)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n_plain):
            g.query_sequential(algo, source, b, L, out=outp)
        torch.cuda.synchronize()
        seq_ms = (time.perf_counter() - t) * 1000.0 / n_plain
        same_seq = bool(torch.equal(out, outp))
        log(f"[bench] sequential per-snapshot evaluation: {seq_ms:.3f} ms/query, identical={same_seq}")
        # the method with its pull step off (pushes only), against which the plain evaluation, whose kernel
        # has no pull step, compares on the analysis alone
        with evq.tuning(pull_frac=2.0):
            g.query(algo, source, b, L, out=outp)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(n_plain):
                g.query(algo, source, b, L, out=outp)
            torch.cuda.synchronize()
            push_ms = (time.perf_counter() - t) * 1000.0 / n_plain
        log(f"[bench] method without its pull step: {push_ms:.3f} ms/query, identical={bool(torch.equal(out, outp))}")

    # batching leg on the same graph: 64 mixed queries of the batched recipe (algorithm uniform, random
    # source, start in [0, K - 25], length in [25, K] clamped), one call against one at a time
    batch_leg = None
    if not args.no_plain:
        bq = synth.batch_queries(inst, 64, seed=args.seed, start_max=K - 25, len_min=25, len_max=K)
        V = inst.num_vertices
        buf = torch.empty(V * K, dtype=torch.int32, device="cuda")
        for (a, s_, b_, L_) in bq[:4]:
            g.query(a, s_, b_, L_, out=buf[:V * L_].view(V, L_))
        for r in g.query_batch(bq):
            r.free()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for (a, s_, b_, L_) in bq:
            g.query(a, s_, b_, L_, out=buf[:V * L_].view(V, L_))
        torch.cuda.synchronize()
        one_ms = (time.perf_counter() - t) * 1000.0
        t = time.perf_counter()
        res_b = g.query_batch(bq)
        torch.cuda.synchronize()
        bat_ms = (time.perf_counter() - t) * 1000.0
        for r in res_b:
            r.free()
        del buf
        batch_leg = {"queries": len(bq), "batch_ms": round(bat_ms, 3), "one_at_a_time_ms": round(one_ms, 3),
                     "speedup": round(one_ms / bat_ms, 3), "config": evq.batch_config()}
        log(f"[bench] batch of {len(bq)} mixed queries: {bat_ms:.1f} ms vs one at a time {one_ms:.1f} ms")

    roof = None
    relax_roof = None
    kernels = None
    if not args.no_roofline:
        evq.timing_reset()
        evq.timing_enable(True)
        reps = 3
        for _ in range(reps):
            g.query(algo, source, b, L, out=out)
        torch.cuda.synchronize()
        kernels = evq.timing_report()
        evq.timing_enable(False)
        evq.timing_reset()
        log("[bench] kernel times per query: " +
            ", ".join(f"{k}={v[1] / reps:.3f}ms/{v[0] // reps}" for k, v in sorted(kernels.items(),
                                                                                 key=lambda kv: -kv[1][1])))
        dom, (launches, tot_ms) = max(kernels.items(), key=lambda kv: kv[1][1])
        byts = algorithmic_bytes(dom, st, L, inst.num_vertices)
        if byts is not None:
            ach = byts * reps / (tot_ms / 1000.0) / 1e9
            avg_us = tot_ms * 1000.0 / launches
            traffic, tsrc = counter_traffic(dom, f"{args.config} {args.algo} window [{b},{b + L})")
            roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": traffic,
                    "avg_launch_us": round(avg_us, 3), "launches_per_query": launches // reps,
                    "algorithmic_bytes_per_query": int(byts),
                    "algorithmic_bytes_per_launch": int(byts * reps / launches), "traffic_source": tsrc}
            if traffic:
                roof["traffic_GBps"] = round(traffic / (avg_us * 1e-6) / 1e9, 2)
                roof["traffic_frac"] = round(traffic / (avg_us * 1e-6) / 1e9 / PEAK_HBM_GBS, 4)
            if dom == "solve_expand_cap_all":
                # visits per edge of the window's intersection graph (over the whole window: the all-present
                # edges), and the rate against one visit per such edge, the bound solve's lower bound
                e_cap = info["num_edges"] - info["num_partial"]
                lb = 12 * e_cap
                roof["visits_per_intersection_edge"] = round(st["edges_cap"] / max(e_cap, 1), 3)
                roof["one_visit_lower_bound"] = {"bytes_per_query": lb,
                                                 "achieved": round(lb * reps / (tot_ms / 1000.0) / 1e9, 2),
                                                 "frac": round(lb * reps / (tot_ms / 1000.0) / 1e9 / PEAK_HBM_GBS, 4)}
            if dom.startswith("solve_expand_"):
                # the expansion's edge-visit rate against the same per-edge
                # memory operations alone over this graph's edges
                visits = st["edges_cup"] if dom == "solve_expand_cup" else st["edges_cap"]
                rate = visits * reps / (tot_ms / 1000.0)
                ceil = g.gather_ceiling(5)
                roof["access_ceiling"] = {"kernel": "gather_ceiling", "edges_per_s": round(ceil, 0),
                                          "expansion_edges_per_s": round(rate, 0),
                                          "frac": round(rate / ceil, 4) if ceil else None}
                log(f"[bench] {dom}: {rate / 1e9:.1f} G edge visits/s; gather ceiling {ceil / 1e9:.1f} G edges/s")
        relax_b = algorithmic_bytes("relax", st, L, inst.num_vertices)
        if "relax" in kernels and relax_b:
            rl, rt = kernels["relax"]
            roof_relax = relax_b * reps / (rt / 1000.0) / 1e9
            relax_roof = {"kernel": "relax", "achieved": round(roof_relax, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                          "frac": round(roof_relax / PEAK_HBM_GBS, 4), "launches_per_query": rl // reps,
                          "avg_launch_us": round(rt * 1000.0 / rl, 3), "algorithmic_bytes_per_query": int(relax_b)}
            log(f"[bench] relaxer: {roof_relax:.1f} GB/s algorithmic over {rl // reps} launches/query")

    # The relaxer at a size where it dominates: the mid graph with 100k + 100k
    # updates per snapshot (about half the vertices unstable), same source and
    # window; on the headline workload the relaxation is a few small launches.
    relax_heavy = None
    if not args.no_roofline and not args.no_heavy and args.config == "mid":
        hv = synth.config_instance("churn", seed=args.seed)
        gh = evq.Graph.from_instance(hv)
        hsrc = synth.pick_sources(hv, 1, seed=args.seed)[0]
        hout = torch.empty_like(out)
        for _ in range(2):  # warm-up (the second full-window query builds the reverse CSR of the pull step)
            gh.query(algo, hsrc, 0, hv.K, out=hout)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            gh.query(algo, hsrc, 0, hv.K, out=hout)
        torch.cuda.synchronize()
        hms = (time.perf_counter() - t) * 1000.0 / 3
        _, hst = gh.query(algo, hsrc, 0, hv.K, out=hout, stats=True)
        evq.timing_reset()
        evq.timing_enable(True)
        for _ in range(3):
            gh.query(algo, hsrc, 0, hv.K, out=hout)
        torch.cuda.synchronize()
        hk = evq.timing_report()
        evq.timing_enable(False)
        evq.timing_reset()
        gh.close()
        del hout
        rl, rt = hk["relax"]
        hb = algorithmic_bytes("relax", hst, hv.K, hv.num_vertices)
        ach = hb * 3 / (rt / 1000.0) / 1e9
        relax_heavy = {"kernel": "relax", "achieved": round(ach, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                       "frac": round(ach / PEAK_HBM_GBS, 4), "launches_per_query": rl // 3,
                       "avg_launch_us": round(rt * 1000.0 / rl, 3), "algorithmic_bytes_per_query": int(hb),
                       "relax_ms_per_query": round(rt / 3, 3), "query_ms": round(hms, 3),
                       "unstable_frac": round(hst["n_unstable"] / hv.num_vertices, 3),
                       "lane_relaxations": hst["lane_relaxations"],
                       "workload": f"mid graph, K={hv.K} snapshots of 100000+100000 updates, {args.algo.upper()} "
                                   f"from vertex {hsrc}, window [0,{hv.K})"}
        # counted HBM traffic of the relaxation kernel on this workload (committed counter summary)
        htraffic, htsrc = counter_traffic("relax", f"churn {args.algo} window [0,{hv.K})")
        relax_heavy["traffic"] = htraffic
        relax_heavy["traffic_source"] = htsrc
        if htraffic:
            hus = rt * 1000.0 / rl
            relax_heavy["traffic_GBps"] = round(htraffic / (hus * 1e-6) / 1e9, 2)
            relax_heavy["traffic_frac"] = round(htraffic / (hus * 1e-6) / 1e9 / PEAK_HBM_GBS, 4)
        log(f"[bench] relaxer on the heavy-churn mid graph: {ach:.1f} GB/s algorithmic "
            f"({hst['n_unstable'] / hv.num_vertices:.0%} unstable, query {hms:.2f} ms)")

    # Fig. 11 analogue (QRS generation = bound solves + unstable set + reduced subgraph, share of the query)
    qrs = {"bounds_only_ms_p50": round(bounds_ms, 4), "query_ms_p50": round(q_ev["p50"], 4),
           "bounds_share_uninstrumented": round(bounds_ms / q_ev["p50"], 4), "paper_cqrs_share": 0.5601}
    if kernels:
        gen = sum(v[1] for k, v in kernels.items()
                  if k.startswith("solve_") or k in ("compact_unstable", "compact_reduce", "copy_bound", "query_init"))
        qrs["kernel_time_share"] = round(gen / sum(v[1] for v in kernels.values()), 4)
    log(f"[bench] QRS generation: {qrs}")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        trip, bits = oracle.replay(inst)
        replay_s = time.perf_counter() - t
        sample = list(range(b, b + L))
        nthreads = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)) or 1)
        t = time.perf_counter()
        want = oracle.query(inst.num_vertices, trip, bits, algo, source, sample, nthreads)
        cpu_s = time.perf_counter() - t
        # per-core rate: two snapshots on one thread
        t = time.perf_counter()
        oracle.query(inst.num_vertices, trip, bits, algo, source, sample[:2], 1)
        one_s = time.perf_counter() - t
        got = evq.to_u32(out).reshape(inst.num_vertices, L)[:, :len(sample)]
        ok = bool(np.array_equal(got, want))
        # the oracle against the paper's reported fractions (a sanity band: unchanged vertices 53.2-99.8%,
        # unstable 0.3-42%, detection recall "nearly all")
        san = oracle.window_sanity(inst.num_vertices, trip, bits, algo, source, b, L, values=want)
        sanity = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in san.items()}
        sanity["paper_unchanged_band"] = list(oracle.UNCHANGED_BAND)
        sanity["paper_unstable_band"] = list(oracle.UNSTABLE_BAND)
        sanity["warnings"] = oracle.sanity_warnings(san)
        log(f"[bench] oracle sanity: {sanity}")
        cpu = {"value": float(counts[sample].sum() / cpu_s), "unit": "snapshot-edges/s", "cores": nthreads,
               "kind": "oracle",
               "sample": f"snapshots {sample[0]}..{sample[-1]} of the window ({len(sample)} of {L}), per-snapshot "
                         f"materialisation + Dijkstra, {cpu_s:.2f}s; replay of the batches ({replay_s:.1f}s) not "
                         f"included",
               "matches_gpu": ok,
               "one_core": {"value": float(counts[sample[:2]].sum() / one_s), "unit": "snapshot-edges/s",
                            "sample": f"snapshots {sample[0]}..{sample[1]} on 1 thread, {one_s:.2f}s"},
               "oracle_sanity": sanity}
        log(f"[bench] oracle sample: {cpu_s:.2f}s for {len(sample)} snapshots on {nthreads} threads, "
            f"matches GPU: {ok}")

    res = {
        "metric": "snapshot-edge relaxations/s",
        "value": snap_edges / (ms / 1000.0),
        "unit": "snapshot-edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: R-MAT scale {inst.meta['scale']} ({inst.num_vertices} vertices, "
                               f"{inst.meta['n_samples']} samples, w in [{inst.meta['wmin']},{inst.meta['wmax']}]), "
                               f"K={K} snapshots of {inst.meta['n_del']}+{inst.meta['n_add']} updates, "
                               f"{args.algo.upper()} from vertex {source}, window [{b},{b + L})",
                   "algo": args.algo, "snapshots": L, "snapshot_edges": snap_edges,
                   "union_edges": info["num_edges"], "partial_edges": info["num_partial"]},
        "ms_per_query": ms,
        "ms_per_query_hip_events": q_ev,
        "qrs_generation": qrs,
        "plain_ms_per_query": plain_ms,
        "speedup_vs_plain": (plain_ms / ms) if plain_ms else None,
        "sequential_ms_per_query": seq_ms,
        "speedup_vs_sequential": (seq_ms / ms) if seq_ms else None,
        "push_only_ms_per_query": push_ms,
        "speedup_vs_plain_push_only": (plain_ms / push_ms) if (plain_ms and push_ms) else None,
        "build_ms": info["build_ms"],
        "batch_leg": batch_leg,
        "query_stats": st,
        "executed_relaxations_per_s": (st["edges_cap"] + st["edges_cup"] + st["lane_relaxations"]) / (ms / 1000.0),
        "roofline": roof,
        "relax_roofline": relax_roof,
        "relax_roofline_heavy_churn": relax_heavy,
        "cpu_baseline": cpu,
    }
    if kernels:
        res["kernel_ms_per_query"] = {k: round(v[1] / 3, 4) for k, v in kernels.items()}
    g.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
