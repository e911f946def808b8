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
--config mid --no-cpu-baseline --no-roofline --no-plain.
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


def algorithmic_bytes(kernel, st, L, V):
    """Bytes a kernel's work must move at minimum, from the query's counters.

    Bound-solve expansion: per edge visit the edge's (col, w) pair and one
    4-byte value read; per improving update one 4-byte atomic write; per
    frontier vertex its 16-byte item (edge offset, row position, vertex) and
    its value.  Relaxer: per edge visit one record (dst, w, lane mask), per
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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (this build has no "
              f"multi-GPU path)", file=sys.stderr)
        sys.exit(2)

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
    t = time.perf_counter()
    for _ in range(args.steps):
        g.query(algo, source, b, L, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1000.0 / args.steps
    log(f"[bench] method: {ms:.3f} ms/query over {args.steps} steps")

    _, st = g.query(algo, source, b, L, out=out, stats=True)
    log(f"[bench] stats: {json.dumps({k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()})}")

    plain_ms = None
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

    roof = None
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
            roof = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": None,
                    "avg_launch_us": round(tot_ms * 1000.0 / launches, 3), "launches_per_query": launches // reps,
                    "algorithmic_bytes_per_query": int(byts)}
        relax_b = algorithmic_bytes("relax", st, L, inst.num_vertices)
        if "relax" in kernels and relax_b:
            rl, rt = kernels["relax"]
            roof_relax = relax_b * reps / (rt / 1000.0) / 1e9
            log(f"[bench] relaxer: {roof_relax:.1f} GB/s algorithmic over {rl // reps} launches/query")

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
        got = evq.to_u32(out).reshape(inst.num_vertices, L)[:, :len(sample)]
        ok = bool(np.array_equal(got, want))
        cpu = {"value": float(counts[sample].sum() / cpu_s), "unit": "snapshot-edges/s", "cores": nthreads,
               "kind": "oracle",
               "sample": f"snapshots {sample[0]}..{sample[-1]} of the window ({len(sample)} of {L}), per-snapshot "
                         f"materialisation + Dijkstra, {cpu_s:.2f}s; replay of the batches ({replay_s:.1f}s) not "
                         f"included",
               "matches_gpu": ok}
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
        "plain_ms_per_query": plain_ms,
        "speedup_vs_plain": (plain_ms / ms) if plain_ms else None,
        "build_ms": info["build_ms"],
        "query_stats": st,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if kernels:
        res["kernel_ms_per_query"] = {k: round(v[1] / 3, 4) for k, v in kernels.items()}
    g.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
