"""Write fullsize_digests.json: the ORACLE's values at the full workload sizes, as
per-snapshot digests, for the GPU parity tests that cannot run the oracle on
every snapshot in their own time.

Only the seeded input generator (synth) and the oracle are called here; no
value comes from the HIP library.  Each section records the fingerprint of the
instance it was computed on, so a test can tell a changed generator (stale
file: regenerate) from a changed result (a parity failure).

Sections (each written as soon as it is done; rerunning one replaces it):
  large    R-MAT scale 23, K = 100, weights [1, 1000]: SSWP, SSNP, SSSP, BFS
           and Viterbi from the seeded source over the window [0, 100): every
           snapshot, both bounds (a rerun on the same instance adds the
           algorithms that are missing)
  batched  R-MAT scale 22, K = 128: the 16-query sample (every 16th of the 256
           seeded batch queries), every snapshot of each window, and the
           unstable count of the oracle's bounds
  served   R-MAT scale 24, a ring of 128 advanced twice: the 16-query sample
           (every 4th of 64 seeded served queries; windows = the newest len
           snapshots), every snapshot of each window, and the unstable count

usage: python tests/golden/make_fullsize_digests.py large batched served
(OMP_NUM_THREADS sets the oracle's threads; the served replay needs ~40 GB.)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
for p in (ROOT, os.path.dirname(HERE)):
    if p not in sys.path:
        sys.path.insert(0, p)

import oracle  # noqa: E402
import synth  # noqa: E402
from digest import array_digest, instance_fingerprint, values_digests  # noqa: E402

OUT = os.path.join(HERE, "fullsize_digests.json")

# Served test layout: ring of K snapshots, A appends before the queries, NQ queries.
SERVED_K, SERVED_A, SERVED_NQ, SERVED_QSEED = 128, 2, 64, 11
BATCHED_N, BATCHED_QSEED, SAMPLE = 256, 1, 16
LARGE_ALGOS = (oracle.SSWP, oracle.SSNP, oracle.SSSP, oracle.BFS, oracle.VITERBI)


def served_queries(inst):
    """(algo, source, win_begin, win_len) of the served test's queries, in submission order:
    windows are the newest len snapshots after SERVED_A appends to a ring of SERVED_K."""
    rng = np.random.default_rng(SERVED_QSEED)
    src = synth.pick_sources(inst, SERVED_NQ, seed=SERVED_QSEED)
    out = []
    for i in range(SERVED_NQ):
        a = int(rng.integers(0, 4))
        L = min(int(rng.integers(16, 129)), SERVED_K)
        out.append((a, int(src[i]), SERVED_A + SERVED_K - L, L))
    return out


def served_instance():
    return synth.rmat_instance(seed=1, **dict(synth.CONFIGS["served"], K=SERVED_K + SERVED_A))


def _load():
    if os.path.exists(OUT):
        with open(OUT) as f:
            return json.load(f)
    return {}


def _save(sec, data):
    d = _load()
    d[sec] = data
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, OUT)


def _log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def large():
    inst = synth.config_instance("large", seed=1)
    fp = instance_fingerprint(inst)
    src = synth.pick_sources(inst, 1, seed=1)[0]
    trip, bits = oracle.replay(inst)
    V, K = inst.num_vertices, inst.K
    _log(f"large: replayed {len(trip)} triples, source {src}")
    out = {"fingerprint": fp, "source": src, "window": [0, K], "algos": {}}
    prev = _load().get("large")
    if prev and prev.get("fingerprint") == fp and prev.get("source") == src:
        out["algos"] = dict(prev["algos"])  # same instance: keep what is there, add the rest
    for algo in LARGE_ALGOS:
        if str(algo) in out["algos"]:
            continue
        rc, ru = oracle.bounds(V, trip, bits, algo, src, 0, K)
        vals = oracle.query(V, trip, bits, algo, src, list(range(K)))
        out["algos"][str(algo)] = {"rcap": array_digest(rc), "rcup": array_digest(ru),
                                   "n_unstable": int((rc != ru).sum()), "columns": values_digests(vals)}
        del vals
        _log(f"large: algo {algo} done")
        _save("large", out)


def _sample_section(name, inst, V, trip, bits, queries, sample_idx, rebase=0):
    d = _load().get(name, {})
    fp = instance_fingerprint(inst)
    if d.get("fingerprint") != fp:
        d = {"fingerprint": fp, "queries": {}}
    for k in sample_idx:
        if str(k) in d["queries"]:
            continue
        a, s, b, L = queries[k]
        rb = b - rebase
        rc, ru = oracle.bounds(V, trip, bits, a, s, rb, L)
        vals = oracle.query(V, trip, bits, a, s, list(range(rb, rb + L)))
        d["queries"][str(k)] = {"query": [a, s, b, L], "n_unstable": int((rc != ru).sum()),
                                "rcap": array_digest(rc), "columns": values_digests(vals)}
        del vals
        _save(name, d)
        _log(f"{name}: query {k} {(a, s, b, L)} done")


def batched():
    inst = synth.config_instance("batched", seed=1)
    qs = synth.batch_queries(inst, BATCHED_N, seed=BATCHED_QSEED)
    trip, bits = oracle.replay(inst)
    _log(f"batched: replayed {len(trip)} triples")
    _sample_section("batched", inst, inst.num_vertices, trip, bits, qs, list(range(0, BATCHED_N, BATCHED_N // SAMPLE)))


def served():
    inst = served_instance()
    V, A = inst.num_vertices, SERVED_A
    qs = served_queries(inst)
    # The ring holds global snapshots A .. A+K-1; the oracle's history is re-based so that its
    # snapshot i is global snapshot A + i: the base becomes snapshot A - 1.
    trip, bits = oracle.replay(synth.Instance(V, inst.base, inst.dels[:A], inst.adds[:A]))
    t = A - 1
    keep = ((bits[:, t // 64] >> np.uint64(t % 64)) & np.uint64(1)).astype(bool)
    reb = synth.Instance(V, trip[keep].copy(), inst.dels[A:], inst.adds[A:])
    del trip, bits, keep
    rtrip, rbits = oracle.replay(reb)
    del reb
    _log(f"served: replayed {len(rtrip)} triples")
    _sample_section("served", inst, V, rtrip, rbits, qs, list(range(0, SERVED_NQ, SERVED_NQ // SAMPLE)), rebase=A)


if __name__ == "__main__":
    for sec in sys.argv[1:] or ["large", "batched", "served"]:
        _log(f"section {sec}")
        {"large": large, "batched": batched, "served": served}[sec]()
