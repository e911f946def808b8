"""Batched queries at full size: R-MAT scale 22 (4,194,304 vertices, 67,108,864
samples, weights [1, 100]), K = 128 snapshots of 20k + 20k updates, 256
queries with the algorithm uniform over the four, a random source of base
out-degree > 0, window start uniform in [0, 100] and length uniform in
[25, 100] clamped to the last snapshot.

Two execution configurations: the fixed one (shared solves of 64 queries,
chunk 8, 2048 workgroups) and the one evq_batch_autotune picks on these
queries, which is what bench.py times.  Under each:
* all 256 expanded results equal the one-at-a-time evq_query results
  (compared on the device, element by element);
* a 16-query sample (every 16th query) equals the oracle on every snapshot
  of its window, through per-snapshot digests that
  tests/golden/make_fullsize_digests.py wrote from the oracle, and its
  unstable count equals the oracle bounds'.
Values are uint32: tolerance zero.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_digests, golden_section, gpu_column_digests

pytestmark = pytest.mark.gpu

NQ, SAMPLE_EVERY = 256, 16


@pytest.fixture(scope="module")
def evq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_10579_amd as m
    return m


@pytest.fixture(scope="module")
def batched(evq):
    inst = synth.config_instance("batched", seed=1)
    sec = golden_section("batched", inst)
    qs = synth.batch_queries(inst, NQ, seed=1)
    g = evq.Graph.from_instance(inst)
    yield inst, qs, sec, g
    g.close()


@pytest.fixture(scope="module", params=["fixed", "autotuned"])
def batch_results(evq, batched, request):
    import torch
    inst, qs, sec, g = batched
    prev = evq.batch_config()
    if request.param == "fixed":
        evq.set_batch_config(lanes=1, chunk=8, blocks=2048, group=64)
    else:
        cfg, ms = g.autotune_batch(qs)
        print(f"batched: autotuner chose {cfg} ({ms:.1f} ms)", flush=True)
    print(f"batched ({request.param}): {len(qs)} queries on V={inst.num_vertices}, config {evq.batch_config()}",
          flush=True)
    res, st = g.query_batch(qs, stats=True)
    torch.cuda.synchronize()
    yield res, st
    for r in res:
        r.free()
    evq.set_batch_config(**prev)


@pytest.mark.timeout(600)
def test_batched_all_equal_one_at_a_time(evq, batched, batch_results):
    import torch
    inst, qs, sec, g = batched
    res, _ = batch_results
    for k, (r, (a, s, b, L)) in enumerate(zip(res, qs)):
        got = r.expand()
        one = g.query(a, s, b, L)
        if not torch.equal(got, one):
            n = int((got != one).sum())
            raise AssertionError(f"query {k} {(a, s, b, L)}: {n} values differ from the one-at-a-time result")
        if k % 64 == 63:
            print(f"  {k + 1} queries equal", flush=True)


@pytest.mark.timeout(600)
def test_batched_sample_vs_oracle(evq, batched, batch_results):
    inst, qs, sec, g = batched
    res, _ = batch_results
    V = inst.num_vertices
    sample = list(range(0, NQ, SAMPLE_EVERY))
    assert sorted(int(k) for k in sec["queries"]) == sample
    for k in sample:
        a, s, b, L = qs[k]
        want = sec["queries"][str(k)]
        assert want["query"] == [a, s, b, L]
        out = res[k].expand()

        def diagnose(col, a=a, s=s, b=b, out=out):
            trip, bits = oracle.replay(inst)
            w = oracle.query(V, trip, bits, a, s, [b + col])[:, 0]
            gc = evq.to_u32(out[:, col].contiguous())
            v = int(np.flatnonzero(gc != w)[0])
            return f"vertex {v}: gpu {gc[v]} oracle {w[v]}"

        assert_digests(gpu_column_digests(out), want["columns"], f"query {k} {(a, s, b, L)}", diagnose)
        assert res[k].info["n_unstable"] == want["n_unstable"]
        print(f"  query {k} {(a, s, b, L)}: equal on all {L} snapshots", flush=True)
