"""Batched queries at full size: R-MAT scale 22 (4,194,304 vertices, 67,108,864
samples, weights [1, 100]), K = 128 snapshots of 20k + 20k updates, 256
queries with the algorithm uniform over the four, a random source of base
out-degree > 0, window start uniform in [0, 100] and length uniform in
[25, 100] clamped to the last snapshot -- in the launch configuration that
bench.py times.

* All 256 expanded results equal the one-at-a-time evq_query results
  (compared on the device, element by element).
* A 16-query sample equals the oracle on three snapshots of each window
  (first, middle, last), and the unstable count equals the oracle bounds'.
Values are uint32: tolerance zero.
"""
import concurrent.futures

import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_equal_values

pytestmark = pytest.mark.gpu


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
    qs = synth.batch_queries(inst, 256, seed=1)
    g = evq.Graph.from_instance(inst)
    yield inst, qs, g
    g.close()


@pytest.fixture(scope="module")
def batch_results(evq, batched):
    import torch
    inst, qs, g = batched
    evq.set_batch_config(lanes=1, chunk=8, blocks=2048, group=64)
    print(f"batched: {len(qs)} queries on V={inst.num_vertices}", flush=True)
    res, st = g.query_batch(qs, stats=True)
    torch.cuda.synchronize()
    yield res, st
    for r in res:
        r.free()


@pytest.mark.timeout(600)
def test_batched_all_equal_one_at_a_time(evq, batched, batch_results):
    import torch
    inst, qs, g = batched
    res, _ = batch_results
    for k, (r, (a, s, b, L)) in enumerate(zip(res, qs)):
        got = r.expand()
        one = g.query(a, s, b, L)
        if not torch.equal(got, one):
            n = int((got != one).sum())
            raise AssertionError(f"query {k} {(a, s, b, L)}: {n} values differ from the one-at-a-time result")
        if k % 64 == 63:
            print(f"  {k + 1} queries equal", flush=True)


@pytest.mark.timeout(900)
def test_batched_sample_vs_oracle(evq, batched, batch_results):
    inst, qs, g = batched
    res, _ = batch_results
    V = inst.num_vertices
    trip, bits = oracle.replay(inst)
    sample = list(range(0, 256, 16))

    def solve(k):
        a, s, b, L = qs[k]
        snaps = sorted({b, b + L // 2, b + L - 1})
        want = oracle.query(V, trip, bits, a, s, snaps, 3)
        rc, ru = oracle.bounds(V, trip, bits, a, s, b, L)
        return k, snaps, want, int((rc != ru).sum())

    with concurrent.futures.ThreadPoolExecutor(5) as ex:
        for k, snaps, want, n_unstable in ex.map(solve, sample):
            a, s, b, L = qs[k]
            cols = [t - b for t in snaps]
            got = evq.to_u32(res[k].expand()[:, cols].contiguous())
            assert_equal_values(got, want, f"query {k} {(a, s, b, L)} snapshots {snaps}")
            assert res[k].info["n_unstable"] == n_unstable
            print(f"  query {k} {(a, s, b, L)}: equal on snapshots {snaps}", flush=True)
