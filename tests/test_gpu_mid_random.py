"""GPU parity on the mid workload (R-MAT scale 20, K = 64) for random queries:
algorithm uniform over the five, sources drawn among vertices with base
out-degree > 0, windows [b, b + L) with L uniform in [1, 64].

* Each query's values on three snapshots of its window (first, middle, last)
  equal the oracle's, and its bounds equal the oracle's bounds.
* The same queries answered in one evq_query_batch call, and by the plain
  evaluation, equal the single answers on every snapshot (compared on the
  device).
* The heavy-churn graph (100k + 100k updates per snapshot, about half the
  vertices unstable, so the relaxation's task writer runs) gets the same
  single-query check on three windows.
Values are uint32: tolerance zero.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_equal_values, gpu_bounds

pytestmark = pytest.mark.gpu

ALGOS = [oracle.SSSP, oracle.BFS, oracle.SSWP, oracle.SSNP, oracle.VITERBI]


@pytest.fixture(scope="module")
def evq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_10579_amd as m
    return m


def random_queries(inst, n, seed):
    rng = np.random.default_rng(seed)
    src = synth.pick_sources(inst, n, seed=seed)
    qs = []
    for i in range(n):
        L = int(rng.integers(1, inst.K + 1))
        b = int(rng.integers(0, inst.K - L + 1))
        qs.append((ALGOS[int(rng.integers(0, 5))], src[i], b, L))
    return qs


def check_sampled(evq, g, inst, rep, qs, ctx):
    V = inst.num_vertices
    for (a, s, b, L) in qs:
        snaps = sorted({b, b + L // 2, b + L - 1})
        print(f"{ctx}: algo {a} source {s} window [{b},{b + L}) snapshots {snaps}", flush=True)
        got = evq.to_u32(g.query(a, s, b, L)).reshape(V, L)
        want = oracle.query(V, rep[0], rep[1], a, s, snaps, 0)
        assert_equal_values(got[:, [t - b for t in snaps]], want, f"{ctx} {(a, s, b, L)}")
        rc, ru = gpu_bounds(g, a, s, b, L)
        rc_o, ru_o = oracle.bounds(V, rep[0], rep[1], a, s, b, L)
        assert np.array_equal(rc, rc_o) and np.array_equal(ru, ru_o), f"{ctx} bounds {(a, s, b, L)}"


@pytest.mark.timeout(900)
def test_mid_random_queries(evq):
    import torch
    inst = synth.config_instance("mid", seed=1)
    rep = oracle.replay(inst)
    qs = random_queries(inst, 10, seed=23)
    with evq.Graph.from_instance(inst) as g:
        check_sampled(evq, g, inst, rep, qs, "mid")
        singles = [g.query(a, s, b, L) for (a, s, b, L) in qs]
        res = g.query_batch(qs)
        torch.cuda.synchronize()
        for r, one, q in zip(res, singles, qs):
            got = r.expand()
            assert torch.equal(got, one), f"batched {q} differs from alone"
            r.free()
        for one, (a, s, b, L) in zip(singles, qs):
            assert torch.equal(g.query_plain(a, s, b, L), one), f"plain {(a, s, b, L)} differs from the method"


@pytest.mark.timeout(900)
def test_churn_random_windows(evq):
    inst = synth.config_instance("churn", seed=1)
    rep = oracle.replay(inst)
    src = synth.pick_sources(inst, 3, seed=4)
    qs = [(oracle.SSSP, src[0], 0, 64), (oracle.BFS, src[1], 10, 40), (oracle.SSWP, src[2], 33, 31)]
    with evq.Graph.from_instance(inst) as g:
        check_sampled(evq, g, inst, rep, qs, "churn")
