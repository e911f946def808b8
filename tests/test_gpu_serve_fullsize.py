"""The query server at full size: R-MAT scale 24 (16,777,216 vertices,
268,435,456 samples, weights [1, 100]), a ring of 128 snapshots of
100k + 100k updates built on the device, then advanced by two appends (so
windows wrap around the ring), and 64 served queries with the algorithm
uniform over the four, a random source of base out-degree > 0 and the
newest len snapshots, len uniform in [16, 128].

* Every served result equals the same query answered alone (compared on the
  device, element by element).
* A 16-query sample (every 4th query) equals the oracle on every snapshot of
  its window, through per-snapshot digests that
  tests/golden/make_fullsize_digests.py wrote from the oracle (whose history
  is re-based at the snapshot before the oldest one held), and its unstable
  count equals the oracle bounds'.
Values are uint32: tolerance zero.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_digests, golden_section, gpu_column_digests

pytestmark = pytest.mark.gpu

K, A, NQ = 128, 2, 64


@pytest.fixture(scope="module")
def evq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_10579_amd as m
    return m


@pytest.fixture(scope="module")
def served(evq):
    import torch
    inst = synth.rmat_instance(seed=1, **dict(synth.CONFIGS["served"], K=K + A))
    print(f"served: generated {len(inst.base)} base edges, {K + A} batches", flush=True)
    g = evq.Graph(inst.num_vertices, inst.base, inst.dels[:K], inst.adds[:K])
    for a in range(A):
        g.append(inst.dels[K + a], inst.adds[K + a])
    assert g.first == A
    rng = np.random.default_rng(11)
    src = synth.pick_sources(inst, NQ, seed=11)
    qs = [(int(rng.integers(0, 4)), src[i], int(rng.integers(16, 129))) for i in range(NQ)]
    with evq.Server(g, mode="batch") as srv:
        for (a, s, L) in qs:
            srv.submit(a, s, L)
        comps = []
        while len(comps) < NQ:
            comps += srv.poll(256, 1000)
    torch.cuda.synchronize()
    comps.sort(key=lambda c: c["ticket"])
    print(f"served: {NQ} queries done, last at {max(c['t_done_ms'] for c in comps):.0f} ms", flush=True)
    yield inst, g, comps
    for c in comps:
        if c["result"] is not None:
            c["result"].free()
    g.close()


@pytest.mark.timeout(600)
def test_served_equal_alone(evq, served):
    import torch
    inst, g, comps = served
    for c in comps:
        assert c["status"] == 0
        a, s, b, L = c["algo"], c["source"], c["win_begin"], c["win_len"]
        assert b + L == A + K
        got = c["result"].expand()
        one = g.query(a, s, b, L)
        if not torch.equal(got, one):
            raise AssertionError(f"served {(a, s, b, L)}: {int((got != one).sum())} values differ from alone")


@pytest.mark.timeout(600)
def test_served_sample_vs_oracle(evq, served):
    inst, g, comps = served
    V = inst.num_vertices
    sec = golden_section("served", inst)
    sample = comps[::NQ // 16]
    assert sorted(int(k) for k in sec["queries"]) == list(range(0, NQ, NQ // 16))

    for k, c in zip(range(0, NQ, NQ // 16), sample):
        want = sec["queries"][str(k)]
        a, s, b, L = c["algo"], c["source"], c["win_begin"], c["win_len"]
        assert want["query"] == [a, s, b, L]
        out = c["result"].expand()

        def diagnose(col, a=a, s=s, b=b, out=out):
            # the oracle's history re-based so that its snapshot i is global snapshot A + i
            trip, bits = oracle.replay(synth.Instance(V, inst.base, inst.dels[:A], inst.adds[:A]))
            t = A - 1
            keep = ((bits[:, t // 64] >> np.uint64(t % 64)) & np.uint64(1)).astype(bool)
            reb = synth.Instance(V, trip[keep].copy(), inst.dels[A:], inst.adds[A:])
            del trip, bits, keep
            rtrip, rbits = oracle.replay(reb)
            w = oracle.query(V, rtrip, rbits, a, s, [b + col - A])[:, 0]
            gc = evq.to_u32(out[:, col].contiguous())
            v = int(np.flatnonzero(gc != w)[0])
            return f"vertex {v}: gpu {gc[v]} oracle {w[v]}"

        assert_digests(gpu_column_digests(out), want["columns"], f"served {(a, s, b, L)}", diagnose)
        assert c["n_unstable"] == want["n_unstable"]
        del out
        print(f"  served query {c['ticket']} {(a, s, b, L)}: equal on all {L} snapshots", flush=True)
