"""GPU parity of the query server (evq_server_*), both modes, on small rings.

Every completed query's compact result equals the oracle's values for the
window the server fixed at admission (the newest `len` held snapshots), and
equals the same query answered alone by evq_query.  Appends between
submissions move the windows.  A budget too small for two queries admits
one at a time; destroying a server with queued queries releases them.
Values are uint32: tolerance zero.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_equal_values

pytestmark = pytest.mark.gpu

ALGOS = [oracle.SSSP, oracle.BFS, oracle.SSWP, oracle.SSNP, oracle.VITERBI]


@pytest.fixture(scope="module")
def evq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_10579_amd as m
    return m


def head(inst, K):
    return synth.Instance(inst.num_vertices, inst.base, inst.dels[:K], inst.adds[:K])


def collect(srv, n, timeout_ms=60000):
    got = []
    waited = 0
    while len(got) < n:
        part = srv.poll(256, 200)
        got += part
        if not part:
            waited += 200
            assert waited < timeout_ms, f"only {len(got)} of {n} queries completed"
    return got


def check(evq, g, inst, rep, comps, alone=True):
    V = inst.num_vertices
    for c in comps:
        assert c["status"] == 0, c
        assert c["t_arrival_ms"] <= c["t_admit_ms"] <= c["t_done_ms"]
        a, s, b, L = c["algo"], c["source"], c["win_begin"], c["win_len"]
        got = evq.to_u32(c["result"].expand()).reshape(V, L)
        want = oracle.window_values(inst, a, s, b, L, replayed=rep)
        assert_equal_values(got, want, f"served {(a, s, b, L)} vs oracle")
        if alone and g.first <= b:
            one = evq.to_u32(g.query(a, s, b, L)).reshape(V, L)
            assert_equal_values(got, one, f"served {(a, s, b, L)} vs alone")
        c["result"].free()


@pytest.mark.parametrize("mode", ["batch", "plain"])
def test_serve_mix_equals_alone_and_oracle(evq, mode):
    K = 16
    inst = synth.random_instance(80, 900, K, 6, 6, 9, 41)
    rep = oracle.replay(inst)
    rng = np.random.default_rng(3)
    src = synth.pick_sources(inst, 60, seed=5)
    with evq.Graph.from_instance(inst) as g:
        with evq.Server(g, mode=mode) as srv:
            for i in range(60):
                srv.submit(ALGOS[int(rng.integers(0, 5))], src[i], int(rng.integers(1, 21)))
            comps = collect(srv, 60)
            assert sorted(c["ticket"] for c in comps) == list(range(1, 61))
            for c in comps:
                assert c["win_begin"] + c["win_len"] == K and c["win_len"] <= K
            check(evq, g, inst, rep, comps)


def test_serve_with_appends(evq):
    K, A = 12, 9
    inst = synth.random_instance(70, 700, K + A, 5, 5, 9, 43)
    rep = oracle.replay(inst)  # global snapshot ids
    src = synth.pick_sources(inst, 8 * (A + 1), seed=7)
    rng = np.random.default_rng(9)
    comps = []
    with evq.Graph.from_instance(head(inst, K)) as g:
        with evq.Server(g, mode="batch", max_batch=8) as srv:
            k = 0
            for a in range(A + 1):
                for _ in range(8):
                    srv.submit(ALGOS[k % 5], src[k], int(rng.integers(1, K + 1)))
                    k += 1
                if a < A:
                    comps += srv.poll(256, 0)
                    g.append(inst.dels[K + a], inst.adds[K + a])
            comps += collect(srv, 8 * (A + 1) - len(comps))
            firsts = sorted({c["win_begin"] + c["win_len"] - K for c in comps})
            print(f"windows ended at {len(firsts)} different ring positions", flush=True)
            check(evq, g, inst, rep, comps)


def test_serve_budget_admits_one_at_a_time(evq):
    K = 8
    inst = synth.random_instance(60, 500, K, 4, 4, 9, 47)
    rep = oracle.replay(inst)
    src = synth.pick_sources(inst, 12, seed=2)
    with evq.Graph.from_instance(inst) as g:
        with evq.Server(g, mode="batch", mem_budget=1) as srv:
            for i in range(12):
                srv.submit(ALGOS[i % 5], src[i], 1 + i % K)
            comps = sorted(collect(srv, 12), key=lambda c: c["t_admit_ms"])
            for prev, nxt in zip(comps, comps[1:]):
                assert nxt["t_admit_ms"] >= prev["t_done_ms"] - 1e-3, "two queries in flight under a one-query budget"
            check(evq, g, inst, rep, comps)


def test_serve_single_query_groups(evq):
    K = 8
    inst = synth.random_instance(60, 500, K, 4, 4, 9, 53)
    rep = oracle.replay(inst)
    src = synth.pick_sources(inst, 16, seed=4)
    with evq.Graph.from_instance(inst) as g:
        with evq.Server(g, mode="batch", max_batch=1, max_groups=4) as srv:
            for i in range(16):
                srv.submit(ALGOS[i % 5], src[i], 1 + i % K)
            check(evq, g, inst, rep, collect(srv, 16))


def test_serve_destroy_with_queued_queries(evq):
    inst = synth.config_instance("small", seed=2)
    src = synth.pick_sources(inst, 200, seed=1)
    with evq.Graph.from_instance(inst) as g:
        srv = evq.Server(g, mode="plain")
        for i in range(200):
            srv.submit(ALGOS[i % 5], src[i], 8)
        srv.close()  # queued ones are dropped, running ones finish, uncollected results released
        with pytest.raises(evq.EvqError):
            evq.Server(g, mode="batch", max_batch=65)


def test_serve_light_load_runs_one_at_a_time(evq):
    # continuous batching at light load: below queue_hi waiting queries, a query starts only when
    # nothing is in flight (as the plain server does); results stay exact
    K = 8
    inst = synth.random_instance(60, 500, K, 4, 4, 9, 59)
    rep = oracle.replay(inst)
    src = synth.pick_sources(inst, 10, seed=6)
    with evq.Graph.from_instance(inst) as g:
        with evq.Server(g, mode="batch", queue_hi=1000) as srv:
            for i in range(10):
                srv.submit(ALGOS[i % 5], src[i], 1 + i % K)
            comps = sorted(collect(srv, 10), key=lambda c: c["t_admit_ms"])
            # a group's queries are admitted together (one dispatch, contiguous in admission order);
            # the next group starts only after everything admitted before it has completed
            i = 0
            while i < len(comps):
                grp = comps[i:i + comps[i]["group_size"]]
                assert len({c["algo"] for c in grp}) == 1
                done_before = max((c["t_done_ms"] for c in comps[:i]), default=0.0)
                assert grp[0]["t_admit_ms"] >= done_before - 1e-3, "a group started beside running queries"
                i += len(grp)
            check(evq, g, inst, rep, comps)


def test_serve_full_queue_is_busy(evq):
    # admission back-off: beyond max_queued waiting queries, submit answers EVQ_EBUSY and queues
    # nothing; the accepted queries complete exactly, and submitting works again after polling
    K = 8
    inst = synth.random_instance(60, 500, K, 4, 4, 9, 61)
    rep = oracle.replay(inst)
    src = synth.pick_sources(inst, 64, seed=8)
    with evq.Graph.from_instance(inst) as g:
        with evq.Server(g, mode="plain", max_queued=2) as srv:
            accepted, busy = 0, 0
            for i in range(64):
                try:
                    srv.submit(ALGOS[i % 5], src[i], 1 + i % K)
                    accepted += 1
                except evq.EvqError as e:
                    assert e.status == evq.EVQ_EBUSY
                    busy += 1
            assert busy > 0 and accepted >= 2
            comps = collect(srv, accepted)
            srv.submit(ALGOS[0], src[0], K)
            comps += collect(srv, 1)
            check(evq, g, inst, rep, comps)
