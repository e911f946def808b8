"""GPU parity of batched queries (evq_query_batch) through the C ABI.

Every expanded compact result is compared bit-exactly with the oracle's
per-snapshot values (small instances: every snapshot of every query) and
with the one-at-a-time evq_query result.  Both execution choices are
covered: shared bound solves with one query per lane, and one bound solve
per query.  Groups of more than 64 queries of one algorithm, windows that
cross the 64-snapshot mask word, length-1 windows and sources without
out-edges are included.  Values are uint32: tolerance zero.
"""
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
    yield m
    m.set_batch_config(lanes=1, chunk=8, blocks=2048, group=64)


def _check_batch(evq, inst, queries, lanes, chunk=8, blocks=2048, group=64, rep=None, vs_single=True,
                 vs_oracle=True):
    import torch
    V = inst.num_vertices
    evq.set_batch_config(lanes=lanes, chunk=chunk, blocks=blocks, group=group)
    print(f"batch: {len(queries)} queries, lanes={lanes} chunk={chunk} blocks={blocks} group={group}", flush=True)
    rep = rep if rep is not None else oracle.replay(inst)
    with evq.Graph.from_instance(inst) as g:
        res = g.query_batch(queries)
        torch.cuda.synchronize()
        for r, (a, s, b, L) in zip(res, queries):
            assert r.info["algo"] == a and r.info["source"] == s and r.info["win_begin"] == b
            got = evq.to_u32(r.expand()).reshape(V, L)
            if vs_single:
                one = evq.to_u32(g.query(a, s, b, L)).reshape(V, L)
                assert_equal_values(got, one, f"batch vs single {(a, s, b, L)}")
            if vs_oracle:
                want = oracle.window_values(inst, a, s, b, L, replayed=rep)
                assert_equal_values(got, want, f"batch vs oracle {(a, s, b, L)}")
            # Theorem 2: the unstable count is that of the bounds
            rc, ru = oracle.bounds(V, rep[0], rep[1], a, s, b, L) if vs_oracle else (None, None)
            if rc is not None:
                assert r.info["n_unstable"] == int((rc != ru).sum())
            r.free()


@pytest.mark.parametrize("lanes", [1, 2])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_batch_small_mixed(evq, lanes, seed):
    inst = synth.config_instance("small", seed=seed)
    qs = synth.batch_queries(inst, 24, seed=seed, start_max=7, len_min=1, len_max=8)
    _check_batch(evq, inst, qs, lanes)


@pytest.mark.parametrize("lanes", [1, 2])
def test_batch_viterbi(evq, lanes):
    inst = synth.config_instance("small", seed=6)
    qs = synth.batch_queries(inst, 20, seed=6, start_max=7, len_min=1, len_max=8, algos=(4, 2))
    _check_batch(evq, inst, qs, lanes)


@pytest.mark.parametrize("chunk,group", [(4, 64), (8, 16), (16, 5), (8, 1)])
def test_batch_chunks_grids_groups(evq, chunk, group):
    inst = synth.config_instance("small", seed=4)
    qs = synth.batch_queries(inst, 40, seed=9, start_max=7, len_min=1, len_max=8)
    _check_batch(evq, inst, qs, 1, chunk=chunk, blocks=64 if chunk == 4 else 2048, group=group)


def test_batch_more_than_64_per_algorithm(evq):
    # 150 SSSP queries: three groups of 50 (64 lanes each); 10 BFS for a second algorithm
    inst = synth.config_instance("small", seed=5)
    qs = synth.batch_queries(inst, 150, seed=5, start_max=7, len_min=1, len_max=8, algos=(0,))
    qs += synth.batch_queries(inst, 10, seed=6, start_max=7, len_min=1, len_max=8, algos=(1,))
    rep = oracle.replay(inst)
    _check_batch(evq, inst, qs, 1, rep=rep, vs_oracle=False)
    # oracle on a sample spanning the groups
    _check_batch(evq, inst, [qs[i] for i in (0, 49, 50, 99, 100, 149, 150, 159)], 1, rep=rep)


@pytest.mark.parametrize("lanes", [1, 2])
def test_batch_two_word_masks(evq, lanes):
    # K = 100: windows inside word 0, inside word 1 and across the boundary
    inst = synth.random_instance(300, 2400, 100, 6, 6, 50, 17)
    src = synth.pick_sources(inst, 6, seed=3)
    qs = [(0, src[0], 0, 100), (1, src[1], 60, 10), (2, src[2], 64, 36), (3, src[3], 10, 54),
          (0, src[4], 63, 2), (2, src[5], 99, 1), (3, src[0], 0, 64), (1, src[2], 30, 70)]
    _check_batch(evq, inst, qs, lanes)


def test_batch_degenerate(evq):
    # a source with no out-edges, length-1 windows, one query, and an empty-batch instance
    inst = synth.random_instance(50, 120, 5, 3, 3, 9, 23)
    deg = np.bincount(inst.base[:, 0], minlength=50)
    lonely = int(np.flatnonzero(deg == 0)[0])
    qs = [(0, lonely, 0, 5), (1, 0, 2, 1), (2, lonely, 4, 1), (3, 1, 0, 5)]
    _check_batch(evq, inst, qs, 1)
    _check_batch(evq, inst, qs[:1], 1)
    empty = synth.Instance(50, inst.base, [np.zeros((0, 3), np.uint32)] * 4, [np.zeros((0, 3), np.uint32)] * 4)
    _check_batch(evq, empty, [(0, 0, 0, 4), (2, 3, 1, 2)], 1)


def test_batch_rejects_bad_query(evq):
    inst = synth.config_instance("small", seed=1)
    with evq.Graph.from_instance(inst) as g:
        for bad, status in [((0, inst.num_vertices, 0, 1), evq.EVQ_ERANGE), ((0, 0, 0, 9), evq.EVQ_ERANGE),
                            ((7, 0, 0, 1), evq.EVQ_EINVAL), ((0, 0, 8, 1), evq.EVQ_ERANGE)]:
            with pytest.raises(evq.EvqError) as ei:
                g.query_batch([(0, 0, 0, 8), bad])
            assert ei.value.status == status
            assert "query 1" in str(ei.value)


def test_batch_result_free_and_reuse(evq):
    # results outlive later batches; freeing one leaves the others intact
    import torch
    inst = synth.config_instance("small", seed=7)
    qs = synth.batch_queries(inst, 12, seed=7, start_max=7, len_min=1, len_max=8)
    rep = oracle.replay(inst)
    evq.set_batch_config(lanes=1, chunk=8, blocks=2048, group=64)
    with evq.Graph.from_instance(inst) as g:
        r1 = g.query_batch(qs)
        r2 = g.query_batch(qs[::-1])
        r1[0].free()
        r1[0].free()  # a freed result is zeroed; freeing again is allowed
        torch.cuda.synchronize()
        for r, (a, s, b, L) in zip(r2[::-1], qs):
            want = oracle.window_values(inst, a, s, b, L, replayed=rep)
            assert_equal_values(evq.to_u32(r.expand()).reshape(inst.num_vertices, L), want, str((a, s, b, L)))
        for r, (a, s, b, L) in list(zip(r1, qs))[1:]:
            want = oracle.window_values(inst, a, s, b, L, replayed=rep)
            assert_equal_values(evq.to_u32(r.expand()).reshape(inst.num_vertices, L), want, str((a, s, b, L)))


def test_batch_autotune_installs_a_valid_choice(evq):
    import torch
    inst = synth.config_instance("small", seed=8)
    qs = synth.batch_queries(inst, 48, seed=8, start_max=7, len_min=1, len_max=8)
    rep = oracle.replay(inst)
    with evq.Graph.from_instance(inst) as g:
        cfg, ms = g.autotune_batch(qs)
        assert cfg == evq.batch_config()
        assert cfg["lanes"] in (1, 2) and cfg["chunk"] in (4, 8, 16) and 64 <= cfg["blocks"] <= 16384 and ms > 0
        res = g.query_batch(qs)
        torch.cuda.synchronize()
        for r, (a, s, b, L) in zip(res, qs):
            want = oracle.window_values(inst, a, s, b, L, replayed=rep)
            assert_equal_values(evq.to_u32(r.expand()).reshape(inst.num_vertices, L), want, str((a, s, b, L)))
            r.free()
    evq.set_batch_config(lanes=1, chunk=8, blocks=2048, group=64)
