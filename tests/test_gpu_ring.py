"""GPU parity of the serving store (evq_append): a ring of K mask bits where
snapshot t (global id) lives in bit t mod K.

* After every append the exported versioned graph equals what the oracle's
  replay of the whole update history fixes: each triple's ring mask has bit
  (t mod K) set iff the triple is in global snapshot t, for the K snapshots
  held; triples in none of them are gone; all-present edges lead each row.
* Queries over windows that wrap around the ring (single, batched with
  shared bound solves and with one solve per query) equal the oracle's
  per-snapshot values.
* Results taken before an append stay valid after it; a rejected append
  leaves the graph unchanged.
Rings of K = 8, 64 (one mask word), 100 and 128 (two words).  When the
history exceeds the oracle's 128 snapshots, the instance is re-based: the
snapshot before the oldest one held becomes the base.  Values are uint32:
tolerance zero.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_equal_values, union_triples_from_export

pytestmark = pytest.mark.gpu

ALGOS = [oracle.SSSP, oracle.BFS, oracle.SSWP, oracle.SSNP, oracle.VITERBI]


@pytest.fixture(scope="module")
def evq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_10579_amd as m
    yield m
    m.set_batch_config(lanes=1, chunk=8, blocks=2048, group=64)


def head(inst, K):
    return synth.Instance(inst.num_vertices, inst.base, inst.dels[:K], inst.adds[:K])


def rebase(inst, A):
    """Instance whose snapshot i is snapshot A + i of `inst` (base = its snapshot A - 1)."""
    if A == 0:
        return inst
    trip, bits = oracle.replay(head(inst, A))
    t = A - 1
    keep = ((bits[:, t // 64] >> np.uint64(t % 64)) & np.uint64(1)).astype(bool)
    return synth.Instance(inst.num_vertices, trip[keep].copy(), inst.dels[A:], inst.adds[A:])


def expected_ring(inst, K, first):
    """triple -> ring mask of the K snapshots first .. first+K-1 (oracle replay of the history)."""
    trip, bits = oracle.replay(inst)
    out = {}
    for r, b in zip(trip, bits):
        m = int(b[0]) | (int(b[1]) << 64)
        ring = 0
        for t in range(first, first + K):
            if (m >> t) & 1:
                ring |= 1 << (t % K)
        if ring:
            out[(int(r[0]), int(r[1]), int(r[2]))] = ring
    return out


def check_ring(g, inst, K, first):
    ex = g.export()
    assert g.first == first
    got = union_triples_from_export(ex, K)
    want = expected_ring(inst, K, first)
    assert got == want, f"ring masks differ after reaching first={first}"
    full = (1 << K) - 1
    rp = ex["row_ptr"].astype(np.int64)
    for u in range(len(ex["row_split"])):
        for j in range(rp[u], rp[u + 1]):
            m = int(ex["mask"][j, 0]) | ((int(ex["mask"][j, 1]) << 64) if ex["mask"].shape[1] == 2 else 0)
            assert (m == full) == (j < ex["row_split"][u]), (u, j)
    info = g.info
    assert info["num_partial"] == sum(1 for m in want.values() if m != full)


@pytest.mark.parametrize("K,A", [(8, 13), (64, 40), (100, 28)])
def test_ring_append_masks(evq, K, A):
    inst = synth.random_instance(60, 500, K + A, 5, 5, 9, 300 + K)
    print(f"ring K={K}, {A} appends", flush=True)
    with evq.Graph.from_instance(head(inst, K)) as g:
        check_ring(g, inst, K, 0)
        for a in range(A):
            g.append(inst.dels[K + a], inst.adds[K + a])
            if a in (0, 1, K - 1, K, A - 1) or a % 7 == 0:
                check_ring(g, inst, K, a + 1)


def test_ring_append_128(evq):
    K, A = 128, 20
    inst = synth.random_instance(80, 600, K + A, 4, 4, 9, 77)
    with evq.Graph.from_instance(head(inst, K)) as g:
        for a in range(A):
            g.append(inst.dels[K + a], inst.adds[K + a])
        reb = rebase(inst, A)  # its snapshot i is global snapshot A + i
        ex = g.export()
        got = union_triples_from_export(ex, K)
        trip, bits = oracle.replay(reb)
        want = {}
        for r, b in zip(trip, bits):
            m = int(b[0]) | (int(b[1]) << 64)
            ring = 0
            for i in range(K):
                if (m >> i) & 1:
                    ring |= 1 << ((A + i) % K)
            if ring:
                want[(int(r[0]), int(r[1]), int(r[2]))] = ring
        assert got == want


def _windows(first, K, rng, n):
    out = []
    for _ in range(n):
        L = int(rng.integers(1, K + 1))
        b = first + int(rng.integers(0, K - L + 1))
        out.append((b, L))
    return out


@pytest.mark.parametrize("K,A", [(8, 13), (64, 30), (100, 27)])
def test_ring_queries_wrap(evq, K, A):
    import torch
    inst = synth.random_instance(70, 700, K + A, 6, 6, 9, 500 + K)
    rep = oracle.replay(inst)  # global snapshot ids
    rng = np.random.default_rng(K)
    with evq.Graph.from_instance(head(inst, K)) as g:
        for a in range(A):
            g.append(inst.dels[K + a], inst.adds[K + a])
        first = g.first
        wins = _windows(first, K, rng, 10) + [(first, K), (first + K - 1, 1)]
        src = synth.pick_sources(inst, len(wins), seed=K)
        qs = [(ALGOS[i % 5], src[i], b, L) for i, (b, L) in enumerate(wins)]
        wrapped = sum(1 for (_, _, b, L) in qs if (b % K) + L > K)
        print(f"ring K={K} first={first}: {len(qs)} windows, {wrapped} wrap", flush=True)
        want = [oracle.window_values(inst, a, s, b, L, replayed=rep) for (a, s, b, L) in qs]
        for (a, s, b, L), w in zip(qs, want):
            got = evq.to_u32(g.query(a, s, b, L)).reshape(inst.num_vertices, L)
            assert_equal_values(got, w, f"single {(a, s, b, L)}")
        for lanes in (1, 2):
            evq.set_batch_config(lanes=lanes)
            res = g.query_batch(qs)
            torch.cuda.synchronize()
            for r, (a, s, b, L), w in zip(res, qs, want):
                got = evq.to_u32(r.expand()).reshape(inst.num_vertices, L)
                assert_equal_values(got, w, f"batch lanes={lanes} {(a, s, b, L)}")
                r.free()


def test_ring_queries_128(evq):
    K, A = 128, 9
    inst = synth.random_instance(90, 900, K + A, 5, 5, 9, 91)
    with evq.Graph.from_instance(head(inst, K)) as g:
        for a in range(A):
            g.append(inst.dels[K + a], inst.adds[K + a])
        reb = rebase(inst, A)
        rep = oracle.replay(reb)
        qs = [(0, 3, A + 100, 28), (2, 5, A + 119, 9), (3, 7, A, 128), (1, 11, A + 64, 64), (0, 13, A + 127, 1)]
        for (a, s, b, L) in qs:
            want = oracle.window_values(reb, a, s, b - A, L, replayed=rep)
            got = evq.to_u32(g.query(a, s, b, L)).reshape(inst.num_vertices, L)
            assert_equal_values(got, want, f"K=128 {(a, s, b, L)}")


def test_ring_old_results_and_bad_append(evq):
    import torch
    K, A = 16, 5
    inst = synth.random_instance(50, 400, K + A, 4, 4, 9, 13)
    rep = oracle.replay(inst)
    with evq.Graph.from_instance(head(inst, K)) as g:
        qs = [(0, 1, 2, 10), (3, 2, 0, 16)]
        res = g.query_batch(qs)
        for a in range(A):
            g.append(inst.dels[K + a], inst.adds[K + a])
        torch.cuda.synchronize()
        for r, (a, s, b, L) in zip(res, qs):
            want = oracle.window_values(inst, a, s, b, L, replayed=rep)
            assert_equal_values(evq.to_u32(r.expand()).reshape(50, L), want, "result taken before the appends")
            r.free()
        before = g.export()
        with pytest.raises(evq.EvqError) as ei:
            g.append(np.zeros((0, 3), np.uint32), np.array([[1, 50, 3]], np.uint32))
        assert ei.value.status == evq.EVQ_EINVAL
        with pytest.raises(evq.EvqError):
            g.query(0, 0, 0, 4)  # snapshot 0 is no longer held
        after = g.export()
        assert g.first == A
        for k in before:
            assert np.array_equal(before[k], after[k])


def _appended_pair(evq, inst, K, batches):
    """Apply batches to two copies of the same ring, incrementally and by a full
    rebuild (evq_tuning.append_rebuild); yield both exports after each append."""
    with evq.Graph.from_instance(head(inst, K)) as g1, evq.Graph.from_instance(head(inst, K)) as g2:
        for dels, adds in batches:
            g1.append(dels, adds)
            with evq.tuning(append_rebuild=1):
                g2.append(dels, adds)
            yield g1, g2


@pytest.mark.parametrize("K,A", [(8, 13), (64, 20), (100, 9), (128, 5)])
def test_ring_incremental_equals_rebuild(evq, K, A):
    # the incremental append (events sorted and looked up, masks updated in one
    # pass, edges placed by rank) produces the same arrays as a full rebuild
    inst = synth.random_instance(90, 900, K + A, 6, 6, 9, 700 + K)
    batches = [(inst.dels[K + a], inst.adds[K + a]) for a in range(A)]
    for i, (g1, g2) in enumerate(_appended_pair(evq, inst, K, batches)):
        e1, e2 = g1.export(), g2.export()
        for k in e1:
            assert np.array_equal(e1[k], e2[k]), f"append {i}: {k} differs"
        assert g1.info["num_partial"] == g2.info["num_partial"]


def test_ring_incremental_odd_batches(evq):
    # deletions of absent triples, additions of held ones, repeated events,
    # empty batches, a vertex's whole row deleted
    K = 6
    inst = synth.random_instance(40, 300, K, 4, 4, 9, 17)
    trip, bits = oracle.replay(inst)
    held = [tuple(int(x) for x in t) for t, b in zip(trip, bits)
            if (int(b[0]) >> (K - 1)) & 1]
    rng = np.random.default_rng(3)
    row0 = [t for t in held if t[0] == held[0][0]]
    absent = [(1, 2, 9), (3, 3, 1), (39, 0, 7)]
    batches = [
        (np.array(absent, np.uint32), np.zeros((0, 3), np.uint32)),
        (np.zeros((0, 3), np.uint32), np.array(held[:5] + held[:2], np.uint32)),
        (np.array(row0 + row0[:1], np.uint32), np.array(absent + absent[:1], np.uint32)),
        (np.zeros((0, 3), np.uint32), np.zeros((0, 3), np.uint32)),
        (np.array(held[5:9], np.uint32), np.array(held[5:7], np.uint32)),
    ]
    for _ in range(8):
        d = [held[int(i)] for i in rng.integers(0, len(held), 3)]
        a = [(int(rng.integers(0, 40)), int(rng.integers(0, 40)), int(rng.integers(1, 10))) for _ in range(4)]
        batches.append((np.array(d, np.uint32), np.array(a, np.uint32)))
    for i, (g1, g2) in enumerate(_appended_pair(evq, inst, K, batches)):
        e1, e2 = g1.export(), g2.export()
        for k in e1:
            assert np.array_equal(e1[k], e2[k]), f"odd batch {i}: {k} differs"
