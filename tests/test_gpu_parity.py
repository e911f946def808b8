"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit-exact.

Sizes span several tiles of every kernel and leave ragged tails; edge cases
cover empty and degenerate inputs.  All values are uint32 and exact, so the
tolerance is zero.
"""
import numpy as np
import pytest

import oracle
import synth
from fixtures import empty_batches_instance, instance_from, load_golden
from gpu_util import assert_equal_values, gpu_bounds, gpu_values, oracle_triples, union_triples_from_export

pytestmark = pytest.mark.gpu

ALGOS = [oracle.SSSP, oracle.BFS, oracle.SSWP, oracle.SSNP, oracle.VITERBI]


@pytest.fixture(scope="module")
def evq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_10579_amd as m
    return m


def _graph(evq, inst):
    return evq.Graph.from_instance(inst)


# ------------------------------------------------------------------ K1: versioned graph


def _check_export(g, inst):
    ex = g.export()
    K = inst.K
    V = inst.num_vertices
    rp = ex["row_ptr"].astype(np.int64)
    assert rp[0] == 0 and rp[-1] == len(ex["col"]) and (np.diff(rp) >= 0).all()
    assert ((ex["row_split"] >= rp[:-1]) & (ex["row_split"] <= rp[1:])).all()
    full = (1 << K) - 1
    # all-present edges first within each row, then the partial ones
    for u in range(V):
        for j in range(rp[u], rp[u + 1]):
            m = int(ex["mask"][j, 0]) | ((int(ex["mask"][j, 1]) << 64) if ex["mask"].shape[1] == 2 else 0)
            assert (m == full) == (j < ex["row_split"][u]), (u, j)
    got = union_triples_from_export(ex, K)
    want = oracle_triples(inst)
    assert got == want
    info = g.info
    assert info["num_edges"] == len(want)
    assert info["num_partial"] == sum(1 for m in want.values() if m != full)


@pytest.mark.parametrize("seed", [1, 2])
def test_versioned_graph_small_config(evq, seed):
    inst = synth.config_instance("small", seed=seed)
    with _graph(evq, inst) as g:
        _check_export(g, inst)


@pytest.mark.parametrize("K", [1, 3, 63, 64, 65, 100, 128])
def test_versioned_graph_mask_widths(evq, K):
    inst = synth.random_instance(40, 300, K, 4, 4, 7, 100 + K)
    with _graph(evq, inst) as g:
        _check_export(g, inst)


def test_versioned_graph_labels_fig7_fig8(evq):
    for case in load_golden("p7_version_labels.json")["cases"]:
        inst = instance_from(case)
        with _graph(evq, inst) as g:
            got = union_triples_from_export(g.export(), inst.K)
        for k, lab in case["labels"].items():
            t = tuple(int(x) for x in k.split(","))
            assert got[t] == int(lab, 2), (case["name"], k)


def test_versioned_graph_wide_ids_and_weights(evq):
    # keys wider than 64 bits (32-bit weights) take the two-word sort path
    rng = np.random.default_rng(5)
    V = 70000
    base = np.stack([rng.integers(0, V, 3000), rng.integers(0, V, 3000),
                     rng.integers(1, 2**32 - 1, 3000, dtype=np.uint64)], 1).astype(np.uint32)
    dels = [base[rng.choice(3000, 50, replace=False)] for _ in range(3)]
    adds = [np.stack([rng.integers(0, V, 60), rng.integers(0, V, 60),
                      rng.integers(1, 2**32 - 1, 60, dtype=np.uint64)], 1).astype(np.uint32) for _ in range(3)]
    inst = synth.Instance(V, base, dels, adds)
    with _graph(evq, inst) as g:
        got = union_triples_from_export(g.export(), 3)
    assert got == oracle_triples(inst)


# ------------------------------------------------------------------ K2: bounds


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("win", [(0, 8), (2, 3), (5, 1)])
def test_bounds_small_config(evq, algo, win):
    inst = synth.config_instance("small", seed=3)
    trip, bits = oracle.replay(inst)
    b, L = win
    rc_o, ru_o = oracle.bounds(inst.num_vertices, trip, bits, algo, 0, b, L)
    with _graph(evq, inst) as g:
        rc, ru = gpu_bounds(g, algo, 0, b, L)
    assert np.array_equal(rc, rc_o)
    assert np.array_equal(ru, ru_o)


# ------------------------------------------------------------------ full method


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_query_small_config(evq, algo, seed):
    inst = synth.config_instance("small", seed=seed)
    trip, bits = oracle.replay(inst)
    want = oracle.window_values(inst, algo, 0, 0, inst.K, replayed=(trip, bits))
    with _graph(evq, inst) as g:
        got = gpu_values(g, algo, 0, 0, inst.K)
        plain = gpu_values(g, algo, 0, 0, inst.K, plain=True)
        seq = gpu_values(g, algo, 0, 0, inst.K, sequential=True)
    assert_equal_values(got, want, f"algo {algo} seed {seed}")
    assert_equal_values(plain, want, f"plain algo {algo} seed {seed}")
    assert_equal_values(seq, want, f"sequential algo {algo} seed {seed}")


@pytest.mark.parametrize("algo", ALGOS)
def test_query_small_config_all_seeds_sssp_from_hub(evq, algo):
    # the sources of the small config: vertex 0 (the R-MAT hub) over seeds 6..20
    for seed in range(6, 21):
        inst = synth.config_instance("small", seed=seed)
        want = oracle.window_values(inst, algo, 0, 0, inst.K)
        with _graph(evq, inst) as g:
            got = gpu_values(g, algo, 0, 0, inst.K)
        assert_equal_values(got, want, f"algo {algo} seed {seed}")


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("K,b,L", [(20, 3, 17), (40, 0, 40), (64, 0, 64), (70, 2, 64), (100, 0, 100),
                                   (128, 0, 128), (128, 27, 100), (128, 60, 9), (12, 11, 1)])
def test_query_lane_layouts(evq, algo, K, b, L):
    inst = synth.rmat_instance(11, 12000, K, 12, 12, wmin=1, wmax=30, seed=K + b)
    src = synth.pick_sources(inst, 1, seed=K)[0]
    want = oracle.window_values(inst, algo, src, b, L)
    with _graph(evq, inst) as g:
        got = gpu_values(g, algo, src, b, L)
        plain = gpu_values(g, algo, src, b, L, plain=True)
        seq = gpu_values(g, algo, src, b, L, sequential=True)
    assert_equal_values(got, want, f"algo {algo} K {K} window [{b},{b + L})")
    assert_equal_values(plain, want, f"plain algo {algo} K {K} window [{b},{b + L})")
    assert_equal_values(seq, want, f"sequential algo {algo} K {K} window [{b},{b + L})")


def test_worked_example(evq):
    gd = load_golden("p6_worked_example.json")
    inst = instance_from(gd)
    with _graph(evq, inst) as g:
        rc, ru = gpu_bounds(g, oracle.SSSP, 0, 0, 2)
        vals = gpu_values(g, oracle.SSSP, 0, 0, 2)
    assert rc.tolist() == gd["expect"]["r_cap"]
    assert ru.tolist() == gd["expect"]["r_cup"]
    assert vals.tolist() == gd["expect"]["values"]


# ------------------------------------------------------------------ edge cases


@pytest.mark.parametrize("algo", ALGOS)
def test_empty_batches_all_stable(evq, algo):
    inst = empty_batches_instance(synth.config_instance("small", seed=7))
    want = oracle.window_values(inst, algo, 0, 0, inst.K)
    with _graph(evq, inst) as g:
        got, st = gpu_values(g, algo, 0, 0, inst.K, stats=True)
    assert_equal_values(got, want)
    assert st["n_unstable"] == 0


@pytest.mark.parametrize("algo", ALGOS)
def test_tiny_and_degenerate_graphs(evq, algo):
    cases = [
        synth.Instance(1, np.zeros((0, 3), np.uint32), [np.zeros((0, 3), np.uint32)],
                       [np.zeros((0, 3), np.uint32)]),
        synth.Instance(1, np.array([[0, 0, 5]], np.uint32), [np.zeros((0, 3), np.uint32)] * 2,
                       [np.zeros((0, 3), np.uint32)] * 2),
        # every edge deleted in the first batch
        synth.Instance(3, np.array([[0, 1, 2], [1, 2, 2]], np.uint32),
                       [np.array([[0, 1, 2], [1, 2, 2]], np.uint32)], [np.zeros((0, 3), np.uint32)]),
        # source without out-edges
        synth.Instance(4, np.array([[1, 2, 3], [2, 0, 4]], np.uint32), [np.zeros((0, 3), np.uint32)] * 3,
                       [np.array([[3, 1, 1]], np.uint32), np.zeros((0, 3), np.uint32),
                        np.zeros((0, 3), np.uint32)]),
    ]
    for ci, inst in enumerate(cases):
        want = oracle.window_values(inst, algo, 0, 0, inst.K)
        with _graph(evq, inst) as g:
            got = gpu_values(g, algo, 0, 0, inst.K)
        assert_equal_values(got, want, f"case {ci}")


@pytest.mark.parametrize("algo", ALGOS)
def test_random_multigraphs(evq, algo):
    for seed in range(12):
        rng = np.random.default_rng(seed)
        V = int(rng.integers(2, 300))
        K = int(rng.choice([1, 2, 5, 33, 64, 65, 128]))
        inst = synth.random_instance(V, int(rng.integers(0, 4 * V)), K, int(rng.integers(0, 6)),
                                     int(rng.integers(0, 6)), int(rng.choice([1, 3, 50])), seed)
        b = int(rng.integers(0, K))
        L = int(rng.integers(1, K - b + 1))
        s = int(rng.integers(0, V))
        want = oracle.window_values(inst, algo, s, b, L)
        with _graph(evq, inst) as g:
            got = gpu_values(g, algo, s, b, L)
        assert_equal_values(got, want, f"seed {seed} V {V} K {K} [{b},{b + L}) s {s}")


def test_invalid_arguments_return_codes(evq):
    inst = synth.config_instance("small", seed=1)
    with _graph(evq, inst) as g:
        for args in [(0, 4096, 0, 8), (0, 0, 0, 9), (0, 0, 8, 1), (0, 0, 3, 0)]:
            with pytest.raises(evq.EvqError) as ei:
                g.query(*args)
            assert ei.value.status == evq.EVQ_ERANGE
        with pytest.raises(evq.EvqError) as ei:
            g.query(7, 0, 0, 8)
        assert ei.value.status == evq.EVQ_EINVAL


def test_determinism_repeat(evq):
    inst = synth.config_instance("small", seed=2)
    with _graph(evq, inst) as g:
        a = gpu_values(g, oracle.SSSP, 0, 0, 8)
        for _ in range(3):
            assert np.array_equal(a, gpu_values(g, oracle.SSSP, 0, 0, 8))


def test_gather_ceiling_measurement(evq):
    # measurement entry point: a positive rate, 0 on a graph without edges,
    # argument errors, and the graph (only read) answers the same afterwards
    inst = synth.config_instance("small", seed=2)
    with _graph(evq, inst) as g:
        a = gpu_values(g, oracle.SSSP, 0, 0, 8)
        assert g.gather_ceiling(2) > 0
        with pytest.raises(evq.EvqError) as ei:
            g.gather_ceiling(0)
        assert ei.value.status == evq.EVQ_EINVAL
        assert np.array_equal(a, gpu_values(g, oracle.SSSP, 0, 0, 8))
    empty = synth.Instance(1, np.zeros((0, 3), np.uint32), [np.zeros((0, 3), np.uint32)],
                           [np.zeros((0, 3), np.uint32)])
    with _graph(evq, empty) as g:
        assert g.gather_ceiling(1) == 0.0


@pytest.mark.parametrize("delta,heavy", [(1, 0), (7, 0), (60, 0), (3, 4), (20, 2)])
@pytest.mark.parametrize("algo", ALGOS)
def test_near_far_scheduling(evq, algo, delta, heavy, tuned):
    # near/far ordering of the bound solves (every vertex gated, or only those
    # with at least `heavy` edges) changes the schedule, never the values
    tuned(delta=delta, heavy=heavy)
    for seed in (1, 2):
        inst = synth.config_instance("small", seed=seed)
        trip, bits = oracle.replay(inst)
        want = oracle.window_values(inst, algo, 0, 0, inst.K, replayed=(trip, bits))
        rc_o, ru_o = oracle.bounds(inst.num_vertices, trip, bits, algo, 0, 0, inst.K)
        with _graph(evq, inst) as g:
            got = gpu_values(g, algo, 0, 0, inst.K)
            rc, ru = gpu_bounds(g, algo, 0, 0, inst.K)
            sub = gpu_values(g, algo, 0, 2, 5)
        assert_equal_values(got, want, f"delta {delta} seed {seed}")
        assert np.array_equal(rc, rc_o) and np.array_equal(ru, ru_o)
        assert_equal_values(sub, want[:, 2:7], f"delta {delta} seed {seed} window [2,7)")


@pytest.mark.parametrize("algo", ALGOS)
def test_heavy_gating_many_blocks(evq, algo, tuned):
    # only vertices with >= 16 edges deferred, threshold following the frontier
    inst = synth.rmat_instance(15, 200000, 16, 150, 150, wmin=1, wmax=100, seed=37)
    src = synth.pick_sources(inst, 1, seed=5)[0]
    trip, bits = oracle.replay(inst)
    delta = {oracle.BFS: 1, oracle.VITERBI: 1 << 23}.get(algo, 20)
    tuned(delta=delta, heavy=16)
    for (b, L) in [(0, 16), (5, 7)]:
        want = oracle.window_values(inst, algo, src, b, L, replayed=(trip, bits))
        rc_o, ru_o = oracle.bounds(inst.num_vertices, trip, bits, algo, src, b, L)
        with _graph(evq, inst) as g:
            got = gpu_values(g, algo, src, b, L)
            rc, ru = gpu_bounds(g, algo, src, b, L)
        assert_equal_values(got, want, f"heavy gating algo {algo} [{b},{b + L})")
        assert np.array_equal(rc, rc_o) and np.array_equal(ru, ru_o)


@pytest.mark.parametrize("frac", [0.0, 0.3, 2.0])
@pytest.mark.parametrize("algo", ALGOS)
def test_pull_step(evq, algo, frac, tuned):
    # full-window intersection solve pulling in every iteration (0), in the
    # dense ones (0.3) or never (2): same values and bounds as the oracle, on
    # small graphs and on one with hubs and many waves per slice (SSSP with
    # its bucketed schedule off, which never pulls)
    tuned(pull_frac=frac, bucket_width=0)
    cases = [(synth.config_instance("small", seed=s), 0) for s in (1, 2, 3)]
    big = synth.rmat_instance(15, 200000, 16, 150, 150, wmin=1, wmax=100, seed=41)
    cases.append((big, synth.pick_sources(big, 1, seed=3)[0]))
    for ci, (inst, src) in enumerate(cases):
        trip, bits = oracle.replay(inst)
        want = oracle.window_values(inst, algo, src, 0, inst.K, replayed=(trip, bits))
        rc_o, ru_o = oracle.bounds(inst.num_vertices, trip, bits, algo, src, 0, inst.K)
        with _graph(evq, inst) as g:
            got = gpu_values(g, algo, src, 0, inst.K)  # pushes only: the reverse CSR is not built yet
            held = g.info["device_bytes"]
            rc, ru = gpu_bounds(g, algo, src, 0, inst.K)  # builds it (unless the pull step is off)
            grown = g.info["device_bytes"] - held
            again = gpu_values(g, algo, src, 0, inst.K)  # reverse CSR reused
            assert g.info["device_bytes"] - held == grown
        assert (grown > 0) == (frac <= 1.0), (frac, grown)
        assert_equal_values(got, want, f"pull {frac} case {ci}")
        assert_equal_values(again, want, f"pull {frac} case {ci} second query")
        assert np.array_equal(rc, rc_o) and np.array_equal(ru, ru_o)


def _indegree_pattern_instance():
    # 16,384 vertices whose in-degrees cycle through counts on both sides of
    # multiples of 64 (0 ... 700, about 3.5M edges from uniform sources,
    # weights 1..100), so that the pull step's slices span several 64-edge
    # steps and destinations run across step and slice ends at every offset;
    # 4 snapshots of 2,000 deletions of base edges and 2,000 additions
    rng = np.random.default_rng(20250210)
    V = 1 << 14
    pattern = np.array([0, 1, 2, 3, 63, 64, 65, 127, 128, 129, 191, 192, 193, 255, 256, 257, 320, 511, 512,
                        513, 700])
    deg = pattern[np.arange(V) % len(pattern)]
    dst = np.repeat(np.arange(V), deg)
    src = rng.integers(0, V, len(dst))
    w = rng.integers(1, 101, len(dst))
    base = np.stack([src, dst, w], axis=1).astype(np.uint32)
    dels, adds = [], []
    for _ in range(4):
        dels.append(base[rng.choice(len(base), 2000, replace=False)].copy())
        adds.append(np.stack([rng.integers(0, V, 2000), rng.integers(0, V, 2000), rng.integers(1, 101, 2000)],
                             axis=1).astype(np.uint32))
    return synth.Instance(V, base, dels, adds)


@pytest.fixture(scope="module")
def indegree_case():
    inst = _indegree_pattern_instance()
    trip, bits = oracle.replay(inst)
    want = {}
    for algo in ALGOS:
        want[algo] = (oracle.window_values(inst, algo, 5, 0, inst.K, replayed=(trip, bits)),
                      oracle.bounds(inst.num_vertices, trip, bits, algo, 5, 0, inst.K))
    return inst, want


@pytest.mark.parametrize("frac", [0.0, 0.3])
@pytest.mark.parametrize("algo", ALGOS)
def test_pull_step_multi_step_slices(evq, algo, frac, tuned, indegree_case):
    # the pull step where each wave's slice holds several 64-edge steps (its
    # loads run four steps ahead): values and bounds equal the oracle's
    tuned(pull_frac=frac, bucket_width=0)
    inst, want = indegree_case
    vals_o, (rc_o, ru_o) = want[algo]
    with _graph(evq, inst) as g:
        first = gpu_values(g, algo, 5, 0, inst.K)  # pushes only
        rc, ru = gpu_bounds(g, algo, 5, 0, inst.K)  # builds the reverse CSR
        got = gpu_values(g, algo, 5, 0, inst.K)
    assert_equal_values(first, vals_o, f"push only, algo {algo}")
    assert np.array_equal(rc, rc_o) and np.array_equal(ru, ru_o), f"bounds, pull {frac}, algo {algo}"
    assert_equal_values(got, vals_o, f"pull {frac}, algo {algo}")


def _device_u32(ptr, n):
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    out = np.empty(max(n, 1), np.uint32)
    if n:
        rc = hip.hipMemcpy(ctypes.c_void_p(out.ctypes.data), ctypes.c_void_p(ptr), ctypes.c_size_t(n * 4), 2)
        assert rc == 0, rc
    return out[:n]


@pytest.mark.parametrize("order", [0, 1])
def test_vertex_numbering(evq, order, tuned):
    # a graph numbered by degree inside (1) or in the caller's ids (0):
    # values, both bounds, compact results (the intersection bound in vertex
    # order, the unstable vertices as caller ids: those whose two bounds
    # differ), the export, and values after an append, all in the caller's
    # numbering and equal to the oracle's
    tuned(vertex_order=order)
    full = synth.rmat_instance(12, 40000, 9, 300, 300, wmin=1, wmax=60, seed=91)
    inst = synth.Instance(full.num_vertices, full.base, full.dels[:8], full.adds[:8])
    V, K = inst.num_vertices, inst.K
    srcs = synth.pick_sources(inst, 2, seed=9)
    trip, bits = oracle.replay(inst)
    with _graph(evq, inst) as g:
        for algo in ALGOS:
            for s in srcs:
                want = oracle.window_values(inst, algo, s, 1, 6, replayed=(trip, bits))
                assert_equal_values(gpu_values(g, algo, s, 1, 6), want, f"order {order} algo {algo} src {s}")
                rc, ru = gpu_bounds(g, algo, s, 0, K)
                rc_o, ru_o = oracle.bounds(V, trip, bits, algo, s, 0, K)
                assert np.array_equal(rc, rc_o) and np.array_equal(ru, ru_o)
        qs = [(algo, s, 0, K) for algo in ALGOS for s in srcs]
        for (algo, s, b, L), r in zip(qs, g.query_batch(qs)):
            want = oracle.window_values(inst, algo, s, b, L, replayed=(trip, bits))
            assert_equal_values(evq.to_u32(r.expand()).reshape(V, L), want, f"order {order} compact {algo}")
            rc_o, ru_o = oracle.bounds(V, trip, bits, algo, s, b, L)
            assert np.array_equal(_device_u32(r._c.d_rcap, V), rc_o)
            ids = _device_u32(r._c.d_unstable, r._c.n_unstable)
            assert np.array_equal(np.sort(ids), np.flatnonzero(rc_o != ru_o).astype(np.uint32))
            r.free()
        _check_export(g, inst)
        g.append(full.dels[8], full.adds[8])
        for algo in ALGOS:
            want = oracle.window_values(full, algo, srcs[0], 1, K)
            assert_equal_values(gpu_values(g, algo, srcs[0], 1, K), want, f"order {order} after append")


@pytest.mark.parametrize("width", [0, 1, 3, 17, 100000, 0xFFFFFFFF])
def test_bucketed_sssp(evq, width, tuned):
    # SSSP intersection solves under delta-stepping with light and heavy edges (bucket width 1:
    # every edge of weight > 1 heavy; 100000: every edge light, plain thresholds; the graph's
    # automatic width; 0: off), full window and sub-windows (which also walk the window-partial
    # edges with the light ones), one- and two-word masks, against the oracle; on the graph with
    # hubs the schedule visits fewer edges than plain frontier iterations
    tuned(bucket_width=width)
    cases = [(synth.config_instance("small", seed=s), 0, [(0, 8), (2, 5), (7, 1)]) for s in (1, 2)]
    big = synth.rmat_instance(15, 200000, 16, 150, 150, wmin=1, wmax=100, seed=41)
    cases.append((big, synth.pick_sources(big, 1, seed=3)[0], [(0, 16), (3, 9)]))
    wide = synth.rmat_instance(12, 40000, 100, 60, 60, wmin=1, wmax=1000, seed=43)
    cases.append((wide, synth.pick_sources(wide, 1, seed=2)[0], [(0, 100), (10, 70), (64, 36)]))
    for ci, (inst, src, wins) in enumerate(cases):
        trip, bits = oracle.replay(inst)
        with _graph(evq, inst) as g:
            for b, L in wins:
                want = oracle.window_values(inst, oracle.SSSP, src, b, L, replayed=(trip, bits))
                rc_o, ru_o = oracle.bounds(inst.num_vertices, trip, bits, oracle.SSSP, src, b, L)
                for rep in range(2):  # the first query builds the weight-ordered rows, the second reuses them
                    got = gpu_values(g, oracle.SSSP, src, b, L)
                    assert_equal_values(got, want, f"width {width} case {ci} [{b},{b + L}) query {rep}")
                rc, ru = gpu_bounds(g, oracle.SSSP, src, b, L)
                assert np.array_equal(rc, rc_o) and np.array_equal(ru, ru_o), (width, ci, b, L)
    if width in (3, 17):
        visits = {}
        with _graph(evq, big) as g:
            src = cases[2][1]
            for w in (0, width):
                tuned(bucket_width=w)
                _, st = gpu_values(g, oracle.SSSP, src, 0, big.K, stats=True)
                visits[w] = st["edges_cap"]
        assert visits[width] < visits[0], visits


@pytest.mark.parametrize("staged", [0, 2, 4])
@pytest.mark.parametrize("algo", ALGOS)
def test_relax_staged_tasks(evq, algo, staged, tuned):
    # the relaxation with the block's tasks staged in LDS (2 or 4 per lane group) or each
    # lane group loading its own (0), for every lane layout (8 to 128 lanes per group);
    # heavy churn so that the reduced subgraph spans many blocks, two-word masks at K = 100
    tuned(relax_staged=staged)
    inst = synth.rmat_instance(14, 120000, 100, 400, 400, wmin=1, wmax=100, seed=53)
    src = synth.pick_sources(inst, 2, seed=8)
    trip, bits = oracle.replay(inst)
    with _graph(evq, inst) as g:
        for s_ in src:
            for (b, L) in [(0, 100), (3, 64), (30, 70), (50, 7), (5, 9), (10, 16), (20, 32), (40, 40)]:
                want = oracle.window_values(inst, algo, s_, b, L, replayed=(trip, bits))
                got, st = gpu_values(g, algo, s_, b, L, stats=True)
                assert_equal_values(got, want, f"staged {staged} algo {algo} [{b},{b + L})")
                assert st["n_unstable"] > 0


@pytest.mark.parametrize("append_edges", [0, 64, 1 << 30])
@pytest.mark.parametrize("algo", ALGOS)
def test_appending_expansions(evq, algo, append_edges, tuned):
    # the bound solves' sparse iterations list the next frontier themselves (every
    # iteration, those of at most 64 frontier edges, or none): same values and bounds,
    # for the full window (with and without the pull step) and a sub-window
    tuned(append_edges=append_edges)
    big = synth.rmat_instance(15, 200000, 16, 150, 150, wmin=1, wmax=100, seed=47)
    cases = [(synth.config_instance("small", seed=4), 0), (big, synth.pick_sources(big, 1, seed=6)[0])]
    for ci, (inst, src) in enumerate(cases):
        trip, bits = oracle.replay(inst)
        rc_o, ru_o = oracle.bounds(inst.num_vertices, trip, bits, algo, src, 0, inst.K)
        want = oracle.window_values(inst, algo, src, 0, inst.K, replayed=(trip, bits))
        with _graph(evq, inst) as g:
            for rep in range(3):  # the second full-window query builds the reverse CSR of the pull step
                got = gpu_values(g, algo, src, 0, inst.K)
                assert_equal_values(got, want, f"append {append_edges} case {ci} query {rep}")
            rc, ru = gpu_bounds(g, algo, src, 0, inst.K)
            sub = gpu_values(g, algo, src, 1, inst.K - 3)
        assert np.array_equal(rc, rc_o) and np.array_equal(ru, ru_o)
        assert_equal_values(sub, want[:, 1:inst.K - 2], f"append {append_edges} case {ci} sub-window")


@pytest.mark.parametrize("direct", [0, 1000000000])
@pytest.mark.parametrize("algo", ALGOS)
def test_relax_task_paths(evq, algo, direct, tuned):
    # relaxation tasks written by a kernel of their own (limit 0) or by the
    # compaction (a limit above any task count): same values
    tuned(direct_tasks=direct)
    inst = synth.rmat_instance(15, 200000, 16, 2000, 2000, wmin=1, wmax=100, seed=41)
    src = synth.pick_sources(inst, 2, seed=9)
    trip, bits = oracle.replay(inst)
    with _graph(evq, inst) as g:
        for s in src:
            for (b, L) in [(0, 16), (4, 9)]:
                want = oracle.window_values(inst, algo, s, b, L, replayed=(trip, bits))
                assert_equal_values(gpu_values(g, algo, s, b, L), want, f"tasks limit {direct} algo {algo} [{b},{b + L})")
                assert_equal_values(gpu_values(g, algo, s, b, L, plain=True), want, f"plain, limit {direct}")
    small = synth.config_instance("small", seed=3)
    with _graph(evq, small) as g:
        want = oracle.window_values(small, algo, 0, 0, small.K)
        assert_equal_values(gpu_values(g, algo, 0, 0, small.K), want, f"small, limit {direct}")


@pytest.mark.parametrize("algo", ALGOS)
def test_query_many_blocks_method_plain_sequential(evq, algo):
    # enough vertices that compact ids are assigned by many blocks in any order
    inst = synth.rmat_instance(15, 200000, 16, 150, 150, wmin=1, wmax=100, seed=31)
    src = synth.pick_sources(inst, 1, seed=3)[0]
    trip, bits = oracle.replay(inst)
    for (b, L) in [(0, 16), (3, 9)]:
        want = oracle.window_values(inst, algo, src, b, L, replayed=(trip, bits))
        with _graph(evq, inst) as g:
            got = gpu_values(g, algo, src, b, L)
            plain = gpu_values(g, algo, src, b, L, plain=True)
            seq = gpu_values(g, algo, src, b, L, sequential=True)
        assert_equal_values(got, want, f"algo {algo} [{b},{b + L})")
        assert_equal_values(plain, want, f"plain algo {algo} [{b},{b + L})")
        assert_equal_values(seq, want, f"sequential algo {algo} [{b},{b + L})")


@pytest.mark.parametrize("algo", ALGOS)
@pytest.mark.parametrize("K,b,L,min_len", [(20, 3, 17, 2), (64, 0, 64, 8), (100, 13, 87, 3), (128, 0, 128, 1)])
def test_split_subwindows_equal_oracle(evq, algo, K, b, L, min_len, tuned):
    # a threshold of 0 unstable vertices forces every window of 2 * min_len or more to split, to depth 4
    inst = synth.rmat_instance(11, 12000, K, 12, 12, wmin=1, wmax=30, seed=K + b + 7)
    src = synth.pick_sources(inst, 1, seed=K + 1)[0]
    want = oracle.window_values(inst, algo, src, b, L)
    tuned(split_frac=1e-9, split_min=min_len)
    with _graph(evq, inst) as g:
        got, st = gpu_values(g, algo, src, b, L, stats=True)
        tuned(split_frac=0.0)
        one, st1 = gpu_values(g, algo, src, b, L, stats=True)
    assert_equal_values(got, want, f"split algo {algo} K {K} [{b},{b + L})")
    assert_equal_values(one, want, f"unsplit algo {algo} K {K} [{b},{b + L})")
    assert st1["subwindows"] == 1
    if st1["n_unstable"] > 0:
        assert st["subwindows"] > 1
