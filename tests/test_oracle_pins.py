"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each check uses a definition the oracle does not share: explicit snapshot
sets, simple-path enumeration, Bellman-Ford rounds, threshold reachability,
scipy's Dijkstra, the paper's theorems and its worked-example properties.
"""
import numpy as np
import pytest

import brute
import oracle
import synth
from fixtures import empty_batches_instance, instance_from, load_golden

ALGOS = [oracle.SSSP, oracle.BFS, oracle.SSWP, oracle.SSNP, oracle.VITERBI]
MAX_TYPE = (oracle.SSWP, oracle.VITERBI)
INF = oracle.INF


def _edges_of(trip, bits, t):
    sel = ((bits[:, t >> 6] >> np.uint64(t & 63)) & np.uint64(1)).astype(bool)
    return trip[sel]


# ---------------------------------------------------------------- replay


@pytest.mark.parametrize("seed", range(40))
def test_replay_matches_explicit_sets(seed):
    rng = np.random.default_rng(seed)
    V = int(rng.integers(1, 9))
    K = int(rng.choice([1, 2, 3, 8, 63, 64, 65, 128])) if seed % 4 == 0 else int(rng.integers(1, 7))
    inst = synth.random_instance(V, int(rng.integers(0, 20)), K, int(rng.integers(0, 4)),
                                 int(rng.integers(0, 4)), int(rng.integers(1, 6)), seed)
    trip, bits = oracle.replay(inst)
    sets = brute.snapshot_sets(inst)
    # every triple listed once
    assert len({tuple(map(int, r)) for r in trip}) == len(trip)
    for t in range(K):
        mine = {tuple(map(int, r)) for r in _edges_of(trip, bits, t)}
        assert mine == sets[t], (seed, t)
    # no bit at or beyond K
    for t in range(K, 128):
        assert len(_edges_of(trip, bits, t)) == 0


def test_replay_delete_absent_and_add_present_are_noops():
    inst = instance_from({"num_vertices": 3, "base": [[0, 1, 5]],
                          "batches": [{"del": [[1, 2, 3]], "add": [[0, 1, 5]]},
                                      {"del": [[0, 1, 5]], "add": [[0, 1, 5]]},
                                      {"del": [[0, 1, 5], [0, 1, 5]], "add": []}]})
    trip, bits = oracle.replay(inst)
    assert trip.tolist() == [[0, 1, 5]]
    # present in snapshots 0 and 1 (deleted then re-added within batch 1), absent in 2
    assert int(bits[0, 0]) == 0b011


def test_version_labels_fig7_fig8():
    g = load_golden("p7_version_labels.json")
    for case in g["cases"]:
        inst = instance_from(case)
        trip, bits = oracle.replay(inst)
        K = inst.K
        got = {}
        for r, b in zip(trip, bits):
            lab = "".join("1" if (int(b[t >> 6]) >> (t & 63)) & 1 else "0" for t in reversed(range(K)))
            got[f"{r[0]},{r[1]},{r[2]}"] = lab
        for k, lab in case["labels"].items():
            assert got[k] == lab, (case["name"], k)


# ---------------------------------------------------------------- solves


def _rand_graph(rng, V, m, wmax):
    return [(int(rng.integers(0, V)), int(rng.integers(0, V)), int(rng.integers(1, wmax + 1))) for _ in range(m)]


@pytest.mark.parametrize("algo", ALGOS)
def test_solve_equals_simple_path_enumeration(algo):
    rng = np.random.default_rng(100 + algo)
    for case in range(2500):
        V = int(rng.integers(1, 7))
        e = _rand_graph(rng, V, int(rng.integers(0, 13)), int(rng.choice([1, 3, 9])))
        s = int(rng.integers(0, V))
        got = oracle.solve(V, np.asarray(e, dtype=np.uint32).reshape(-1, 3), algo, s)
        want = brute.enumerate_paths(V, e, algo, s)
        assert (got == want).all(), (algo, case, V, e, s, got, want)


@pytest.mark.parametrize("algo", ALGOS)
def test_solve_equals_bellman_ford(algo):
    rng = np.random.default_rng(200 + algo)
    for case in range(1000):
        V = int(rng.integers(1, 41))
        e = _rand_graph(rng, V, int(rng.integers(0, 4 * V)), int(rng.choice([1, 5, 100])))
        s = int(rng.integers(0, V))
        got = oracle.solve(V, np.asarray(e, dtype=np.uint32).reshape(-1, 3), algo, s)
        want = brute.bellman_ford(V, e, algo, s)
        assert (got == want).all(), (algo, case)


def test_sssp_saturates_instead_of_wrapping():
    e = [(0, 1, 0xF0000000), (1, 2, 0x20000000), (0, 3, 0xFFFFFFFE), (3, 4, 7)]
    got = oracle.solve(5, np.asarray(e, dtype=np.uint32), oracle.SSSP, 0)
    assert got.tolist() == [0, 0xF0000000, oracle.SAT, oracle.SAT, oracle.SAT]
    assert (got == brute.bellman_ford(5, e, oracle.SSSP, 0)).all()


def _rmat_graph(scale, n, seed, wmax):
    e = synth.rmat_edges(scale, n, seed=seed, wmax=wmax)
    return 1 << scale, e


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_closed_forms_on_rmat(seed):
    V, e = _rmat_graph(10, 6000, seed, 50)
    el = [tuple(map(int, r)) for r in e]
    deg = np.bincount(e[:, 0], minlength=V)
    s = int(np.flatnonzero(deg > 0)[seed])
    sssp = oracle.solve(V, e, oracle.SSSP, s)
    assert (sssp == brute.scipy_sssp(V, el, s)).all()
    unit = e.copy()
    unit[:, 2] = 1
    assert (oracle.solve(V, e, oracle.BFS, s) == oracle.solve(V, unit, oracle.SSSP, s)).all()
    assert (oracle.solve(V, e, oracle.SSWP, s) == brute.threshold_widest(V, el, s)).all()
    assert (oracle.solve(V, e, oracle.SSNP, s) == brute.threshold_narrowest(V, el, s)).all()


@pytest.mark.parametrize("seed", [1, 2])
def test_viterbi_closed_forms(seed):
    # weights 2^k: every division is exact while the value stays normal, so the value is 2^-d with d the
    # shortest path in the exponents (scipy, independent of the oracle), or unreachable once d > 126
    V, e = _rmat_graph(10, 6000, seed, 3)
    el = [tuple(map(int, r)) for r in e]
    deg = np.bincount(e[:, 0], minlength=V)
    s = int(np.flatnonzero(deg > 0)[seed])
    d = brute.scipy_sssp(V, el, s).astype(np.int64)
    pw = e.copy()
    pw[:, 2] = 1 << e[:, 2]
    got = oracle.solve(V, pw, oracle.VITERBI, s)
    want = np.zeros(V, dtype=np.uint32)
    ok = (d != INF) & (d <= 126)
    want[ok] = (np.ldexp(np.ones(ok.sum(), dtype=np.float32), -d[ok].astype(np.int32))).view(np.uint32)
    assert (got == want).all()
    # unit weights: 1.0 exactly where reachable
    unit = e.copy()
    unit[:, 2] = 1
    reach = brute.reachable(V, el, s)
    got = oracle.solve(V, unit, oracle.VITERBI, s)
    assert (got == np.where(reach, brute.ONE, 0).astype(np.uint32)).all()


def test_viterbi_rounding_and_underflow():
    # 1/3 rounds to the nearest single; long chains of /100 leave the normal range and become unreachable
    e = [(0, 1, 3), (1, 2, 3)] + [(i, i + 1, 100) for i in range(2, 30)]
    got = oracle.solve(31, np.asarray(e, dtype=np.uint32), oracle.VITERBI, 0)
    assert got[1] == np.array([1 / 3], dtype=np.float32).view(np.uint32)[0]
    third = float(np.array([1 / 3], dtype=np.float32)[0])
    assert got[2] == np.array([third / 3], dtype=np.float32).view(np.uint32)[0]
    assert (got == brute.bellman_ford(31, e, oracle.VITERBI, 0)).all()
    vals = got.view(np.float32)
    assert (vals[vals > 0] >= np.finfo(np.float32).tiny).all() and got[30] == 0 and got[20] != 0


def test_source_without_out_edges():
    e = np.asarray([[1, 2, 3], [2, 0, 4]], dtype=np.uint32)
    for algo in ALGOS:
        got = oracle.solve(3, e, algo, 0)
        src = INF if algo == oracle.SSWP else (brute.ONE if algo == oracle.VITERBI else 0)
        unr = 0 if algo in MAX_TYPE else INF
        assert got.tolist() == [src, unr, unr]


# ---------------------------------------------------------------- query / bounds


def _small():
    return synth.config_instance("small", seed=1)


def test_query_equals_per_snapshot_solve():
    inst = synth.random_instance(30, 120, 5, 6, 6, 20, 11)
    trip, bits = oracle.replay(inst)
    sets = brute.snapshot_sets(inst)
    for algo in ALGOS:
        vals = oracle.window_values(inst, algo, 3, 1, 4, replayed=(trip, bits))
        for i in range(4):
            e = np.asarray(sorted(sets[1 + i]), dtype=np.uint32).reshape(-1, 3)
            assert (vals[:, i] == brute.bellman_ford(30, [tuple(map(int, r)) for r in e], algo, 3)).all()


def test_bounds_are_solves_on_intersection_and_union():
    inst = synth.random_instance(25, 100, 6, 5, 5, 9, 5)
    trip, bits = oracle.replay(inst)
    sets = brute.snapshot_sets(inst)
    b, L = 1, 4
    cap = set.intersection(*sets[b:b + L])
    cup = set.union(*sets[b:b + L])
    for algo in ALGOS:
        rcap, rcup = oracle.bounds(25, trip, bits, algo, 0, b, L)
        assert (rcap == brute.bellman_ford(25, sorted(cap), algo, 0)).all()
        assert (rcup == brute.bellman_ford(25, sorted(cup), algo, 0)).all()


@pytest.mark.parametrize("algo", ALGOS)
def test_theorems_1_and_2_on_small_rmat(algo):
    inst = _small()
    trip, bits = oracle.replay(inst)
    V, K = inst.num_vertices, inst.K
    vals = oracle.window_values(inst, algo, 0, 0, K, replayed=(trip, bits))
    rcap, rcup = oracle.bounds(V, trip, bits, algo, 0, 0, K)
    lo, hi = (rcap, rcup) if algo in MAX_TYPE else (rcup, rcap)  # Table 1 directions
    assert (vals >= lo[:, None]).all() and (vals <= hi[:, None]).all()
    stable = rcap == rcup
    assert (vals[stable] == rcap[stable][:, None]).all()
    # detected-stable is a subset of truly constant (safe, not complete)
    const = (vals == vals[:, :1]).all(axis=1)
    assert not (stable & ~const).any()


def test_worked_example_bounds_and_values():
    g = load_golden("p6_worked_example.json")
    inst = instance_from(g)
    trip, bits = oracle.replay(inst)
    rcap, rcup = oracle.bounds(4, trip, bits, oracle.SSSP, 0, 0, 2)
    vals = oracle.window_values(inst, oracle.SSSP, 0, 0, 2, replayed=(trip, bits))
    assert rcap.tolist() == g["expect"]["r_cap"]
    assert rcup.tolist() == g["expect"]["r_cup"]
    assert vals.tolist() == g["expect"]["values"]
    assert (rcap == rcup).tolist() == g["expect"]["stable"]


def test_special_cases_L1_and_empty_batches_and_nesting():
    inst = _small()
    trip, bits = oracle.replay(inst)
    V = inst.num_vertices
    for algo in ALGOS:
        for t in (0, 5):
            rcap, rcup = oracle.bounds(V, trip, bits, algo, 0, t, 1)
            v = oracle.window_values(inst, algo, 0, t, 1, replayed=(trip, bits))
            assert (rcap == rcup).all() and (v[:, 0] == rcap).all()
        # window nesting: stable(W) is a subset of stable(W') for W' inside W
        a, b = oracle.bounds(V, trip, bits, algo, 0, 0, 8)
        c, d = oracle.bounds(V, trip, bits, algo, 0, 2, 3)
        assert not ((a == b) & (c != d)).any()
    e = empty_batches_instance(inst)
    t2, b2 = oracle.replay(e)
    for algo in ALGOS:
        rcap, rcup = oracle.bounds(V, t2, b2, algo, 0, 0, e.K)
        assert (rcap == rcup).all()
