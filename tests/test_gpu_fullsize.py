"""GPU parity at the full workload sizes, in the configuration bench.py times.

mid   (R-MAT scale 20, K = 64): SSSP, BFS and Viterbi from the seeded source, every one
      of the 64 snapshots compared with the oracle, plus the bounds.
large (R-MAT scale 23, K = 100, weights [1, 1000], two-word masks): SSWP and
      SSNP; three sampled snapshots compared with the oracle, and on all 100
      columns the properties that hold at any size (Theorem 1's sandwich with
      Table 1's directions, Theorem 2's constancy of stable vertices).
Values are uint32 and exact: tolerance zero.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import assert_equal_values, gpu_bounds, gpu_values

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def evq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2502_10579_amd as m
    return m


@pytest.fixture(scope="module")
def mid():
    inst = synth.config_instance("mid", seed=1)
    return inst, oracle.replay(inst), synth.pick_sources(inst, 1, seed=1)[0]


@pytest.fixture(scope="module")
def large():
    inst = synth.config_instance("large", seed=1)
    return inst, oracle.replay(inst), synth.pick_sources(inst, 1, seed=1)[0]


@pytest.mark.parametrize("algo", [oracle.SSSP, oracle.BFS, oracle.VITERBI])
def test_mid_all_snapshots(evq, mid, algo):
    inst, rep, src = mid
    V, K = inst.num_vertices, inst.K
    print(f"mid: algo {algo} source {src}", flush=True)
    want = oracle.window_values(inst, algo, src, 0, K, replayed=rep)
    rc_o, ru_o = oracle.bounds(V, rep[0], rep[1], algo, src, 0, K)
    with evq.Graph.from_instance(inst) as g:
        got, st = gpu_values(g, algo, src, 0, K, stats=True)
        rc, ru = gpu_bounds(g, algo, src, 0, K)
    assert np.array_equal(rc, rc_o) and np.array_equal(ru, ru_o)
    assert_equal_values(got, want, f"mid algo {algo}")
    assert st["n_unstable"] == int((rc_o != ru_o).sum())


@pytest.mark.parametrize("algo", [oracle.SSWP, oracle.SSNP])
def test_large_sampled_snapshots_and_invariants(evq, large, algo):
    inst, rep, src = large
    V, K = inst.num_vertices, inst.K
    print(f"large: algo {algo} source {src}", flush=True)
    snaps = [0, 37, K - 1]
    want = oracle.query(V, rep[0], rep[1], algo, src, snaps)
    with evq.Graph.from_instance(inst) as g:
        assert g.info["mask_words"] == 2
        got = gpu_values(g, algo, src, 0, K)
        rc, ru = gpu_bounds(g, algo, src, 0, K)
    assert_equal_values(got[:, snaps], want, f"large algo {algo} snapshots {snaps}")
    lo, hi = (rc, ru) if algo == oracle.SSWP else (ru, rc)
    assert (got >= lo[:, None]).all() and (got <= hi[:, None]).all()
    stable = rc == ru
    assert (got[stable] == rc[stable][:, None]).all()
