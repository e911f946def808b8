"""Seeded synthetic inputs shared by the HIP library's tests/bench and the oracle.

This module only draws random numbers (counter-based SplitMix64) and keeps the
current edge set so that update batches are valid; it holds none of the query
arithmetic.  Instances follow the evolving-graph model of the paper (Section 2:
a base snapshot and a sequence of batches of edge deletions and additions).

Workload recipe (stand-in for the paper's real graphs, Table 3, which are not
available here): R-MAT with (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), no noise,
no vertex permutation; `n_samples` R-MAT draws whose exact duplicate triples
collapse; weights uniform in [wmin, wmax]; batch i deletes `n_del` triples drawn
uniformly without replacement from the current snapshot and adds `n_add` fresh
R-MAT triples that are absent from it.
"""
import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmat.c")
# EVQ_SYNTH_LIBRARY loads another build of the same source (the sanitized one of the tests)
_LIB = os.environ.get("EVQ_SYNTH_LIBRARY") or os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.synth_instance.restype = ctypes.c_int64
        lib.synth_instance.argtypes = [
            ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
            ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.synth_rmat.restype = None
        lib.synth_rmat.argtypes = [
            ctypes.c_uint32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
            ctypes.c_uint64, ctypes.c_void_p]
        lib.synth_draw.restype = ctypes.c_uint64
        lib.synth_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        _lib = lib
    return _lib


RMAT_ABC = (0.57, 0.19, 0.19)


@dataclass
class Instance:
    """A base edge set plus K update batches.

    base: (n, 3) uint32 rows (src, dst, w).  dels[i], adds[i]: (k, 3) uint32.
    Snapshot i is the edge set after applying batches 0..i to the base
    (deletions of a batch before its additions).
    """
    num_vertices: int
    base: np.ndarray
    dels: list
    adds: list
    meta: dict = field(default_factory=dict)

    @property
    def K(self) -> int:
        return len(self.dels)


def rmat_instance(scale: int, n_samples: int, K: int, n_del: int, n_add: int,
                  wmin: int = 1, wmax: int = 100, seed: int = 1, abc=RMAT_ABC) -> Instance:
    lib = _load()
    base = np.empty((n_samples, 3), dtype=np.uint32)
    dels = np.empty((max(K * n_del, 1), 3), dtype=np.uint32)
    adds = np.empty((max(K * n_add, 1), 3), dtype=np.uint32)
    n = lib.synth_instance(scale, abc[0], abc[1], abc[2], wmin, wmax, seed, n_samples, K, n_del, n_add,
                           base.ctypes.data, dels.ctypes.data, adds.ctypes.data)
    if n < 0:
        raise ValueError("synth_instance: parameters out of range")
    base = base[:n].copy()
    dl = [dels[i * n_del:(i + 1) * n_del] for i in range(K)]
    al = [adds[i * n_add:(i + 1) * n_add] for i in range(K)]
    return Instance(1 << scale, base, dl, al,
                    dict(scale=scale, n_samples=n_samples, K=K, n_del=n_del, n_add=n_add,
                         wmin=wmin, wmax=wmax, seed=seed, abc=tuple(abc)))


def rmat_edges(scale: int, n: int, seed: int = 1, stream: int = 0, wmin: int = 1, wmax: int = 100,
               abc=RMAT_ABC) -> np.ndarray:
    lib = _load()
    out = np.empty((n, 3), dtype=np.uint32)
    lib.synth_rmat(scale, abc[0], abc[1], abc[2], wmin, wmax, seed, stream, n, out.ctypes.data)
    return out


def draw(seed: int, stream: int, i: int) -> int:
    return int(_load().synth_draw(seed, stream, i))


def pick_sources(inst: Instance, count: int, seed: int = 1, stream: int = 1 << 30) -> list:
    """`count` sources drawn uniformly among vertices with base out-degree > 0."""
    deg = np.bincount(inst.base[:, 0], minlength=inst.num_vertices)
    cand = np.flatnonzero(deg > 0)
    if cand.size == 0:
        return [0] * count
    return [int(cand[draw(seed, stream, i) % cand.size]) for i in range(count)]


def batch_queries(inst: Instance, n: int, seed: int = 1, start_max: int = 100, len_min: int = 25,
                  len_max: int = 100, algos=(0, 1, 2, 3)) -> list:
    """n query descriptors (algo, source, win_begin, win_len) for a batch: algorithm uniform over
    `algos`, source uniform among base vertices of out-degree > 0, start uniform in [0, start_max]
    (clamped to K - 1), length uniform in [len_min, len_max], clamped so the window ends by K."""
    K = inst.K
    srcs = pick_sources(inst, n, seed=seed, stream=(1 << 30) + 1)
    out = []
    for i in range(n):
        a = algos[draw(seed, (1 << 30) + 2, i) % len(algos)]
        b = min(draw(seed, (1 << 30) + 3, i) % (start_max + 1), K - 1)
        L = len_min + draw(seed, (1 << 30) + 4, i) % (len_max - len_min + 1)
        out.append((int(a), int(srcs[i]), int(b), int(max(1, min(L, K - b)))))
    return out


def random_instance(V: int, n_base: int, K: int, n_del: int, n_add: int, wmax: int, seed: int) -> Instance:
    """Small uniform multigraph instance (for exhaustive pin tests): base may hold
    exact duplicates; deletions draw from the current set; additions are uniform."""
    rng = np.random.default_rng(seed)
    base = np.stack([rng.integers(0, V, n_base), rng.integers(0, V, n_base),
                     rng.integers(1, wmax + 1, n_base)], axis=1).astype(np.uint32).reshape(-1, 3)
    cur = {tuple(map(int, r)) for r in base}
    dels, adds = [], []
    for _ in range(K):
        pool = sorted(cur)
        k = min(n_del, len(pool))
        pick = rng.choice(len(pool), size=k, replace=False) if k else np.zeros(0, dtype=np.int64)
        d = np.array([pool[j] for j in pick], dtype=np.uint32).reshape(-1, 3)
        a = np.stack([rng.integers(0, V, n_add), rng.integers(0, V, n_add),
                      rng.integers(1, wmax + 1, n_add)], axis=1).astype(np.uint32).reshape(-1, 3)
        for r in d:
            cur.discard(tuple(map(int, r)))
        for r in a:
            cur.add(tuple(map(int, r)))
        dels.append(d)
        adds.append(a)
    return Instance(V, base, dels, adds, dict(kind="uniform", seed=seed))


CONFIGS = {
    # R-MAT scale 12, average out-degree 8, K = 8, 0.1% of edges per batch (33 + 33)
    "small": dict(scale=12, n_samples=32768, K=8, n_del=33, n_add=33, wmin=1, wmax=100),
    # R-MAT scale 20, 16M samples, K = 64, 10k + 10k
    "mid": dict(scale=20, n_samples=16777216, K=64, n_del=10000, n_add=10000, wmin=1, wmax=100),
    # the mid graph with heavy churn: 100k + 100k per snapshot (about half the vertices unstable)
    "churn": dict(scale=20, n_samples=16777216, K=64, n_del=100000, n_add=100000, wmin=1, wmax=100),
    # R-MAT scale 23, 134M samples, K = 100, 50k + 50k, weights [1, 1000]
    "large": dict(scale=23, n_samples=134217728, K=100, n_del=50000, n_add=50000, wmin=1, wmax=1000),
    # R-MAT scale 22, 67M samples, K = 128, 20k + 20k
    "batched": dict(scale=22, n_samples=67108864, K=128, n_del=20000, n_add=20000, wmin=1, wmax=100),
    # R-MAT scale 24, 268M samples, ring of 128, 100k + 100k
    "served": dict(scale=24, n_samples=268435456, K=128, n_del=100000, n_add=100000, wmin=1, wmax=100),
}


def config_instance(name: str, seed: int = 1) -> Instance:
    return rmat_instance(seed=seed, **CONFIGS[name])
