"""Independent brute-force definitions used to pin the oracle.

Nothing here is shared with the oracle or with the HIP library: each function
restates a definition directly (path enumeration, Bellman-Ford rounds,
threshold reachability, explicit per-snapshot sets) so that a mistake in the
oracle's Dijkstra/BFS or in its replay shows up as a disagreement.
"""
from collections import deque

import numpy as np

SSSP, BFS, SSWP, SSNP, VIT = 0, 1, 2, 3, 4
INF = 0xFFFFFFFF
SAT = 0xFFFFFFFE
ONE = 0x3F800000  # 1.0 as an IEEE single
FLT_MIN = float(np.finfo(np.float32).tiny)


def max_type(algo):
    return algo in (SSWP, VIT)


def vit_step(bits, w):
    """One Viterbi step: the single float with pattern `bits` divided by w in double precision, rounded to
    single (nearest even); a quotient below the smallest normal single is unreachable (0)."""
    if bits == 0:
        return 0
    x = float(np.array([bits], dtype=np.uint32).view(np.float32)[0])
    q = x / float(w)
    if q < FLT_MIN:
        return 0
    return int(np.array([q], dtype=np.float32).view(np.uint32)[0])


def snapshot_sets(inst):
    """Snapshot i = set of triples after applying batches 0..i to the base
    (each batch: deletions, then additions)."""
    cur = {tuple(int(x) for x in r) for r in np.asarray(inst.base).reshape(-1, 3)}
    out = []
    for d, a in zip(inst.dels, inst.adds):
        for r in np.asarray(d).reshape(-1, 3):
            cur.discard(tuple(int(x) for x in r))
        for r in np.asarray(a).reshape(-1, 3):
            cur.add(tuple(int(x) for x in r))
        out.append(set(cur))
    return out


def unreachable(algo):
    return 0 if max_type(algo) else INF


def source_value(algo):
    return INF if algo == SSWP else (ONE if algo == VIT else 0)


def path_value(algo, weights):
    """Value of one path given the weights along it (empty path = the source)."""
    if algo == SSSP:
        return min(sum(weights), SAT)
    if algo == BFS:
        return min(len(weights), SAT)
    if algo == SSWP:
        return min(weights) if weights else INF
    if algo == VIT:
        x = ONE
        for w in weights:
            x = vit_step(x, w)
        return x
    return max(weights) if weights else 0


def best_of(algo, vals):
    vals = list(vals)
    if not vals:
        return None
    return max(vals) if max_type(algo) else min(vals)


def enumerate_paths(V, edges, algo, s):
    """Best path value over every simple path s -> v (exponential: V <= 8)."""
    adj = [[] for _ in range(V)]
    for (u, v, w) in edges:
        adj[u].append((v, w))
    best = [None] * V
    best[s] = source_value(algo)

    def dfs(u, seen, ws):
        for (x, w) in adj[u]:
            if x in seen:
                continue
            pv = path_value(algo, ws + [w])
            b = best_of(algo, [pv] + ([best[x]] if best[x] is not None else []))
            best[x] = b
            seen.add(x)
            dfs(x, seen, ws + [w])
            seen.discard(x)

    dfs(s, {s}, [])
    return np.array([unreachable(algo) if b is None else b for b in best], dtype=np.uint64).astype(np.uint32)


def bellman_ford(V, edges, algo, s):
    """Rounds of relaxing every edge until nothing changes (generalised Bellman-Ford)."""
    val = [unreachable(algo)] * V
    val[s] = source_value(algo)
    for _ in range(V + 1):
        changed = False
        for (u, v, w) in edges:
            xu = val[u]
            if algo == SSSP:
                if xu == INF:
                    continue
                c = min(xu + w, SAT)
            elif algo == BFS:
                if xu == INF:
                    continue
                c = min(xu + 1, SAT)
            elif algo == SSWP:
                c = min(xu, w)
            elif algo == VIT:
                c = vit_step(xu, w)
            else:
                if xu == INF:
                    continue
                c = max(xu, w)
            if (c > val[v]) if max_type(algo) else (c < val[v]):
                val[v] = c
                changed = True
        if not changed:
            break
    return np.array(val, dtype=np.uint64).astype(np.uint32)


def reachable(V, edges, s):
    adj = [[] for _ in range(V)]
    for (u, v, _w) in edges:
        adj[u].append(v)
    seen = np.zeros(V, dtype=bool)
    seen[s] = True
    q = deque([s])
    while q:
        u = q.popleft()
        for x in adj[u]:
            if not seen[x]:
                seen[x] = True
                q.append(x)
    return seen


def threshold_widest(V, edges, s):
    """SSWP(v) = max t such that v is reachable from s using only edges with w >= t."""
    out = np.zeros(V, dtype=np.uint64)
    for t in sorted({int(e[2]) for e in edges}):
        r = reachable(V, [e for e in edges if e[2] >= t], s)
        out[r] = np.maximum(out[r], t)
    out[s] = INF
    return out.astype(np.uint32)


def threshold_narrowest(V, edges, s):
    """SSNP(v) = min t such that v is reachable from s using only edges with w <= t."""
    out = np.full(V, INF, dtype=np.uint64)
    for t in sorted({int(e[2]) for e in edges}, reverse=True):
        r = reachable(V, [e for e in edges if e[2] <= t], s)
        out[r] = np.minimum(out[r], t)
    out[s] = 0
    return out.astype(np.uint32)


def scipy_sssp(V, edges, s):
    """SSSP through scipy's Dijkstra (parallel edges reduced to their minimum weight)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra
    best = {}
    for (u, v, w) in edges:
        if u == v:
            continue
        k = (int(u), int(v))
        best[k] = min(best.get(k, 1 << 62), int(w))
    if best:
        rows = np.array([k[0] for k in best]), np.array([k[1] for k in best])
        data = np.array(list(best.values()), dtype=np.float64)
        m = csr_matrix((data, rows), shape=(V, V))
    else:
        m = csr_matrix((V, V))
    d = dijkstra(m, directed=True, indices=s)
    out = np.where(np.isinf(d), INF, np.minimum(d, SAT)).astype(np.uint64)
    return out.astype(np.uint32)
