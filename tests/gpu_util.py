"""Helpers for the GPU parity tests: run the HIP path, run the oracle, compare."""
import numpy as np

import oracle


def gpu_values(g, algo, source, b, L, plain=False, stats=False, sequential=False):
    import paper_2502_10579_amd as evq
    fn = g.query_plain if plain else (g.query_sequential if sequential else g.query)
    r = fn(algo, source, b, L, stats=stats)
    if stats:
        out, st = r
        return evq.to_u32(out).reshape(g.num_vertices, L), st
    return evq.to_u32(r).reshape(g.num_vertices, L)


def gpu_bounds(g, algo, source, b, L):
    import paper_2502_10579_amd as evq
    rc, ru = g.query_bounds(algo, source, b, L)
    return evq.to_u32(rc), evq.to_u32(ru)


def assert_equal_values(got, want, ctx=""):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        v, i = bad[0]
        raise AssertionError(f"{ctx}: {len(bad)} mismatches; first at vertex {v} snapshot {i}: "
                             f"gpu {got[v, i]} oracle {want[v, i]}")


def union_triples_from_export(ex, K):
    """Set of (src, dst, w) -> 128-bit presence integer from an exported versioned graph."""
    V = len(ex["row_split"])
    rp = ex["row_ptr"].astype(np.int64)
    src = np.repeat(np.arange(V, dtype=np.uint32), np.diff(rp))
    out = {}
    MW = ex["mask"].shape[1] if ex["mask"].ndim == 2 and len(ex["mask"]) else 1
    for j in range(len(src)):
        m = int(ex["mask"][j, 0]) | ((int(ex["mask"][j, 1]) << 64) if MW == 2 else 0)
        out[(int(src[j]), int(ex["col"][j]), int(ex["w"][j]))] = m
    return out


def oracle_triples(inst):
    trip, bits = oracle.replay(inst)
    d = {}
    for r, b in zip(trip, bits):
        m = int(b[0]) | (int(b[1]) << 64)
        if m:
            d[(int(r[0]), int(r[1]), int(r[2]))] = m
    return d


def gpu_column_digests(t, chunk=16):
    """Digests (tests/digest.py) of the columns of a (V, L) int32 device tensor of uint32 values."""
    from digest import column_digests
    L = t.shape[1]
    out = []
    for i in range(0, L, chunk):
        part = t[:, i:i + chunk].t().contiguous().cpu().numpy().view(np.uint32)
        out += column_digests(part)
    return out


def assert_digests(got, want, ctx, diagnose=None):
    """Columns whose digests differ are named; diagnose(i) may add the first differing vertex."""
    assert len(got) == len(want), f"{ctx}: {len(got)} columns, expected {len(want)}"
    bad = [i for i, (a, b) in enumerate(zip(got, want)) if a != b]
    if bad:
        msg = f"{ctx}: {len(bad)} of {len(want)} snapshot columns differ from the oracle (first: column {bad[0]})"
        if diagnose is not None:
            msg += "; " + diagnose(bad[0])
        raise AssertionError(msg)


def golden_section(name, inst):
    """A section of tests/golden/fullsize_digests.json, checked against the instance it was computed on."""
    import json
    import os
    from digest import instance_fingerprint
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_digests.json")
    with open(path) as f:
        sec = json.load(f)[name]
    fp = instance_fingerprint(inst)
    assert sec["fingerprint"] == fp, (f"golden section {name} was computed on another instance "
                                      f"(regenerate with tests/golden/make_fullsize_digests.py {name})")
    return sec
