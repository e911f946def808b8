"""Fingerprints used to compare values too large to recompute on the test machine.

A column digest is the 128-bit XXH3 hash of one snapshot's values (uint32, in
vertex order, little-endian).  Equal digests mean equal columns (up to a hash
collision); a differing digest names the snapshot that differs.  This module
holds no query arithmetic: it only hashes arrays.
"""
import concurrent.futures

import numpy as np
import xxhash


def _h(buf) -> str:
    return xxhash.xxh3_128(memoryview(np.ascontiguousarray(buf))).hexdigest()


def array_digest(a) -> str:
    """Digest of one uint32 array (e.g. a bound vector)."""
    return _h(np.asarray(a, dtype=np.uint32))


def column_digests(cols_major, threads: int = 8) -> list:
    """Digests of the rows of an (L, V) uint32 array: row i = snapshot i's values."""
    a = np.ascontiguousarray(cols_major, dtype=np.uint32)
    with concurrent.futures.ThreadPoolExecutor(threads) as ex:
        return list(ex.map(_h, [a[i] for i in range(a.shape[0])]))


def values_digests(values_vl, threads: int = 8) -> list:
    """Digests of the columns of a (V, L) uint32 array (the library's values layout)."""
    return column_digests(np.asarray(values_vl, dtype=np.uint32).T, threads)


def instance_fingerprint(inst) -> str:
    """Digest of an instance's base edges and batches, so a stored digest can tell
    a changed generator from a changed result."""
    h = xxhash.xxh3_128()
    h.update(np.asarray([inst.num_vertices, len(inst.dels)], dtype=np.uint64).tobytes())
    h.update(memoryview(np.ascontiguousarray(inst.base)))
    for d, a in zip(inst.dels, inst.adds):
        h.update(np.asarray([len(d), len(a)], dtype=np.uint64).tobytes())
        h.update(memoryview(np.ascontiguousarray(d)))
        h.update(memoryview(np.ascontiguousarray(a)))
    return h.hexdigest()
