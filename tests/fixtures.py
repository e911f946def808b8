"""Test-side helpers: golden fixtures as instances, small instance factories."""
import json
import os

import numpy as np

from synth import Instance

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _arr(rows):
    return np.asarray(rows, dtype=np.uint32).reshape(-1, 3)


def instance_from(d):
    return Instance(int(d["num_vertices"]), _arr(d["base"]),
                    [_arr(b["del"]) for b in d["batches"]], [_arr(b["add"]) for b in d["batches"]])


def empty_batches_instance(inst):
    K = inst.K
    z = np.zeros((0, 3), dtype=np.uint32)
    return Instance(inst.num_vertices, inst.base, [z] * K, [z] * K)
