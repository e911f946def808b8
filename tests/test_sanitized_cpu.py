"""The C oracle and the seeded input generator built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, host code only), run in a child process over
small instances that reach their edge cases: every algorithm, sub-windows,
masks of one and two words (K = 8, 65 and 128), saturating sums and the
largest weights on explicit edge lists, Viterbi's float values, and a graph
with no base edges.  The child must report nothing and
return the same values as the normal build.
"""
import json
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

CASES = [  # (scale, edges, K, dels, adds, wmin, wmax, seed, [(algo, b, L)])
    (6, 300, 8, 4, 4, 1, 100, 1, [(0, 0, 8), (1, 2, 5), (2, 0, 8), (3, 1, 6), (4, 0, 8)]),
    (7, 600, 65, 3, 3, 1, 1000, 2, [(0, 0, 65), (2, 10, 55), (3, 63, 2), (4, 0, 65)]),
    (5, 200, 128, 2, 2, 60000, 65534, 3, [(0, 0, 128), (1, 64, 64), (3, 0, 128)]),
    (4, 0, 4, 0, 1, 1, 10, 4, [(0, 0, 4), (2, 1, 3)]),
]

CHILD = textwrap.dedent("""
    import json, sys
    import numpy as np
    sys.path.insert(0, {root!r})
    import oracle, synth
    out = []
    for scale, E, K, nd, na, wmin, wmax, seed, qs in json.loads(sys.argv[1]):
        inst = synth.rmat_instance(scale, E, K, nd, na, wmin=wmin, wmax=wmax, seed=seed)
        trip, bits = oracle.replay(inst)
        src = int(synth.pick_sources(inst, 1, seed=seed)[0]) if len(inst.base) else 0
        for a, b, L in qs:
            vals = oracle.query(inst.num_vertices, trip, bits, a, src, list(range(b, b + L)))
            rc, ru = oracle.bounds(inst.num_vertices, trip, bits, a, src, b, L)
            out.append([int(np.asarray(vals, dtype=np.uint64).sum() % (1 << 61)), int(rc.astype(np.uint64).sum()),
                        int(ru.astype(np.uint64).sum()), len(trip)])
    # saturation and the largest weights on explicit edge lists (a chain and a two-way cycle)
    big = np.array([[0, 1, 0xFFFFFFF0], [1, 2, 0xFFFFFFF0], [2, 3, 7], [3, 2, 0xFFFFFFFF]], dtype=np.uint32)
    for a in range(5):
        out.append([int(x) for x in oracle.solve(4, big, a, 0)])
    print("RESULT " + json.dumps(out))
""")


def _gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _run_child(env_extra):
    env = dict(os.environ, OMP_NUM_THREADS="4", **env_extra)
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT), json.dumps(CASES)],
                       capture_output=True, text=True, env=env, timeout=600)
    return r


def test_oracle_and_generator_under_asan_ubsan(tmp_path):
    asan = _gcc_runtime("libasan.so")
    if asan is None or _gcc_runtime("libubsan.so") is None:
        pytest.skip("gcc sanitizer runtimes not installed")
    flags = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined", "-fopenmp", "-shared", "-fPIC"]
    libs = {}
    for name, src in (("oracle", os.path.join(ROOT, "oracle", "oracle.c")),
                      ("synth", os.path.join(ROOT, "synth", "rmat.c"))):
        libs[name] = str(tmp_path / f"lib{name}_san.so")
        subprocess.check_call(flags + ["-o", libs[name], src])
    plain = _run_child({})
    assert plain.returncode == 0, plain.stderr[-3000:]
    san = _run_child({"EVQ_ORACLE_LIBRARY": libs["oracle"], "EVQ_SYNTH_LIBRARY": libs["synth"],
                      "LD_PRELOAD": asan, "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=23",
                      "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    report = san.stderr[-5000:]
    assert san.returncode == 0, f"sanitized run failed ({san.returncode}):\n{report}"
    assert "AddressSanitizer" not in san.stderr and "runtime error" not in san.stderr, report
    got = [l for l in san.stdout.splitlines() if l.startswith("RESULT ")]
    want = [l for l in plain.stdout.splitlines() if l.startswith("RESULT ")]
    assert got and got == want, (got, want)
