"""Shared helpers for the tests (no method arithmetic here)."""
import numpy as np


def canon(a):
    """-0.0 -> +0.0: the sign of a zero endpoint is not part of the result."""
    a = np.array(a, dtype=np.float64, copy=True)
    a[a == 0] = 0.0
    return a


def bits_equal(a, b) -> bool:
    a = canon(a); b = canon(b)
    return a.shape == b.shape and np.array_equal(a.view(np.uint64), b.view(np.uint64))


def first_mismatch(a, b):
    a = canon(a).reshape(-1); b = canon(b).reshape(-1)
    bad = np.flatnonzero(a.view(np.uint64) != b.view(np.uint64))
    if len(bad) == 0:
        return None
    i = int(bad[0])
    return i, float(a[i]), float(b[i]), len(bad)


def csf_equal(gpu: dict, orc: dict) -> bool:
    k = orc["k"]
    for l in range(k):
        if not np.array_equal(np.asarray(gpu["idx"][l]), np.asarray(orc["idx"][l])):
            return False
        if l + 1 < k and not np.array_equal(np.asarray(gpu["ptr"][l]), np.asarray(orc["ptr"][l])):
            return False
    return True


# Results of expensive oracle runs shared between test modules of one pytest
# process (filled by whichever test computes them first).
ORACLE_RESULTS: dict = {}


def oracle_curve_kept(orc, synth, level: int = 10):
    """The oracle's kept boxes of the curve workload at `level` (computed once
    per process; test_gpu_fullsize stores the ones it computes level by level)."""
    key = ("curve_kept", level)
    if key not in ORACLE_RESULTS:
        w = synth.curve()
        recs = orc.subdivide(w.polys, w.k, level, dom=w.domain(), nthreads=orc.max_threads())
        for r in recs:
            ORACLE_RESULTS[("curve_kept", r["level"])] = r["kept"]
    return ORACLE_RESULTS[key]
