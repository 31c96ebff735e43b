"""GPU parity for undefined enclosures: a NaN coefficient.

Criterion C0 (Sec. 3.2) drops a box only when 0 is certainly outside the
enclosure; a NaN endpoint certifies nothing, so the box is kept (the same
rule the oracle pins on the CPU).  A NaN coefficient reaches every box of a
dense polynomial, so that polynomial's enclosures are NaN everywhere; in a
system the other polynomials still exclude.  NaN payloads are not part of
the result: positions of NaN must agree, and every other endpoint bit for
bit (after -0 -> +0).
"""
import sys

import numpy as np
import pytest

from oracle import core as orc
from paper_2406_09857_amd import synth
from tests.helpers import canon, csf_equal

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def vx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_09857_amd import binding
    binding.lib()
    return binding


def _nan_equal(a, b):
    a = canon(a); b = canon(b)
    if a.shape != b.shape:
        return False
    na, nb = np.isnan(a), np.isnan(b)
    return np.array_equal(na, nb) and np.array_equal(a[~na].view(np.uint64), b[~nb].view(np.uint64))


def _systems():
    """(name, k, depth, polys, domain): one polynomial with a NaN coefficient,
    a two-polynomial system whose first polynomial has one, and a system of
    interval polynomials whose second one has a [NaN, NaN] coefficient."""
    p2 = synth.small_random(2, 12, seed=301)[0]
    p2[3, 4] = np.nan
    q3 = synth.small_random(3, 9, seed=302, npolys=2)
    q3[0][1, 0, 2] = np.nan
    # interval coefficients, one of them [NaN, NaN], on a non-dyadic domain
    r3 = synth.small_random(3, 6, seed=303, npolys=2)
    lo = r3[1] - np.abs(r3[1]) * 1e-9
    hi = r3[1] + np.abs(r3[1]) * 1e-9
    lo[0, 2, 1] = hi[0, 2, 1] = np.nan
    return [("k2 NaN", 2, 7, [p2], np.array([-1.0, 1.0] * 2)),
            ("k3 system, NaN in the first", 3, 5, q3, np.array([-1.0, 1.0] * 3)),
            ("k3 system, NaN interval coefficient in the second", 3, 4, [r3[0], (lo, hi)],
             np.array([-0.7, 1.1, -1.0, 0.9, -1.3, 1.0]))]


@pytest.mark.parametrize("case", range(3))
def test_nan_coefficient_interval_eval_level(vx, case):
    name, k, depth, polys, dom = _systems()[case]
    recs = orc.subdivide(polys, k, depth, dom=dom, nthreads=orc.max_threads())
    for r in recs:
        S = r["S"]
        if len(S["boxes"]) == 0:
            continue
        _say(f"[nan] {name}: interval_eval_level, level {r['level']} sizes {orc.csf_sizes(S)}")
        csf = vx.CSF.from_arrays(k, S["level"], S["idx"], S["ptr"])
        lo, hi, keep = vx.interval_eval_level(polys, csf, dom)
        lo = lo.cpu().numpy(); hi = hi.cpu().numpy(); keep = keep.cpu().numpy().astype(bool)
        assert _nan_equal(lo, r["lo"]) and _nan_equal(hi, r["hi"]), (name, r["level"])
        assert np.array_equal(keep, r["keep"]), (name, r["level"])
    if case == 0:  # one polynomial, NaN everywhere: nothing is ever excluded
        assert all(r["keep"].all() and np.isnan(r["lo"]).all() for r in recs)
        assert len(recs[-1]["kept"]) == 4 ** depth
    if case == 1:  # the second polynomial still excludes
        assert len(recs[-1]["kept"]) < 8 ** depth


@pytest.mark.parametrize("case", range(3))
def test_nan_coefficient_run_subdivision(vx, case):
    name, k, depth, polys, dom = _systems()[case]
    _say(f"[nan] {name}: run_subdivision to level {depth}")
    recs = orc.subdivide(polys, k, depth, dom=dom, nthreads=orc.max_threads())
    seen = {}

    def record(level, S, lo, hi, keep, K):
        seen[level] = (S, lo, hi, keep, K)

    stats, kept = vx.run_subdivision(polys, dom, depth, record=record)
    for r in recs:
        if r["level"] not in seen:
            assert len(r["S"]["boxes"]) == 0
            continue
        S, lo, hi, keep, K = seen[r["level"]]
        assert csf_equal(S, r["S"]), (name, r["level"])
        assert _nan_equal(lo, r["lo"]) and _nan_equal(hi, r["hi"]), (name, r["level"])
        assert np.array_equal(keep.astype(bool), r["keep"]), (name, r["level"])
        assert csf_equal(K, orc.csf_from_boxes(r["kept"], r["level"])), (name, r["level"])
        assert stats[r["level"]]["steps"] == int(r["steps"].sum())
