"""Taylor-form exclusion of order m >= 3 on the GPU against the oracle
(Sec. 3.2, Taylor form definition, multinomial form).

Bar: the order-m enclosures are bit-identical to the oracle's (after
-0 -> +0), the combined keep flags and the kept sets of whole runs equal.
Cases: every level of `tiny` (orders 3 and 4), the surface and the curve at
levels with thousands of boxes, k = 1..4 with interval coefficients on a
non-dyadic domain (orders 3..6), systems whose term polynomials exceed one
group of 64 (the chunked path), degrees below the order (terms of zero),
an empty level, the loop with the test on (tiny, surface, curve), and a
sampled full-size curve run with the order-3 test at every level.
"""
import sys
import time

import numpy as np
import pytest

from oracle import core as orc
from paper_2406_09857_amd import synth
from tests.helpers import bits_equal, csf_equal, first_mismatch

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


def _check(vx, polys, S, dom, m, tag):
    _say(f"[tm] {tag}: order {m}, level {S['level']} sizes {orc.csf_sizes(S)}")
    tlo, thi = orc.taylor_m_level(polys, S, dom, m, nthreads=orc.max_threads())
    lo0, hi0, _ = orc.eval_level(polys, S, dom, nthreads=orc.max_threads())
    keep_o = orc.keep_mask(lo0, hi0) & orc.keep_mask(tlo, thi)
    csf = vx.CSF.from_arrays(S["k"], S["level"], S["idx"], S["ptr"])
    _, _, keep = vx.interval_eval_level(polys, csf, dom)
    glo, ghi = vx.taylor_exclusion(polys, csf, dom, m, keep=keep)
    glo = glo.cpu().numpy(); ghi = ghi.cpu().numpy()
    assert bits_equal(glo, tlo), (tag, m, "lo", first_mismatch(glo, tlo))
    assert bits_equal(ghi, thi), (tag, m, "hi", first_mismatch(ghi, thi))
    assert np.array_equal(keep.cpu().numpy().astype(bool), keep_o), (tag, m)


@pytest.mark.parametrize("m", [3, 4])
def test_tiny_levels(vx, m):
    w = synth.tiny()
    recs = orc.subdivide(w.polys, 2, 6)
    for r in recs[1:]:
        _check(vx, w.polys, r["S"], w.domain(), m, "tiny")


def test_surface_and_curve_levels(vx):
    w = synth.surface()
    r = orc.subdivide(w.polys, 3, 6, nthreads=orc.max_threads())[-1]
    _check(vx, w.polys, r["S"], w.domain(), 3, "surface level 6")
    _check(vx, w.polys, r["S"], w.domain(), 4, "surface level 6")
    w = synth.curve()
    r = orc.subdivide(w.polys, 3, 5, nthreads=orc.max_threads())[-1]
    _check(vx, w.polys, r["S"], w.domain(), 3, "curve level 5")


@pytest.mark.parametrize("k,d,level,m", [(1, 11, 6, 6), (2, 8, 5, 4), (3, 7, 4, 3), (3, 6, 3, 5), (4, 5, 3, 3)])
def test_random_k_odd_domain_interval_coefficients(vx, k, d, level, m):
    """Non-dyadic domain (centre enclosures one ulp wide) and interval
    coefficients, k = 1..4, orders 3 to 6."""
    rng = np.random.default_rng(600 + k + m)
    c = synth.small_random(k, d, seed=610 + k + m, npolys=2)
    polys = [(c[0] - 1e-3 * np.abs(c[0]), c[0] + 1e-3 * np.abs(c[0])), c[1]]
    dom = np.array([-0.7, 1.3] * k)
    boxes = rng.integers(0, 1 << level, size=(400, k))
    S = orc.csf_from_boxes(boxes, level)
    _check(vx, polys, S, dom, m, f"k{k} d{d}")


def test_many_polynomials_chunked_terms(vx):
    """Six trivariate polynomials at order 4: 6 x 20 centre terms and 6 x 15
    box terms, evaluated as systems of at most 64 polynomials."""
    rng = np.random.default_rng(620)
    polys = synth.small_random(3, 6, seed=621, npolys=6)
    S = orc.csf_from_boxes(rng.integers(0, 16, size=(300, 3)), 4)
    _check(vx, polys, S, np.array([-1.0, 1.0] * 3), 4, "six polynomials")


def test_degrees_below_the_order_and_empty_level(vx):
    const = np.zeros((1, 1, 1)); const[0, 0, 0] = 0.0
    S = orc.csf_from_boxes(np.random.default_rng(6).integers(0, 8, size=(60, 3)), 3)
    _check(vx, [const, synth.plane_x3()], S, np.array([-1.0, 1.0] * 3), 3, "degree 0 and 1")
    _check(vx, [synth.sphere()], S, np.array([-1.0, 1.0] * 3), 5, "sphere (degree 2)")
    E = orc.csf_from_boxes(np.zeros((0, 3), np.int64), 4)
    csf = vx.CSF.from_arrays(3, 4, E["idx"], E["ptr"])
    glo, ghi = vx.taylor_exclusion([synth.sphere()], csf, np.array([-1.0, 1.0] * 3), 3)
    assert glo.shape == (1, 0) and ghi.shape == (1, 0)


def test_order_outside_the_range_is_refused(vx):
    w = synth.tiny()
    S = orc.subdivide(w.polys, 2, 2)[-1]["S"]
    csf = vx.CSF.from_arrays(2, 2, S["idx"], S["ptr"])
    for m in (0, 7):
        with pytest.raises(vx.VxError):
            vx.taylor_exclusion(w.polys, csf, w.domain(), m)


@pytest.mark.parametrize("name,depth,m", [("tiny", 8, 3), ("surface", 6, 3), ("curve", 6, 3), ("surface", 5, 4)])
def test_run_subdivision_with_taylor_m_matches_oracle(vx, name, depth, m):
    w = getattr(synth, name)()
    _say(f"[tm] run_subdivision(taylor_order={m}) {name} depth {depth}")
    got = {}

    def rec(level, S, lo, hi, keep, K):
        got[level] = K
        return False

    stats, _ = vx.run_subdivision(w.polys, w.domain(), depth, record=rec, taylor_order=m)
    ref = orc.subdivide_tm(w.polys, w.k, depth, m, dom=w.domain(), nthreads=orc.max_threads())
    for r in ref:
        K = orc.csf_from_boxes(r["kept"], r["level"])
        assert orc.csf_sizes(K) == [got[r["level"]]["idx"][l].shape[0] for l in range(w.k)], r["level"]
        assert csf_equal(got[r["level"]], K), r["level"]
    t2, _ = vx.run_subdivision(w.polys, w.domain(), depth, taylor2=True)
    _say(f"[tm] kept per level, order {m}: {[s['kept'][w.k - 1] for s in stats]}; "
         f"order 2: {[s['kept'][w.k - 1] for s in t2]}")


def _boxes_of(S):
    k = S["k"]
    cols = [np.asarray(S["idx"][k - 1], np.int64)]
    up = np.arange(len(cols[0]))
    for l in range(k - 2, -1, -1):
        ptr = np.asarray(S["ptr"][l], np.int64)
        up = np.searchsorted(ptr, up, side="right") - 1
        cols.append(np.asarray(S["idx"][l], np.int64)[up])
    return np.stack(cols[::-1], axis=1) if len(cols[0]) else np.zeros((0, k), np.int64)


@pytest.mark.timeout(900)
def test_curve_taylor3_sampled_every_level(vx):
    """The full curve (two degree-100 polynomials, levels 0..10) with the
    order-3 test AND-ed with C0: every level's CSF is the children of the
    previous kept set, the kept CSF the flagged boxes, and 128 seeded boxes
    per level are re-evaluated by the oracle (C0 and order-3 enclosures,
    combined flag) on a CSF of the sample alone."""
    w = synth.curve()
    dom = w.domain()
    got = {}

    def rec(level, S, lo, hi, keep, K):
        got[level] = (S, lo, hi, keep.astype(bool), K)
        return False

    t = time.time()
    stats, _ = vx.run_subdivision(w.polys, dom, w.depth, record=rec, taylor_order=3)
    _say(f"[tm] curve order 3: GPU run with per-level copies {time.time() - t:.1f} s, kept per level "
         f"{[s['kept'][2] for s in stats]}")
    rng = np.random.default_rng(2408)
    prev_children = np.zeros((1, w.k), np.int64)
    for level in range(w.depth + 1):
        S, lo, hi, keep, K = got.pop(level)
        tag = f"curve order-3 level {level}"
        B = _boxes_of(S)
        assert csf_equal(S, orc.csf_from_boxes(prev_children, level)), tag
        assert csf_equal(K, orc.csf_from_boxes(B[keep], level)), tag
        n = len(B)
        pick = np.sort(rng.choice(n, size=min(n, 128), replace=False))
        T = orc.csf_from_boxes(B[pick], level)
        lo_o, hi_o, _ = orc.eval_level(w.polys, T, dom, nthreads=orc.max_threads())
        tlo, thi = orc.taylor_m_level(w.polys, T, dom, 3, nthreads=orc.max_threads())
        keep_o = orc.keep_mask(lo_o, hi_o) & orc.keep_mask(tlo, thi)
        assert bits_equal(lo[:, pick], lo_o), (tag, "lo", first_mismatch(lo[:, pick], lo_o))
        assert bits_equal(hi[:, pick], hi_o), (tag, "hi", first_mismatch(hi[:, pick], hi_o))
        assert np.array_equal(keep[pick], keep_o), tag
        prev_children = orc.children_of(B[keep])
    assert not got
