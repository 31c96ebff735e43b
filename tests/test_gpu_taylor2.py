"""Order-2 Taylor-form exclusion on the GPU against the oracle.

Bar: the order-2 enclosures are bit-identical to the oracle's (after
-0 -> +0), the combined keep flags and the kept sets of whole runs equal.
Cases span several tiles and ragged tails of every stage (hundreds of boxes
at levels 3-6), k = 1..4, a non-dyadic domain, interval coefficients,
degrees below 2 (all second-order polynomials zero) and an empty level.
"""
import sys

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


def _check(vx, polys, S, dom, tag):
    _say(f"[t2] {tag}: level {S['level']} sizes {orc.csf_sizes(S)}")
    tlo, thi = orc.taylor2_level(polys, S, dom, nthreads=orc.max_threads())
    lo0, hi0, _ = orc.eval_level(polys, S, dom, nthreads=orc.max_threads())
    keep_o = orc.keep_mask(lo0, hi0) & orc.keep_mask(tlo, thi)
    csf = vx.CSF.from_arrays(S["k"], S["level"], S["idx"], S["ptr"])
    _, _, keep = vx.interval_eval_level(polys, csf, dom)
    glo, ghi = vx.taylor_exclusion(polys, csf, dom, 2, keep=keep)
    glo = glo.cpu().numpy(); ghi = ghi.cpu().numpy()
    assert bits_equal(glo, tlo), (tag, "lo", first_mismatch(glo, tlo))
    assert bits_equal(ghi, thi), (tag, "hi", first_mismatch(ghi, thi))
    assert np.array_equal(keep.cpu().numpy().astype(bool), keep_o), tag


def test_tiny_levels(vx):
    w = synth.tiny()
    recs = orc.subdivide(w.polys, 2, 6)
    for r in recs[1:]:
        _check(vx, w.polys, r["S"], w.domain(), "tiny")


def test_surface_level6_and_curve_level5(vx):
    w = synth.surface()
    r = orc.subdivide(w.polys, 3, 6, nthreads=orc.max_threads())[-1]
    _check(vx, w.polys, r["S"], w.domain(), "surface")
    w = synth.curve()
    r = orc.subdivide(w.polys, 3, 5, nthreads=orc.max_threads())[-1]
    _check(vx, w.polys, r["S"], w.domain(), "curve")


@pytest.mark.parametrize("k,d,level", [(1, 9, 6), (2, 7, 5), (3, 6, 4), (4, 4, 3)])
def test_random_k_odd_domain_interval_coefficients(vx, k, d, level):
    """Non-dyadic domain (centre enclosures one ulp wide) and interval
    coefficients."""
    rng = np.random.default_rng(400 + k)
    c = synth.small_random(k, d, seed=410 + k, npolys=2)
    polys = [(c[0] - 1e-3 * np.abs(c[0]), c[0] + 1e-3 * np.abs(c[0])), c[1]]
    dom = np.array([-0.7, 1.3] * k)
    boxes = rng.integers(0, 1 << level, size=(400, k))
    S = orc.csf_from_boxes(boxes, level)
    _check(vx, polys, S, dom, f"k{k}")


def test_degenerate_degrees_and_empty_level(vx):
    const = np.zeros((1, 1, 1)); const[0, 0, 0] = 0.0
    S = orc.csf_from_boxes(np.random.default_rng(6).integers(0, 8, size=(60, 3)), 3)
    _check(vx, [const, synth.plane_x3()], S, np.array([-1.0, 1.0] * 3), "degree0+1")
    _check(vx, [synth.sphere()], S, np.array([-1.0, 1.0] * 3), "sphere")
    E = orc.csf_from_boxes(np.zeros((0, 3), np.int64), 4)
    csf = vx.CSF.from_arrays(3, 4, E["idx"], E["ptr"])
    glo, ghi = vx.taylor_exclusion([synth.sphere()], csf, np.array([-1.0, 1.0] * 3), 2)
    assert glo.shape == (1, 0) and ghi.shape == (1, 0)


def test_run_subdivision_with_taylor2_matches_oracle(vx):
    w = synth.surface()
    depth = 6
    _say("[t2] run_subdivision(taylor2) surface depth 6")
    got = {}

    def rec(level, S, lo, hi, keep, K):
        got[level] = K
        return False

    stats, _ = vx.run_subdivision(w.polys, w.domain(), depth, record=rec, taylor2=True)
    ref = orc.subdivide_t2(w.polys, 3, depth, nthreads=orc.max_threads())
    for r in ref:
        K = orc.csf_from_boxes(r["kept"], r["level"])
        assert orc.csf_sizes(K) == list(got[r["level"]]["idx"][l].shape[0] for l in range(3)), r["level"]
        assert csf_equal(got[r["level"]], K), r["level"]
    plain, _ = vx.run_subdivision(w.polys, w.domain(), depth)
    assert stats[-1]["kept"][2] < plain[-1]["kept"][2]
