"""GPU parity: HIP path (through the C ABI) against the CPU oracle.

Bar: interval endpoints bit-identical after -0 -> +0, keep flags and CSFs
identical.  The oracle computes the same canonical Horner order with the same
directed rounding, and every directed-rounding result is unique, so any
difference is a bug.
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


def _dev_csf(vx, S):
    return vx.CSF.from_arrays(S["k"], S["level"], S["idx"], S["ptr"])


def _check_level(vx, polys, S, dom, tag):
    """GPU interval_eval_level on the oracle's CSF S vs the oracle."""
    _say(f"[parity] {tag}: level {S['level']} sizes {orc.csf_sizes(S)}")
    lo_o, hi_o, _ = orc.eval_level(polys, S, dom, nthreads=orc.max_threads())
    keep_o = orc.keep_mask(lo_o, hi_o)
    lo_g, hi_g, keep_g = vx.interval_eval_level(polys, _dev_csf(vx, S), dom)
    lo_g = lo_g.cpu().numpy(); hi_g = hi_g.cpu().numpy(); keep_g = keep_g.cpu().numpy().astype(bool)
    assert bits_equal(lo_g, lo_o), (tag, "lo", first_mismatch(lo_g, lo_o))
    assert bits_equal(hi_g, hi_o), (tag, "hi", first_mismatch(hi_g, hi_o))
    assert np.array_equal(keep_g, keep_o), tag
    return keep_g


def _check_filter(vx, S, keep, tag):
    K_o = orc.csf_from_boxes(S["boxes"][keep], S["level"])
    N_o = orc.csf_from_boxes(orc.children_of(S["boxes"][keep]), S["level"] + 1) if keep.any() else None
    import torch
    kt = torch.as_tensor(keep.astype(np.uint8), device="cuda")
    K_g, N_g = vx.filter_subdivide(_dev_csf(vx, S), kt)
    assert orc.csf_sizes(K_o) == K_g.n, tag
    assert csf_equal(K_g.to_numpy(), K_o), tag
    if N_o is not None:
        assert orc.csf_sizes(N_o) == N_g.n, tag
        assert csf_equal(N_g.to_numpy(), N_o), tag


def test_tiny_every_level_eval_and_filter(vx):
    w = synth.tiny()
    recs = orc.subdivide(w.polys, w.k, w.depth)
    for r in recs:
        keep = _check_level(vx, w.polys, r["S"], w.domain(), "tiny")
        _check_filter(vx, r["S"], keep, f"tiny level {r['level']}")


def test_run_subdivision_tiny_matches_oracle(vx):
    w = synth.tiny()
    recs = orc.subdivide(w.polys, w.k, w.depth)
    seen = {}

    def record(level, S, lo, hi, keep, K):
        seen[level] = (S, lo, hi, keep, K)

    stats, kept = vx.run_subdivision(w.polys, w.domain(), w.depth, record=record)
    for r in recs:
        S, lo, hi, keep, K = seen[r["level"]]
        assert csf_equal(S, r["S"])
        assert bits_equal(lo, r["lo"]) and bits_equal(hi, r["hi"])
        assert np.array_equal(keep.astype(bool), r["keep"])
        assert stats[r["level"]]["n"] == orc.csf_sizes(r["S"])
        assert stats[r["level"]]["steps"] == int(r["steps"].sum())
    assert csf_equal(kept, orc.csf_from_boxes(recs[-1]["kept"], w.depth))


@pytest.mark.parametrize("k,d,level", [(1, 9, 6), (2, 7, 5), (3, 6, 4), (4, 4, 3)])
def test_random_k_interval_coefficients_odd_domains(vx, k, d, level):
    rng = np.random.default_rng(200 + k)
    poly = synth.small_random(k, d, seed=300 + k)[0]
    rad = np.abs(synth.small_random(k, d, seed=400 + k)[0]) * 1e-2
    polys = [(poly - rad, poly + rad), synth.small_random(k, d, seed=500 + k)[0]]
    boxes = rng.integers(0, 1 << level, size=(400, k))
    for dom in (np.array([-1.0, 1.0] * k), np.array([-0.7, 1.3] * k), np.array([0.25, 3.0] * k),
                np.array([-5.0, -0.5] * k)):
        S = orc.csf_from_boxes(boxes, level)
        keep = _check_level(vx, polys, S, dom, f"k={k} dom={dom[:2]}")
        _check_filter(vx, S, keep, f"k={k}")


def test_level0_and_straddling_cells(vx):
    """Level 0 is one cell [-1,1]^k (straddles 0): the general product path."""
    for k, d in [(1, 12), (2, 9), (3, 6), (4, 3)]:
        poly = synth.small_random(k, d, seed=600 + k)[0]
        S = orc.csf_from_boxes(np.zeros((1, k), np.int64), 0)
        _check_level(vx, [poly], S, np.array([-1.0, 1.0] * k), f"level0 k={k}")


def test_surface_levels_full_parity(vx):
    w = synth.surface()
    recs = orc.subdivide(w.polys, 3, 6, nthreads=orc.max_threads())
    for r in recs:
        keep = _check_level(vx, w.polys, r["S"], w.domain(), "surface")
        _check_filter(vx, r["S"], keep, f"surface level {r['level']}")


def test_curve_low_levels_full_parity(vx):
    w = synth.curve()
    recs = orc.subdivide(w.polys, 3, 4, nthreads=orc.max_threads())
    for r in recs:
        keep = _check_level(vx, w.polys, r["S"], w.domain(), "curve")
        _check_filter(vx, r["S"], keep, f"curve level {r['level']}")


@pytest.mark.parametrize("k", [2, 3])
def test_mixed_degrees_one_system(vx, k):
    """Polynomials of different degrees in one system (one launch per stage
    serves all of them); degrees cross the 8-entry group boundaries of the
    padded middle-stage rows."""
    rng = np.random.default_rng(700 + k)
    degs = [1, 7, 8, 9, 15, 16, 17, 23] if k == 3 else [0, 1, 5, 9, 16, 31]
    polys = [synth.small_random(k, dg, seed=800 + dg)[0] for dg in degs]
    level = 5
    boxes = rng.integers(0, 1 << level, size=(3000, k))
    S = orc.csf_from_boxes(boxes, level)
    for dom in (np.array([-1.0, 1.0] * k), np.array([-0.6, 1.1] * k)):
        keep = _check_level(vx, polys, S, dom, f"mixed k={k}")
        _check_filter(vx, S, keep, f"mixed k={k}")


def test_more_than_eight_polynomials(vx):
    """Systems larger than one launch's polynomial set are evaluated in chunks;
    the keep flag is the conjunction over all of them."""
    rng = np.random.default_rng(901)
    polys = [synth.small_random(3, 4 + (i % 5), seed=900 + i)[0] for i in range(11)]
    S = orc.csf_from_boxes(rng.integers(0, 16, size=(500, 3)), 4)
    _check_level(vx, polys, S, np.array([-1.0, 1.0] * 3), "eleven polynomials")


def test_run_without_level_times_gives_the_same_sets(vx):
    """VX_RUN_NO_TIMES only drops the timing events: every level's counts and
    the final kept CSF equal those of a timed run (the surface to level 7)."""
    w = synth.surface()
    s1, k1 = vx.run_subdivision(w.polys, w.domain(), 7)
    s2, k2 = vx.run_subdivision(w.polys, w.domain(), 7, level_times=False)
    assert [(a["n"], a["kept"], a["steps"]) for a in s1] == [(a["n"], a["kept"], a["steps"]) for a in s2]
    assert all(a["eval_ms"] == 0.0 and a["filter_ms"] == 0.0 for a in s2)
    assert all(a["eval_ms"] > 0.0 for a in s1)
    assert csf_equal(k2, k1)
