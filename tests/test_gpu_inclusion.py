"""Inclusion criterion C1 (Sec. 3.2) on the GPU against the oracle, in both
forms: sign change over the vertices, and the order-2 Taylor variant (bounds
at the two extreme vertices of the linear part).

Bar: the certification flags (per polynomial and box) equal the oracle's
exactly.  Cases: every level of `tiny`, the `surface` kept set at level 6
(thousands of boxes, several tiles and ragged tails), random k = 1..4 with
two polynomials, interval coefficients and non-dyadic domains, level-14 box
sets whose vertex nodes have narrow and wide label windows (the two merge
paths of the vertex CSF), a plane on a grid plane (zeros at vertices certify
nothing), the sphere, level 0 and an empty set; at full size, the surface's final kept set (level 9) with a seeded
sample re-checked by the oracle on a CSF of the sample alone (a box's flag
depends on its own vertices only).
"""
import sys
import time

import numpy as np
import pytest

from oracle import core as orc
from paper_2406_09857_amd import synth

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


METHODS = ["vertices", "taylor"]


def _ref(polys, S, dom, method):
    fn = orc.taylor_inclusion_level if method == "taylor" else orc.inclusion_level
    return fn(polys, S, dom, nthreads=orc.max_threads())


def _check(vx, polys, S, dom, tag, method="vertices"):
    _say(f"[c1] {tag} ({method}): level {S['level']} sizes {orc.csf_sizes(S)}")
    ref = _ref(polys, S, dom, method)
    csf = vx.CSF.from_arrays(S["k"], S["level"], S["idx"], S["ptr"])
    got = vx.inclusion_test(polys, csf, dom, taylor=method == "taylor").cpu().numpy().astype(bool)
    assert got.shape == ref.shape, tag
    bad = np.argwhere(got != ref)
    assert len(bad) == 0, (tag, bad[:5].tolist(), int(got.sum()), int(ref.sum()))
    return int(ref.sum())


@pytest.mark.parametrize("method", METHODS)
def test_tiny_every_level(vx, method):
    w = synth.tiny()
    for r in orc.subdivide(w.polys, 2, 8):
        _check(vx, w.polys, r["S"], w.domain(), "tiny", method)


@pytest.mark.parametrize("method", METHODS)
def test_surface_kept_level6(vx, method):
    w = synth.surface()
    r = orc.subdivide(w.polys, 3, 6, nthreads=orc.max_threads())[-1]
    K = orc.csf_from_boxes(r["kept"], 6)
    assert _check(vx, w.polys, K, w.domain(), "surface kept", method) > 0


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("k,d,level", [(1, 9, 7), (2, 7, 5), (3, 6, 4), (4, 4, 3)])
def test_random_k_odd_domain_interval_coefficients(vx, k, d, level, method):
    rng = np.random.default_rng(500 + k)
    c = synth.small_random(k, d, seed=510 + k, npolys=2)
    polys = [(c[0] - 1e-3 * np.abs(c[0]), c[0] + 1e-3 * np.abs(c[0])), c[1]]
    dom = np.array([-0.7, 1.3] * k)
    boxes = rng.integers(0, 1 << level, size=(600, k))
    S = orc.csf_from_boxes(boxes, level)
    _check(vx, polys, S, dom, f"k{k}", method)


@pytest.mark.parametrize("k", [2, 3])
def test_vertex_csf_wide_label_windows(vx, k):
    """The vertex CSF is merged per vertex node from bitmaps over the label
    window of its children when that window spans at most 4096 labels, and
    by a sequential merge otherwise: at level 14, boxes spread over the whole
    axis take the second path, a clustered set beside them the first."""
    rng = np.random.default_rng(900 + k)
    level = 14
    spread = rng.integers(0, 1 << level, size=(400, k))
    cluster = rng.integers(0, 64, size=(400, k)) + (1 << (level - 1))
    # boxes cut by the plane x1 = 0.5 + 2^-20 (inside cells of x1 label 3 * 2^(level-2))
    cut = rng.integers(0, 1 << level, size=(300, k))
    cut[:, 0] = 3 << (level - 2)
    S = orc.csf_from_boxes(np.concatenate([spread, cluster, cut]), level)
    dom = np.array([-1.0, 1.0] * k)
    c = synth.small_random(k, 5, seed=920 + k, npolys=2)
    plane = synth.monomial_poly(k, 1, {tuple([1] + [0] * (k - 1)): 1.0, tuple([0] * k): -(0.5 + 2.0 ** -20)})
    assert _check(vx, [c[0], c[1], plane], S, dom, f"wide windows k{k}") > 0


@pytest.mark.parametrize("method", METHODS)
def test_closed_forms_and_edge_cases(vx, method):
    k = 3
    S = orc.csf_from_boxes(np.random.default_rng(7).integers(0, 16, size=(500, k)), 4)
    dom = np.array([-1.0, 1.0] * k)
    on_grid = synth.monomial_poly(k, 1, {(0, 0, 1): 1.0, (0, 0, 0): 0.5})  # x3 = -0.5, a grid plane
    between = synth.monomial_poly(k, 1, {(0, 0, 1): 1.0, (0, 0, 0): -0.34375})
    _check(vx, [on_grid, between, synth.sphere()], S, dom, "planes+sphere", method)
    root = orc.csf_from_boxes(np.zeros((1, k), np.int64), 0)
    _check(vx, [synth.sphere(), between], root, dom, "level 0", method)
    E = orc.csf_from_boxes(np.zeros((0, k), np.int64), 5)
    csf = vx.CSF.from_arrays(k, 5, E["idx"], E["ptr"])
    assert vx.inclusion_test([synth.sphere()], csf, dom, taylor=method == "taylor").shape == (1, 0)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("method", METHODS)
def test_surface_final_kept_set_sampled(vx, method):
    w = synth.surface()
    dom = w.domain()
    t = time.time()
    _, kept = vx.run_subdivision(w.polys, dom, w.depth)
    K = vx.CSF.from_arrays(3, w.depth, kept["idx"], kept["ptr"])
    got = vx.inclusion_test(w.polys, K, dom, taylor=method == "taylor").cpu().numpy().astype(bool)[0]
    _say(f"[c1] surface level {w.depth}: {K.nboxes} kept boxes, {int(got.sum())} certified, {time.time() - t:.1f} s")
    # leaf labels of the kept CSF
    idx = [np.asarray(a, np.int64) for a in kept["idx"]]
    ptr = [np.asarray(a, np.int64) for a in kept["ptr"]]
    up2 = np.searchsorted(ptr[1], np.arange(len(idx[2])), side="right") - 1
    up1 = np.searchsorted(ptr[0], up2, side="right") - 1
    B = np.stack([idx[0][up1], idx[1][up2], idx[2]], axis=1)
    rng = np.random.default_rng(2408)
    pick = np.sort(rng.choice(len(B), size=min(len(B), 4000), replace=False))
    T = orc.csf_from_boxes(B[pick], w.depth)
    assert np.array_equal(T["boxes"], B[pick])
    ref = _ref(w.polys, T, dom, method)[0]
    assert np.array_equal(got[pick], ref), np.flatnonzero(got[pick] != ref)[:5]
    assert 0 < got.sum() < len(got)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("name,depth,c1_from", [("tiny", 8, 3), ("surface", 6, 3)])
def test_run_subdivision_with_inclusion_matches_oracle(vx, method, name, depth, c1_from):
    """Algorithm 3 with C0 and C1 (from level c1_from on): at every level the
    evaluated CSF, the certified boxes (keep = 2), their count and the
    continuing CSF equal the oracle's."""
    from tests.helpers import csf_equal
    w = getattr(synth, name)()
    got = {}

    def rec(level, S, lo, hi, keep, K):
        got[level] = (S, keep.copy(), K)
        return False

    stats, _ = vx.run_subdivision(w.polys, w.domain(), depth, record=rec, inclusion=method, inclusion_from=c1_from)
    ref = orc.subdivide_c1(w.polys, w.k, depth, c1_from, dom=w.domain(), nthreads=orc.max_threads(),
                           taylor=method == "taylor")
    total = 0
    for r in ref:
        L = r["level"]
        S, keep, K = got[L]
        assert csf_equal(S, r["S"]), L
        cert = r["S"]["boxes"][keep == 2]
        assert np.array_equal(cert, r["certified"]), L
        assert stats[L]["certified"] == len(r["certified"]), L
        assert csf_equal(K, orc.csf_from_boxes(r["kept"], L)), L
        total += len(cert)
    _say(f"[c1] {name} ({method}) to level {depth}, C1 from {c1_from}: {total} certified boxes")
    assert total > 0
