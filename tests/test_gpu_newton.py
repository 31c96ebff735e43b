"""Newton interval inclusion test (Krawczyk's form, Sec. 3.2) on the GPU
against the oracle.

Bar: the certification flags and the Krawczyk enclosures K (every endpoint,
after -0 -> +0) equal the oracle's.  Cases: the circle-line system at
several levels (every box), random square systems for k = 1..4 with
interval coefficients on a non-dyadic domain, linear systems, a singular
system, an empty set, and the `points` workload (three trivariate degree-20
polynomials): every level-6..9 set of the oracle's subdivision, and the
final kept set of a GPU run to level 9 (the benchmark's configuration).
"""
import sys

import numpy as np
import pytest

from oracle import core as orc
from paper_2406_09857_amd import synth
from tests.helpers import bits_equal, first_mismatch

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


def _check(vx, polys, S, dom, tag, want_k=True):
    _say(f"[newton] {tag}: level {S['level']} sizes {orc.csf_sizes(S)}")
    ref, Kref = orc.newton_level(polys, S, dom, nthreads=orc.max_threads(), want_k=True)
    csf = vx.CSF.from_arrays(S["k"], S["level"], S["idx"], S["ptr"])
    got, K = vx.newton_test(polys, csf, dom, want_k=True)
    got = got.cpu().numpy().astype(bool)
    K = K.cpu().numpy()
    assert np.array_equal(got, ref), (tag, np.flatnonzero(got != ref)[:5])
    if want_k:
        assert bits_equal(K, Kref), (tag, first_mismatch(K, Kref))
    return int(ref.sum())


def _all_boxes(k, level):
    n = 1 << level
    return np.array(np.meshgrid(*[np.arange(n)] * k, indexing="ij")).reshape(k, -1).T


def test_circle_and_line_every_box(vx):
    F1 = synth.monomial_poly(2, 2, {(2, 0): 1.0, (0, 2): 1.0, (0, 0): -0.3})
    F2 = synth.monomial_poly(2, 2, {(1, 0): 1.0, (0, 1): -1.0})
    for level in (3, 6, 8):
        S = orc.csf_from_boxes(_all_boxes(2, level), level)
        assert _check(vx, [F1, F2], S, np.array([-1.0, 1.0] * 2), "circle-line") == 2


@pytest.mark.parametrize("k,d,level", [(1, 9, 8), (2, 6, 6), (3, 4, 4), (4, 3, 3)])
def test_random_square_systems_odd_domain_interval_coefficients(vx, k, d, level):
    rng = np.random.default_rng(600 + k)
    c = synth.small_random(k, d, seed=610 + k, npolys=k)
    polys = [(c[0] - 1e-6 * np.abs(c[0]), c[0] + 1e-6 * np.abs(c[0]))] + c[1:]
    dom = np.array([-0.7, 1.3] * k)
    boxes = rng.integers(0, 1 << level, size=(2000, k))
    S = orc.csf_from_boxes(boxes, level)
    _check(vx, polys, S, dom, f"k{k}")


def test_linear_singular_and_empty(vx):
    k, level = 2, 4
    S = orc.csf_from_boxes(_all_boxes(k, level), level)
    dom = np.array([-1.0, 1.0] * k)
    lin = [synth.monomial_poly(2, 1, {(1, 0): 1.0, (0, 1): 1.0, (0, 0): -0.40625}),
           synth.monomial_poly(2, 1, {(0, 1): 1.0, (0, 0): 0.15625})]
    assert _check(vx, lin, S, dom, "linear") >= 1
    par = [synth.monomial_poly(2, 1, {(1, 0): 1.0, (0, 1): 1.0}),
           synth.monomial_poly(2, 1, {(1, 0): 1.0, (0, 1): 1.0, (0, 0): -0.1})]
    assert _check(vx, par, S, dom, "parallel") == 0
    E = orc.csf_from_boxes(np.zeros((0, k), np.int64), 5)
    csf = vx.CSF.from_arrays(k, 5, E["idx"], E["ptr"])
    assert vx.newton_test(lin, csf, dom).shape == (0,)


def test_points_workload_levels_6_to_9(vx):
    w = synth.points()
    recs = orc.subdivide(w.polys, 3, 9, nthreads=orc.max_threads())
    total = 0
    for r in recs[6:]:
        total += _check(vx, w.polys, r["S"], w.domain(), "points")
    assert total > 0


def test_points_final_kept_set_of_a_gpu_run(vx):
    w = synth.points()
    dom = w.domain()
    _, kept = vx.run_subdivision(w.polys, dom, w.depth)
    T = {"k": 3, "level": w.depth, "idx": kept["idx"], "ptr": kept["ptr"]}
    idx = [np.asarray(a, np.int64) for a in kept["idx"]]
    ptr = [np.asarray(a, np.int64) for a in kept["ptr"]]
    up2 = np.searchsorted(ptr[1], np.arange(len(idx[2])), side="right") - 1
    up1 = np.searchsorted(ptr[0], up2, side="right") - 1
    T["boxes"] = np.stack([idx[0][up1], idx[1][up2], idx[2]], axis=1)
    n = _check(vx, w.polys, T, dom, "points final kept")
    _say(f"[newton] points level {w.depth}: {len(T['boxes'])} kept boxes, {n} certified")


def test_run_subdivision_with_newton_matches_oracle(vx):
    """Algorithm 3 on the points workload with C1 = the Newton test from
    level 6 on: every level's CSF, certified boxes and continuing CSF equal
    the oracle's."""
    from tests.helpers import csf_equal
    w = synth.points()
    depth, c1_from = 9, 6
    got = {}

    def rec(level, S, lo, hi, keep, K):
        got[level] = (S, keep.copy(), K)
        return False

    stats, _ = vx.run_subdivision(w.polys, w.domain(), depth, record=rec, inclusion="vertices",
                                  inclusion_from=c1_from)
    ref = orc.subdivide_c1(w.polys, 3, depth, c1_from, dom=w.domain(), nthreads=orc.max_threads())
    total = 0
    for r in ref:
        L = r["level"]
        S, keep, K = got[L]
        assert csf_equal(S, r["S"]), L
        assert np.array_equal(r["S"]["boxes"][keep == 2], r["certified"]), L
        assert stats[L]["certified"] == len(r["certified"]), L
        assert csf_equal(K, orc.csf_from_boxes(r["kept"], L)), L
        total += len(r["certified"])
    _say(f"[newton] points loop: {total} boxes certified")
    assert total > 0


# ---------------------------------------------------------------------------
# Fewer polynomials than variables: the test on the span of the gradients
# ---------------------------------------------------------------------------

def _check_span(vx, polys, S, dom, tag):
    _say(f"[newton-span] {tag}: level {S['level']} sizes {orc.csf_sizes(S)}")
    ref, Kref, _ = orc.newton_span_level(polys, S, dom, nthreads=orc.max_threads(), want_k=True)
    csf = vx.CSF.from_arrays(S["k"], S["level"], S["idx"], S["ptr"])
    got, K = vx.newton_test(polys, csf, dom, want_k=True)
    got = got.cpu().numpy().astype(bool)
    K = K.cpu().numpy()
    assert np.array_equal(got, ref), (tag, np.flatnonzero(got != ref)[:5])
    assert bits_equal(K, Kref), (tag, first_mismatch(K, Kref))
    return int(ref.sum())


def test_span_line_and_circle(vx):
    """Two planes (a line) on every box of levels 2 and 4; the circle of
    x^2 + y^2 + z^2 = 0.5 and z = 0.3 on the oracle's kept sets of levels
    4..7: flags and K bit for bit."""
    dom = np.array([-1.0, 1.0] * 3)
    F1 = synth.monomial_poly(3, 1, {(1, 0, 0): 1.0, (0, 0, 0): -0.3})
    F2 = synth.monomial_poly(3, 1, {(0, 1, 0): 1.0, (0, 0, 0): 0.21})
    for level in (2, 4):
        S = orc.csf_from_boxes(_all_boxes(3, level), level)
        _check_span(vx, [F1, F2], S, dom, f"line level {level}")
    C1 = synth.monomial_poly(3, 2, {(2, 0, 0): 1.0, (0, 2, 0): 1.0, (0, 0, 2): 1.0, (0, 0, 0): -0.5})
    C2 = synth.monomial_poly(3, 1, {(0, 0, 1): 1.0, (0, 0, 0): -0.3})
    total = 0
    for r in orc.subdivide([C1, C2], 3, 7, nthreads=orc.max_threads())[4:]:
        total += _check_span(vx, [C1, C2], r["S"], dom, f"circle level {r['level']}")
    assert total > 0


@pytest.mark.parametrize("k,m,d,level", [(2, 1, 6, 5), (3, 1, 5, 4), (3, 2, 4, 5), (4, 2, 3, 3), (4, 3, 3, 3)])
def test_span_random_systems_odd_domain_interval_coefficients(vx, k, m, d, level):
    """Random systems of m < k polynomials, one with interval coefficients,
    on a non-dyadic domain, on the oracle's kept set of the level."""
    c = synth.small_random(k, d, seed=700 + 10 * k + m, npolys=m)
    polys = [(c[0] - 1e-6 * np.abs(c[0]), c[0] + 1e-6 * np.abs(c[0]))] + list(c[1:])
    dom = np.array([-0.9, 1.1] * k)
    S = orc.subdivide(polys, k, level, dom=dom, nthreads=orc.max_threads())[-1]["S"]
    _check_span(vx, polys, S, dom, f"k{k} m{m} d{d}")


def test_span_on_the_curve_level_8(vx):
    """The curve workload (two degree-100 trivariate polynomials) on 20,000
    seeded boxes of the oracle's kept set of level 8 (as a CSF of their
    own): flags and K bit for bit.  Nothing is certified there (nor on a
    sample of level 10): the gradients of these polynomials enclosed on a
    box are far wider than their midpoints separate, so K is wider than the
    cube; the test certifies on the circle and the random systems above."""
    from tests.helpers import oracle_curve_kept
    w = synth.curve()
    kept = np.asarray(oracle_curve_kept(orc, synth, 8), np.int64)
    rng = np.random.default_rng(880)
    pick = kept[np.sort(rng.choice(len(kept), 20000, replace=False))]
    S = orc.csf_from_boxes(pick, 8)
    n = _check_span(vx, w.polys, S, w.domain(), "curve level 8 sample")
    _say(f"[newton-span] curve level 8: {n} of 20000 sampled boxes certified")


def test_span_in_the_loop_matches_oracle(vx):
    """Algorithm 3 on the circle (sphere and plane) with C1 = the span test
    from level 4 on: every level's CSF, certified boxes and continuing CSF
    equal the oracle's."""
    from tests.helpers import csf_equal
    C1 = synth.monomial_poly(3, 2, {(2, 0, 0): 1.0, (0, 2, 0): 1.0, (0, 0, 2): 1.0, (0, 0, 0): -0.5})
    C2 = synth.monomial_poly(3, 1, {(0, 0, 1): 1.0, (0, 0, 0): -0.3})
    dom = np.array([-1.0, 1.0] * 3)
    depth, c1_from = 7, 4
    got = {}

    def rec(level, S, lo, hi, keep, K):
        got[level] = (S, keep.copy(), K)
        return False

    stats, _ = vx.run_subdivision([C1, C2], dom, depth, record=rec, inclusion="vertices", inclusion_from=c1_from)
    ref = orc.subdivide_c1([C1, C2], 3, depth, c1_from, dom=dom, nthreads=orc.max_threads())
    total = 0
    for r in ref:
        L = r["level"]
        S, keep, K = got[L]
        assert csf_equal(S, r["S"]), L
        assert np.array_equal(r["S"]["boxes"][keep == 2], r["certified"]), L
        assert stats[L]["certified"] == len(r["certified"]), L
        assert csf_equal(K, orc.csf_from_boxes(r["kept"], L)), L
        total += len(r["certified"])
    _say(f"[newton-span] circle loop: {total} boxes certified")
    assert total > 0
