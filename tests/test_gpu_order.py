"""GPU parity of the variable-order costs (Theorem 1 under each order of the
variables) and of a subdivision run in a chosen order.

The node counts of every order come from CSFs the library builds on the
device; the oracle lists the same boxes' labels in that order and builds
its CSF on the host.  Counts and steps must be equal.  A run with the
variables reordered (coefficients transposed) must keep exactly the boxes
the oracle keeps for the transposed polynomials.
"""
import itertools
import sys

import numpy as np
import pytest

from oracle import core as orc
from paper_2406_09857_amd import synth
from tests.helpers import csf_equal

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


def _cases():
    rng = np.random.default_rng(77)
    return {
        "curve_level6": (synth.curve(), 6, None),
        "tiny_level8": (synth.tiny(), 8, None),
        "random_k4_level3": (synth.Workload("r4", 4, 3, synth.small_random(4, 5, seed=45, npolys=2)), 3,
                             rng.integers(0, 8, size=(900, 4))),
        "single_box_k3": (synth.surface(), 5, np.array([[3, 17, 30]])),
    }


@pytest.mark.parametrize("name", list(_cases()))
def test_order_costs_match_oracle(vx, name):
    w, level, boxes = _cases()[name]
    if boxes is None:
        boxes = orc.subdivide(w.polys, w.k, level, w.domain(), nthreads=orc.max_threads())[-1]["S"]["boxes"]
    S = orc.csf_from_boxes(boxes, level)
    degrees = [orc.poly_degree(p) for p in w.polys]
    orders = list(itertools.permutations(range(w.k)))
    _say(f"[order] {name}: {len(S['boxes'])} boxes, {len(orders)} orders")
    want = orc.order_costs(S["boxes"], level, degrees, orders)
    got = vx.variable_order_costs(w.polys, _dev_csf(vx, S), orders)
    assert [(tuple(o), c, st) for o, c, st in got] == want
    assert got[0][1] == orc.csf_sizes(S)  # the default order is the CSF itself
    only_counts = vx.variable_order_costs(None, _dev_csf(vx, S), orders[-2:])
    assert [c for _, c, _ in only_counts] == [c for _, c, _ in want[-2:]]


def test_run_in_the_cheapest_order_matches_oracle(vx):
    """The points system (three trivariate degree-20 polynomials): choose the
    order with the fewest steps on the level-5 set, then run levels 0..6 in it;
    every level's kept set equals the oracle's for the transposed
    polynomials, and mapped back it encloses the same points as a run in the
    default order (the kept boxes of level 6 in the two runs overlap)."""
    w = synth.points()
    recs = orc.subdivide(w.polys, 3, 5, w.domain(), nthreads=orc.max_threads())
    S5 = recs[-1]["S"]
    costs = vx.variable_order_costs(w.polys, _dev_csf(vx, S5))
    best = min(costs, key=lambda c: c[2])[0]
    _say(f"[order] points: costs {[(o, s) for o, _, s in costs]}, best {best}")
    tp = [np.ascontiguousarray(np.transpose(p, best)) for p in w.polys]
    for a, b in zip(vx.permute_variables(w.polys, best), tp):
        assert np.array_equal(a, b)
    want = orc.subdivide(tp, 3, 6, w.domain(), nthreads=orc.max_threads())
    seen = {}
    stats, kept = vx.run_subdivision(vx.permute_variables(w.polys, best), w.domain(), 6,
                                     record=lambda lv, S, lo, hi, keep, K: seen.__setitem__(lv, K))
    for r in want:
        assert csf_equal(seen[r["level"]], orc.csf_from_boxes(r["kept"], r["level"])), r["level"]
        assert stats[r["level"]]["steps"] == int(r["steps"].sum())
    plain = orc.subdivide(w.polys, 3, 6, w.domain(), nthreads=orc.max_threads())[-1]["kept"]
    inv = np.argsort(best)
    back = want[-1]["kept"][:, inv]
    common = set(map(tuple, back)) & set(map(tuple, plain))
    assert len(common) > 0.5 * min(len(back), len(plain))


def test_order_costs_reject_bad_orders(vx):
    w = synth.tiny()
    S = orc.csf_from_boxes(np.array([[1, 2], [3, 0]]), 2)
    with pytest.raises(vx.VxError) as e:
        vx.variable_order_costs(w.polys, _dev_csf(vx, S), [(0, 0)])
    assert e.value.code == vx.VX_EINVAL


def test_run_permuted_interval_system(vx):
    """Interval coefficients on a non-dyadic domain, variables reordered
    (x3, x1, x2): every level's kept set equals the oracle's for the
    transposed pairs."""
    a, b = synth.small_random(3, 5, seed=51, npolys=2)
    rad = np.abs(synth.small_random(3, 5, seed=52)[0]) * 1e-2
    polys = [(a - rad, a + rad), b]
    order = (2, 0, 1)
    tp = [(np.ascontiguousarray(np.transpose(a - rad, order)), np.ascontiguousarray(np.transpose(a + rad, order))),
          np.ascontiguousarray(np.transpose(b, order))]
    dom = np.array([-0.7, 1.3] * 3)
    want = orc.subdivide(tp, 3, 5, dom, nthreads=orc.max_threads())
    seen = {}
    vx.run_subdivision(vx.permute_variables(polys, order), dom, 5,
                       record=lambda lv, S, lo, hi, keep, K: seen.__setitem__(lv, K))
    for r in want:
        if len(r["S"]["boxes"]):
            assert csf_equal(seen[r["level"]], orc.csf_from_boxes(r["kept"], r["level"])), r["level"]


def _near_plane_x3(seed):
    """x3 - 1/3 plus a small random degree-4 perturbation: a surface that is a
    graph over (x1, x2), cheapest with x3 as the first CSF variable."""
    p = 0.05 * synth.small_random(3, 4, seed=seed)[0]
    p[0, 0, 1] += 1.0
    p[0, 0, 0] -= 1.0 / 3.0
    return p


def _auto_cases():
    r = synth.small_random(3, 5, seed=91, npolys=2)
    lo = r[1] - 1e-6 * np.abs(r[1])
    hi = r[1] + 1e-6 * np.abs(r[1])
    return {
        "near_plane_x3": ([_near_plane_x3(90)], 3, 7, 4, np.array([-1.0, 1.0] * 3)),
        "points_system": (synth.points().polys, 3, 7, 5, synth.points().domain()),
        "interval_system_odd_domain": ([_near_plane_x3(92), (lo, hi)], 3, 6, 3,
                                       np.array([-0.7, 1.1, -1.0, 0.9, -1.3, 1.0])),
        "tiny": (synth.tiny().polys, 2, 8, 6, synth.tiny().domain()),
    }


@pytest.mark.parametrize("name", list(_auto_cases()))
def test_run_with_automatic_variable_order_matches_oracle(vx, name):
    """VX_RUN_AUTO_ORDER: the order is Theorem 1's argmin over the children of
    the probe level's kept set (ties to the first permutation in
    lexicographic order), found here by the oracle; the run then equals, level
    by level, the oracle's run of the transposed polynomials on the permuted
    domain (evaluated set and kept set of every level)."""
    polys, k, depth, probe, dom = _auto_cases()[name]
    _say(f"[order] automatic order: {name}, probe level {probe}, depth {depth}")
    pre = orc.subdivide(polys, k, probe, dom=dom, nthreads=orc.max_threads())[-1]
    degrees = [orc.poly_degree(p) for p in polys]
    orders = list(itertools.permutations(range(k)))
    if len(pre["kept"]):
        costs = orc.order_costs(orc.children_of(pre["kept"]), probe + 1, degrees, orders)
        best = min(range(len(orders)), key=lambda o: (costs[o][2], o))
    else:
        best = 0
    order = list(orders[best])
    got = {}

    def rec(level, S, lo, hi, keep, K):
        got[level] = (S, K)
        return False

    stats, _ = vx.run_subdivision(polys, dom, depth, record=rec, auto_order=True, auto_order_at=probe)
    assert all(s["axes"] == order for s in stats), (stats[0]["axes"], order)
    tp = vx.permute_variables(polys, order)
    tdom = np.asarray(dom, np.float64).reshape(k, 2)[order].reshape(-1)
    ref = orc.subdivide(tp, k, depth, dom=tdom, nthreads=orc.max_threads())
    for r in ref:
        if r["level"] not in got:
            assert len(r["S"]["boxes"]) == 0
            continue
        S, K = got[r["level"]]
        assert csf_equal(S, r["S"]), (name, r["level"])
        assert csf_equal(K, orc.csf_from_boxes(r["kept"], r["level"])), (name, r["level"])
    if name == "near_plane_x3":
        assert order[0] == 2
    plain, _ = vx.run_subdivision(polys, dom, depth)
    _say(f"[order] {name}: order {order}, steps {sum(s['steps'] for s in stats)} against "
         f"{sum(s['steps'] for s in plain)} in the given order")
    assert all(s["axes"] == list(range(k)) for s in plain)
