"""GPU parity of the early exit for systems (run_subdivision_ex with
VX_RUN_EARLY_EXIT): polynomial p is evaluated only on the boxes that
polynomials 0..p-1 kept.

A box is excluded as soon as one polynomial of the system excludes it
(Sec. 3.2, exclusion criterion for systems), so every level's kept set is the
oracle's plain C0 set, bit for bit.  The work is pinned too: the steps the
run reports equal Theorem 1's count summed over the polynomials, each on the
CSF of the boxes the earlier ones kept, computed from the oracle's enclosures.
"""
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


def _early_steps(polys, k, rec):
    """Theorem 1 steps of the early-exit evaluation of one oracle level."""
    S = rec["S"]
    alive = np.ones(len(S["boxes"]), bool)
    total = 0
    for p, poly in enumerate(polys):
        sub = orc.csf_from_boxes(S["boxes"][alive], S["level"])
        total += sum(orc.theorem1_steps(k, orc.poly_degree(poly), orc.csf_sizes(sub)))
        alive &= orc.keep_mask(rec["lo"][p:p + 1], rec["hi"][p:p + 1])
        if not alive.any():
            break
    return total


def _interval_system():
    a, b = synth.small_random(3, 6, seed=47, npolys=2)
    rad = np.abs(synth.small_random(3, 6, seed=48)[0]) * 1e-2
    return [(a - rad, a + rad), b]


def _systems():
    pos = synth.monomial_poly(2, 2, {(2, 0): 1.0, (0, 2): 1.0, (0, 0): 1.0})  # > 0 off level 0
    return {
        "curve_d100": (synth.curve(), 6),
        "points_k3_d20": (synth.points(), 6),
        "random_k2_np3": (synth.Workload("r2", 2, 8, synth.small_random(2, 7, seed=41, npolys=3)), 8),
        "random_k4_np2": (synth.Workload("r4", 4, 4, synth.small_random(4, 4, seed=43, npolys=2)), 4),
        # interval coefficients on a non-dyadic domain
        "interval_k3_odd_domain": (synth.Workload("iv", 3, 6, _interval_system(), dom=(-0.7, 1.3)), 6),
        # disjoint planes: the second polynomial empties the first one's survivors
        "disjoint_planes": (synth.Workload("pl", 3, 6, [synth.plane_x1(3, 0.3), synth.plane_x1(3, -0.45)]), 6),
        # the first polynomial excludes every box of level 1: the later ones never run
        "first_excludes_all": (synth.Workload("pos", 2, 4, [pos, synth.circle()]), 4),
    }


@pytest.mark.parametrize("name", list(_systems()))
def test_early_exit_kept_sets_and_steps_match_oracle(vx, name):
    w, depth = _systems()[name]
    polys, k, dom = w.polys, w.k, w.domain()
    _say(f"[early] {name}: k={k} np={len(polys)} depth={depth}")
    recs = orc.subdivide(polys, k, depth, dom, nthreads=orc.max_threads())
    seen = {}

    def record(level, S, lo, hi, keep, K):
        assert lo is None and hi is None and keep is None
        seen[level] = (S, K)

    stats, kept = vx.run_subdivision(polys, dom, depth, record=record, early_exit=True)
    plain, kept_plain = vx.run_subdivision(polys, dom, depth)
    for r in recs:
        lv = r["level"]
        if len(r["S"]["boxes"]) == 0:  # the set ran empty: no callback, empty records
            assert lv not in seen and stats[lv]["n"] == [0] * k and stats[lv]["steps"] == 0, (name, lv)
            continue
        S, K = seen[lv]
        assert csf_equal(S, r["S"]), (name, lv)
        assert csf_equal(K, orc.csf_from_boxes(r["kept"], lv)), (name, lv)
        assert stats[lv]["n"] == orc.csf_sizes(r["S"]), (name, lv)
        assert stats[lv]["steps"] == _early_steps(polys, k, r), (name, lv)
        assert stats[lv]["n"] == plain[lv]["n"] and stats[lv]["kept"] == plain[lv]["kept"], (name, lv)
        assert stats[lv]["steps"] <= plain[lv]["steps"], (name, lv)
    if kept is None:
        assert kept_plain is None and len(recs[-1]["kept"]) == 0
    else:
        assert csf_equal(kept, kept_plain)
        assert csf_equal(kept, orc.csf_from_boxes(recs[-1]["kept"], depth))


def test_early_exit_from_a_level(vx):
    """VX_RUN_EARLY_EXIT_FROM(4): levels 0..3 run as without the flag (full
    enclosures in the callback, bit-identical to the oracle's), levels 4..6
    with the early exit; every kept set is the oracle's."""
    from tests.helpers import bits_equal
    w = synth.curve()
    polys, k, dom = w.polys, w.k, w.domain()
    recs = orc.subdivide(polys, k, 6, dom, nthreads=orc.max_threads())
    seen = {}

    def record(level, S, lo, hi, keep, K):
        seen[level] = (lo, hi, keep, K)

    stats, _ = vx.run_subdivision(polys, dom, 6, record=record, early_exit=True, early_exit_from=4)
    for r in recs:
        lv = r["level"]
        lo, hi, keep, K = seen[lv]
        assert csf_equal(K, orc.csf_from_boxes(r["kept"], lv)), lv
        if lv < 4:
            assert bits_equal(lo, r["lo"]) and bits_equal(hi, r["hi"]), lv
            assert np.array_equal(keep.astype(bool), r["keep"]), lv
            assert stats[lv]["steps"] == int(r["steps"].sum()), lv
        else:
            assert lo is None and keep is None, lv
            assert stats[lv]["steps"] == _early_steps(polys, k, r), lv
    with pytest.raises(ValueError):
        vx.run_subdivision(polys, dom, 2, early_exit_from=1)


def test_early_exit_saves_work_on_the_curve(vx):
    """On the curve the first polynomial already excludes boxes from level 3
    on, so the second one runs on a strict subset of every later level."""
    w = synth.curve()
    stats, _ = vx.run_subdivision(w.polys, w.domain(), 8, early_exit=True, want_kept=False, level_times=False)
    plain, _ = vx.run_subdivision(w.polys, w.domain(), 8, want_kept=False, level_times=False)
    assert [s["kept"] for s in stats] == [s["kept"] for s in plain]
    assert all(a["steps"] < b["steps"] for a, b in zip(stats[3:], plain[3:]))


def test_early_exit_one_polynomial_is_the_plain_run(vx):
    w = synth.surface()
    s1, k1 = vx.run_subdivision(w.polys, w.domain(), 6, early_exit=True)
    s2, k2 = vx.run_subdivision(w.polys, w.domain(), 6)
    assert [(a["n"], a["kept"], a["steps"]) for a in s1] == [(a["n"], a["kept"], a["steps"]) for a in s2]
    assert csf_equal(k1, k2)


def test_early_exit_rejects_taylor_and_inclusion(vx):
    w = synth.curve(degree=8, depth=3)
    with pytest.raises(vx.VxError) as e:
        vx.run_subdivision(w.polys, w.domain(), 3, early_exit=True, mean_value=True)
    assert e.value.code == vx.VX_EINVAL
    with pytest.raises(vx.VxError) as e:
        vx.run_subdivision(w.polys, w.domain(), 3, early_exit=True, taylor2=True)
    assert e.value.code == vx.VX_EINVAL
    p = synth.points(k=2, degree=4)
    with pytest.raises(vx.VxError) as e:
        vx.run_subdivision(p.polys, p.domain(), 3, early_exit=True, inclusion="vertices", inclusion_from=2)
    assert e.value.code == vx.VX_EINVAL
