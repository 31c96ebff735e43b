"""Batched persistent subdivision (many systems per launch, HIP graph,
autotuner) against the oracle and against the plain single-system path.

Bar: for every system, the last level's boxes, enclosures (bitwise, -0 ->
+0) and keep flags, and the per-level node counts, equal those of the
system run alone.
"""
import sys
import time

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


def _host(r):
    """Host copies of a batch result's last level and kept set."""
    return {"last": r["last"].to_numpy(), "kept": r["kept"].to_numpy(), "lo": r["lo"].cpu().numpy(),
            "hi": r["hi"].cpu().numpy(), "keep": r["keep"].cpu().numpy().astype(bool), "stats": r["stats"],
            "steps": r["steps"]}


def _sub(csf, s):
    """System s's part of a batched CSF (numpy dict, depth 0 = system) as a
    plain 3-depth CSF (idx, ptr rebased) plus its leaf range; None if absent."""
    idx, ptr = csf["idx"], csf["ptr"]
    q = int(np.searchsorted(idx[0], s))
    if q >= len(idx[0]) or idx[0][q] != s:
        return None
    a, b = [q], [q + 1]
    for l in range(3):
        a.append(int(ptr[l][a[-1]]))
        b.append(int(ptr[l][b[-1]]))
    sub_idx = [idx[l + 1][a[l + 1]:b[l + 1]] for l in range(3)]
    sub_ptr = [ptr[l + 1][a[l + 1]:b[l + 1] + 1] - a[l + 2] for l in range(2)]
    return {"idx": sub_idx, "ptr": sub_ptr, "leaves": (a[3], b[3])}


def _csf_match(sub, plain) -> bool:
    if sub is None:
        return len(plain["idx"][2]) == 0
    return (all(np.array_equal(sub["idx"][l], np.asarray(plain["idx"][l])) for l in range(3))
            and all(np.array_equal(sub["ptr"][l], np.asarray(plain["ptr"][l])) for l in range(2)))


def _check_system(h, s, S, lo, hi, keep, K, tag):
    """System s of host batch result h against a plain last level (S, lo,
    hi, keep, K as CSF dicts / arrays)."""
    sub = _sub(h["last"], s)
    assert _csf_match(sub, S), (tag, s, "evaluated set")
    if sub is not None:
        a, b = sub["leaves"]
        assert bits_equal(h["lo"][a:b], lo), (tag, s, "lo", first_mismatch(h["lo"][a:b], lo))
        assert bits_equal(h["hi"][a:b], hi), (tag, s, "hi", first_mismatch(h["hi"][a:b], hi))
        assert np.array_equal(h["keep"][a:b], keep), (tag, s, "keep")
    assert _csf_match(_sub(h["kept"], s), K), (tag, s, "kept set")


def _empty_csf():
    return {"idx": [np.zeros(0, np.int32)] * 3, "ptr": [np.zeros(1, np.int32)] * 2}


def _compare_to_oracle(vx, systems, depth, r, tag):
    h = _host(r)
    tot = np.zeros((depth + 1, 2, 4), np.int64)
    steps = np.zeros(depth + 1, np.int64)
    for s, sysp in enumerate(systems):
        recs = orc.subdivide(sysp, 3, depth, nthreads=orc.max_threads())
        for rec in recs:
            steps[rec["level"]] += int(np.sum(rec["steps"]))
            sz = orc.csf_sizes(rec["S"])
            K = orc.csf_from_boxes(rec["kept"], rec["level"]) if len(rec["kept"]) else None
            ksz = orc.csf_sizes(K) if K is not None else [0, 0, 0]
            tot[rec["level"], 0] += [1 if sz[-1] else 0] + list(sz)
            tot[rec["level"], 1] += [1 if ksz[-1] else 0] + list(ksz)
        last = recs[depth]
        S = last["S"] if len(last["S"]["boxes"]) else _empty_csf()
        K = orc.csf_from_boxes(last["kept"], depth) if len(last["kept"]) else _empty_csf()
        _check_system(h, s, S, last["lo"][0], last["hi"][0], last["keep"], K, tag)
    assert np.array_equal(h["stats"], tot), (tag, "per-level counts")
    assert r["steps"] == steps.tolist(), (tag, "Theorem 1 steps")


def _same_result(a, b):
    if not np.array_equal(a["stats"], b["stats"]):
        return False
    for l in range(4):
        n = a["last"].n[l]
        if n != b["last"].n[l]:
            return False
        if not bool((a["last"].idx[l][:n] == b["last"].idx[l][:n]).all()):
            return False
    return (bits_equal(a["lo"].cpu().numpy(), b["lo"].cpu().numpy())
            and bits_equal(a["hi"].cpu().numpy(), b["hi"].cpu().numpy())
            and bool((a["keep"] == b["keep"]).all()))


def test_batch_small_systems_vs_oracle(vx):
    """16 systems of degrees 10..60 to level 6, graph mode, against the oracle."""
    w = synth.batch(count=16, depth=6)
    _say("[batch] oracle parity: 16 systems, depth 6")
    b, r = vx.run_subdivision_batch(w.systems, w.domain(), 6, graph=True)
    _compare_to_oracle(vx, w.systems, 6, r, "batch16")
    b.close()


def test_batch_degenerate_systems_vs_oracle(vx):
    """A constant (excluded at level 0), the zero polynomial (never excluded),
    planes and spheres mixed with random systems."""
    k = 3
    const = np.zeros((1, 1, 1)); const[0, 0, 0] = 2.5
    zero = np.zeros((2, 2, 2))
    systems = [[synth.sphere()], [const], [synth.plane_x1(3, 0.25)], [zero], [synth.plane_x3()]]
    systems += [[p] for p in synth.small_random(k, 7, seed=77, npolys=3)]
    _say("[batch] degenerate systems, depth 4")
    b, r = vx.run_subdivision_batch(systems, np.array([-1.0, 1.0] * 3), 4, graph=False)
    _compare_to_oracle(vx, systems, 4, r, "degenerate")
    b.close()


def test_batch64_depth8_matches_plain_runs(vx):
    """The full batch (64 systems, degrees 10..60, depth 8) against 64 plain
    run_subdivision calls, every system's last level bit for bit."""
    w = synth.batch()
    depth = w.depth
    _say(f"[batch] {w.name}: batched run, depth {depth}")
    b, r = vx.run_subdivision_batch(w.systems, w.domain(), depth, graph=True)
    h = _host(r)
    b.close()
    del r
    tot = np.zeros((depth + 1, 2, 4), np.int64)
    steps = np.zeros(depth + 1, np.int64)
    for s, sysp in enumerate(w.systems):
        grab = {}

        def rec(level, S, lo, hi, keep, K):
            if level == depth:
                grab.update(S=S, lo=lo[0], hi=hi[0], keep=keep.astype(bool), K=K)
            return False

        stats, _ = vx.run_subdivision(sysp, w.domain(), depth, record=rec)
        for st in stats:
            lv = st["level"]
            tot[lv, 0] += [1 if st["n"][2] > 0 else 0] + st["n"]
            tot[lv, 1] += [1 if st["kept"][2] > 0 else 0] + st["kept"]
            steps[lv] += st["steps"]
        if not grab:
            grab = dict(S=_empty_csf(), lo=np.zeros(0), hi=np.zeros(0), keep=np.zeros(0, bool), K=_empty_csf())
        _check_system(h, s, grab["S"], grab["lo"], grab["hi"], grab["keep"], grab["K"], "batch64")
    _say(f"[batch] per-level totals {tot[:, 0, 3].tolist()}")
    assert np.array_equal(h["stats"], tot)
    assert h["steps"] == steps.tolist()


def test_batch_eager_graph_replays_and_autotune_identical(vx):
    """Eager launches, three graph replays (with eager work and waits between
    them) and an autotuned configuration give the same result."""
    import torch
    w = synth.batch(count=24, depth=7)
    _say("[batch] eager vs graph vs autotuned: 24 systems, depth 7")
    b0, r0 = vx.run_subdivision_batch(w.systems, w.domain(), 7, graph=False)
    cap = b0.cap
    b1 = vx.Batch(w.systems, w.domain(), 7, cap=cap, graph=True)
    for i in range(3):
        b1.run()
        r1 = b1.result()
        assert r1["rc"] == 0
        assert _same_result(r0, r1), f"replay {i}"
        x = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        (x * 2).sum().item()
    chosen, ms = b1.autotune(candidates=[(8, 1, 1024), (4, 2, 4096), (2, 4, 8192), (1, 8, 256)], reps=1)
    assert len(chosen) == 8 and all(m > 0 for m in ms)
    b1.run()
    r2 = b1.result()
    assert _same_result(r0, r2), "autotuned graph"
    b0.close(); b1.close()


def test_batch_capacity_overflow_is_reported(vx):
    """Too small capacities: VX_ECAPACITY with the counts needed; the binding's
    retry with those counts then reproduces the roomy run."""
    w = synth.batch(count=8, depth=6)
    small = [8, 8 << 6, 64, 256]
    b = vx.Batch(w.systems, w.domain(), 6, cap=small, graph=False)
    b.run()
    r = b.result()
    assert r["rc"] == vx.VX_ECAPACITY
    assert any(n > c for n, c in zip(r["need"], small))
    b.close()
    b2, r2 = vx.run_subdivision_batch(w.systems, w.domain(), 6, cap=small)
    b3, r3 = vx.run_subdivision_batch(w.systems, w.domain(), 6)
    assert _same_result(r2, r3)
    b2.close(); b3.close()


@pytest.mark.timeout(900)
def test_batch64_depth8_vs_oracle_every_level(vx):
    """The batched workload at its stated size (64 systems, degrees 10..60,
    depth 8, graph replay with autotuned per-level launch shapes) against the
    oracle at every level, for 8 seeded systems including the one of highest
    degree and the one with the most level-8 boxes: the evaluated set, every
    enclosure bit, the keep flags, the kept set, and Theorem 1's steps of the
    system's own CSF against the oracle's counted steps.

    The depth-8 run's last level is compared directly.  Level L < 8 is read
    from a run of the same handle configuration stopped at depth L (same
    systems, capacities and per-level launch shapes): a level's kernels do not
    depend on the depth a run stops at, and the per-level counts of those
    runs must equal the depth-8 run's."""
    from paper_2406_09857_amd.binding import split_systems
    w = synth.batch()
    depth, dom = w.depth, w.domain()
    _say(f"[batch] {w.name}: sizing run, depth {depth}")
    b0, r0 = vx.run_subdivision_batch(w.systems, dom, depth, graph=False)
    cap = [max(int(n), 1) for n in r0["need"]]
    b0.close()
    del b0, r0
    b = vx.Batch(w.systems, dom, depth, cap=cap, graph=True)
    chosen, _ = b.autotune(reps=1)
    _say(f"[batch] autotuned launch shapes {chosen}")
    b.run()
    r = b.result()
    assert r["rc"] == 0
    full = _host(r)
    b.close()
    del b, r
    per = split_systems(full["last"], len(w.systems))
    degs = [s[0].shape[0] - 1 for s in w.systems]
    top_deg = int(np.argmax(degs))
    top_boxes = int(np.argmax([len(p["boxes"]) for p in per]))
    rng = np.random.default_rng(858)
    pick = {top_deg, top_boxes}
    for s in rng.permutation(len(w.systems)):
        if len(pick) == 8:
            break
        pick.add(int(s))
    pick = sorted(pick)
    _say(f"[batch] systems checked against the oracle: {pick} (degrees {[degs[s] for s in pick]}, "
         f"level-8 boxes {[len(per[s]['boxes']) for s in pick]})")
    recs = {}
    for s in pick:
        t = time.time()
        recs[s] = orc.subdivide(w.systems[s], 3, depth, dom=dom, nthreads=orc.max_threads())
        _say(f"[batch] oracle system {s} (degree {degs[s]}): {time.time() - t:.1f} s")
    for L in range(depth + 1):
        if L == depth:
            h = full
        else:
            bl = vx.Batch(w.systems, dom, L, cap=cap, tune=chosen[: L + 1], graph=True)
            bl.run()
            rl = bl.result()
            assert rl["rc"] == 0, L
            h = _host(rl)
            bl.close()
            del bl, rl
            assert np.array_equal(h["stats"][L], full["stats"][L]), (L, "per-level counts vs the depth-8 run")
            assert h["steps"][L] == full["steps"][L], (L, "steps vs the depth-8 run")
        for s in pick:
            rec = recs[s][L]
            S = rec["S"] if len(rec["S"]["boxes"]) else _empty_csf()
            K = orc.csf_from_boxes(rec["kept"], L) if len(rec["kept"]) else _empty_csf()
            _check_system(h, s, S, rec["lo"][0], rec["hi"][0], rec["keep"], K, f"batch64 level {L}")
            sub = _sub(h["last"], s)
            sizes = [len(a) for a in sub["idx"]] if sub is not None else [0, 0, 0]
            assert sum(orc.theorem1_steps(3, degs[s], sizes)) == int(rec["steps"].sum()), (L, s, "steps")
        _say(f"[batch] level {L}: {int(full['stats'][L, 0, 3])} boxes over all systems, "
             f"{len(pick)} systems bit-exact")
