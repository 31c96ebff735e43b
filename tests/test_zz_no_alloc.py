"""interval_eval_level_noalloc (the library's static per-GPU scratch instead
of a caller workspace) against interval_eval_level, through the C ABI.

Two calls in a row, the second on a smaller level, so that the second one
runs on scratch that still holds the first one's contents; then a level
whose scratch need exceeds the static array is refused before any work.
Bar: every enclosure bit (after -0 -> +0) and every keep flag equal.
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


def _level(w, level):
    rec = orc.subdivide(w.polys, w.k, level, dom=w.domain(), nthreads=orc.max_threads())[-1]
    return rec["S"]


def _same(vx, polys, S, dom, tag):
    csf = vx.CSF.from_arrays(S["k"], S["level"], S["idx"], S["ptr"])
    need = vx.workspace_bytes(vx.VX_WS_EVAL, vx.as_polys(polys), csf)
    _say(f"[noalloc] {tag}: level {S['level']} sizes {orc.csf_sizes(S)}, scratch need {need} bytes")
    assert 0 < need <= vx.NOALLOC_SCRATCH_BYTES
    lo_a, hi_a, keep_a = vx.interval_eval_level_noalloc(polys, csf, dom)
    lo_b, hi_b, keep_b = vx.interval_eval_level(polys, csf, dom)
    lo_a = lo_a.cpu().numpy(); hi_a = hi_a.cpu().numpy()
    lo_b = lo_b.cpu().numpy(); hi_b = hi_b.cpu().numpy()
    assert bits_equal(lo_a, lo_b), (tag, first_mismatch(lo_a, lo_b))
    assert bits_equal(hi_a, hi_b), (tag, first_mismatch(hi_a, hi_b))
    assert np.array_equal(keep_a.cpu().numpy(), keep_b.cpu().numpy()), tag


def test_noalloc_matches_workspace_entry_point_twice(vx):
    w = synth.curve()
    big = _level(w, 6)      # two degree-100 polynomials, 71,032 boxes (36 MiB of scratch)
    small = _level(w, 3)    # 456 boxes: the second call runs on the first one's leftovers
    _same(vx, w.polys, big, w.domain(), "curve level 6 (first call)")
    _same(vx, w.polys, small, w.domain(), "curve level 3 (second call, smaller)")
    t = synth.tiny()
    _same(vx, t.polys, _level(t, 6), t.domain(), "tiny level 6 (another system)")


def test_noalloc_refuses_levels_beyond_its_scratch(vx):
    import torch
    w = synth.curve()
    S = _level(w, 7)  # 288,376 boxes: its scratch need exceeds 64 MiB
    csf = vx.CSF.from_arrays(S["k"], S["level"], S["idx"], S["ptr"])
    need = vx.workspace_bytes(vx.VX_WS_EVAL, vx.as_polys(w.polys), csf)
    assert need > vx.NOALLOC_SCRATCH_BYTES
    lo = torch.full((2, csf.nboxes), 7.0, dtype=torch.float64, device="cuda")
    hi = lo.clone()
    kp = torch.full((csf.nboxes,), 9, dtype=torch.uint8, device="cuda")
    with pytest.raises(vx.VxError) as e:
        vx.interval_eval_level_noalloc(w.polys, csf, w.domain(), out=(lo, hi, kp))
    assert e.value.code == vx.VX_ECAPACITY and "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert bool((lo == 7.0).all()) and bool((kp == 9).all())  # nothing was enqueued
    # a call that fits still works after the refusal
    _same(vx, w.polys, _level(w, 4), w.domain(), "curve level 4 (after the refusal)")
