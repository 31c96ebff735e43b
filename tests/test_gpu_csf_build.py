"""csf_build (radix sort + scans) against the oracle's CSF of the same box
list: identical labels and offsets at every depth."""
import numpy as np
import pytest

from oracle import core as orc
from tests.helpers import csf_equal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_09857_amd import binding
    binding.lib()
    return binding


@pytest.mark.parametrize("k,level,n", [(1, 5, 40), (2, 8, 3000), (3, 10, 200000), (4, 6, 50000), (3, 1, 10),
                                       (2, 0, 5), (3, 20, 100000), (2, 29, 20000), (3, 10, 2_000_000)])
def test_csf_build_matches_oracle(vx, k, level, n):
    import torch
    print(f"[csf_build] k={k} level={level} n={n}", flush=True)
    rng = np.random.default_rng(k * 1000 + level)
    hi = 1 << level
    boxes = rng.integers(0, hi, size=(n, k))
    if n > 4:  # duplicates and a clustered tail
        boxes[n // 2:] = boxes[: n - n // 2] // 2 if level > 0 else 0
    got = vx.csf_build(torch.as_tensor(boxes.astype(np.int32), device="cuda"), level)
    want = orc.csf_from_boxes(boxes, level)
    assert got.n == orc.csf_sizes(want)
    assert csf_equal(got.to_numpy(), want)


def test_csf_build_empty_and_errors(vx):
    import torch
    got = vx.csf_build(torch.zeros((0, 3), dtype=torch.int32, device="cuda"), 4)
    assert got.n == [0, 0, 0]
    with pytest.raises(vx.VxError) as e:
        vx.csf_build(torch.tensor([[0, 16]], dtype=torch.int32, device="cuda"), 4)
    assert e.value.code == vx.VX_EINVAL
    with pytest.raises(vx.VxError) as e:
        vx.csf_build(torch.zeros((3, 4), dtype=torch.int32, device="cuda"), 20)
    assert e.value.code == vx.VX_EUNSUPPORTED
