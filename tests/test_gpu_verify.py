"""GPU byte compare (aceapex_compare, the decode's verification kernel)
against numpy: the count of differing bytes and the first index, with
differences planted at the ends, inside 16-byte words and across them, for
buffers that share their alignment and buffers that do not, and sizes from
0 up to several grid strides."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def host_cmp(a, b):
    d = np.flatnonzero(a != b)
    return int(d.size), int(d[0]) if d.size else int(a.size)


@pytest.mark.parametrize("n", [0, 1, 15, 16, 17, 1000, 65_537, (1 << 22) + 5, 33 << 20])
@pytest.mark.parametrize("offsets", [(0, 0), (3, 3), (0, 5), (7, 1)], ids=["aligned", "same_offset", "b_shifted", "both_shifted"])
def test_counts_and_first_index(n, offsets):
    import torch

    import paper_2606_04268_amd as ax

    rng = np.random.default_rng(n + 7 * offsets[0] + offsets[1])
    base = rng.integers(0, 256, n, dtype=np.uint8)
    other = base.copy()
    if n:
        picks = {0, n - 1, n // 2, min(n - 1, 16), min(n - 1, 31)} | set(rng.integers(0, n, min(n, 50)).tolist())
        for i in picks:
            other[i] ^= np.uint8(1 << int(rng.integers(0, 8)))
    oa, ob = offsets
    da = torch.zeros(n + oa + 16, dtype=torch.uint8, device="cuda")
    db = torch.zeros(n + ob + 16, dtype=torch.uint8, device="cuda")
    da[oa:oa + n] = torch.from_numpy(base).cuda()
    db[ob:ob + n] = torch.from_numpy(other).cuda()
    say(f"[gpu] compare n={n} offsets={offsets}")
    assert ax.compare(da[oa:oa + n], db[ob:ob + n]) == host_cmp(base, other)
    assert ax.compare(da[oa:oa + n], da[oa:oa + n]) == (0, n)


def test_every_byte_value_difference():
    """A difference in any one bit of any byte lane of a word is seen."""
    import torch

    import paper_2606_04268_amd as ax

    a = np.zeros(16 * 8 * 16, dtype=np.uint8)
    b = a.copy()
    for k in range(16):
        for bit in range(8):
            b[(k * 8 + bit) * 16 + k] = 1 << bit
    got = ax.compare(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
    assert got == host_cmp(a, b) == (128, 0)
