"""GPU parity over the depth limit D in {1, 2, 10, unlimited} x chain
flattening {off, R1, R2} (Sec. 7.4, Table 5; Sec. 3.3) on 4 MiB of wiki-like
text and of FASTQ-like data, 1 MiB blocks: every stream is encoded by the
oracle, and the GPU decode (eager, and a plan replayed as a graph) must equal
the original bytes and the oracle's decode."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import gpu_decode, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


_DATA = {}


def _data(kind):
    if kind not in _DATA:
        _DATA[kind] = synth.make(kind, 4 << 20, synth.CFG_SEEDS[2] if kind == "wiki" else synth.CFG_SEEDS[1])
    return _DATA[kind]


@pytest.mark.parametrize("flatten", [0, 1, 2], ids=["off", "R1", "R2"])
@pytest.mark.parametrize("depth", [1, 2, 10, 0], ids=["D1", "D2", "D10", "Dinf"])
@pytest.mark.parametrize("kind", ["wiki", "fastq"])
def test_depth_and_flattening(kind, depth, flatten):
    import torch

    import paper_2606_04268_amd as ax

    x = _data(kind)
    s = oracle.encode(x, max_depth=depth, flatten=flatten)
    h = oracle.header_fields(s)
    if depth:
        assert h["max_level"] <= depth - 1
    ref = oracle.decode(s)
    assert np.array_equal(ref, x)
    say(f"[gpu] sweep {kind} D={depth or 'inf'} flatten={flatten}: max_level {h['max_level']}, {h['n_seq']} matches")
    got, status = gpu_decode(s)
    assert status == 0
    assert np.array_equal(got, x)
    ds = ax.to_device(s)
    out = torch.full((ds.n,), 0xA5, dtype=torch.uint8, device="cuda")
    plan = ax.Plan([ds], outs=[out])
    try:
        plan.launch(graph=True)
        torch.cuda.synchronize()
        ax.check_status(plan.statuses)
        assert np.array_equal(out.cpu().numpy(), x)
    finally:
        plan.close()
