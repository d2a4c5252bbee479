"""GPU parity at the benchmark sizes: the 256 MiB FASTQ-like stream and the
1 GiB wiki-like stream encoded twice (depth unlimited, and depth limit 8),
decoded in the launch configurations bench.py times (aceapex_decode, and a
plan replayed as a captured graph).  Every output byte is compared with the
original and with the oracle's sequential decode of the same stream."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


CASES = {
    "fastq256": ("fastq", 256 << 20, synth.CFG_SEEDS[1], dict(flatten=1)),
    "wiki1g": ("wiki", 1 << 30, synth.CFG_SEEDS[2], dict()),
    "wiki1g_d8": ("wiki", 1 << 30, synth.CFG_SEEDS[2], dict(max_depth=8)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_full_size_decode(name):
    import torch

    import paper_2606_04268_amd as ax

    kind, n, seed, opts = CASES[name]
    say(f"[gpu] full size {name}: generating and encoding {n} bytes")
    x = synth.make(kind, n, seed)
    s = ax.encode(x, **opts)
    h = oracle.header_fields(s)
    if opts.get("max_depth"):
        assert h["max_level"] <= opts["max_depth"] - 1
    ref = oracle.decode(s)
    assert np.array_equal(ref, x)
    ds = ax.to_device(s)
    xd = torch.from_numpy(x).cuda()
    say(f"[gpu] full size {name}: decode (max level {h['max_level']}, {h['n_seq']} matches)")
    out, st = ax.decode(ds)
    torch.cuda.synchronize()
    ax.check_status(st)
    assert torch.equal(out[:n], xd)
    out.fill_(0xA5)
    plan = ax.Plan([ds], outs=[out])
    try:
        for _ in range(2):
            plan.launch(graph=True)
            torch.cuda.synchronize()
            ax.check_status(plan.statuses)
            assert torch.equal(out[:n], xd)
            out.fill_(0x5A)
    finally:
        plan.close()
    assert ax.content_hash(x) == h["content_hash"]
