"""GPU test of aceapex_decode_noalloc, the entry point that allocates nothing
(its workspace is a library-static device array): its output must equal
aceapex_decode's on the same stream, on two calls in a row (the second with a
smaller stream, over what the first left in the array), and a stream whose
workspace exceeds the array is refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from gpu_util import GUARD, POISON, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _guarded(n):
    import torch

    buf = torch.full((n + 2 * GUARD,), POISON, dtype=torch.uint8, device="cuda")
    return buf, buf[GUARD:GUARD + max(n, 16)]


def _check_guards(buf, n):
    h = buf.cpu().numpy()
    assert (h[:GUARD] == POISON).all() and (h[GUARD + n:] == POISON).all(), "write outside the output"
    return h[GUARD:GUARD + n]


def test_noalloc_matches_decode_twice():
    import torch

    import paper_2606_04268_amd as ax
    from paper_2606_04268_amd import _abi

    cases = [("markov 4 MiB", synth.markov(4 << 20, synth.CFG_SEEDS[0]), dict()),
             ("fastq 1 MiB, flattened", synth.fastq(1 << 20, 99), dict(flatten=1, block_log2=18))]
    stream = torch.cuda.current_stream()
    for label, x, opts in cases:
        s = oracle.encode(x, **opts)
        ds = ax.to_device(s)
        assert ax.workspace_bytes([ds]) <= _abi.NOALLOC_WORKSPACE_MAX
        say(f"[gpu] noalloc {label}: {ds.n} bytes, {ds.info.n_seq} matches")
        ref, st_ref = ax.decode(ds)
        buf, out = _guarded(ds.n)
        status = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
        rc = _abi.decode_noalloc(ds.abi(), out.data_ptr(), out.numel(), status.data_ptr(), stream.cuda_stream)
        assert rc == 0, _abi.strerror(rc)
        torch.cuda.synchronize()
        assert int(st_ref.item()) == 0 and int(status.item()) == 0
        got = _check_guards(buf, ds.n)
        assert np.array_equal(got, ref[:ds.n].cpu().numpy())
        assert np.array_equal(got, x)


def test_noalloc_refuses_a_workspace_beyond_the_array():
    import torch

    import paper_2606_04268_amd as ax
    from paper_2606_04268_amd import _abi

    x = synth.markov(1 << 16, 5)
    ds = ax.to_device(oracle.encode(x))
    big = _abi.Stream(ds.comp.data_ptr(), _abi.Info.from_buffer_copy(ds.info), None)
    big.info.n_seq = 6_000_000  # 12 bytes of match record each: beyond the 64 MiB array
    out = torch.empty(ds.n, dtype=torch.uint8, device="cuda")
    rc = _abi.decode_noalloc(big, out.data_ptr(), out.numel(), None, torch.cuda.current_stream().cuda_stream)
    assert rc == _abi.E_WORKSPACE
