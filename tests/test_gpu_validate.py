"""GPU check of stored levels (ACEAPEX_VALIDATE_LEVELS): with the variable
set, aceapex_decode fails a stream in which some match's stored level does
not exceed the level of a match that writes its source (Sec. 7.1), and
decodes every stream whose stored levels respect the writers, exact or not,
byte for byte."""
import numpy as np
import pytest

import oracle
import streamgen
import synth
from gpu_util import gpu_decode, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


@pytest.fixture
def validate(monkeypatch):
    monkeypatch.setenv("ACEAPEX_VALIDATE_LEVELS", "1")


def chained(seed, n=40_000, bl=12):
    rng = np.random.default_rng(seed)
    blocks, lits = streamgen.random_tokens(rng, n, bl, max_len=30)
    _, levels = streamgen.execute(blocks, lits, n, bl)
    return blocks, lits, n, bl, levels


@pytest.mark.parametrize("kind,opts", [("markov", dict()), ("fastq", dict(flatten=1)), ("wiki", dict(max_depth=4)),
                                       ("wiki", dict()), ("random", dict(block_log2=14))])
def test_exact_levels_pass(validate, kind, opts):
    x = synth.make(kind, 3 << 20, 51)
    s = oracle.encode(x, **opts)
    say(f"[gpu] validated decode {kind} {opts}")
    got, status = gpu_decode(s)
    assert status == 0 and np.array_equal(got, x)


@pytest.mark.parametrize("seed", range(4))
def test_under_leveled_stream_fails(validate, seed):
    """One match whose writer has its level or more: the check fails it."""
    blocks, lits, n, bl, levels = chained(seed)
    deep = [i for i, v in enumerate(levels) if v > 0]
    bad = list(levels)
    bad[deep[len(deep) // 2]] -= 1  # now equal to (or below) one of its writers
    s, _ = streamgen.build(blocks, lits, n, block_log2=bl, levels=bad)
    say(f"[gpu] under-leveled stream seed={seed}")
    assert gpu_decode(s)[1] == -3
    flat = [0] * len(levels)  # every match at level 0
    s, _ = streamgen.build(blocks, lits, n, block_log2=bl, levels=flat)
    assert gpu_decode(s)[1] == -3


@pytest.mark.parametrize("seed", range(3))
def test_over_leveled_stream_passes(validate, seed):
    """Levels that keep every writer below its reader (here twice the
    definition) are safe; the check accepts them and the decode is exact."""
    blocks, lits, n, bl, levels = chained(seed + 10)
    s, want = streamgen.build(blocks, lits, n, block_log2=bl, levels=[2 * v for v in levels])
    got, status = gpu_decode(s)
    assert status == 0 and got.tobytes() == want


def test_workspace_grows_and_is_checked(monkeypatch):
    import torch

    import paper_2606_04268_amd as ax
    from paper_2606_04268_amd import _abi

    x = synth.make("wiki", 1 << 20, 52)
    s = oracle.encode(x)
    ds = ax.to_device(s)
    monkeypatch.delenv("ACEAPEX_VALIDATE_LEVELS", raising=False)
    small = ax.workspace_bytes([ds])
    monkeypatch.setenv("ACEAPEX_VALIDATE_LEVELS", "1")
    big = ax.workspace_bytes([ds])
    assert big >= _abi.workspace_bytes_derive(ds.info) and big > small
    out = torch.empty(ds.n, dtype=torch.uint8, device="cuda")
    ws = torch.empty(small, dtype=torch.uint8, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    handle = torch.cuda.current_stream().cuda_stream
    # through the C ABI: the Python helper would replace a short workspace
    rc = _abi.decode(ds.abi(), out.data_ptr(), out.numel(), ws.data_ptr(), ws.numel(), st.data_ptr(), handle)
    assert rc == _abi.E_WORKSPACE
    monkeypatch.setenv("ACEAPEX_VALIDATE_LEVELS", "0")  # "0" leaves the check off
    rc = _abi.decode(ds.abi(), out.data_ptr(), out.numel(), ws.data_ptr(), ws.numel(), st.data_ptr(), handle)
    assert rc == 0
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and np.array_equal(out.cpu().numpy(), x)
