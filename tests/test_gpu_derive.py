"""GPU parity of the device-side level derivation: streams in the paper's
four-stream format (Sec. 3.2: no lvl[], no level table) decode to the
original bytes through aceapex_decode, and the levels the device derives
(aceapex_decode_derive) equal the levels of the definition (Sec. 7.1) that
the oracle computes -- for streams with and without stored levels, chains
deep enough to reach the one-workgroup tail, and corrupt inputs."""
import numpy as np
import pytest

import oracle
import streamgen
import synth
from gpu_util import GUARD, POISON, gpu_decode, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def derive(s):
    """aceapex_decode_derive on cuda:0 with guard bands; returns (bytes, levels, status)."""
    import torch

    import paper_2606_04268_amd as ax

    ds = ax.to_device(s)
    n = ds.n
    buf = torch.full((n + 2 * GUARD,), POISON, dtype=torch.uint8, device="cuda")
    out = buf[GUARD:GUARD + max(n, 16)]
    _, st, lv = ax.decode_derive(ds, out=out)
    torch.cuda.synchronize()
    h = buf.cpu().numpy()
    assert (h[:GUARD] == POISON).all() and (h[GUARD + n:] == POISON).all(), "write outside the output"
    return h[GUARD:GUARD + n], lv.cpu().numpy()[:ds.info.n_seq], int(st.item())


@pytest.mark.parametrize("kind", ["markov", "fastq", "wiki", "random"])
@pytest.mark.parametrize("opts", [dict(), dict(flatten=1), dict(max_depth=8), dict(block_log2=14, chunk_log2=5)],
                         ids=["plain", "flat", "d8", "small"])
def test_four_stream_format_decodes(kind, opts):
    x = synth.make(kind, 3 << 20, 0xD0 + len(kind))
    o = dict(dict(block_log2=18), **opts)
    free = oracle.encode(x, levels=0, **o)
    stored = oracle.encode(x, **o)
    want_lv = oracle.tokens(free)["lvl"]
    assert np.array_equal(want_lv, oracle.tokens(stored)["lvl"])
    say(f"[gpu] derive {kind} {opts}: {want_lv.size} matches, max level {int(want_lv.max(initial=0))}")
    got, status = gpu_decode(free)  # aceapex_decode: no stored levels -> derived
    assert status == 0 and np.array_equal(got, x)
    for s in (free, stored):
        got, lv, status = derive(s)
        assert status == 0 and np.array_equal(got, x)
        assert np.array_equal(lv, want_lv)


@pytest.mark.parametrize("levels", [600, 2500])
def test_chains_reach_the_tail(levels):
    """A chain of one match per level: after the first levels the queue is
    small and one workgroup runs the rest."""
    m = levels
    blocks = [([(4, 4, 0)] + [(0, 4, 4 * i) for i in range(1, m)], 0)]
    s, want = streamgen.build(blocks, b"abcd", 4 + 4 * m, block_log2=14, chunk_log2=5, with_levels=False)
    got, lv, status = derive(s)
    assert status == 0 and got.tobytes() == want
    assert lv.tolist() == list(range(m))
    # the same chain spread over small blocks, with literals between
    x = np.frombuffer(want, np.uint8)
    s2 = oracle.encode(x, block_log2=6, tiebreak=1, hash_bits=12, levels=0)
    got, lv, status = derive(s2)
    assert status == 0 and np.array_equal(got, x)
    assert np.array_equal(lv, oracle.tokens(s2)["lvl"])


def test_deep_unflattened_fastq():
    x = synth.fastq(6 << 20, 31)
    s = oracle.encode(x, levels=0)
    want = oracle.tokens(s)["lvl"]
    say(f"[gpu] derive deep fastq: max level {int(want.max())}")
    got, lv, status = derive(s)
    assert status == 0 and np.array_equal(got, x) and np.array_equal(lv, want)


@pytest.mark.parametrize("seed", range(6))
def test_random_token_streams(seed):
    rng = np.random.default_rng(600 + seed)
    bl = [4, 6, 9, 12, 16, 20][seed]
    n = int(rng.integers(1000, 200_000))
    blocks, lits = streamgen.random_tokens(rng, n, bl, max_len=[8, 40, 300][seed % 3], p_match=0.6)
    s, want = streamgen.build(blocks, lits, n, block_log2=bl, chunk_log2=int(rng.integers(0, 8)), with_levels=False)
    _, exact = streamgen.execute(blocks, lits, n, bl)
    got, lv, status = derive(s)
    assert status == 0 and got.tobytes() == want
    assert lv.tolist() == exact


def test_corrupt_four_stream_format():
    s, _ = streamgen.build([([(8, 4, 0)], 0)], bytes(range(8)), 12, block_log2=8, with_levels=False)
    bad = s.copy()
    base = int.from_bytes(bad[64:72].tobytes(), "little")
    off_at = base + 32 + 32
    bad[off_at:off_at + 4] = np.frombuffer((6).to_bytes(4, "little"), np.uint8)
    _, status = gpu_decode(bad)
    assert status == -3


def test_empty_and_literal_only():
    for x in (np.zeros(0, np.uint8), np.frombuffer(b"abc", np.uint8), np.arange(256, dtype=np.uint8)):
        s = oracle.encode(x, levels=0, block_log2=8)
        got, status = gpu_decode(s)
        assert status == 0 and np.array_equal(got, x)
