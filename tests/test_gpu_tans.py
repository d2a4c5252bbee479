"""GPU parity of the entropy stage for literals: containers written by the
oracle's tANS coder (oracle/tans_oracle.c) decode on the device to the
original bytes and to the oracle's decode, byte for byte, for literal
streams of the benchmark workloads, edge cases (empty, one symbol, fewer
symbols than lanes, every table size) and damaged containers."""
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


def gpu_tans(container):
    import torch

    import paper_2606_04268_amd as ax
    from paper_2606_04268_amd import _abi

    info = _abi.tans_probe(container)
    n = int(info.n)
    buf = torch.full((n + 2 * GUARD,), POISON, dtype=torch.uint8, device="cuda")
    out = buf[GUARD:GUARD + max(n, 16)]
    _, st = ax.tans_decode(container, out=out)
    torch.cuda.synchronize()
    h = buf.cpu().numpy()
    assert (h[:GUARD] == POISON).all() and (h[GUARD + n:] == POISON).all(), "write outside the output"
    return h[GUARD:GUARD + n], int(st.item())


def literals_of(stream):
    """The lit[] sections of every block of a stream, concatenated."""
    s = np.asarray(stream)
    nb = int(s[32:36].view(np.uint32)[0])
    parts = []
    for b in range(nb):
        at = int(s[64 + 16 * b:72 + 16 * b].view(np.uint64)[0])
        h = s[at:at + 32].view(np.uint32)
        ns, nl, nc, cmdb, lenb, lvlb = int(h[0]), int(h[1]), int(h[2]), int(h[4]), int(h[5]), int(h[6])
        pad = lambda v: (v + 15) // 16 * 16
        lit = at + 32 + 32 * nc + pad(4 * ns) + pad(cmdb) + pad(lenb) + pad(lvlb)
        parts.append(s[lit:lit + nl])
    return np.concatenate(parts) if parts else np.zeros(0, np.uint8)


@pytest.mark.parametrize("kind", ["fastq", "markov", "wiki", "random"])
def test_literal_streams(kind):
    x = synth.make(kind, 8 << 20, 0x7A)
    lit = literals_of(oracle.encode(x, flatten=1 if kind == "fastq" else 0, block_log2=18))
    for table_log, lanes in [(11, max(1, lit.size // 1024)), (12, 4096), (8, 1000)]:
        c = oracle.tans_encode(lit, table_log, lanes)
        say(f"[gpu] tans {kind}: {lit.size} literal bytes -> {c.size} (R={table_log}, {lanes} lanes)")
        got, status = gpu_tans(c)
        assert status == 0
        assert np.array_equal(got, lit) and np.array_equal(got, oracle.tans_decode(c))


@pytest.mark.parametrize("x,table_log,lanes", [
    (b"", 11, 16), (b"a", 11, 300), (b"q" * 5000, 11, 7), (bytes(range(256)) * 33, 8, 513),
    (bytes(range(256)) * 33, 12, 1), (b"ab" * 999, 9, 1024), (b"xyz" * 10, 10, 4096)],
    ids=["empty", "one_byte", "one_symbol", "all_bytes_R8", "all_bytes_one_lane", "two_symbols", "more_lanes"])
def test_edge_cases(x, table_log, lanes):
    c = oracle.tans_encode(x, table_log, lanes)
    got, status = gpu_tans(c)
    assert status == 0 and got.tobytes() == x


def test_damaged_containers():
    """A lane whose initial state is out of range, or whose end bit lies before
    the previous lane's, fails the decode; a flipped data bit decodes to other
    bytes or fails, never outside the output."""
    x = synth.fastq(200_000, 9).tobytes()
    c = oracle.tans_encode(x, 11, 256)
    lt = 544
    bad = c.copy()
    bad[lt + 8 * 5 + 4:lt + 8 * 5 + 8] = np.frombuffer((5000).to_bytes(4, "little"), np.uint8)
    assert gpu_tans(bad)[1] == -3
    bad = c.copy()
    bad[lt + 8 * 9:lt + 8 * 9 + 4] = np.frombuffer((0).to_bytes(4, "little"), np.uint8)
    assert gpu_tans(bad)[1] == -3
    rng = np.random.default_rng(4)
    body = lt + 8 * 256
    for _ in range(20):
        bad = c.copy()
        i = int(rng.integers(body, c.size - 8))
        bad[i] ^= np.uint8(1 << int(rng.integers(0, 8)))
        got, status = gpu_tans(bad)
        assert status in (0, -3)
