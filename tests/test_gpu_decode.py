"""GPU parity: every decode through the C ABI must equal, byte for byte, both
the original bytes and the oracle's sequential decode of the same stream.
Streams come from the oracle encoder or are hand-built token lists; no
expected value comes from the GPU path."""
import os

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


def parity(x, s, label):
    say(f"[gpu] {label}: n={len(x)} comp={s.size} max_level={oracle.header_fields(s)['max_level']}")
    got, status = gpu_decode(s)
    assert status == 0, f"device status {status}"
    want = np.frombuffer(bytes(x), np.uint8) if not isinstance(x, np.ndarray) else x
    ref = oracle.decode(s)
    assert np.array_equal(ref, want)
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"{bad.size} bytes differ, first at {bad[0]}")
    return got


def test_single_hip_runtime_in_process():
    import torch

    import paper_2606_04268_amd as ax
    from paper_2606_04268_amd import _abi

    _abi.load()
    torch.zeros(1, device="cuda")
    maps = open("/proc/self/maps").read()
    libs = {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}
    assert len(libs) == 1, libs
    assert any(_abi.LIB_PATH in line for line in maps.splitlines())
    assert ax is not None


def test_config0_markov_4mib():
    """The 4 MB text workload: order-2 Markov text with 20% copies, 1 MB
    blocks, minimum match 4, no flattening."""
    x = synth.markov(4 << 20, synth.CFG_SEEDS[0])
    s = oracle.encode(x)
    got = parity(x, s, "cfg0")
    assert oracle.content_hash(got) == oracle.header_fields(s)["content_hash"]


@pytest.mark.parametrize("kind", ["markov", "fastq", "wiki", "random"])
@pytest.mark.parametrize("opts", [dict(), dict(flatten=1), dict(max_depth=8), dict(flatten=2),
                                  dict(tiebreak=1)],
                         ids=["plain", "flat", "d8", "flatlit", "recent"])
def test_generated_kinds(kind, opts, ordered_slots):
    x = synth.make(kind, 3 << 19, 0xACE0 + len(kind))
    s = oracle.encode(x, block_log2=18, **opts)
    parity(x, s, f"{kind}/{opts}")


@pytest.mark.parametrize("chunk_log2", [0, 3, 7, 10])
@pytest.mark.parametrize("block_log2", [3, 9, 16, 20])
def test_block_and_chunk_sizes(block_log2, chunk_log2, ordered_slots):
    x = synth.markov(200_000 + 1234, 77)
    s = oracle.encode(x, block_log2=block_log2, chunk_log2=chunk_log2, hash_bits=16)
    parity(x, s, f"bl{block_log2}/ck{chunk_log2}")


@pytest.mark.parametrize("seed", range(16))
def test_random_token_streams(seed, ordered_slots):
    rng = np.random.default_rng(100 + seed)
    bl = [3, 4, 6, 10, 14, 20][seed % 6]
    n = int(rng.integers(1, 60_000))
    blocks, lits = streamgen.random_tokens(rng, n, bl, max_len=[5, 40, 700][seed % 3],
                                           p_match=[0.3, 0.6, 0.9][seed % 3])
    s, want = streamgen.build(blocks, lits, n, block_log2=bl, chunk_log2=int(rng.integers(0, 11)))
    parity(np.frombuffer(want, np.uint8), s, f"tokens seed={seed} bl={bl}")


@pytest.mark.parametrize("width", [4, "random"])
def test_padded_varints(width, ordered_slots):
    """Non-minimal LEB128: every value padded to 4 bytes fills a full chunk's
    slices to 4096 bytes (the largest the workgroup decoder takes) and a
    chunk that also holds the trailing run to 4100 (decoded one wave per
    slice); random widths mix value lengths inside every window."""
    rng = np.random.default_rng(23)
    w = 4 if width == 4 else np.random.default_rng(29)
    m = 2048  # two full chunks of 1024 sequences; the second holds the trailing run
    blocks = [([(4, 4, 0)] + [(1, 4, int(rng.integers(0, 4))) for _ in range(m - 1)], 3)]
    n = 8 + 5 * (m - 1) + 3
    lits = bytes(rng.integers(0, 256, size=n, dtype=np.uint8))
    s, want = streamgen.build(blocks, lits, n, block_log2=16, chunk_log2=10, varint_width=w)
    parity(np.frombuffer(want, np.uint8), s, f"padded varints width={width}")
    blocks, lits = streamgen.random_tokens(rng, 200_000, 16, max_len=300, p_match=0.8)
    s, want = streamgen.build(blocks, lits, 200_000, block_log2=16, chunk_log2=10, varint_width=w)
    parity(np.frombuffer(want, np.uint8), s, f"padded varints random tokens width={width}")


def test_long_literal_runs_in_staged_chunks(ordered_slots):
    """Chunks whose literals are staged in LDS, with the run-length patterns
    that select each way of placing the words past a run's first four: a few
    very long runs in a wave (placed by the whole wave, several 256-byte steps
    for the 2000-byte run), twelve lanes per wave with a 40-byte run in one
    slot and every lane with a 20-byte run in another (placed by each lane,
    four words per pass), and exactly eight lanes with a 100-byte run."""
    rng = np.random.default_rng(41)
    runs = []
    for i in range(1024):  # chunk 0: three very long runs among one-byte runs
        runs.append({5: 700, 300: 2000, 777: 300}.get(i, 1))
    for i in range(1024):  # chunk 1: twelve lanes per wave with a 40-byte run in slot 0
        runs.append(40 if i % 4 == 0 and (i // 4) % 64 < 12 else int(rng.integers(0, 3)))
    for i in range(1024):  # chunk 2: exactly eight lanes per wave with a 100-byte run in slot 1
        runs.append(100 if i % 4 == 1 and (i // 4) % 64 < 8 else int(rng.integers(0, 4)))
    for i in range(1024):  # chunk 3: every lane has a 20-byte run in slot 2
        runs.append(20 if i % 4 == 2 else int(rng.integers(0, 2)))
    runs[0] = max(runs[0], 8)
    seqs, pos = [], 0
    for r in runs:
        pos += r
        seqs.append((r, 4, int(rng.integers(0, pos - 3))))
        pos += 4
    trail = 5
    n = pos + trail
    lits = bytes(rng.integers(0, 256, size=n, dtype=np.uint8))
    s, want = streamgen.build([(seqs, trail)], lits, n, block_log2=20, chunk_log2=10)
    parity(np.frombuffer(want, np.uint8), s, "long literal runs")


def test_doubling_string_long_matches():
    u = np.random.default_rng(7).permutation(256)[:16].astype(np.uint8).tobytes()
    x = u * (1 << 16)  # 1 MiB of one repeated 16-byte unit: long matches, deep levels
    s = oracle.encode(x, hash_bits=12)
    parity(np.frombuffer(x, np.uint8), s, "doubling")


@pytest.mark.parametrize("m", [500, 2000, 5000, 9000])
def test_level_chains_of_every_histogram_shape(m):
    """m chained 4-byte copies: levels 0..m-1.  500 and 2000 levels take the
    parse shapes with 1024- and 4096-level LDS histograms; 5000 levels go past
    the largest, so the deepest levels take one global atomic per match.
    9000 one-match levels all run in the tail workgroup, more of them than the
    tail keeps slot ranges for in LDS (8192), so the last ones are read from
    the level table in memory."""
    blocks = [([(4, 4, 0)] + [(0, 4, 4 * i) for i in range(1, m)], 0)]
    n = 4 + 4 * m
    s, want = streamgen.build(blocks, b"abcd", n, block_log2=16, chunk_log2=5)
    assert oracle.header_fields(s)["max_level"] == m - 1
    parity(np.frombuffer(want, np.uint8), s, f"chain{m}")


def test_edge_cases(ordered_slots):
    for x in [b"", b"a", b"abc", b"abcd" * 3, bytes(range(256)), b"z" * 70_000]:
        for o in [dict(), dict(block_log2=3, chunk_log2=0), dict(flatten=1, block_log2=4)]:
            s = oracle.encode(x, hash_bits=10, **o)
            parity(np.frombuffer(x, np.uint8), s, f"edge n={len(x)} {o}")


def test_multiple_of_chunk_size(ordered_slots):
    blocks = [([(4, 4, 0)] * 8, 3)]
    lits = bytes(range(35))
    n = 8 * 8 + 3
    s, want = streamgen.build(blocks, lits, n, block_log2=8, chunk_log2=2)
    parity(np.frombuffer(want, np.uint8), s, "nseq%K==0")


@pytest.mark.parametrize("run", [1, 200], ids=["one_byte_runs", "two_byte_runs"])
@pytest.mark.parametrize("trail", [0, 5, 40, 20000], ids=lambda t: f"trail{t}")
def test_full_chunk_holding_the_trailing_run(run, trail):
    """A block of exactly 2 x 1024 sequences at the largest chunk size: its
    last chunk holds 1024 sequences plus the trailing run, one command more
    than the workgroup's threads cover.  Runs of 200 bytes take the
    workgroup varint decoder, runs of 1 the one-byte path; a trailing run of
    20000 bytes makes the chunk's span exceed the LDS tile."""
    rng = np.random.default_rng(run * 100 + trail)
    m = 2048
    seqs = [(4, 4, 0)] + [(run, 4, int(rng.integers(0, 4))) for _ in range(m - 1)]
    n = 8 + (run + 4) * (m - 1) + trail
    lits = bytes(rng.integers(0, 256, size=n, dtype=np.uint8))
    s, want = streamgen.build([(seqs, trail)], lits, n, block_log2=20, chunk_log2=10)
    parity(np.frombuffer(want, np.uint8), s, f"full last chunk run={run} trail={trail}")


def test_decode_many_matches_single():
    import torch

    import paper_2606_04268_amd as ax

    xs, ss = [], []
    for i, kind in enumerate(["markov", "fastq", "random", "wiki", "markov"]):
        x = synth.make(kind, 50_000 * (i + 1) + i, 500 + i)
        xs.append(x)
        ss.append(oracle.encode(x, block_log2=15, flatten=i % 2))
    say("[gpu] decode_many x5")
    dss = [ax.to_device(s) for s in ss]
    outs, st = ax.decode_many(dss)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    for x, o in zip(xs, outs):
        assert np.array_equal(o[: len(x)].cpu().numpy(), x)


def test_stale_output_and_workspace_do_not_matter():
    """Poisoned output and a dirty reused workspace give the same bytes."""
    import torch

    import paper_2606_04268_amd as ax

    x = synth.fastq(1 << 20, 12)
    s = oracle.encode(x, block_log2=17, flatten=1)
    ds = ax.to_device(s)
    ws = torch.full((ax.workspace_bytes([ds]),), 0x5A, dtype=torch.uint8, device="cuda")
    for fill in (0x00, 0xFF, 0x3C):
        out = torch.full((ds.n,), fill, dtype=torch.uint8, device="cuda")
        say(f"[gpu] stale fill={fill:#x}")
        ax.decode(ds, out=out, workspace=ws)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), x)


@pytest.mark.parametrize("with_table", [True, False], ids=["level_table", "no_table"])
def test_level_schedule_with_and_without_host_table(with_table):
    """The wavefront is launched per level from the host copy of the level
    table (deep sparse levels grouped in one workgroup) or, without it, with
    full-size launches for every level; both give the same bytes."""
    import torch

    import paper_2606_04268_amd as ax

    x = synth.fastq(3 << 20, 21)
    s = oracle.encode(x, block_log2=16, flatten=1)
    ds = ax.to_device(s)
    if not with_table:
        ds.levels = None
    say(f"[gpu] schedule with_table={with_table} max_level={ds.info.max_level}")
    out, st = ax.decode(ds)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert np.array_equal(out[: ds.n].cpu().numpy(), x)


def test_many_blocks_many_levels():
    """2100 blocks of 8 bytes, each one match copying the previous block:
    levels 0..2099, more (level, block) pairs than the per-block record
    cursors cover, so records are reserved per level instead."""
    m = 2100
    blocks = [([], 8)] + [([(0, 8, 8 * (b - 1))], 0) for b in range(1, m + 1)]
    n = 8 * (m + 1)
    s, want = streamgen.build(blocks, bytes(range(8)), n, block_log2=3, chunk_log2=2)
    assert oracle.header_fields(s)["max_level"] == m - 1
    parity(np.frombuffer(want, np.uint8), s, "chain-of-blocks")


@pytest.mark.parametrize("depth", [63, 64, 65])
def test_ordered_slots_level_limit(depth, ordered_slots):
    """Streams of 63, 64 and 65 levels: single streams of at most 64 levels
    place each chunk's records at slots counted and scanned before the parse,
    deeper ones append them; both must decode the same bytes."""
    x = synth.wiki(8 << 20, 0xACE5)  # 72 levels at unlimited depth
    s = oracle.encode(x, block_log2=20, max_depth=depth)
    assert oracle.header_fields(s)["max_level"] == depth - 1
    parity(x, s, f"depth{depth}")


def test_ordered_slots_scan_over_many_tiles(ordered_slots):
    """Eight sequences per chunk and about 40 levels: more (level, chunk)
    counts than one workgroup's pass of the tile scan covers (over 256 tiles
    of 4096 counts, the last one partial)."""
    x = synth.wiki(6 << 20, 0xACE6)
    s = oracle.encode(x, block_log2=20, chunk_log2=3, max_depth=40)
    h = oracle.header_fields(s)
    assert h["max_level"] == 39 and (h["max_level"] + 1) * h["n_chunks"] > 256 * 4096
    assert (h["max_level"] + 1) * h["n_chunks"] % 4096 != 0
    parity(x, s, "ordered-many-tiles")
