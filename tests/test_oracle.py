"""Pins for the oracle: closed forms, the paper's worked examples, brute force,
invariants and error paths.  CPU only.

Each test fixes the oracle to something other than itself: a closed form
derived by hand, a worked example from the paper's text, a second decoder in
pure Python, direct execution of token lists, or levels recomputed in Python
from the definition in Sec. 7.1.
"""
import itertools

import numpy as np
import pytest

import oracle
import streamgen
import synth


def toks(s):
    return [tuple(int(v) for v in t) for t in oracle.tokens(s)]


def py_levels_and_literals(tokens, n):
    """Levels from the definition (Sec. 7.1) and a literal-byte map, in Python."""
    wl = [-1] * n
    lit = [True] * n
    out = []
    for dst, src, ln, _ in tokens:
        lv = 1 + max(wl[src:src + ln], default=-1)
        out.append(lv)
        for k in range(ln):
            wl[dst + k] = lv
            lit[dst + k] = False
    return out, lit


def unique_bytes(L, seed=7):
    rng = np.random.default_rng(seed)
    return rng.permutation(256)[:L].astype(np.uint8).tobytes()


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("tiebreak", [0, 1])
@pytest.mark.parametrize("k", [1, 3, 6])
def test_doubling_string_levels_closed_form(tiebreak, k):
    """u repeated 2^k times (|u| = 16, distinct bytes): the greedy parse is one
    literal run u then k matches, the j-th at 16*2^j of length 16*2^j from
    position 0, and its level is exactly j (each doubling reads bytes written
    by the previous one)."""
    L = 16
    x = unique_bytes(L) * (1 << k)
    s = oracle.encode(x, tiebreak=tiebreak, hash_bits=12)
    want = [(L << j, 0, L << j, j) for j in range(k)]
    assert toks(s) == want
    assert oracle.decode(s).tobytes() == x
    assert oracle.header_fields(s)["max_level"] == k - 1


def test_depth_one_is_two_phase():
    """With depth limit 1 every match must source literal bytes only, so the
    doubling string becomes copies of u from position 0, all at level 0."""
    L, k = 16, 5
    x = unique_bytes(L) * (1 << k)
    s = oracle.encode(x, max_depth=1, hash_bits=12)
    assert toks(s) == [(j * L, 0, L, 0) for j in range(1, 1 << k)]
    assert oracle.decode(s).tobytes() == x


def test_flattening_collapses_doubling_chain():
    """Within one block, flattening traces every match byte to its literal
    root, so every piece sources the literal run u at positions 0..15: copies
    of u, all at level 0 (Sec. 3.3: every in-block source is a literal)."""
    L, k = 16, 4
    x = unique_bytes(L) * (1 << k)
    s = oracle.encode(x, flatten=1, hash_bits=12)
    t = toks(s)
    assert all(lv == 0 for *_, lv in t)
    assert all(src == 0 and ln == L for _, src, ln, _ in t)
    assert [d for d, *_ in t] == [j * L for j in range(1, 1 << k)]
    assert oracle.decode(s).tobytes() == x


# ------------------------------------------------------ the paper's worked examples

def _w1_input():
    rng = np.random.default_rng(1234)
    x = bytearray(rng.integers(0, 256, 6000, dtype=np.uint8).tobytes())
    x[5100:5132] = x[5000:5032]
    x[5300:5332] = x[5000:5032]
    return bytes(x)


def test_w1_absolute_offset_example():
    """Sec. 3.1: bytes at 5,000 referenced from 5,100 (distance 100) and from
    5,300 (distance 300) are stored both times as the absolute offset 5,000."""
    x = _w1_input()
    s = oracle.encode(x, hash_bits=16)
    t = [tt for tt in toks(s) if tt[0] in (5100, 5300)]
    assert [(d, src) for d, src, _, _ in t] == [(5100, 5000), (5300, 5000)]
    assert all(ln == 32 for _, _, ln, _ in t)
    assert [lv for *_, lv in t] == [0, 0]
    assert oracle.decode(s).tobytes() == x


def test_w2_chain_example():
    """Sec. 3.3: A copies from B, which copies from literal C.  Without
    flattening (most-recent tie-break) A sources B at level 1; after
    flattening A sources C directly at level 0."""
    x = _w1_input()  # C = 5000.., B = 5100.., A = 5300..
    s = oracle.encode(x, hash_bits=16, tiebreak=1)
    t = {d: (src, lv) for d, src, _, lv in toks(s)}
    assert t[5100] == (5000, 0) and t[5300] == (5100, 1)
    s = oracle.encode(x, hash_bits=16, tiebreak=1, flatten=1)
    t = {d: (src, lv) for d, src, _, lv in toks(s)}
    assert t[5100] == (5000, 0) and t[5300] == (5000, 0)


def test_w2_chain_crossing_blocks_keeps_dependency():
    """Sec. 3.3 limitation: a chain that leaves the block is cut at the first
    position outside it, so the dependency on the earlier block remains."""
    x = _w1_input()
    # blocks of 256 bytes: B (5100) and A (5300) sit in different blocks
    s = oracle.encode(x, hash_bits=16, tiebreak=1, flatten=1, block_log2=8)
    t = {d: (src, lv) for d, src, _, lv in toks(s)}
    # A's source B lies in block 19 (4864..5119) while A lies in block 20:
    # the trace stops at B, which is itself a level-0 match
    assert t[5300] == (5100, 1)


def _r2_input():
    """512-byte blocks.  Block 1 holds the literal run C (700..731).  Block 2
    holds B = copy of C at 1100, a literal run C' at 1160, B' = copy of C' at
    1220, then A = copy of C at 1300 and A' = copy of C' at 1420."""
    rng = np.random.default_rng(4321)
    x = bytearray(rng.integers(0, 256, 2048, dtype=np.uint8).tobytes())
    x[1100:1132] = x[700:732]
    x[1220:1252] = x[1160:1192]
    x[1300:1332] = x[700:732]
    x[1420:1452] = x[1160:1192]
    return bytes(x)


@pytest.mark.parametrize("flatten,want", [
    # no flattening, most-recent tie-break: A and A' take the latest copy
    (0, {1100: (700, 0), 1220: (1160, 0), 1300: (1100, 1), 1420: (1220, 1)}),
    # R1: every chain is traced inside block 2; A's trace leaves the block
    # at 700 (first position outside), the trace of A' ends at the literal C'
    (1, {1100: (700, 0), 1220: (1160, 0), 1300: (700, 0), 1420: (1160, 0)}),
    # R2: only chains rooted at a literal of the block are re-pointed: A'
    # moves to C', A keeps its source B because B's chain leaves the block
    (2, {1100: (700, 0), 1220: (1160, 0), 1300: (1100, 1), 1420: (1160, 0)}),
])
def test_flatten_modes_on_two_chains(flatten, want):
    """Sec. 3.3 and its limitation: the three flattening readings give three
    different source sets on one input with a cross-block chain (C -> B -> A)
    and an in-block literal chain (C' -> B' -> A')."""
    x = _r2_input()
    s = oracle.encode(x, hash_bits=16, tiebreak=1, flatten=flatten, block_log2=9)
    t = {d: (src, lv) for d, src, ln, lv in toks(s) if ln >= 32}
    assert {d: t[d] for d in want} == want
    assert oracle.decode(s).tobytes() == x


def flattened_from_definition(x, plain_tokens, B, mode, m0=4):
    """The matches that flattening must produce, recomputed from the
    unflattened parse by following each byte's chain backwards (Sec. 3.3).

    A byte of a match in block [bs, bs+B) traces its source y: while y lies in
    the block and was written by a match, y moves to that match's source byte.
    The trace ends at a literal of the block (the chain is literal-rooted) or
    at a position before the block.  Mode 1 re-points the byte to where the
    trace ends; mode 2 re-points it only when the chain is literal-rooted and
    otherwise keeps its own source.  Each match is cut where the new sources
    stop being consecutive; pieces shorter than m0 become literals."""
    src_of = {}
    for dst, src, ln, _ in plain_tokens:
        for k in range(ln):
            src_of[dst + k] = src + k
    out = []
    for dst, src, ln, _ in plain_tokens:
        bs = dst // B * B
        new = []
        for k in range(ln):
            y = src + k
            while y >= bs and y in src_of:
                y = src_of[y]
            rooted = y >= bs
            new.append(y if (mode == 1 or rooted) else src + k)
        a = 0
        while a < ln:
            b = a + 1
            while b < ln and new[b] == new[b - 1] + 1:
                b += 1
            if b - a >= m0:
                out.append((dst + a, new[a], b - a))
            a = b
    return out


@pytest.mark.parametrize("mode", [1, 2])
@pytest.mark.parametrize("seed", range(6))
def test_flattening_matches_definition(mode, seed):
    """Both flattening readings equal their definition recomputed from the
    unflattened parse (most-recent tie-break, no depth limit: the parse then
    does not depend on levels, so flattening is a pure rewrite of it)."""
    rng = np.random.default_rng(100 + seed)
    alpha = [2, 3, 4, 16][seed % 4]
    n = int(rng.integers(300, 4000))
    base = rng.integers(0, alpha, n, dtype=np.uint8)
    for _ in range(n // 40):  # repeats so that chains of copies appear
        ln = int(rng.integers(4, 40))
        d = int(rng.integers(ln, n - ln)) if n > 2 * ln else 0
        s0 = int(rng.integers(0, d - ln + 1)) if d >= ln else 0
        base[d:d + ln] = base[s0:s0 + ln]
    x = base.tobytes()
    bl = [3, 5, 6, 8, 9, 12][seed]
    o = dict(hash_bits=12, tiebreak=1, block_log2=bl, chunk_log2=2)
    plain = toks(oracle.encode(x, **o))
    got = [(d, s_, ln) for d, s_, ln, _ in toks(oracle.encode(x, flatten=mode, **o))]
    assert got == flattened_from_definition(x, plain, 1 << bl, mode)


# ------------------------------------------------------------------ brute force

OPTION_GRID = [
    dict(),
    dict(tiebreak=1),
    dict(flatten=1),
    dict(flatten=2, tiebreak=1),
    dict(max_depth=1),
    dict(max_depth=2, tiebreak=1),
    dict(max_depth=3, flatten=1),
    dict(block_log2=3, chunk_log2=0),
    dict(block_log2=4, flatten=1, tiebreak=1, chunk_log2=1),
    dict(block_log2=3, max_depth=2, chunk_log2=1),
    dict(block_log2=3, flatten=2, tiebreak=1, chunk_log2=0),
    dict(block_log2=3, flatten=1, tiebreak=1, chunk_log2=1),
    dict(levels=0),
    dict(block_log2=3, levels=0, chunk_log2=1),
]


def _all_strings(alpha, maxlen):
    for L in range(maxlen + 1):
        for t in itertools.product(alpha, repeat=L):
            yield bytes(t)


def _check_stream(x, s, opts):
    rep = oracle.check(x, s)
    assert rep.level_mismatch == 0
    t = toks(s)
    py_lv, lit = py_levels_and_literals(t, len(x))
    assert [lv for *_, lv in t] == py_lv
    B = 1 << opts.get("block_log2", 20)
    for dst, src, ln, _ in t:
        assert src + ln <= dst and ln >= 4
        assert x[src:src + ln] == x[dst:dst + ln]
        if opts.get("flatten") == 1:
            bs = dst // B * B
            assert all(lit[y] for y in range(max(src, bs), src + ln))
    if opts.get("max_depth"):
        assert all(lv <= opts["max_depth"] - 1 for *_, lv in t)
    if opts.get("flatten") and opts.get("tiebreak") == 1 and not opts.get("max_depth"):
        # R1 / R2: the matches are the definition's rewrite of the unflattened parse
        plain = toks(oracle.encode(x, **dict(opts, flatten=0)))
        assert [(d, s_, ln) for d, s_, ln, _ in t] == flattened_from_definition(x, plain, B, opts["flatten"])
    return t


@pytest.mark.parametrize("opts", OPTION_GRID, ids=lambda o: ",".join(f"{k}={v}" for k, v in o.items()) or "default")
def test_bruteforce_roundtrip(opts):
    """Every string over {a,b} up to length 11 and over {a,b,c} up to 7 round-trips
    under each option set, agrees with the pure-Python decoder and passes the
    invariants (source before destination, source bytes equal, levels exact,
    flattening and depth bounds)."""
    o = dict(hash_bits=8)
    o.update(opts)
    n_matched = 0
    for x in itertools.chain(_all_strings(b"ab", 11), _all_strings(b"abc", 7)):
        s = oracle.encode(x, **o)
        assert oracle.decode(s).tobytes() == x
        assert oracle.refdec(s) == x
        n_matched += bool(_check_stream(x, s, o))
    assert n_matched > 100


# ------------------------------------------------------ token-level semantics

@pytest.mark.parametrize("seed", range(12))
def test_random_token_streams(seed):
    """Hand-built streams of random tokens (not from the encoder): the oracle's
    decode equals direct execution of the tokens and the Python decoder, and
    its checker recomputes the same levels."""
    rng = np.random.default_rng(seed)
    bl = [3, 5, 8, 12][seed % 4]
    n = int(rng.integers(0, 3000))
    blocks, lits = streamgen.random_tokens(rng, n, bl, max_len=[6, 40, 300][seed % 3])
    s, want = streamgen.build(blocks, lits, n, block_log2=bl, chunk_log2=int(rng.integers(0, 5)))
    assert oracle.decode(s).tobytes() == want
    assert oracle.refdec(s) == want
    assert oracle.check(np.frombuffer(want, np.uint8), s).level_mismatch == 0
    for T in (1, 3):
        assert oracle.decode_mt(s, T).tobytes() == want


@pytest.mark.parametrize("width", [2, 4, "random"])
def test_padded_varints_decode_the_same(width):
    """LEB128 values padded with zero continuation groups (non-minimal, at most
    4 bytes) are valid and decode like the minimal encoding."""
    rng = np.random.default_rng(17)
    n = 20_000
    blocks, lits = streamgen.random_tokens(rng, n, 12, max_len=300, p_match=0.7)
    w = np.random.default_rng(5) if width == "random" else width
    s, want = streamgen.build(blocks, lits, n, block_log2=12, chunk_log2=6, varint_width=w)
    s0, want0 = streamgen.build(blocks, lits, n, block_log2=12, chunk_log2=6)
    assert want == want0 and s.size > s0.size
    assert oracle.decode(s).tobytes() == want
    assert oracle.refdec(s) == want
    assert oracle.check(np.frombuffer(want, np.uint8), s).level_mismatch == 0


def test_edge_cases():
    for x in [b"", b"a", b"abc", b"abcd", b"aaaaaaaa", bytes(range(256)) * 3]:
        for o in [dict(), dict(block_log2=3, chunk_log2=0), dict(flatten=1, block_log2=4)]:
            s = oracle.encode(x, hash_bits=10, **o)
            assert oracle.decode(s).tobytes() == x
            assert oracle.refdec(s) == x
    s = oracle.encode(b"")
    h = oracle.header_fields(s)
    assert h["n_blocks"] == 0 and h["comp_bytes"] == 96 and h["n_seq"] == 0


def test_sequences_multiple_of_chunk():
    """n_seq an exact multiple of the chunk size: the trailing run belongs to the last chunk."""
    blocks = [([(4, 4, 0)] * 4, 3)]
    lits = bytes(range(19))
    n = 4 * 8 + 3
    s, want = streamgen.build(blocks, lits, n, block_log2=8, chunk_log2=1)
    assert oracle.decode(s).tobytes() == want
    assert oracle.refdec(s) == want


# ----------------------------------------------------------------- error paths

def _valid_small():
    rng = np.random.default_rng(5)
    blocks, lits = streamgen.random_tokens(rng, 600, 7)
    return streamgen.build(blocks, lits, 600, block_log2=7, chunk_log2=2)


def test_rejects_overlapping_source():
    blocks = [([(4, 4, 2)], 0)]  # src 2 + 4 > dst 4
    with pytest.raises(AssertionError):
        streamgen.build(blocks, b"abcd", 8, block_log2=8)
    s, _ = streamgen.build([([(4, 4, 0)], 0)], b"abcd", 8, block_log2=8)
    bad = s.copy()
    # the off[] section starts right after the block header + one chunk entry
    base = int.from_bytes(bad[64:72].tobytes(), "little")
    off_at = base + 32 + 32
    bad[off_at:off_at + 4] = np.frombuffer((2).to_bytes(4, "little"), np.uint8)
    with pytest.raises(oracle.OracleError) as e:
        oracle.decode(bad)
    assert e.value.code == -3


def test_rejects_truncation_and_bad_header():
    s, _ = _valid_small()
    for cut in (0, 10, 63, 64, s.size // 2, s.size - 1):
        with pytest.raises(oracle.OracleError):
            oracle.decode(s[:cut])
    bad = s.copy()
    bad[0] ^= 1
    with pytest.raises(oracle.OracleError):
        oracle.decode(bad)


def test_random_bit_flips_never_crash():
    s, want = _valid_small()
    rng = np.random.default_rng(9)
    rejected = 0
    for _ in range(400):
        bad = s.copy()
        i = int(rng.integers(0, s.size))
        bad[i] ^= np.uint8(1 << int(rng.integers(0, 8)))
        try:
            got = oracle.decode(bad)
        except oracle.OracleError:
            rejected += 1
            continue
        assert got.size == len(want)
    assert rejected > 100


def test_rejects_wrong_level_bound():
    rng = np.random.default_rng(3)
    blocks, lits = streamgen.random_tokens(rng, 400, 8)
    s, _ = streamgen.build(blocks, lits, 400, block_log2=8, max_level=0)
    if oracle.tokens(streamgen.build(blocks, lits, 400, block_log2=8)[0])["lvl"].max() > 0:
        with pytest.raises(oracle.OracleError):
            oracle.decode(s)


# ---------------------------------------------------- generated workloads

@pytest.mark.parametrize("kind", ["markov", "fastq", "wiki", "random"])
@pytest.mark.parametrize("opts", [dict(), dict(flatten=1), dict(max_depth=8), dict(flatten=2)],
                         ids=["plain", "flat", "d8", "flatlit"])
def test_generated_workloads(kind, opts):
    n = 3 << 20
    x = synth.make(kind, n, 0xACE0)
    s = oracle.encode(x, block_log2=18, **opts)
    rep = oracle.check(x, s)
    assert rep.level_mismatch == 0
    if opts.get("flatten") == 1:
        assert rep.inblock_nonliteral_src_bytes == 0
    if opts.get("max_depth"):
        assert rep.depth_violations == 0 and rep.max_level <= 7
    assert (oracle.decode_mt(s, 4) == x).all()
    assert oracle.header_fields(s)["content_hash"] == oracle.content_hash(x)


# -------------------------------------------- streams without levels (Sec. 3.2)

@pytest.mark.parametrize("kind", ["markov", "fastq", "wiki", "random"])
@pytest.mark.parametrize("opts", [dict(), dict(flatten=1), dict(max_depth=4), dict(block_log2=12, chunk_log2=4)],
                         ids=["plain", "flat", "d4", "small"])
def test_four_stream_format(kind, opts):
    """The paper's four streams (lit, len, off, cmd) with no lvl[] and no level
    table decode to the same bytes, and the oracle assigns every match the
    level of the definition (Sec. 7.1) from the writers of its source bytes:
    equal to the levels the encoder computed while parsing and stored in the
    levelled stream of the same input."""
    x = synth.make(kind, 1 << 20, 0xACE0 + len(kind))
    o = dict(dict(block_log2=16), **opts)
    with_lv = oracle.encode(x, **o)
    free = oracle.encode(x, levels=0, **o)
    h = oracle.header_fields(free)
    assert h["flags"] & 8 == 0 and h["max_level"] == 0 and h["n_deep"] == 0
    assert free.size < with_lv.size
    assert np.array_equal(oracle.decode(free), x)
    assert np.array_equal(oracle.decode_mt(free, 3), x)
    assert oracle.refdec(free) == x.tobytes()
    a, b = oracle.tokens(with_lv), oracle.tokens(free)
    assert np.array_equal(a, b)
    rep = oracle.check(x, free)
    assert rep.level_mismatch == 0 and rep.max_level == oracle.header_fields(with_lv)["max_level"]


def test_four_stream_format_from_tokens():
    """Hand-built token lists without levels: the oracle's levels equal the
    ones computed in Python from the definition."""
    rng = np.random.default_rng(21)
    for bl in (4, 8, 12):
        n = 3000
        blocks, lits = streamgen.random_tokens(rng, n, bl, max_len=50)
        s, want = streamgen.build(blocks, lits, n, block_log2=bl, chunk_log2=3, with_levels=False)
        assert oracle.decode(s).tobytes() == want
        t = toks(s)
        py_lv, _ = py_levels_and_literals(t, n)
        assert [lv for *_, lv in t] == py_lv


def test_four_stream_format_rejects_level_fields():
    x = synth.markov(50_000, 1)
    s = oracle.encode(x, levels=0, block_log2=12)
    bad = s.copy()
    bad[36] = 1  # a max_level without levels
    with pytest.raises(oracle.OracleError):
        oracle.decode(bad)
