"""The host encoder of the library against the oracle.

Without a depth limit both encoders are written independently from the same
description of the parse (greedy over 4-byte hash chains, absolute offsets,
lowest-level tie-break, within-block flattening), so their streams must be
identical byte for byte.  With a depth limit (Sec. 7.4) the library's
encoder takes a different parse than the oracle's greedy-with-cut: it keeps
the level-independent parse's matches that stay within the limit and re-cuts
the deeper ones inside their own span.  Its streams are then held to the
definition: exact levels recomputed by the oracle's checker, every level at
most D - 1, every source before its destination, the original bytes back,
and every match inside a match of the unlimited parse."""
import numpy as np
import pytest

import oracle
import synth
import paper_2606_04268_amd as ax

OPTS = [dict(), dict(flatten=1), dict(flatten=2), dict(tiebreak=1), dict(tiebreak=1, flatten=1),
        dict(chunk_log2=3, block_log2=12)]
IDS = ["plain", "flat", "flatlit", "recent", "recentflat", "small"]

LIMITED = [dict(max_depth=8), dict(max_depth=1, flatten=1), dict(max_depth=2), dict(max_depth=10, flatten=2),
           dict(max_depth=3, tiebreak=1), dict(max_depth=8, block_log2=12, chunk_log2=3)]
LIMITED_IDS = ["d8", "d1flat", "d2", "d10flatlit", "d3recent", "d8small"]


def _split(opts):
    return opts.get("block_log2", 17), {k: v for k, v in opts.items() if k != "block_log2"}


@pytest.mark.parametrize("kind", ["markov", "fastq", "wiki", "random"])
@pytest.mark.parametrize("opts", OPTS, ids=IDS)
def test_product_encoder_matches_oracle(kind, opts):
    x = synth.make(kind, (1 << 20) + 4321, 99)
    bl, rest = _split(opts)
    want = oracle.encode(x, block_log2=bl, **rest)
    got = ax.encode(x, block_log2=bl, threads=4, **rest)
    assert got.size == want.size
    assert np.array_equal(got, want)
    rep = oracle.check(x, got)
    assert rep.level_mismatch == 0


def _spans(s):
    t = oracle.tokens(s)
    return [(int(d), int(d) + int(n)) for d, n in zip(t["dst"], t["len"])]


def check_limited(x, s, depth, plain):
    """A depth-limited stream against the definition (see the module text)."""
    x = np.frombuffer(bytes(x), np.uint8) if isinstance(x, (bytes, bytearray)) else np.asarray(x, dtype=np.uint8)
    rep = oracle.check(x, s)
    assert rep.level_mismatch == 0 and rep.depth_violations == 0
    assert rep.max_level <= depth - 1
    assert np.array_equal(oracle.decode(s), x)
    t = oracle.tokens(s)
    assert (t["src"].astype(np.int64) + t["len"] <= t["dst"]).all()
    # every match lies inside one match of the unlimited parse (same options, no limit)
    outer = _spans(plain)
    starts = np.array([a for a, _ in outer], dtype=np.int64)
    ends = np.array([b for _, b in outer], dtype=np.int64)
    for a, b in _spans(s):
        i = np.searchsorted(starts, a, side="right") - 1
        assert i >= 0 and b <= ends[i], (a, b)


@pytest.mark.parametrize("kind", ["markov", "fastq", "wiki", "random"])
@pytest.mark.parametrize("opts", LIMITED, ids=LIMITED_IDS)
def test_product_encoder_depth_limited(kind, opts):
    x = synth.make(kind, (1 << 20) + 4321, 99)
    bl, rest = _split(opts)
    got = ax.encode(x, block_log2=bl, threads=4, **rest)
    plain = ax.encode(x, block_log2=bl, threads=4, **dict(rest, max_depth=0, flatten=0))
    # flattening only cuts matches into pieces, so containment holds with it too
    check_limited(x, got, opts["max_depth"], plain)


def test_product_encoder_edge_cases():
    for x in [b"", b"a", b"abcd", b"abcdabcdabcd", bytes(range(256)) * 5, b"q" * 5000]:
        for o in [dict(), dict(block_log2=3, chunk_log2=0), dict(flatten=1, block_log2=4)]:
            want = oracle.encode(x, hash_bits=10, **o)
            got = ax.encode(x, hash_bits=10, **o)
            assert np.array_equal(got, want), (x[:20], o)
        for o in [dict(max_depth=2), dict(max_depth=1, block_log2=3, chunk_log2=0)]:
            got = ax.encode(x, hash_bits=10, **o)
            check_limited(x, got, o["max_depth"], ax.encode(x, hash_bits=10, **dict(o, max_depth=0)))


@pytest.mark.parametrize("opts", [dict(flatten=1), dict(max_depth=8), dict(max_depth=2, flatten=2)])
def test_product_encoder_thread_count_does_not_matter(opts):
    x = synth.fastq(3 << 20, 5)
    a = ax.encode(x, block_log2=16, threads=1, **opts)
    b = ax.encode(x, block_log2=16, threads=7, **opts)
    assert np.array_equal(a, b)


def test_product_encoder_rejects_bad_options():
    with pytest.raises(ax.AceapexError):
        ax.encode(b"abcdefgh", min_match=3)
    with pytest.raises(ax.AceapexError):
        ax.encode(b"abcdefgh", block_log2=2)
