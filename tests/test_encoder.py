"""The host encoder of the library against the oracle's encoder.

Both are written independently from the same description of the parse
(greedy over 4-byte hash chains, absolute offsets, lowest-level tie-break,
within-block flattening, depth limit); their streams must be identical byte
for byte, and every product stream must pass the oracle's checker."""
import numpy as np
import pytest

import oracle
import synth
import paper_2606_04268_amd as ax

OPTS = [dict(), dict(flatten=1), dict(flatten=2), dict(max_depth=8), dict(max_depth=1, flatten=1),
        dict(tiebreak=1), dict(tiebreak=1, flatten=1), dict(chunk_log2=3, block_log2=12)]
IDS = ["plain", "flat", "flatlit", "d8", "d1flat", "recent", "recentflat", "small"]


@pytest.mark.parametrize("kind", ["markov", "fastq", "wiki", "random"])
@pytest.mark.parametrize("opts", OPTS, ids=IDS)
def test_product_encoder_matches_oracle(kind, opts):
    x = synth.make(kind, (1 << 20) + 4321, 99)
    want = oracle.encode(x, block_log2=opts.get("block_log2", 17), **{k: v for k, v in opts.items() if k != "block_log2"})
    got = ax.encode(x, block_log2=opts.get("block_log2", 17), threads=4,
                    **{k: v for k, v in opts.items() if k != "block_log2"})
    assert got.size == want.size
    assert np.array_equal(got, want)
    rep = oracle.check(x, got)
    assert rep.level_mismatch == 0


def test_product_encoder_edge_cases():
    for x in [b"", b"a", b"abcd", b"abcdabcdabcd", bytes(range(256)) * 5, b"q" * 5000]:
        for o in [dict(), dict(block_log2=3, chunk_log2=0), dict(flatten=1, block_log2=4), dict(max_depth=2)]:
            want = oracle.encode(x, hash_bits=10, **o)
            got = ax.encode(x, hash_bits=10, **o)
            assert np.array_equal(got, want), (x[:20], o)


def test_product_encoder_thread_count_does_not_matter():
    x = synth.fastq(3 << 20, 5)
    a = ax.encode(x, block_log2=16, flatten=1, threads=1)
    b = ax.encode(x, block_log2=16, flatten=1, threads=7)
    assert np.array_equal(a, b)


def test_product_encoder_rejects_bad_options():
    with pytest.raises(ax.AceapexError):
        ax.encode(b"abcdefgh", min_match=3)
    with pytest.raises(ax.AceapexError):
        ax.encode(b"abcdefgh", block_log2=2)
