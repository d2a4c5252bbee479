"""Seeded mixes of streams for the batched GPU tests: varied kinds, sizes,
block and chunk sizes and encoder options, plus the edge cases (an empty
stream, long doubling matches, a 600-deep chain)."""
import numpy as np

import oracle
import streamgen
import synth


def mixed_streams(count, seed):
    """(original bytes, stream) pairs of varied kind, size, block size and options."""
    rng = np.random.default_rng(seed)
    out = []
    kinds = ["markov", "fastq", "random", "wiki"]
    for i in range(count):
        kind = kinds[i % 4]
        n = int(np.exp(rng.uniform(np.log(200), np.log(600_000))))
        x = synth.make(kind, n, seed * 1000 + i)
        opts = dict(block_log2=int(rng.choice([12, 16, 20])), flatten=int(rng.integers(0, 3)),
                    max_depth=int(rng.choice([0, 0, 2, 8])), chunk_log2=int(rng.choice([4, 8, 10])))
        out.append((x, oracle.encode(x, **opts)))
    out.append((np.zeros(0, np.uint8), oracle.encode(b"")))
    u = np.random.default_rng(7).permutation(256)[:16].astype(np.uint8).tobytes()
    dbl = u * 4096
    out.append((np.frombuffer(dbl, np.uint8), oracle.encode(dbl, hash_bits=12)))
    m = 600
    blocks = [([(4, 4, 0)] + [(0, 4, 4 * i) for i in range(1, m)], 0)]
    s, want = streamgen.build(blocks, b"abcd", 4 + 4 * m, block_log2=14, chunk_log2=5)
    out.append((np.frombuffer(want, np.uint8), s))
    return out
