"""Pins for the oracle's tANS coder (oracle/tans_oracle.c), the entropy stage
for literals (Sec. 4.4, Sec. 8 leave entropy coding of the four streams to
future work): exact round trips, code lengths fixed in closed form by dyadic
probabilities, the normalization rules, brute force over tiny inputs and
damaged containers.  CPU only."""
import itertools

import numpy as np
import pytest

import oracle
import synth


def body_bits(c):
    """Bitstream bytes of a container (field at offset 24)."""
    return int(c[24:28].view(np.uint32)[0])


@pytest.mark.parametrize("lanes", [1, 3, 64, 1024])
@pytest.mark.parametrize("table_log", [8, 11, 12])
def test_round_trip(table_log, lanes):
    rng = np.random.default_rng(table_log * 100 + lanes)
    for x in [b"", b"z", bytes(range(256)), synth.fastq(300_000, 1).tobytes(), synth.wiki(200_000, 2).tobytes(),
              rng.integers(0, 256, 50_000, dtype=np.uint8).tobytes(), rng.integers(0, 3, 10_000, dtype=np.uint8).tobytes()]:
        c = oracle.tans_encode(x, table_log, lanes)
        assert oracle.tans_decode(c).tobytes() == x


def test_single_symbol_costs_no_bits():
    """One symbol owns every table entry, so each state maps to itself with
    zero bits: the bitstream is empty whatever the length."""
    for n in (1, 100, 12345):
        c = oracle.tans_encode(b"q" * n, 11, 7)
        assert body_bits(c) == 0
        assert oracle.tans_decode(c).tobytes() == b"q" * n


@pytest.mark.parametrize("table_log", [8, 11])
def test_dyadic_code_lengths(table_log):
    """With probabilities 1/2, 1/4, 1/8, 1/8 the normalized counts are exact
    (L/2, L/4, L/8, L/8) and a symbol of count c = L / 2^b always costs
    exactly b bits (its states y lie in [c, 2c), so R - floor(log2 y) = b):
    the bitstream holds n_a + 2 n_b + 3 (n_c + n_d) bits in total."""
    L = 1 << table_log
    n = 8 * 5000
    x = np.array([0] * (n // 2) + [1] * (n // 4) + [2] * (n // 8) + [3] * (n // 8), dtype=np.uint8)
    np.random.default_rng(5).shuffle(x)
    counts = oracle.tans_counts(x, table_log)
    assert counts[:4].tolist() == [L // 2, L // 4, L // 8, L // 8] and counts[4:].sum() == 0
    c = oracle.tans_encode(x, table_log, 1)
    want_bits = n // 2 * 1 + n // 4 * 2 + n // 4 * 3
    assert body_bits(c) == (want_bits + 7) // 8
    assert np.array_equal(oracle.tans_decode(c), x)


def test_uniform_bytes_cost_eight_bits():
    x = np.tile(np.arange(256, dtype=np.uint8), 40)
    c = oracle.tans_encode(x, 11, 1)
    assert body_bits(c) == x.size  # 8 bits each
    assert np.array_equal(oracle.tans_decode(c), x)


def test_normalized_counts():
    """Counts sum to 2^R, every present symbol keeps at least 1, absent ones
    get 0, and the corrections land on the largest count."""
    x = np.array([7] * 100_000 + [9] * 3, dtype=np.uint8)  # 9 would round to 0
    c = oracle.tans_counts(x, 11)
    assert c.sum() == 2048 and c[9] == 1 and c[7] == 2047 and (c > 0).sum() == 2
    x = np.arange(256, dtype=np.uint8).repeat([1 if i else 10_000 for i in range(256)])
    c = oracle.tans_counts(x, 8)  # 256 symbols in 256 entries: every count is 1
    assert c.sum() == 256 and (c == 1).all()
    with pytest.raises(oracle.OracleError):
        oracle.tans_counts(np.arange(256, dtype=np.uint8), 7)


def test_bruteforce_tiny_inputs():
    n_checked = 0
    for L in range(0, 8):
        for t in itertools.product(b"abc", repeat=L):
            x = bytes(t)
            for lanes in (1, 2, 5):
                assert oracle.tans_decode(oracle.tans_encode(x, 8, lanes)).tobytes() == x
                n_checked += 1
    assert n_checked > 9000


def test_close_to_the_entropy():
    """Within 1% of the empirical entropy on a large skewed source."""
    rng = np.random.default_rng(11)
    p = np.array([0.4, 0.3, 0.15, 0.1, 0.05])
    x = rng.choice(5, size=400_000, p=p).astype(np.uint8)
    h = np.bincount(x) / x.size
    H = -(h * np.log2(h)).sum()
    c = oracle.tans_encode(x, 12, 1)
    assert body_bits(c) * 8 / x.size < H * 1.01


def test_damaged_containers_never_crash():
    x = synth.fastq(40_000, 4).tobytes()
    c = oracle.tans_encode(x, 11, 16)
    rng = np.random.default_rng(3)
    bad_count = 0
    for _ in range(300):
        d = c.copy()
        i = int(rng.integers(0, d.size))
        d[i] ^= np.uint8(1 << int(rng.integers(0, 8)))
        try:
            got = oracle.tans_decode(d)
        except oracle.OracleError:
            bad_count += 1
            continue
        assert got.size == len(x)
    assert bad_count > 30
    with pytest.raises(oracle.OracleError):
        oracle.tans_decode(c[:100])
