"""The seeded input generators (synth/): their random sources against
published reference outputs, and golden digests of every configuration's
input (and of the oracle's stream of it) for determinism across machines.
CPU only."""
import json
import os

import numpy as np

import synth
from golden.make_golden import digests

HERE = os.path.dirname(os.path.abspath(__file__))


def test_splitmix64_reference_outputs():
    """SplitMix64 (Steele, Lea and Flood 2014) from state 0: the first four
    outputs of the reference generator."""
    gamma = 0x9E3779B97F4A7C15
    got = [synth.splitmix64((k * gamma) % 2**64) for k in range(4)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]


def test_xoshiro256starstar_reference_outputs():
    """xoshiro256** (Blackman and Vigna 2018) from the state {1, 2, 3, 4}: the
    first output is rotl(2 * 5, 7) * 9 = 11520, the second 0 (s1 becomes 0),
    the third rotl(262149 * 5, 7) * 9; then the reference sequence."""
    got = [int(v) for v in synth.raw64_state(6, [1, 2, 3, 4])]
    assert got == [11520, 0, 1509978240, 1215971899390074240, 1216172134540287360, 607988272756665600]


def test_seeding_goes_through_splitmix64():
    """Generator state = four SplitMix64 outputs of the seed."""
    seed = 0xACE0
    st, x = [], seed
    gamma = 0x9E3779B97F4A7C15
    for _ in range(4):
        st.append(synth.splitmix64(x))
        x = (x + gamma) % 2**64
    assert np.array_equal(synth.raw64(5, seed), synth.raw64_state(5, st))


def test_golden_digests():
    with open(os.path.join(HERE, "golden", "synth_hashes.json")) as f:
        want = json.load(f)
    assert digests() == want
