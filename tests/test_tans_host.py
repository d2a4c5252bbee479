"""Host checks of the library's tANS container API (no GPU): its encoder,
written separately from the oracle's from the same definition, produces the
same containers byte for byte, and the probe rejects malformed headers."""
import numpy as np
import pytest

import oracle
import synth
from paper_2606_04268_amd import _abi


@pytest.mark.parametrize("table_log,lanes", [(8, 1), (11, 1024), (12, 333), (11, 50_000)])
def test_encoder_matches_oracle(table_log, lanes):
    rng = np.random.default_rng(table_log + lanes)
    for x in [b"", b"q" * 1000, bytes(range(256)) * 10, synth.fastq(400_000, 3).tobytes(),
              synth.wiki(300_000, 4).tobytes(), rng.integers(0, 256, 70_000, dtype=np.uint8).tobytes()]:
        a = _abi.tans_encode(x, table_log, lanes)
        b = oracle.tans_encode(x, table_log, lanes)
        assert np.array_equal(a, b)
        info = _abi.tans_probe(a)
        assert info.n == len(x) and info.lanes == lanes and info.table_log == table_log
        assert info.container_bytes == a.size


def test_probe_rejects_bad_headers():
    c = oracle.tans_encode(synth.fastq(50_000, 1).tobytes(), 11, 64)
    with pytest.raises(_abi.AceapexError) as e:
        _abi.tans_probe(c[:100])
    assert e.value.code == _abi.E_INVAL
    for at, v in [(0, ord("B")), (8, 13), (8, 7), (12, 0), (28, 1), (33, 0x7F)]:
        bad = c.copy()
        bad[at] = v
        with pytest.raises(_abi.AceapexError) as e:
            _abi.tans_probe(bad)
        assert e.value.code == _abi.E_FORMAT, at
