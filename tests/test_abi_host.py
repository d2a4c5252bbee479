"""Host-only checks of the C ABI: the library loads, exports every declared
symbol, and the host-side calls (probe, workspace sizing, argument checks)
behave as include/aceapex.h states.  No compute call is made."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_2606_04268_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "aceapex.h")).read()
    return sorted(set(re.findall(r"^\w[\w\s\*]*?\b(aceapex_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    names = declared_functions()
    assert set(names) == set(_abi.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_probe_reads_header():
    x = synth.markov(300_000, 3)
    s = oracle.encode(x, block_log2=16, flatten=1)
    info = _abi.probe(s)
    h = oracle.header_fields(s)
    assert info.decoded_bytes == len(x) == h["decoded_bytes"]
    assert info.comp_bytes == s.size
    for k in ("n_blocks", "max_level", "n_seq", "n_deep", "n_chunks", "flags", "block_log2",
              "min_match", "chunk_log2", "max_depth", "content_hash"):
        assert getattr(info, k) == h[k], k


def test_probe_rejects_bad_headers():
    s = oracle.encode(b"hello world hello world", block_log2=10)
    with pytest.raises(_abi.AceapexError) as e:
        _abi.probe(s[:10])
    assert e.value.code == _abi.E_INVAL
    for i, v in [(0, ord("B")), (4, 2), (7, 0x80), (6, 0x18), (11, 1), (32, 99)]:
        bad = s.copy()
        bad[i] = v
        with pytest.raises(_abi.AceapexError) as e:
            _abi.probe(bad)
        assert e.value.code == _abi.E_FORMAT, i
    # without the levels flag (the four streams of Sec. 3.2) the level fields must be zero
    deep = oracle.encode(synth.markov(20_000, 2), block_log2=10)
    assert _abi.probe(deep).max_level > 0
    bad = deep.copy()
    bad[6] &= 0xF7
    with pytest.raises(_abi.AceapexError) as e:
        _abi.probe(bad)
    assert e.value.code == _abi.E_FORMAT
    free = oracle.encode(synth.markov(20_000, 2), block_log2=10, levels=0)
    info = _abi.probe(free)
    assert info.flags & 8 == 0 and info.max_level == 0 and _abi.level_table(free, info) is None


def test_workspace_bytes_covers_every_match_record():
    x = synth.markov(1 << 20, 4)
    a = oracle.encode(x, block_log2=18)
    ia = _abi.probe(a)
    wa = _abi.workspace_bytes([_abi.Desc(_abi.Stream(0, ia, None), 0, ia.decoded_bytes, 0)])
    assert wa >= 12 * ia.n_seq + 64 * ia.n_chunks
    two = _abi.workspace_bytes([_abi.Desc(_abi.Stream(0, ia, None), 0, 0, 0)] * 2)
    assert 2 * wa - 4096 <= two <= 2 * wa + 4096


def test_host_argument_errors_need_no_gpu():
    s = oracle.encode(synth.markov(5000, 1), block_log2=12)
    info = _abi.probe(s)
    lib = _abi.load()
    st = _abi.Stream(0, info, None)
    # null compressed pointer
    assert lib.aceapex_decode(ctypes.byref(st), 4096, info.decoded_bytes, 4096, 1 << 20, None, None) == _abi.E_INVAL
    st = _abi.Stream(16, info, None)
    # output too small
    assert lib.aceapex_decode(ctypes.byref(st), 4096, info.decoded_bytes - 1, 4096, 1 << 20, None, None) == _abi.E_CAPACITY
    # misaligned output
    assert lib.aceapex_decode(ctypes.byref(st), 4097, info.decoded_bytes, 4096, 1 << 20, None, None) == _abi.E_INVAL
    # workspace too small / misaligned
    assert lib.aceapex_decode(ctypes.byref(st), 4096, info.decoded_bytes, 4096, 16, None, None) == _abi.E_WORKSPACE
    assert lib.aceapex_decode(ctypes.byref(st), 4096, info.decoded_bytes, 4100, 1 << 20, None, None) == _abi.E_WORKSPACE
    # outside the GPU limits: 2^21-byte blocks
    big = oracle.encode(synth.markov(5000, 1), block_log2=21)
    ib = _abi.probe(big)
    sb = _abi.Stream(16, ib, None)
    assert lib.aceapex_decode(ctypes.byref(sb), 4096, ib.decoded_bytes, 4096, 1 << 20, None, None) == _abi.E_UNSUPPORTED
    assert _abi.strerror(_abi.E_CORRUPT) == "corrupt stream"
    assert lib.aceapex_decode_many(None, 0, None, 0, None) == _abi.OK


def test_level_table_matches_tokens():
    x = synth.fastq(2 << 20, 8)
    s = oracle.encode(x, block_log2=17, flatten=1)
    info = _abi.probe(s)
    counts = list(_abi.level_table(s, info))
    import numpy as np

    assert counts == list(np.bincount(oracle.tokens(s)["lvl"], minlength=info.max_level + 1))
    with pytest.raises(_abi.AceapexError):
        _abi.level_table(s[:70], info)
    bad = s.copy()
    at = 64 + 16 * (info.n_blocks + 1)
    bad[at] ^= 1
    with pytest.raises(_abi.AceapexError):
        _abi.level_table(bad, info)


def test_plan_argument_errors_need_no_gpu():
    s = oracle.encode(synth.markov(5000, 1), block_log2=12)
    info = _abi.probe(s)
    levels = _abi.level_table(s, info)
    t = _abi.tuning_defaults()
    assert (t.level_wg_max, t.tail_level_max, t.long_copy, t.xcd_parts) == (512, 2048, 128, 8)
    lib = _abi.load()
    h = ctypes.c_void_p()
    with_table = _abi.Desc(_abi.Stream(16, info, levels), 4096, info.decoded_bytes, 0)
    without = _abi.Desc(_abi.Stream(16, info, None), 4096, info.decoded_bytes, 0)
    arr = (_abi.Desc * 1)(with_table)
    ws = _abi.workspace_bytes([with_table])
    assert lib.aceapex_plan_create(arr, 1, 4096, ws, None, None, None) == _abi.E_INVAL  # no plan pointer
    assert lib.aceapex_plan_create((_abi.Desc * 1)(without), 1, 4096, ws, None, None, ctypes.byref(h)) == _abi.E_INVAL
    assert lib.aceapex_plan_create(arr, 1, 4096, ws - 256, None, None, ctypes.byref(h)) == _abi.E_WORKSPACE
    for k, v in [("level_wg_max", 0), ("level_wg_max", 65536), ("long_copy", 8), ("xcd_parts", 0), ("xcd_parts", 9)]:
        bad = _abi.tuning_defaults()
        setattr(bad, k, v)
        assert lib.aceapex_plan_create(arr, 1, 4096, ws, ctypes.byref(bad), None, ctypes.byref(h)) == _abi.E_INVAL, k
    assert h.value is None
    assert lib.aceapex_plan_launch(None, None) == _abi.E_INVAL
    assert lib.aceapex_plan_launch_graph(None, None) == _abi.E_INVAL
    assert lib.aceapex_plan_set_tuning(None, ctypes.byref(t)) == _abi.E_INVAL
    assert lib.aceapex_plan_tune(None, None, 1, None) == _abi.E_INVAL
    lib.aceapex_plan_destroy(None)


def test_workspace_follows_level_validation(monkeypatch):
    """With ACEAPEX_VALIDATE_LEVELS set, a stream with levels needs room for
    the derive-mode check as well as its decode; "0" leaves it off."""
    x = synth.markov(1 << 20, 5)
    info = _abi.probe(oracle.encode(x, block_log2=16))
    desc = [_abi.Desc(_abi.Stream(0, info, None), 0, info.decoded_bytes, 0)]
    monkeypatch.delenv("ACEAPEX_VALIDATE_LEVELS", raising=False)
    plain = _abi.workspace_bytes(desc)
    monkeypatch.setenv("ACEAPEX_VALIDATE_LEVELS", "0")
    assert _abi.workspace_bytes(desc) == plain
    monkeypatch.setenv("ACEAPEX_VALIDATE_LEVELS", "1")
    checked = _abi.workspace_bytes(desc)
    assert checked == max(plain, _abi.workspace_bytes_derive(info)) and checked > plain


def test_workspace_holds_ordered_slot_counts(monkeypatch):
    """A stream of at most 64 levels has room for its (level, chunk) counts
    whatever ACEAPEX_ORDERED_SLOTS says (the setting is read at each decode);
    a deeper stream has none."""
    x = synth.wiki(8 << 20, 0xACE5)
    ws = {}
    for depth in (64, 65):
        info = _abi.probe(oracle.encode(x, block_log2=20, max_depth=depth))
        assert info.max_level == depth - 1
        desc = [_abi.Desc(_abi.Stream(0, info, None), 0, info.decoded_bytes, 0)]
        sizes = set()
        for v in (None, "0", "1"):
            if v is None:
                monkeypatch.delenv("ACEAPEX_ORDERED_SLOTS", raising=False)
            else:
                monkeypatch.setenv("ACEAPEX_ORDERED_SLOTS", v)
            sizes.add(_abi.workspace_bytes(desc))
        assert len(sizes) == 1
        ws[depth] = (sizes.pop(), info)
    (w64, i64), (w65, i65) = ws[64], ws[65]
    assert i64.n_chunks == i65.n_chunks and abs(i64.n_seq - i65.n_seq) < 100
    # the two layouts differ otherwise by a few KiB (level counters, alignment)
    assert 4 * 64 * i64.n_chunks - 8192 <= w64 - w65 <= 4 * 64 * i64.n_chunks + 8192


def test_compare_argument_errors_need_no_gpu():
    """aceapex_compare refuses a null or misaligned result pointer and null
    buffers before it touches the GPU."""
    lib = _abi.load()
    assert _abi.compare(0, 0, 16, 0, 0) == _abi.E_INVAL  # no result
    assert _abi.compare(0x1000, 0x2000, 16, 0x3004, 0) == _abi.E_INVAL  # result not 8-byte aligned
    assert _abi.compare(0, 0x2000, 16, 0x3000, 0) == _abi.E_INVAL  # null buffer with n > 0
    assert lib is not None
