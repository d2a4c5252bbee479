"""ORACLE -- test infrastructure only.

A second, independent decoder in pure Python for tiny streams.  It reads the
stream layout directly and executes the sequences in order (Sec. 3.2: literal
run, then a copy from an absolute position of the decoded output, Sec. 3.1).
It deliberately ignores the chunk index and the levels, and checks only what
it needs to execute; the C oracle is the strict validator.
"""
from __future__ import annotations


def _u(b: bytes, a: int, n: int) -> int:
    return int.from_bytes(b[a:a + n], "little")


def _varints(b: bytes, start: int, count: int):
    vals, i = [], start
    for _ in range(count):
        v, shift = 0, 0
        while True:
            c = b[i]
            i += 1
            v |= (c & 0x7F) << shift
            shift += 7
            if c < 0x80:
                break
        vals.append(v)
    return vals


def _pad(v: int) -> int:
    return (v + 15) // 16 * 16


def refdec(stream) -> bytes:
    s = bytes(stream)
    assert s[:4] == b"ACX1", "bad magic"
    block_log2, min_match = s[8], s[9]
    n = _u(s, 16, 8)
    n_blocks = _u(s, 32, 4)
    out = bytearray(n)
    for b in range(n_blocks):
        base = _u(s, 64 + 16 * b, 8)
        n_seq, n_lit, n_chunks = _u(s, base, 4), _u(s, base + 4, 4), _u(s, base + 8, 4)
        cmd_bytes, len_bytes = _u(s, base + 16, 4), _u(s, base + 20, 4)
        lvl_bytes = _u(s, base + 24, 4)
        q = base + 32 + 32 * n_chunks
        off_at = q
        q += _pad(4 * n_seq)
        cmd_at = q
        q += _pad(cmd_bytes)
        len_at = q
        q += _pad(len_bytes)
        q += _pad(lvl_bytes)
        lit_at = q
        runs = _varints(s, cmd_at, n_seq + 1)
        lens = _varints(s, len_at, n_seq)
        p = b << block_log2
        li = 0
        for i in range(n_seq + 1):
            r = runs[i]
            out[p:p + r] = s[lit_at + li:lit_at + li + r]
            p += r
            li += r
            if i == n_seq:
                break
            m = lens[i] + min_match
            src = _u(s, off_at + 4 * i, 4)
            assert src + m <= p, "source overlaps destination"
            for k in range(m):
                out[p + k] = out[src + k]
            p += m
        assert p == min(n, (b + 1) << block_log2), "block does not tile its range"
        assert li == n_lit
    return bytes(out)
