"""Test helper: build streams directly from token lists (no encoder involved).

A third, independent writer of the stream layout, used to craft inputs that
no encoder would emit: random valid token streams for property tests, deep
dependency chains, and corrupted streams for the error paths.  Tokens are
given per block as (literal_run, match_len, src) sequences plus a trailing
literal run; levels are computed here from the definition (Sec. 7.1) unless
given explicitly.
"""
from __future__ import annotations

import numpy as np


def _varint(v: int, width: int = 0) -> bytes:
    """LEB128 of v in at least `width` bytes (zero groups with the continuation
    bit pad a short value: a valid, non-minimal encoding)."""
    out = bytearray()
    while True:
        c = v & 0x7F
        v >>= 7
        more = bool(v) or len(out) + 1 < width
        out.append(c | (0x80 if more else 0))
        if not more:
            return bytes(out)


def _pad(b: bytes) -> bytes:
    return b + b"\0" * ((-len(b)) % 16)


def execute(blocks, lits: bytes, n: int, block_log2: int):
    """Run the sequences in order; returns (decoded bytes, per-match levels)."""
    out = bytearray(n)
    wl = [-1] * n
    levels = []
    li = 0
    for b, (seqs, trail) in enumerate(blocks):
        p = b << block_log2
        for r, m, s in seqs:
            out[p:p + r] = lits[li:li + r]
            li += r
            p += r
            assert s + m <= p
            lv = 1 + max((wl[s + k] for k in range(m)), default=-1)
            for k in range(m):
                out[p + k] = out[s + k]
                wl[p + k] = lv
            levels.append(lv)
            p += m
        out[p:p + trail] = lits[li:li + trail]
        li += trail
        p += trail
        assert p == min(n, (b + 1) << block_log2)
    return bytes(out), levels


def random_tokens(rng: np.random.Generator, n: int, block_log2: int, min_match: int = 4,
                  p_match: float = 0.5, max_len: int = 40, max_run: int = 12):
    """Random valid token lists covering n bytes; sources anywhere before dst."""
    B = 1 << block_log2
    blocks = []
    nlit = 0
    for b in range((n + B - 1) // B):
        p, end = b * B, min(n, (b + 1) * B)
        seqs = []
        run = 0
        while p < end:
            room = end - p
            if p >= min_match and rng.random() < p_match and room >= min_match:
                m = int(rng.integers(min_match, min(max_len, room, p) + 1)) if min(max_len, room, p) >= min_match else 0
                if m:
                    s = int(rng.integers(0, p - m + 1))
                    seqs.append((run, m, s))
                    nlit += run
                    run = 0
                    p += m
                    continue
            r = int(rng.integers(1, min(max_run, room) + 1))
            run += r
            p += r
        blocks.append((seqs, run))
        nlit += run
    lits = rng.integers(0, 256, size=nlit, dtype=np.uint8).tobytes()
    return blocks, lits


def build(blocks, lits: bytes, n: int, *, block_log2: int, min_match: int = 4,
          chunk_log2: int = 10, levels=None, flags: int = 8, max_depth: int = 0,
          max_level=None, n_deep=None, level_counts=None, varint_width=None,
          with_levels: bool = True) -> np.ndarray:
    """Serialize token lists into the stream layout (levels from the definition by default).

    varint_width: None for minimal LEB128; an int w to pad every value to at
    least w bytes; a numpy Generator to draw each value's width from 1..4.
    with_levels=False writes the four streams of Sec. 3.2 only: no lvl[]
    sections, no level table, the levels flag clear and the header's level
    fields zero.
    """
    def vw():
        if varint_width is None:
            return 0
        if isinstance(varint_width, int):
            return varint_width
        return int(varint_width.integers(1, 5))

    decoded, exact = execute(blocks, lits, n, block_log2)
    if levels is None:
        levels = exact
    K = 1 << chunk_log2
    nb = len(blocks)
    assert nb == (n + (1 << block_log2) - 1) >> block_log2
    payloads, seq_base, chunk_base = [], [], []
    tot_seq = tot_chunks = 0
    li = mi = 0
    gmax = 0
    deep = 0
    for b, (seqs, trail) in enumerate(blocks):
        cmd, ln, lv, off, lit = bytearray(), bytearray(), bytearray(), bytearray(), bytearray()
        chunks = []
        p = 0
        bmax = 0
        for i, (r, m, s) in enumerate(seqs):
            if i % K == 0:
                chunks.append((len(cmd), len(ln), len(lv), len(lit), p))
            cmd += _varint(r, vw())
            lit += lits[li:li + r]
            li += r
            p += r
            ln += _varint(m - min_match, vw())
            off += int(s).to_bytes(4, "little")
            if with_levels:
                lv += _varint(levels[mi], vw())
                bmax = max(bmax, levels[mi])
                deep += levels[mi] > 0
            mi += 1
            p += m
        if not seqs:
            chunks.append((0, 0, 0, 0, 0))
        cmd += _varint(trail, vw())
        lit += lits[li:li + trail]
        li += trail
        gmax = max(gmax, bmax)
        hdr = b"".join(int(v).to_bytes(4, "little") for v in (
            len(seqs), len(lit), len(chunks), bmax, len(cmd), len(ln), len(lv), 0))
        idx = b"".join(b"".join(int(v).to_bytes(4, "little") for v in c) + b"\0" * 12 for c in chunks)
        payloads.append(hdr + idx + _pad(bytes(off)) + _pad(bytes(cmd)) + _pad(bytes(ln)) +
                        _pad(bytes(lv)) + _pad(bytes(lit)))
        seq_base.append(tot_seq)
        chunk_base.append(tot_chunks)
        tot_seq += len(seqs)
        tot_chunks += len(chunks)
    table_len = 16 * (nb + 1)
    mlev = gmax if max_level is None else max_level
    hist = [0] * (mlev + 1)
    for lv in levels:
        if lv <= mlev:
            hist[lv] += 1
    if level_counts is not None:
        hist = list(level_counts)
    hist_bytes = _pad(b"".join(int(v).to_bytes(4, "little") for v in hist)) if with_levels else b""
    if not with_levels:
        flags &= ~8
        gmax = 0
    pos = 64 + table_len + len(hist_bytes)
    offsets = []
    for pl in payloads:
        offsets.append(pos)
        pos += len(pl)
    comp = pos
    table = b"".join(int(o).to_bytes(8, "little") + int(sb).to_bytes(4, "little") + int(cb).to_bytes(4, "little")
                     for o, sb, cb in zip(offsets + [comp], seq_base + [tot_seq], chunk_base + [tot_chunks]))
    hdr = bytearray(64)
    hdr[0:4] = b"ACX1"
    hdr[4:6] = (1).to_bytes(2, "little")
    hdr[6:8] = flags.to_bytes(2, "little")
    hdr[8] = block_log2
    hdr[9] = min_match
    hdr[10] = chunk_log2
    hdr[12:16] = max_depth.to_bytes(4, "little")
    hdr[16:24] = n.to_bytes(8, "little")
    hdr[24:32] = comp.to_bytes(8, "little")
    hdr[32:36] = nb.to_bytes(4, "little")
    hdr[36:40] = (gmax if max_level is None or not with_levels else max_level).to_bytes(4, "little")
    hdr[40:44] = tot_seq.to_bytes(4, "little")
    hdr[44:48] = (deep if n_deep is None else n_deep).to_bytes(4, "little")
    hdr[48:52] = tot_chunks.to_bytes(4, "little")
    s = bytes(hdr) + table + hist_bytes + b"".join(payloads)
    assert len(s) == comp
    return np.frombuffer(s, dtype=np.uint8).copy(), decoded
