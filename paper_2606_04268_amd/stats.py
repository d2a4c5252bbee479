"""Host-side statistics of a stream, for measurement and reports.

Reads the stream layout of include/aceapex.h with numpy: section sizes, match
and literal byte counts, and the number and bytes of the matches at every
dependency level (Sec. 7.1).  Decodes nothing.
"""
from __future__ import annotations

import numpy as np

from . import _abi


def leb128(b: np.ndarray) -> np.ndarray:
    """Vectorised LEB128 decode of a byte run that holds whole values."""
    if b.size == 0:
        return np.zeros(0, dtype=np.uint64)
    term = b < 0x80
    ends = np.nonzero(term)[0]
    starts = np.concatenate(([0], ends[:-1] + 1))
    pos = np.arange(b.size) - np.repeat(starts, ends - starts + 1)
    parts = (b.astype(np.uint64) & np.uint64(0x7F)) << (np.uint64(7) * pos.astype(np.uint64))
    return np.add.reduceat(parts, starts)


def _pad(v: int) -> int:
    return (v + 15) // 16 * 16


def literals(stream) -> np.ndarray:
    """The lit[] sections of every block, concatenated in stream order: the
    literal bytes in output order (Sec. 3.2)."""
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    info = _abi.probe(s)
    nb = info.n_blocks
    offs = s[64:64 + 16 * (nb + 1)].view(np.uint64).reshape(-1, 2)[:, 0].astype(np.int64)
    parts = []
    for b in range(nb):
        o = int(offs[b])
        ns, nl, nc, _, cb, lb, vb, _ = (int(v) for v in s[o:o + 32].view(np.uint32))
        at = o + 32 + 32 * nc + _pad(4 * ns) + _pad(cb) + _pad(lb) + _pad(vb)
        parts.append(s[at:at + nl])
    return np.concatenate(parts) if parts else np.zeros(0, np.uint8)


def stream_stats(stream) -> dict:
    s = np.ascontiguousarray(stream, dtype=np.uint8)
    info = _abi.probe(s)
    nb = info.n_blocks
    table = s[64:64 + 16 * (nb + 1)].view(np.uint64).reshape(-1, 2)
    offs = table[:, 0].astype(np.int64)
    table_bytes = _pad(4 * (info.max_level + 1)) if info.flags & 8 else 0  # level table, when levels are stored
    sec = dict(header=64 + 16 * (nb + 1) + table_bytes, block_headers=0, chunk_index=0, off=0, cmd=0, len=0, lvl=0,
               lit=0, padding=0)
    lens, lvls = [], []
    lit_bytes = 0
    for b in range(nb):
        o = int(offs[b])
        hdr = s[o:o + 32].view(np.uint32)
        ns, nl, nc, _, cb, lb, vb, _ = (int(v) for v in hdr)
        q = o + 32 + 32 * nc
        off_at = q
        q += _pad(4 * ns)
        cmd_at = q
        q += _pad(cb)
        len_at = q
        q += _pad(lb)
        lvl_at = q
        q += _pad(vb)
        sec["block_headers"] += 32
        sec["chunk_index"] += 32 * nc
        sec["off"] += 4 * ns
        sec["cmd"] += cb
        sec["len"] += lb
        sec["lvl"] += vb
        sec["lit"] += nl
        sec["padding"] += (_pad(4 * ns) - 4 * ns) + (_pad(cb) - cb) + (_pad(lb) - lb) + (_pad(vb) - vb) + (_pad(nl) - nl)
        lit_bytes += nl
        lens.append(leb128(s[len_at:len_at + lb]) + np.uint64(info.min_match))
        lvls.append(leb128(s[lvl_at:lvl_at + vb]))
        del off_at, cmd_at
    ln = np.concatenate(lens) if lens else np.zeros(0, np.uint64)
    lv = np.concatenate(lvls) if lvls else np.zeros(0, np.uint64)
    counts = np.bincount(lv.astype(np.int64), minlength=info.max_level + 1) if lv.size else np.zeros(1, np.int64)
    mbytes = (np.bincount(lv.astype(np.int64), weights=ln.astype(np.float64), minlength=info.max_level + 1)
              if lv.size else np.zeros(1))
    M = int(ln.sum())
    N = int(info.decoded_bytes)
    C = int(info.comp_bytes)
    return dict(
        decoded_bytes=N, comp_bytes=C, n_blocks=nb, n_seq=int(info.n_seq), n_deep=int(info.n_deep),
        n_chunks=int(info.n_chunks), max_level=int(info.max_level), match_bytes=M, literal_bytes=lit_bytes,
        level_counts=[int(v) for v in counts], level_bytes=[int(v) for v in mbytes],
        avg_level=float((lv.astype(np.float64)).mean()) if lv.size else 0.0, sections=sec,
        algorithmic_bytes=C + N + M,
    )
