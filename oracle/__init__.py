"""ORACLE -- test infrastructure only.

ctypes binding of ``aceapex_oracle.c`` (a plain CPU encoder, sequential and
block-parallel decoders, and an independent level/invariant checker for the
absolute-offset LZ77 codec of ACEAPEX, arXiv 2606.04268) plus ``refdec``, a
second decoder in pure Python for tiny streams.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU decoder
and never imports it.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ERRORS = {0: "ok", -1: "invalid argument", -2: "bad format", -3: "corrupt stream",
          -4: "output capacity too small", -9: "out of memory"}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {ERRORS.get(code, code)} ({code})")
        self.code = code


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, host only)."""
    import subprocess

    srcs = [os.path.join(_HERE, "aceapex_oracle.c"), os.path.join(_HERE, "tans_oracle.c")]
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared", "-o", tmp] + srcs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Opts(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "block_log2", "min_match", "flatten", "max_depth", "chain_depth", "hash_bits",
        "tiebreak", "chunk_log2", "levels")]


class Report(ctypes.Structure):
    _fields_ = [("n_seq", ctypes.c_uint64), ("n_lit_bytes", ctypes.c_uint64),
                ("match_bytes", ctypes.c_uint64), ("n_deep", ctypes.c_uint64),
                ("level_sum", ctypes.c_uint64), ("max_level", ctypes.c_uint32),
                ("n_blocks", ctypes.c_uint32), ("inblock_nonliteral_src_bytes", ctypes.c_uint64),
                ("level_mismatch", ctypes.c_uint64), ("depth_violations", ctypes.c_uint64)]


TOKEN_DTYPE = np.dtype([("dst", "<u4"), ("src", "<u4"), ("len", "<u4"), ("lvl", "<u4")])

_u8p = ctypes.POINTER(ctypes.c_uint8)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        lib.orc_encode.argtypes = [_u8p, ctypes.c_uint64, ctypes.POINTER(Opts), ctypes.POINTER(_u8p)]
        lib.orc_encode.restype = ctypes.c_int64
        lib.orc_free.argtypes = [ctypes.c_void_p]
        lib.orc_free.restype = None
        lib.orc_decode.argtypes = [_u8p, ctypes.c_uint64, _u8p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
        lib.orc_decode.restype = ctypes.c_int
        lib.orc_decode_mt.argtypes = [_u8p, ctypes.c_uint64, _u8p, ctypes.c_uint64, ctypes.c_int]
        lib.orc_decode_mt.restype = ctypes.c_int
        lib.orc_check.argtypes = [_u8p, ctypes.c_uint64, _u8p, ctypes.c_uint64, ctypes.POINTER(Report)]
        lib.orc_check.restype = ctypes.c_int
        lib.orc_tokens.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64]
        lib.orc_tokens.restype = ctypes.c_int64
        lib.orc_tans_counts.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint16)]
        lib.orc_tans_counts.restype = ctypes.c_int
        lib.orc_tans_encode.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(_u8p)]
        lib.orc_tans_encode.restype = ctypes.c_int64
        lib.orc_tans_decode.argtypes = [_u8p, ctypes.c_uint64, _u8p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)]
        lib.orc_tans_decode.restype = ctypes.c_int
        _lib = lib
    return _lib


def _buf(a) -> np.ndarray:
    if isinstance(a, np.ndarray):
        return np.ascontiguousarray(a, dtype=np.uint8)
    return np.frombuffer(bytes(a), dtype=np.uint8)


def _p(a: np.ndarray):
    return a.ctypes.data_as(_u8p)


DEFAULTS = dict(block_log2=20, min_match=4, flatten=0, max_depth=0, chain_depth=32,
                hash_bits=22, tiebreak=0, chunk_log2=10, levels=1)


def header_fields(stream) -> dict:
    s = _buf(stream)
    h = s[:64].tobytes()
    le = lambda a, b: int.from_bytes(h[a:b], "little")
    return dict(magic=h[:4], version=le(4, 6), flags=le(6, 8), block_log2=h[8], min_match=h[9],
                chunk_log2=h[10], max_depth=le(12, 16), decoded_bytes=le(16, 24),
                comp_bytes=le(24, 32), n_blocks=le(32, 36), max_level=le(36, 40),
                n_seq=le(40, 44), n_deep=le(44, 48), n_chunks=le(48, 52),
                content_hash=le(56, 64))


def content_hash(x) -> int:
    """XXH3-64 of the decoded bytes (Sec. 4.3 verification), via the xxhash package."""
    import xxhash

    return xxhash.xxh3_64_intdigest(memoryview(_buf(x)))


def encode(x, *, with_hash: bool = True, **opts) -> np.ndarray:
    """Encode raw bytes; returns the stream as a uint8 array."""
    o = dict(DEFAULTS)
    unknown = set(opts) - set(o)
    if unknown:
        raise TypeError(f"unknown encoder options {unknown}")
    o.update(opts)
    xa = _buf(x)
    out = _u8p()
    n = _load().orc_encode(_p(xa), xa.size, ctypes.byref(Opts(**o)), ctypes.byref(out))
    if n < 0:
        raise OracleError(int(n), "encode")
    s = np.ctypeslib.as_array(out, shape=(n,)).copy()
    _load().orc_free(out)
    if with_hash and xa.size:
        s[56:64] = np.frombuffer(content_hash(xa).to_bytes(8, "little"), dtype=np.uint8)
    return s


def decode(stream) -> np.ndarray:
    """Sequential decode (the definition of the decoded result)."""
    s = _buf(stream)
    n = header_fields(s)["decoded_bytes"] if s.size >= 64 else 0
    out = np.empty(max(n, 1), dtype=np.uint8)
    got = ctypes.c_uint64(0)
    rc = _load().orc_decode(_p(s), s.size, _p(out), n, ctypes.byref(got))
    if rc:
        raise OracleError(rc, "decode")
    return out[:n]


def decode_mt(stream, threads: int) -> np.ndarray:
    """Block-parallel CPU decode with per-block progress counters."""
    s = _buf(stream)
    n = header_fields(s)["decoded_bytes"]
    out = np.empty(max(n, 1), dtype=np.uint8)
    rc = _load().orc_decode_mt(_p(s), s.size, _p(out), n, threads)
    if rc:
        raise OracleError(rc, "decode_mt")
    return out[:n]


def decode_into(stream: np.ndarray, out: np.ndarray, threads: int = 1) -> None:
    """Decode into a preallocated buffer (for timing without allocation)."""
    lib = _load()
    if threads <= 1:
        got = ctypes.c_uint64(0)
        rc = lib.orc_decode(_p(stream), stream.size, _p(out), out.size, ctypes.byref(got))
    else:
        rc = lib.orc_decode_mt(_p(stream), stream.size, _p(out), out.size, threads)
    if rc:
        raise OracleError(rc, "decode")


@dataclass
class CheckReport:
    n_seq: int
    n_lit_bytes: int
    match_bytes: int
    n_deep: int
    max_level: int
    avg_level: float
    n_blocks: int
    inblock_nonliteral_src_bytes: int
    level_mismatch: int
    depth_violations: int


def check(x, stream) -> CheckReport:
    """Decode + compare with x + recompute every level from the writer map."""
    xa, s = _buf(x), _buf(stream)
    r = Report()
    rc = _load().orc_check(_p(xa), xa.size, _p(s), s.size, ctypes.byref(r))
    if rc:
        raise OracleError(rc, "check")
    return CheckReport(r.n_seq, r.n_lit_bytes, r.match_bytes, r.n_deep, r.max_level,
                       (r.level_sum / r.n_seq) if r.n_seq else 0.0, r.n_blocks,
                       r.inblock_nonliteral_src_bytes, r.level_mismatch, r.depth_violations)


def tokens(stream) -> np.ndarray:
    """Every match as (dst, src, len, lvl) in stream order."""
    s = _buf(stream)
    cnt = header_fields(s)["n_seq"]
    out = np.zeros(cnt, dtype=TOKEN_DTYPE)
    n = _load().orc_tokens(_p(s), s.size, out.ctypes.data, cnt)
    if n < 0:
        raise OracleError(int(n), "tokens")
    return out[:n]


from .refdec import refdec  # noqa: E402  (pure-Python second decoder)


# ------------------------------------------------------------ tANS (literals)

def tans_counts(x, table_log: int = 11) -> np.ndarray:
    """Normalized counts (256 x u16, summing to 2^table_log) of the bytes x."""
    xa = _buf(x)
    c = (ctypes.c_uint16 * 256)()
    rc = _load().orc_tans_counts(_p(xa), xa.size, table_log, c)
    if rc:
        raise OracleError(rc, "tans_counts")
    return np.array(c[:], dtype=np.uint16)


def tans_encode(x, table_log: int = 11, lanes: int = 1024) -> np.ndarray:
    """tANS-code the bytes x into an ACT1 container (tans_oracle.c)."""
    xa = _buf(x)
    out = _u8p()
    n = _load().orc_tans_encode(_p(xa), xa.size, table_log, lanes, ctypes.byref(out))
    if n < 0:
        raise OracleError(int(n), "tans_encode")
    s = np.ctypeslib.as_array(out, shape=(n,)).copy()
    _load().orc_free(out)
    return s


def tans_decode(container) -> np.ndarray:
    """Decode an ACT1 container."""
    c = _buf(container)
    n = int(c[4:8].view(np.uint32)[0]) if c.size >= 8 else 0
    out = np.empty(max(n, 1), dtype=np.uint8)
    got = ctypes.c_uint64(0)
    rc = _load().orc_tans_decode(_p(c), c.size, _p(out), out.size, ctypes.byref(got))
    if rc:
        raise OracleError(rc, "tans_decode")
    return out[:got.value]
