"""ctypes binding of the C ABI in include/aceapex.h (argument marshalling only).

The shared library ``libaceapex.so`` is built in-tree by
``__graft_entry__.build()``.  Loading it never falls back to anything else:
if the library is missing, or no GPU is present when a decode is requested,
the call raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaceapex.so")

OK = 0
E_INVAL, E_FORMAT, E_CORRUPT, E_CAPACITY = -1, -2, -3, -4
E_WORKSPACE, E_UNSUPPORTED, E_TIMEOUT, E_HIP = -5, -6, -7, -8


class Info(ctypes.Structure):
    """aceapex_info."""
    _fields_ = [("decoded_bytes", ctypes.c_uint64), ("comp_bytes", ctypes.c_uint64),
                ("n_blocks", ctypes.c_uint32), ("block_log2", ctypes.c_uint32),
                ("min_match", ctypes.c_uint32), ("chunk_log2", ctypes.c_uint32),
                ("max_depth", ctypes.c_uint32), ("max_level", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("n_seq", ctypes.c_uint32),
                ("n_deep", ctypes.c_uint32), ("n_chunks", ctypes.c_uint32),
                ("content_hash", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stream(ctypes.Structure):
    """aceapex_stream."""
    _fields_ = [("d_comp", ctypes.c_void_p), ("info", Info)]


class Desc(ctypes.Structure):
    """aceapex_desc."""
    _fields_ = [("s", Stream), ("d_out", ctypes.c_void_p), ("out_capacity", ctypes.c_uint64),
                ("d_status", ctypes.c_void_p)]


class AceapexError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = strerror(code) if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")
        self.code = code


EXPORTS = ("aceapex_probe", "aceapex_workspace_bytes", "aceapex_decode", "aceapex_decode_many",
           "aceapex_strerror", "aceapex_last_hip_error")

_lib = None


def load():
    """Load libaceapex.so (after torch, so that one HIP runtime serves both)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    try:
        import torch  # noqa: F401  (its HIP runtime must be the one the library binds to)
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.aceapex_probe.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(Info)]
    lib.aceapex_probe.restype = ctypes.c_int
    lib.aceapex_workspace_bytes.argtypes = [ctypes.POINTER(Desc), ctypes.c_uint32]
    lib.aceapex_workspace_bytes.restype = ctypes.c_size_t
    lib.aceapex_decode.argtypes = [ctypes.POINTER(Stream), vp, ctypes.c_uint64, vp, ctypes.c_size_t, vp, vp]
    lib.aceapex_decode.restype = ctypes.c_int
    lib.aceapex_decode_many.argtypes = [ctypes.POINTER(Desc), ctypes.c_uint32, vp, ctypes.c_size_t, vp]
    lib.aceapex_decode_many.restype = ctypes.c_int
    lib.aceapex_strerror.argtypes = [ctypes.c_int]
    lib.aceapex_strerror.restype = ctypes.c_char_p
    lib.aceapex_last_hip_error.argtypes = []
    lib.aceapex_last_hip_error.restype = ctypes.c_int
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().aceapex_strerror(code).decode()


def probe(prefix) -> Info:
    """aceapex_probe on a host buffer (bytes, bytearray or uint8 numpy array)."""
    import numpy as np

    buf = np.ascontiguousarray(np.frombuffer(bytes(prefix[:64]), dtype=np.uint8))
    info = Info()
    rc = load().aceapex_probe(buf.ctypes.data, buf.size, ctypes.byref(info))
    if rc:
        raise AceapexError(rc, "probe")
    return info


def workspace_bytes(descs) -> int:
    arr = (Desc * len(descs))(*descs)
    return int(load().aceapex_workspace_bytes(arr, len(descs)))


def decode(stream: Stream, d_out: int, out_capacity: int, d_ws: int, ws_bytes: int,
           d_status: int, hip_stream: int) -> int:
    return load().aceapex_decode(ctypes.byref(stream), d_out, out_capacity, d_ws, ws_bytes,
                                 d_status, hip_stream)


def decode_many(descs, d_ws: int, ws_bytes: int, hip_stream: int) -> int:
    arr = (Desc * len(descs))(*descs)
    return load().aceapex_decode_many(arr, len(descs), d_ws, ws_bytes, hip_stream)
