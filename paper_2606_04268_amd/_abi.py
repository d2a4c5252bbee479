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
E_WORKSPACE, E_UNSUPPORTED, E_TIMEOUT, E_HIP, E_NOMEM = -5, -6, -7, -8, -9


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
    _fields_ = [("d_comp", ctypes.c_void_p), ("info", Info), ("h_levels", ctypes.POINTER(ctypes.c_uint32))]


class Desc(ctypes.Structure):
    """aceapex_desc."""
    _fields_ = [("s", Stream), ("d_out", ctypes.c_void_p), ("out_capacity", ctypes.c_uint64),
                ("d_status", ctypes.c_void_p)]


class EncOpts(ctypes.Structure):
    """aceapex_enc_opts."""
    _fields_ = [(n, ctypes.c_uint32) for n in (
        "block_log2", "min_match", "flatten", "max_depth", "chain_depth", "hash_bits",
        "tiebreak", "chunk_log2", "threads", "verbose", "levels")]


class Tuning(ctypes.Structure):
    """aceapex_tuning."""
    _fields_ = [(n, ctypes.c_uint32) for n in ("level_wg_max", "tail_level_max", "long_copy", "xcd_parts")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TansInfo(ctypes.Structure):
    """aceapex_tans_info."""
    _fields_ = [("n", ctypes.c_uint64), ("container_bytes", ctypes.c_uint64), ("table_log", ctypes.c_uint32),
                ("lanes", ctypes.c_uint32), ("bitstream_bytes", ctypes.c_uint32)]


class AceapexError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = strerror(code) if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")
        self.code = code


EXPORTS = ("aceapex_probe", "aceapex_level_table", "aceapex_workspace_bytes", "aceapex_decode", "aceapex_decode_many",
           "aceapex_decode_noalloc", "aceapex_decode_host", "aceapex_decode_derive", "aceapex_workspace_bytes_derive",
           "aceapex_tans_probe", "aceapex_tans_workspace_bytes", "aceapex_tans_decode", "aceapex_tans_encode",
           "aceapex_compare",
           "aceapex_strerror", "aceapex_last_hip_error", "aceapex_enc_defaults", "aceapex_encode",
           "aceapex_free", "aceapex_timing", "aceapex_timing_read", "aceapex_tuning_defaults",
           "aceapex_plan_create", "aceapex_plan_launch", "aceapex_plan_launch_graph", "aceapex_plan_set_tuning",
           "aceapex_plan_get_tuning", "aceapex_plan_tune", "aceapex_plan_destroy")

PHASES = ("setup", "parse", "levels")

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
    lib.aceapex_level_table.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32]
    lib.aceapex_level_table.restype = ctypes.c_int
    lib.aceapex_workspace_bytes.argtypes = [ctypes.POINTER(Desc), ctypes.c_uint32]
    lib.aceapex_workspace_bytes.restype = ctypes.c_size_t
    lib.aceapex_decode.argtypes = [ctypes.POINTER(Stream), vp, ctypes.c_uint64, vp, ctypes.c_size_t, vp, vp]
    lib.aceapex_decode.restype = ctypes.c_int
    lib.aceapex_decode_noalloc.argtypes = [ctypes.POINTER(Stream), vp, ctypes.c_uint64, vp, vp]
    lib.aceapex_decode_noalloc.restype = ctypes.c_int
    lib.aceapex_decode_derive.argtypes = [ctypes.POINTER(Stream), vp, ctypes.c_uint64, vp, ctypes.c_size_t, vp, vp, vp]
    lib.aceapex_decode_derive.restype = ctypes.c_int
    lib.aceapex_workspace_bytes_derive.argtypes = [ctypes.POINTER(Info)]
    lib.aceapex_workspace_bytes_derive.restype = ctypes.c_size_t
    lib.aceapex_tans_probe.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(TansInfo)]
    lib.aceapex_tans_probe.restype = ctypes.c_int
    lib.aceapex_tans_workspace_bytes.argtypes = [ctypes.POINTER(TansInfo)]
    lib.aceapex_tans_workspace_bytes.restype = ctypes.c_size_t
    lib.aceapex_compare.argtypes = [vp, vp, ctypes.c_uint64, vp, vp]
    lib.aceapex_compare.restype = ctypes.c_int
    lib.aceapex_tans_decode.argtypes = [vp, ctypes.POINTER(TansInfo), vp, ctypes.c_uint64, vp, ctypes.c_size_t, vp, vp]
    lib.aceapex_tans_decode.restype = ctypes.c_int
    lib.aceapex_tans_encode.argtypes = [vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(vp)]
    lib.aceapex_tans_encode.restype = ctypes.c_int64
    lib.aceapex_decode_host.argtypes = [vp, ctypes.c_size_t, vp, ctypes.c_uint64, ctypes.c_uint32]
    lib.aceapex_decode_host.restype = ctypes.c_int
    lib.aceapex_decode_many.argtypes = [ctypes.POINTER(Desc), ctypes.c_uint32, vp, ctypes.c_size_t, vp]
    lib.aceapex_decode_many.restype = ctypes.c_int
    lib.aceapex_strerror.argtypes = [ctypes.c_int]
    lib.aceapex_strerror.restype = ctypes.c_char_p
    lib.aceapex_last_hip_error.argtypes = []
    lib.aceapex_last_hip_error.restype = ctypes.c_int
    lib.aceapex_enc_defaults.argtypes = [ctypes.POINTER(EncOpts)]
    lib.aceapex_enc_defaults.restype = None
    lib.aceapex_encode.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(EncOpts), ctypes.POINTER(vp)]
    lib.aceapex_encode.restype = ctypes.c_int64
    lib.aceapex_free.argtypes = [vp]
    lib.aceapex_free.restype = None
    lib.aceapex_timing.argtypes = [ctypes.c_int]
    lib.aceapex_timing.restype = ctypes.c_int
    lib.aceapex_timing_read.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_uint32),
                                        ctypes.c_uint32]
    lib.aceapex_timing_read.restype = ctypes.c_int
    lib.aceapex_tuning_defaults.argtypes = [ctypes.POINTER(Tuning)]
    lib.aceapex_tuning_defaults.restype = None
    lib.aceapex_plan_create.argtypes = [ctypes.POINTER(Desc), ctypes.c_uint32, vp, ctypes.c_size_t,
                                        ctypes.POINTER(Tuning), vp, ctypes.POINTER(vp)]
    lib.aceapex_plan_create.restype = ctypes.c_int
    for name in ("aceapex_plan_launch", "aceapex_plan_launch_graph"):
        getattr(lib, name).argtypes = [vp, vp]
        getattr(lib, name).restype = ctypes.c_int
    lib.aceapex_plan_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    lib.aceapex_plan_set_tuning.restype = ctypes.c_int
    lib.aceapex_plan_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    lib.aceapex_plan_get_tuning.restype = ctypes.c_int
    lib.aceapex_plan_tune.argtypes = [vp, vp, ctypes.c_uint32, ctypes.POINTER(Tuning)]
    lib.aceapex_plan_tune.restype = ctypes.c_int
    lib.aceapex_plan_destroy.argtypes = [vp]
    lib.aceapex_plan_destroy.restype = None
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


def level_table(stream, info: Info):
    """aceapex_level_table on a host stream: a ctypes uint32 array of max_level + 1
    counts, or None for a stream without levels (the four streams of Sec. 3.2)."""
    import numpy as np

    if not info.flags & 8:
        return None
    buf = np.ascontiguousarray(stream, dtype=np.uint8)
    n = info.max_level + 1
    counts = (ctypes.c_uint32 * n)()
    rc = load().aceapex_level_table(buf.ctypes.data, buf.size, counts, n)
    if rc:
        raise AceapexError(rc, "level_table")
    return counts


def workspace_bytes(descs) -> int:
    arr = (Desc * len(descs))(*descs)
    return int(load().aceapex_workspace_bytes(arr, len(descs)))


def decode(stream: Stream, d_out: int, out_capacity: int, d_ws: int, ws_bytes: int,
           d_status: int, hip_stream: int) -> int:
    return load().aceapex_decode(ctypes.byref(stream), d_out, out_capacity, d_ws, ws_bytes,
                                 d_status, hip_stream)


def decode_noalloc(stream: Stream, d_out: int, out_capacity: int, d_status: int, hip_stream: int) -> int:
    return load().aceapex_decode_noalloc(ctypes.byref(stream), d_out, out_capacity, d_status, hip_stream)


NOALLOC_WORKSPACE_MAX = 64 << 20  # ACEAPEX_NOALLOC_WORKSPACE_MAX


def decode_derive(stream: Stream, d_out: int, out_capacity: int, d_ws: int, ws_bytes: int, d_levels,
                  d_status: int, hip_stream: int) -> int:
    return load().aceapex_decode_derive(ctypes.byref(stream), d_out, out_capacity, d_ws, ws_bytes, d_levels,
                                        d_status, hip_stream)


def workspace_bytes_derive(info: Info) -> int:
    return int(load().aceapex_workspace_bytes_derive(ctypes.byref(info)))


def decode_host(stream, out, threads: int = 0) -> int:
    """aceapex_decode_host on host numpy buffers (stream: uint8, out: uint8 writable)."""
    return load().aceapex_decode_host(stream.ctypes.data, stream.size, out.ctypes.data if out.size else None,
                                      out.size, threads)


def decode_many(descs, d_ws: int, ws_bytes: int, hip_stream: int) -> int:
    arr = (Desc * len(descs))(*descs)
    return load().aceapex_decode_many(arr, len(descs), d_ws, ws_bytes, hip_stream)


def enc_defaults() -> EncOpts:
    o = EncOpts()
    load().aceapex_enc_defaults(ctypes.byref(o))
    return o


def encode(data, opts: EncOpts):
    """aceapex_encode on a host buffer; returns the stream as a uint8 numpy array."""
    import numpy as np

    x = np.ascontiguousarray(np.frombuffer(bytes(data), np.uint8) if not isinstance(data, np.ndarray)
                             else data, dtype=np.uint8)
    out = ctypes.c_void_p()
    n = load().aceapex_encode(x.ctypes.data if x.size else None, x.size, ctypes.byref(opts), ctypes.byref(out))
    if n < 0:
        raise AceapexError(int(n), "encode")
    try:
        s = np.ctypeslib.as_array(ctypes.cast(out, ctypes.POINTER(ctypes.c_uint8)), shape=(n,)).copy()
    finally:
        load().aceapex_free(out)
    return s


def timing(enable: bool) -> None:
    load().aceapex_timing(1 if enable else 0)


def timing_read():
    """{group name: (total ms, launches)} of the decodes recorded since timing(True)."""
    n = len(PHASES)
    ms = (ctypes.c_float * n)()
    cnt = (ctypes.c_uint32 * n)()
    rc = load().aceapex_timing_read(ms, cnt, n)
    if rc:
        raise AceapexError(rc, "timing_read")
    return {PHASES[i]: (float(ms[i]), int(cnt[i])) for i in range(n)}


def tuning_defaults() -> Tuning:
    t = Tuning()
    load().aceapex_tuning_defaults(ctypes.byref(t))
    return t


def plan_create(descs, d_ws: int, ws_bytes: int, tuning, hip_stream: int) -> int:
    """aceapex_plan_create; returns the plan handle (an integer)."""
    arr = (Desc * len(descs))(*descs)
    h = ctypes.c_void_p()
    rc = load().aceapex_plan_create(arr, len(descs), d_ws, ws_bytes,
                                    ctypes.byref(tuning) if tuning is not None else None, hip_stream,
                                    ctypes.byref(h))
    if rc:
        raise AceapexError(rc, "plan_create")
    return h.value


def plan_launch(plan: int, hip_stream: int, graph: bool = False) -> int:
    f = load().aceapex_plan_launch_graph if graph else load().aceapex_plan_launch
    return f(plan, hip_stream)


def plan_set_tuning(plan: int, tuning: Tuning) -> int:
    return load().aceapex_plan_set_tuning(plan, ctypes.byref(tuning))


def plan_get_tuning(plan: int) -> Tuning:
    t = Tuning()
    rc = load().aceapex_plan_get_tuning(plan, ctypes.byref(t))
    if rc:
        raise AceapexError(rc, "plan_get_tuning")
    return t


def plan_tune(plan: int, hip_stream: int, reps: int) -> Tuning:
    t = Tuning()
    rc = load().aceapex_plan_tune(plan, hip_stream, reps, ctypes.byref(t))
    if rc:
        raise AceapexError(rc, "plan_tune")
    return t


def plan_destroy(plan: int) -> None:
    load().aceapex_plan_destroy(plan)


def tans_probe(container) -> TansInfo:
    import numpy as np

    buf = np.ascontiguousarray(np.frombuffer(bytes(container[:544]), dtype=np.uint8))
    info = TansInfo()
    rc = load().aceapex_tans_probe(buf.ctypes.data, buf.size, ctypes.byref(info))
    if rc:
        raise AceapexError(rc, "tans_probe")
    return info


def compare(d_a: int, d_b: int, n: int, d_result: int, hip_stream: int) -> int:
    return load().aceapex_compare(d_a, d_b, n, d_result, hip_stream)


def tans_workspace_bytes(info: TansInfo) -> int:
    return int(load().aceapex_tans_workspace_bytes(ctypes.byref(info)))


def tans_decode(d_in: int, info: TansInfo, d_out: int, out_capacity: int, d_ws: int, ws_bytes: int,
                d_status: int, hip_stream: int) -> int:
    return load().aceapex_tans_decode(d_in, ctypes.byref(info), d_out, out_capacity, d_ws, ws_bytes, d_status,
                                      hip_stream)


def tans_encode(data, table_log: int = 11, lanes: int = 1024):
    """aceapex_tans_encode on host bytes; returns the container as a uint8 numpy array."""
    import numpy as np

    x = np.ascontiguousarray(np.frombuffer(bytes(data), np.uint8) if not isinstance(data, np.ndarray) else data,
                             dtype=np.uint8)
    out = ctypes.c_void_p()
    n = load().aceapex_tans_encode(x.ctypes.data if x.size else None, x.size, table_log, lanes, ctypes.byref(out))
    if n < 0:
        raise AceapexError(int(n), "tans_encode")
    try:
        return np.ctypeslib.as_array(ctypes.cast(out, ctypes.POINTER(ctypes.c_uint8)), shape=(n,)).copy()
    finally:
        load().aceapex_free(out)
