"""MI355X-native decoder for absolute-offset LZ77 streams (ACEAPEX, arXiv 2606.04268).

Every step of a decode runs in the HIP kernels of ``libaceapex.so`` behind the
C ABI of ``include/aceapex.h``; this module only moves arguments across it.
PyTorch supplies device memory and streams.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import _abi
from ._abi import AceapexError, Info

__all__ = ["AceapexError", "Info", "DeviceStream", "probe", "encode", "to_device",
           "workspace_bytes", "decode", "decode_derive", "decode_host", "decode_many", "check_status",
           "content_hash", "Plan", "tans_decode"]


def _torch():
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("the ACEAPEX decoder needs a ROCm GPU; none is visible")
    return torch


def content_hash(data) -> int:
    """XXH3-64 of a host buffer, the verification hash of Sec. 4.3 (xxhash package)."""
    import xxhash

    return xxhash.xxh3_64_intdigest(memoryview(np.ascontiguousarray(data, dtype=np.uint8)))


def encode(data, *, with_hash: bool = True, **opts) -> np.ndarray:
    """Encode host bytes into a stream (host encoder in libaceapex.so).

    Options (see aceapex_enc_opts): block_log2, min_match, flatten, max_depth,
    chain_depth, hash_bits, tiebreak, chunk_log2, threads, verbose, levels
    (0: the four streams of Sec. 3.2 only; the decoder derives the levels).
    """
    o = _abi.enc_defaults()
    for k, v in opts.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown encoder option {k}")
        setattr(o, k, int(v))
    s = _abi.encode(data, o)
    x = np.frombuffer(bytes(data), np.uint8) if not isinstance(data, np.ndarray) else data
    if with_hash and x.size:
        s[56:64] = np.frombuffer(content_hash(x).to_bytes(8, "little"), dtype=np.uint8)
    return s


def probe(stream) -> Info:
    """Header fields of a host-resident stream (aceapex_probe)."""
    return _abi.probe(stream)


@dataclass
class DeviceStream:
    """A compressed stream resident in device memory plus its probed header
    and a host copy of its level table (matches per level)."""
    comp: "object"  # torch.Tensor, uint8, on the GPU
    info: Info
    levels: "object" = None  # ctypes uint32 array, or None

    @property
    def n(self) -> int:
        return int(self.info.decoded_bytes)

    def abi(self) -> _abi.Stream:
        return _abi.Stream(self.comp.data_ptr(), self.info, self.levels)


def to_device(stream, device="cuda") -> DeviceStream:
    """Copy a host stream (uint8 numpy array or bytes) to the GPU."""
    torch = _torch()
    host = np.ascontiguousarray(np.frombuffer(bytes(stream), np.uint8) if not isinstance(stream, np.ndarray)
                                else stream, dtype=np.uint8)
    info = probe(host)
    if info.comp_bytes != host.size:
        raise AceapexError(_abi.E_FORMAT, f"header says {info.comp_bytes} bytes, buffer has {host.size}")
    levels = _abi.level_table(host, info)
    comp = torch.from_numpy(host).to(device)
    return DeviceStream(comp, info, levels)


def workspace_bytes(streams) -> int:
    descs = [_abi.Desc(s.abi(), None, s.n, None) for s in streams]
    return _abi.workspace_bytes(descs)


def _stream_handle(stream):
    torch = _torch()
    st = stream if stream is not None else torch.cuda.current_stream()
    return st.cuda_stream


def _used_on(stream, tensors):
    """Mark tensors allocated here as in use by ``stream`` when it is not the
    current stream, so that the caching allocator does not hand their memory
    to another tensor while the decode enqueued there may still use it."""
    torch = _torch()
    if stream is None or stream == torch.cuda.current_stream(stream.device):
        return
    for t in tensors:
        t.record_stream(stream)


def decode(ds: DeviceStream, out=None, workspace=None, status=None, stream=None):
    """Enqueue a decode of ``ds``; returns (out, status) tensors.  Asynchronous."""
    torch = _torch()
    dev = ds.comp.device
    mine = []  # tensors allocated here
    if out is None:
        out = torch.empty(max(ds.n, 1), dtype=torch.uint8, device=dev)
        mine.append(out)
    need = workspace_bytes([ds])
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        mine.append(workspace)
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=dev)
        mine.append(status)
    _used_on(stream, mine)
    rc = _abi.decode(ds.abi(), out.data_ptr(), out.numel(), workspace.data_ptr(), workspace.numel(),
                     status.data_ptr(), _stream_handle(stream))
    if rc:
        raise AceapexError(rc, "decode")
    return out, status


def decode_many(streams, outs=None, workspace=None, statuses=None, stream=None):
    """Enqueue one batched decode of many streams; returns (outs, statuses)."""
    torch = _torch()
    dev = streams[0].comp.device if streams else "cuda"
    mine = []  # tensors allocated here
    if outs is None:
        outs = [torch.empty(max(s.n, 1), dtype=torch.uint8, device=dev) for s in streams]
        mine += outs
    if statuses is None:
        statuses = torch.empty(max(len(streams), 1), dtype=torch.int32, device=dev)
        mine.append(statuses)
    descs = [_abi.Desc(s.abi(), o.data_ptr(), o.numel(), statuses.data_ptr() + 4 * i)
             for i, (s, o) in enumerate(zip(streams, outs))]
    need = _abi.workspace_bytes(descs) if descs else 0
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        mine.append(workspace)
    _used_on(stream, mine)
    rc = _abi.decode_many(descs, workspace.data_ptr(), workspace.numel(), _stream_handle(stream))
    if rc:
        raise AceapexError(rc, "decode_many")
    return outs, statuses


def decode_derive(ds: DeviceStream, out=None, workspace=None, status=None, levels: bool = True, stream=None):
    """Enqueue a decode of ``ds`` that derives every match's level on the
    device (aceapex_decode_derive); returns (out, status, levels) where levels
    is a uint32-valued int32 tensor of each match's level in stream order (or
    None).  The call reads a queue length back from the device every few
    levels, so it returns once the last level is enqueued."""
    torch = _torch()
    dev = ds.comp.device
    mine = []
    if out is None:
        out = torch.empty(max(ds.n, 1), dtype=torch.uint8, device=dev)
        mine.append(out)
    need = _abi.workspace_bytes_derive(ds.info)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        mine.append(workspace)
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=dev)
        mine.append(status)
    lv = torch.empty(max(int(ds.info.n_seq), 1), dtype=torch.int32, device=dev) if levels else None
    if lv is not None:
        mine.append(lv)
    _used_on(stream, mine)
    rc = _abi.decode_derive(ds.abi(), out.data_ptr(), out.numel(), workspace.data_ptr(), workspace.numel(),
                            lv.data_ptr() if lv is not None else None, status.data_ptr(), _stream_handle(stream))
    if rc:
        raise AceapexError(rc, "decode_derive")
    return out, status, lv


def decode_host(stream, threads: int = 0) -> np.ndarray:
    """Decode a host stream on the host CPU (aceapex_decode_host)."""
    s = np.ascontiguousarray(np.frombuffer(bytes(stream), np.uint8) if not isinstance(stream, np.ndarray)
                             else stream, dtype=np.uint8)
    out = np.empty(int(probe(s).decoded_bytes), dtype=np.uint8)
    rc = _abi.decode_host(s, out, threads)
    if rc:
        raise AceapexError(rc, "decode_host")
    return out


def tans_decode(container, out=None, workspace=None, status=None, stream=None, device="cuda"):
    """Decode a tANS container (entropy-coded literals) on the GPU; the
    container is a host array (copied to the device) or a device tensor whose
    first 544 bytes are given as ``container[1]`` in a (tensor, host prefix)
    pair.  Returns (out, status)."""
    torch = _torch()
    if isinstance(container, tuple):
        d_in, prefix = container
    else:
        prefix = np.ascontiguousarray(container, dtype=np.uint8)
        d_in = torch.from_numpy(prefix).to(device)
    info = _abi.tans_probe(prefix)
    dev = d_in.device
    mine = []
    if out is None:
        out = torch.empty(max(int(info.n), 1), dtype=torch.uint8, device=dev)
        mine.append(out)
    need = _abi.tans_workspace_bytes(info)
    if workspace is None or workspace.numel() < need:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        mine.append(workspace)
    if status is None:
        status = torch.empty(1, dtype=torch.int32, device=dev)
        mine.append(status)
    _used_on(stream, mine)
    rc = _abi.tans_decode(d_in.data_ptr(), info, out.data_ptr(), out.numel(), workspace.data_ptr(),
                          workspace.numel(), status.data_ptr(), _stream_handle(stream))
    if rc:
        raise AceapexError(rc, "tans_decode")
    return out, status


def compare(a, b, stream=None):
    """Byte compare of two device tensors on the GPU (aceapex_compare):
    returns (differing bytes, index of the first; n when none).  Synchronizes
    the stream to read the result."""
    torch = _torch()
    if a.numel() != b.numel() or a.dtype != torch.uint8 or b.dtype != torch.uint8:
        raise ValueError("compare takes two uint8 tensors of one size")
    a = a.contiguous()
    b = b.contiguous()
    res = torch.empty(2, dtype=torch.int64, device=a.device)
    _used_on(stream, [res])
    rc = _abi.compare(a.data_ptr(), b.data_ptr(), a.numel(), res.data_ptr(), _stream_handle(stream))
    if rc:
        raise AceapexError(rc, "compare")
    (stream if stream is not None else torch.cuda.current_stream(a.device)).synchronize()
    mism, first = (int(v) for v in res.cpu())
    return mism, first


def check_status(status) -> None:
    """Raise if any device status word is nonzero (synchronises)."""
    vals = status.cpu().numpy().ravel()
    bad = np.nonzero(vals)[0]
    if bad.size:
        raise AceapexError(int(vals[bad[0]]), f"device status of stream {int(bad[0])}")


class Plan:
    """A batch of device streams laid out once in its workspace
    (aceapex_plan_create); every launch decodes all of them again by
    enqueueing kernels only, directly or through a captured HIP graph.

    The tensors given (or allocated here) are kept referenced for the plan's
    lifetime, as the C ABI requires."""

    def __init__(self, streams, outs=None, statuses=None, workspace=None, stream=None, tuning=None):
        torch = _torch()
        self.streams = list(streams)
        dev = self.streams[0].comp.device if self.streams else "cuda"
        if outs is None:
            outs = [torch.empty(max(s.n, 1), dtype=torch.uint8, device=dev) for s in self.streams]
        if statuses is None:
            statuses = torch.zeros(max(len(self.streams), 1), dtype=torch.int32, device=dev)
        self.outs, self.statuses = list(outs), statuses
        descs = [_abi.Desc(s.abi(), o.data_ptr(), o.numel(), statuses.data_ptr() + 4 * i)
                 for i, (s, o) in enumerate(zip(self.streams, self.outs))]
        need = _abi.workspace_bytes(descs) if descs else 0
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        self.workspace = workspace
        t = None
        if tuning is not None:
            t = _abi.tuning_defaults()
            for k, v in dict(tuning).items():
                setattr(t, k, int(v))
        self._h = _abi.plan_create(descs, workspace.data_ptr(), workspace.numel(), t, _stream_handle(stream))

    def launch(self, stream=None, graph: bool = False):
        """Enqueue one decode of every stream (asynchronous)."""
        rc = _abi.plan_launch(self._handle(), _stream_handle(stream), graph)
        if rc:
            raise AceapexError(rc, "plan_launch")

    @property
    def tuning(self) -> dict:
        return _abi.plan_get_tuning(self._handle()).as_dict()

    def set_tuning(self, **knobs):
        t = _abi.plan_get_tuning(self._handle())
        for k, v in knobs.items():
            if not hasattr(t, k):
                raise TypeError(f"unknown tuning knob {k}")
            setattr(t, k, int(v))
        rc = _abi.plan_set_tuning(self._handle(), t)
        if rc:
            raise AceapexError(rc, "plan_set_tuning")

    def signature(self) -> str:
        """Key of this batch's shape for a tuning cache: stream count and the
        rounded logs of its decoded bytes and matches, and its deepest level."""
        import math

        n = sum(s.n for s in self.streams)
        m = sum(int(s.info.n_seq) for s in self.streams)
        lv = max((int(s.info.max_level) for s in self.streams), default=0)
        return f"s{len(self.streams)}-b{round(math.log2(n + 1))}-m{round(math.log2(m + 1))}-l{lv}"

    def tune(self, reps: int = 3, stream=None, cache: str | None = None) -> dict:
        """Autotune the level schedule (aceapex_plan_tune) and return it.  With
        a cache file (JSON), a schedule stored for the same signature is reused
        instead, and a new one is stored."""
        import json
        import os

        key = self.signature()
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                self.set_tuning(**table[key])
                return dict(table[key])
        best = _abi.plan_tune(self._handle(), _stream_handle(stream), reps).as_dict()
        if cache:
            table[key] = best
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return best

    def _handle(self):
        if not self._h:
            raise AceapexError(_abi.E_INVAL, "plan already closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            _abi.plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
