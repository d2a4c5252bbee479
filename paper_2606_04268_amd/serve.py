"""Serving loop: continuous batching of decode requests on one GPU.

Requests arrive over time (a Poisson process in the benchmark); each asks for
one compressed stream of a resident pool to be decoded into device memory.
The loop

  * admits waiting requests first-come first-served while their output and
    workspace fit in the device-memory budget (an arena carved from one
    preallocated buffer; memory returns when a request completes),
  * launches the admitted requests as one batched decode (aceapex_decode_many)
    on a free HIP stream, so that up to `lanes` batches run on the GPU at once
    and requests that arrive while others run join the next batch,
  * records, per request, the time from its arrival to the moment the host
    observes its batch's completion.

`mode="fifo"` is the plain baseline: one request per launch, one at a time.
Outputs stay resident; `keep_outputs=True` returns a host copy of each
result for checking.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import AceapexError, DeviceStream, _abi

ALIGN = 256


class Arena:
    """First-fit allocator over one device buffer (offsets, 256-byte aligned)."""

    def __init__(self, nbytes: int, device="cuda"):
        import torch

        self.size = int(nbytes)
        self.buf = torch.empty(self.size, dtype=torch.uint8, device=device)
        self.free = [(0, self.size)]  # sorted, coalesced (offset, length)
        self.used = 0

    def alloc(self, n: int):
        n = max(ALIGN, (int(n) + ALIGN - 1) // ALIGN * ALIGN)
        for i, (o, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (o + n, ln - n)
                self.used += n
                return o, n
        return None

    def release(self, o: int, n: int):
        self.used -= n
        fr = self.free
        lo, hi = 0, len(fr)
        while lo < hi:
            mid = (lo + hi) // 2
            if fr[mid][0] < o:
                lo = mid + 1
            else:
                hi = mid
        fr.insert(lo, (o, n))
        # coalesce with the neighbours
        if lo + 1 < len(fr) and fr[lo][0] + fr[lo][1] == fr[lo + 1][0]:
            fr[lo] = (fr[lo][0], fr[lo][1] + fr[lo + 1][1])
            fr.pop(lo + 1)
        if lo > 0 and fr[lo - 1][0] + fr[lo - 1][1] == fr[lo][0]:
            fr[lo - 1] = (fr[lo - 1][0], fr[lo - 1][1] + fr[lo][1])
            fr.pop(lo)

    def view(self, o: int, n: int):
        return self.buf[o:o + n]


@dataclass
class Request:
    rid: int
    stream: int       # index into the pool
    arrival: float    # seconds from the start of the run
    admitted: float = -1.0
    launched: float = -1.0
    done: float = -1.0
    status: int = 0
    result: np.ndarray = None
    _mem: list = field(default_factory=list)


@dataclass
class Batch:
    reqs: list
    lane: int
    event: object
    statuses: object
    outs: list


class Server:
    """Continuous-batching decode server over a pool of resident streams.

    Memory: `budget_bytes` covers every lane's workspace (fixed, sized for
    the largest batch workspace a lane may run) plus the output arena from
    which requests are admitted.
    """

    def __init__(self, pool, budget_bytes: int, lanes: int = 4, max_batch: int = 256, device="cuda"):
        import torch

        self.pool = list(pool)
        self.device = device
        self.max_batch = max_batch
        self._ws_one = [max(_abi.workspace_bytes([_abi.Desc(p.abi(), None, p.n, None)]), ALIGN)
                        for p in self.pool]
        self.lane_ws = max(max(self._ws_one) * 2, int(budget_bytes * 0.25 / lanes))
        self.lane_ws = (self.lane_ws + ALIGN - 1) // ALIGN * ALIGN
        arena = budget_bytes - lanes * self.lane_ws
        if arena <= 0:
            raise ValueError("budget too small for the lane workspaces")
        self.arena = Arena(arena, device)
        self.ws = [torch.empty(self.lane_ws, dtype=torch.uint8, device=device) for _ in range(lanes)]
        self.lanes = [torch.cuda.Stream(device=device) for _ in range(lanes)]

    def need_bytes(self, stream: int) -> int:
        return (self.pool[stream].n + ALIGN - 1) // ALIGN * ALIGN

    def run(self, arrivals, mode: str = "continuous", keep_outputs: bool = False, timeout_s: float = 600.0):
        """Serve (arrival_seconds, pool_index) pairs; returns the requests."""
        import torch

        reqs = [Request(i, int(s), float(t)) for i, (t, s) in enumerate(sorted(arrivals))]
        for r in reqs:
            if self.need_bytes(r.stream) > self.arena.size or self._ws_one[r.stream] > self.lane_ws:
                raise ValueError(f"request {r.rid} needs more memory than the budget holds")
        waiting = []
        inflight = []
        nxt = 0
        done_count = 0
        lanes_busy = [False] * len(self.lanes)
        max_lanes = 1 if mode == "fifo" else len(self.lanes)
        max_batch = 1 if mode == "fifo" else self.max_batch
        t0 = time.perf_counter()
        while done_count < len(reqs):
            now = time.perf_counter() - t0
            if now > timeout_s:
                raise TimeoutError("serving run exceeded its time limit")
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                waiting.append(reqs[nxt])
                nxt += 1
            still = []
            for b in inflight:
                if b.event.query():
                    tdone = time.perf_counter() - t0
                    st = b.statuses.cpu().numpy()
                    for i, r in enumerate(b.reqs):
                        r.done = tdone
                        r.status = int(st[i])
                        if keep_outputs:
                            r.result = b.outs[i][: self.pool[r.stream].n].cpu().numpy()
                        for o, n in r._mem:
                            self.arena.release(o, n)
                        r._mem = []
                    done_count += len(b.reqs)
                    lanes_busy[b.lane] = False
                else:
                    still.append(b)
            inflight = still
            lane = next((i for i in range(max_lanes) if not lanes_busy[i]), None)
            if lane is not None and waiting:
                batch, descs, ws_est = [], [], 0
                while waiting and len(batch) < max_batch:
                    r = waiting[0]
                    if batch and ws_est + self._ws_one[r.stream] > self.lane_ws:
                        break
                    got = self.arena.alloc(self.need_bytes(r.stream))
                    if got is None:
                        break  # first come, first served: the head waits for memory
                    r._mem.append(got)
                    r.admitted = time.perf_counter() - t0
                    ws_est += self._ws_one[r.stream]
                    batch.append(waiting.pop(0))
                if batch:
                    self._launch(batch, lane, inflight, t0, waiting)
                    lanes_busy[lane] = True
                    continue
            if not inflight and not waiting and nxt < len(reqs):
                wait = reqs[nxt].arrival - (time.perf_counter() - t0)
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
        torch.cuda.synchronize()
        return reqs

    def _launch(self, batch, lane, inflight, t0, waiting):
        import torch

        stream = self.lanes[lane]
        statuses = torch.empty(len(batch), dtype=torch.int32, device=self.device)
        outs = [self.arena.view(r._mem[0][0], max(self.pool[r.stream].n, 1)) for r in batch]
        descs = [_abi.Desc(self.pool[r.stream].abi(), o.data_ptr(), o.numel(), statuses.data_ptr() + 4 * i)
                 for i, (r, o) in enumerate(zip(batch, outs))]
        while _abi.workspace_bytes(descs) > self.lane_ws and len(batch) > 1:
            r = batch.pop()  # back to the head of the queue
            descs.pop()
            outs.pop()
            for o, n in r._mem:
                self.arena.release(o, n)
            r._mem = []
            r.admitted = -1.0
            waiting.insert(0, r)
        ws = self.ws[lane]
        rc = _abi.decode_many(descs, ws.data_ptr(), ws.numel(), stream.cuda_stream)
        if rc:
            raise AceapexError(rc, "decode_many")
        ev = torch.cuda.Event()
        ev.record(stream)
        now = time.perf_counter() - t0
        for r in batch:
            r.launched = now
        inflight.append(Batch(batch, lane, ev, statuses, outs))


def summarize(reqs, pool) -> dict:
    lat = np.array([r.done - r.arrival for r in reqs])
    nbytes = sum(pool[r.stream].n for r in reqs)
    span = max(r.done for r in reqs) - min(r.arrival for r in reqs)
    return {
        "requests": len(reqs),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "decoded_bytes": int(nbytes),
        "aggregate_gbps": float(nbytes / span / 1e9) if span > 0 else 0.0,
        "errors": int(sum(1 for r in reqs if r.status)),
    }


def poisson_arrivals(count: int, rate_per_s: float, pool_size: int, seed: int):
    """count (time, pool index) pairs: exponential gaps at rate_per_s, uniform pool picks."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))
    picks = rng.integers(0, pool_size, size=count)
    return list(zip(t.tolist(), picks.tolist()))
