"""Serving loop: continuous batching of decode requests on one GPU.

Requests arrive over time (a Poisson process in the benchmark); each asks for
one compressed stream of a resident pool to be decoded into device memory.
The loop

  * admits waiting requests first-come first-served while their output and
    workspace fit in the device-memory budget (an arena carved from one
    preallocated buffer; memory returns when a request completes),
  * launches the admitted requests as one batched decode (aceapex_decode_many;
    streams without stored levels are decoded one by one on the same lane)
    on a free HIP stream, so that up to `lanes` batches run on the GPU at once
    and requests that arrive while others run join the next batch,
  * records, per request, the time from its arrival to the moment the host
    observes its batch's completion.

`mode="fifo"` is the plain baseline: one request per launch, one at a time.
Outputs stay resident; `keep_outputs=True` returns a host copy of each
result for checking.

Device choice (Sec. 7.2 finds a small, deep stream slower on the GPU than on
the CPU; Sec. 8.2 suggests choosing per input): with host copies of the
streams, `route="auto"` pre-scans each request's size and deepest level and
sends it to the host decoder (aceapex_decode_host on a worker thread) when a
cost model says the host finishes first.  A host-decoded result is copied
into the same device arena, so every result ends up resident on the device;
its latency runs to the end of that copy.
"""
from __future__ import annotations

import threading
import time
from concurrent.futures import ThreadPoolExecutor
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
    route: str = "gpu"  # device that decoded it: "gpu" or "cpu"
    _mem: list = field(default_factory=list)


@dataclass
class CostModel:
    """Estimated completion times of one request on each device.

    host: size / cpu_gbps (one host thread, aceapex_decode_host).
    GPU:  a batch's fixed cost, one level boundary per level of the stream
          (the wavefront of Sec. 7.1 runs levels 0..max_level), and the size
          at the batched decode rate."""
    cpu_gbps: float = 0.4
    gpu_gbps: float = 100.0
    gpu_fixed_us: float = 150.0
    gpu_level_us: float = 2.5

    def cpu_s(self, n: int) -> float:
        return n / (self.cpu_gbps * 1e9)

    def gpu_s(self, n: int, levels: int) -> float:
        return (self.gpu_fixed_us + levels * self.gpu_level_us) * 1e-6 + n / (self.gpu_gbps * 1e9)

    def route(self, n: int, levels: int) -> str:
        return "cpu" if self.cpu_s(n) < self.gpu_s(n, levels) else "gpu"


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

    def __init__(self, pool, budget_bytes: int, lanes: int = 4, max_batch: int = 256, device="cuda",
                 host_streams=None, cpu_workers: int = 4, cost: CostModel | None = None):
        import torch

        self.pool = list(pool)
        self.host_streams = list(host_streams) if host_streams is not None else None
        self.cost = cost or CostModel()
        self.cpu_workers = cpu_workers
        self._tls = threading.local()
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

    def route_of(self, stream: int, route: str) -> str:
        """The device a request for pool stream `stream` goes to."""
        if route == "gpu" or self.host_streams is None:
            return "gpu"
        if route == "cpu":
            return "cpu"
        d = self.pool[stream]
        return self.cost.route(d.n, int(d.info.max_level) + 1)

    def calibrate_cpu(self, max_bytes: int = 8 << 20) -> float:
        """Measure the host decoder's rate (one thread) on the pool's streams of
        at most max_bytes (decoded), and put it in the cost model."""
        if self.host_streams is None:
            return self.cost.cpu_gbps
        picks = [i for i in range(len(self.pool)) if 0 < self.pool[i].n <= max_bytes][:8]
        nbytes, secs = 0, 0.0
        for i in picks:
            out = np.empty(self.pool[i].n, dtype=np.uint8)
            t0 = time.perf_counter()
            rc = _abi.decode_host(self.host_streams[i], out, 1)
            secs += time.perf_counter() - t0
            if rc:
                raise AceapexError(rc, "decode_host")
            nbytes += out.size
        if secs > 0:
            self.cost.cpu_gbps = nbytes / secs / 1e9
        return self.cost.cpu_gbps

    def _cpu_decode(self, r: Request, view):
        """Worker thread: decode on the host, then copy into the request's
        arena slot on this thread's own stream; returns the status."""
        import torch

        st = getattr(self._tls, "stream", None)
        if st is None:
            st = self._tls.stream = torch.cuda.Stream(device=self.device)
        d = self.pool[r.stream]
        out = np.empty(max(d.n, 1), dtype=np.uint8)
        rc = _abi.decode_host(self.host_streams[r.stream], out[:d.n], 1)
        if rc == 0 and d.n:
            with torch.cuda.stream(st):
                view[:d.n].copy_(torch.from_numpy(out[:d.n]))
            st.synchronize()
        return rc

    def run(self, arrivals, mode: str = "continuous", keep_outputs: bool = False, timeout_s: float = 600.0,
            route: str = "gpu"):
        """Serve (arrival_seconds, pool_index) pairs; returns the requests.

        route: "gpu" (every request on the GPU), "cpu" (every request on the
        host decoder) or "auto" (per request, the device the cost model
        picks); "fifo" mode always uses the GPU."""
        import torch

        if route != "gpu" and self.host_streams is None:
            raise ValueError("host routes need host copies of the streams")
        if mode == "fifo":
            route = "gpu"
        reqs = [Request(i, int(s), float(t)) for i, (t, s) in enumerate(sorted(arrivals))]
        for r in reqs:
            r.route = self.route_of(r.stream, route)
            if self.need_bytes(r.stream) > self.arena.size or self._ws_one[r.stream] > self.lane_ws:
                raise ValueError(f"request {r.rid} needs more memory than the budget holds")
        cpu_pool = ThreadPoolExecutor(self.cpu_workers) if any(r.route == "cpu" for r in reqs) else None
        cpu_waiting, cpu_running = [], []
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
                (cpu_waiting if reqs[nxt].route == "cpu" else waiting).append(reqs[nxt])
                nxt += 1
            # host route: completed decodes, then admission (first come, first served)
            still_cpu = []
            for r, fut, view in cpu_running:
                if fut.done():
                    r.done = time.perf_counter() - t0
                    r.status = int(fut.result())
                    if keep_outputs:
                        r.result = view[: self.pool[r.stream].n].cpu().numpy()
                    for o, n in r._mem:
                        self.arena.release(o, n)
                    r._mem = []
                    done_count += 1
                else:
                    still_cpu.append((r, fut, view))
            cpu_running = still_cpu
            while cpu_waiting and len(cpu_running) < self.cpu_workers:
                r = cpu_waiting[0]
                got = self.arena.alloc(self.need_bytes(r.stream))
                if got is None:
                    break
                cpu_waiting.pop(0)
                r._mem.append(got)
                r.admitted = r.launched = time.perf_counter() - t0
                view = self.arena.view(got[0], max(self.pool[r.stream].n, 1))
                cpu_running.append((r, cpu_pool.submit(self._cpu_decode, r, view), view))
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
            if not inflight and not waiting and not cpu_running and not cpu_waiting and nxt < len(reqs):
                wait = reqs[nxt].arrival - (time.perf_counter() - t0)
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
        if cpu_pool is not None:
            cpu_pool.shutdown(wait=True)
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
        # streams with stored levels go in one batched decode; streams in the
        # four-section format (levels derived on the device) one at a time,
        # after it on the same lane and workspace
        plain = [d for d in descs if d.s.info.flags & 8]
        if plain:
            rc = _abi.decode_many(plain, ws.data_ptr(), ws.numel(), stream.cuda_stream)
            if rc:
                raise AceapexError(rc, "decode_many")
        for d in descs:
            if not d.s.info.flags & 8:
                rc = _abi.decode(d.s, d.d_out, d.out_capacity, ws.data_ptr(), ws.numel(), d.d_status,
                                 stream.cuda_stream)
                if rc:
                    raise AceapexError(rc, "decode")
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
        "routes": {dev: {"requests": sum(1 for r in reqs if r.route == dev),
                         "bytes": int(sum(pool[r.stream].n for r in reqs if r.route == dev))}
                   for dev in ("gpu", "cpu")},
    }


def poisson_arrivals(count: int, rate_per_s: float, pool_size: int, seed: int):
    """count (time, pool index) pairs: exponential gaps at rate_per_s, uniform pool picks."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))
    picks = rng.integers(0, pool_size, size=count)
    return list(zip(t.tolist(), picks.tolist()))
