"""GPU checks of the serving loop: every request served under continuous
batching decodes exactly as the same stream decoded alone, whatever the mix
it was batched with (streams with stored levels and streams in the
four-section format), whichever device (GPU, or the host decoder) the
request was routed to, and a tight memory budget only delays admission."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pool():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_04268_amd as ax

    rng = np.random.default_rng(77)
    originals, streams, hosts = [], [], []
    for i in range(12):
        n = int(np.exp(rng.uniform(np.log(2_000), np.log(3_000_000))))
        x = synth.make(["markov", "fastq", "wiki", "random"][i % 4], n, 900 + i)
        s = oracle.encode(x, block_log2=int(rng.choice([16, 20])), flatten=int(i % 3),
                          max_depth=int(rng.choice([0, 4])))
        originals.append(x)
        streams.append(ax.to_device(s))
        hosts.append(s)
    # streams in the four-section format (no stored levels): their levels
    # are derived on the device, or they go to the host decoder
    for kind, seed in (("wiki", 950), ("fastq", 951)):
        x = synth.make(kind, 600_000, seed)
        s = oracle.encode(x, block_log2=16, levels=0)
        assert oracle.header_fields(s)["flags"] & 8 == 0
        originals.append(x)
        streams.append(ax.to_device(s))
        hosts.append(s)
    # a small stream with a deep chain: one match per level, 700 levels
    seg = np.frombuffer(np.random.default_rng(3).integers(0, 256, 16, dtype=np.uint8).tobytes(), np.uint8)
    x = np.concatenate([np.concatenate([np.frombuffer((i ^ 0x80808080).to_bytes(4, "little"), np.uint8), seg])
                        for i in range(700)])
    s = oracle.encode(x, tiebreak=1, hash_bits=12, block_log2=12)
    assert oracle.header_fields(s)["max_level"] > 600
    originals.append(x)
    streams.append(ax.to_device(s))
    hosts.append(s)
    return originals, streams, hosts


def alone(streams):
    import paper_2606_04268_amd as ax

    res = []
    for d in streams:
        out, st = ax.decode(d)
        ax.check_status(st)
        res.append(out[:d.n].cpu().numpy())
    return res


@pytest.mark.parametrize("mode", ["continuous", "fifo"])
def test_served_requests_match_alone(pool, mode):
    from paper_2606_04268_amd.serve import Server, poisson_arrivals, summarize

    originals, streams, _ = pool
    ref = alone(streams)
    for x, r in zip(originals, ref):
        assert np.array_equal(x, r)
    arrivals = poisson_arrivals(80, 4000.0, len(streams), seed=5)
    say(f"[gpu] serve 80 requests mode={mode}")
    srv = Server(streams, budget_bytes=256 << 20, lanes=3, max_batch=32)
    reqs = srv.run(arrivals, mode=mode, keep_outputs=True, timeout_s=60)
    for r in reqs:
        assert r.status == 0
        assert r.done >= r.launched >= r.admitted >= r.arrival - 1e-9
        assert np.array_equal(r.result, ref[r.stream])
    s = summarize(reqs, streams)
    assert s["errors"] == 0 and s["requests"] == 80
    assert srv.arena.used == 0


def test_tight_budget_delays_but_serves(pool):
    """An arena barely above the largest request: requests queue for memory,
    all complete, first come first served."""
    from paper_2606_04268_amd.serve import Server

    originals, streams, _ = pool
    biggest = max(d.n for d in streams)
    # lane workspaces take twice the largest single workspace each
    from paper_2606_04268_amd import workspace_bytes

    ws = 2 * max(workspace_bytes([d]) for d in streams)
    budget = 2 * ((ws + 255) // 256 * 256) + biggest + biggest // 2
    srv = Server(streams, budget_bytes=budget, lanes=2, max_batch=8)
    arrivals = [(0.0005 * i, i % len(streams)) for i in range(40)]
    say("[gpu] serve 40 requests under a tight budget")
    reqs = srv.run(arrivals, keep_outputs=True, timeout_s=60)
    order = sorted(reqs, key=lambda r: (r.admitted, r.rid))
    assert [r.rid for r in order] == sorted(r.rid for r in reqs)
    for r in reqs:
        assert r.status == 0
        assert np.array_equal(r.result, originals[r.stream])
    assert srv.arena.used == 0


@pytest.mark.parametrize("route", ["cpu", "auto"])
def test_routes_give_the_same_results(pool, route):
    """Requests routed to the host decoder, or split between the devices by
    the cost model (size and deepest level), decode exactly as alone; the
    host-decoded results land in the same device arena."""
    from paper_2606_04268_amd.serve import Server, poisson_arrivals, summarize

    originals, streams, hosts = pool
    srv = Server(streams, budget_bytes=256 << 20, lanes=3, max_batch=32, host_streams=hosts, cpu_workers=3)
    arrivals = poisson_arrivals(90, 4000.0, len(streams), seed=9)
    say(f"[gpu] serve 90 requests route={route}")
    reqs = srv.run(arrivals, keep_outputs=True, timeout_s=120, route=route)
    for r in reqs:
        assert r.status == 0
        assert np.array_equal(r.result, originals[r.stream])
    s = summarize(reqs, streams)
    assert s["errors"] == 0 and srv.arena.used == 0
    if route == "cpu":
        assert s["routes"]["gpu"]["requests"] == 0
    else:
        deep = len(streams) - 1
        assert srv.route_of(deep, "auto") == "cpu"  # 700 levels of a 14 KB stream
        assert srv.route_of(int(np.argmax([d.n for d in streams])), "auto") == "gpu"
        assert s["routes"]["cpu"]["requests"] > 0 and s["routes"]["gpu"]["requests"] > 0
