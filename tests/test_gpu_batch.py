"""GPU parity of the batched decode (aceapex_decode_many): many independent
streams in one launch sequence must each decode exactly as alone, including
when some streams of the batch are corrupt."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import GUARD, POISON, say
from mixes import mixed_streams

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def run_batch(pairs, with_tables=True):
    import torch

    import paper_2606_04268_amd as ax

    dss = [ax.to_device(s) for _, s in pairs]
    if not with_tables:
        for d in dss:
            d.levels = None
    bufs, outs = [], []
    for d in dss:
        b = torch.full((d.n + 2 * GUARD,), POISON, dtype=torch.uint8, device="cuda")
        bufs.append(b)
        outs.append(b[GUARD:GUARD + max(d.n, 16)])
    statuses = torch.full((len(dss),), 12345, dtype=torch.int32, device="cuda")
    ax.decode_many(dss, outs=outs, statuses=statuses)
    torch.cuda.synchronize()
    st = statuses.cpu().numpy()
    res = []
    for d, b in zip(dss, bufs):
        h = b.cpu().numpy()
        assert (h[:GUARD] == POISON).all(), "write below an output buffer"
        assert (h[GUARD + d.n:] == POISON).all(), "write above an output buffer"
        res.append(h[GUARD:GUARD + d.n])
    return res, st


@pytest.mark.parametrize("with_tables", [True, False], ids=["batched", "one_by_one"])
def test_batch_of_mixed_streams(with_tables):
    pairs = mixed_streams(24, 3)
    say(f"[gpu] decode_many {len(pairs)} streams with_tables={with_tables}")
    res, st = run_batch(pairs, with_tables)
    assert (st == 0).all(), st
    for (x, _), got in zip(pairs, res):
        assert np.array_equal(got, x)


def test_large_batch_many_small_streams():
    """Hundreds of 4 KB .. 64 KB streams in one call."""
    rng = np.random.default_rng(11)
    pairs = []
    for i in range(300):
        n = int(rng.integers(4096, 65536))
        x = synth.make(["markov", "fastq", "random"][i % 3], n, 5000 + i)
        pairs.append((x, oracle.encode(x, block_log2=16, flatten=i % 2)))
    say("[gpu] decode_many 300 small streams")
    res, st = run_batch(pairs)
    assert (st == 0).all()
    for (x, _), got in zip(pairs, res):
        assert np.array_equal(got, x)


def _corrupt(s, rng):
    """A copy of stream s with a few bytes flipped past the header (the header
    stays valid so that the host accepts it)."""
    bad = s.copy()
    h = oracle.header_fields(s)
    start = 64 + 16 * (h["n_blocks"] + 1) + (4 * (h["max_level"] + 1) + 15) // 16 * 16
    for _ in range(int(rng.integers(1, 6))):
        i = int(rng.integers(start, s.size))
        bad[i] ^= np.uint8(1 << int(rng.integers(0, 8)))
    return bad


def test_corrupt_streams_do_not_disturb_their_batch():
    """Valid streams decode exactly and no output buffer is overrun, whatever
    the corrupt streams beside them contain."""
    rng = np.random.default_rng(2024)
    good = mixed_streams(10, 9)
    for trial in range(4):
        pairs = []
        corrupt_at = set()
        for i, (x, s) in enumerate(good):
            if i % 3 == trial % 3 and x.size > 1000:
                pairs.append((x, _corrupt(s, rng)))
                corrupt_at.add(i)
            else:
                pairs.append((x, s))
        say(f"[gpu] corrupt batch trial {trial}: corrupt streams {sorted(corrupt_at)}")
        res, st = run_batch(pairs)
        for i, ((x, _), got) in enumerate(zip(pairs, res)):
            if i in corrupt_at:
                assert st[i] in (0, -3)
            else:
                assert st[i] == 0
                assert np.array_equal(got, x)


def test_more_streams_than_one_launch_sequence():
    """2,100 streams: more than one launch sequence holds (2,048), so the
    batch runs as two sequences with the workspace split between them, in
    aceapex_decode_many and in a plan (direct launches and graph replay)."""
    import torch

    import paper_2606_04268_amd as ax

    rng = np.random.default_rng(2100)
    pairs = []
    for i in range(2100):
        n = int(np.exp(rng.uniform(np.log(64), np.log(12_000))))
        x = synth.make(["markov", "fastq", "random", "wiki"][i % 4], n, 77_000 + i)
        opts = dict(block_log2=int(rng.choice([8, 10, 12])), flatten=int(rng.integers(0, 3)),
                    max_depth=int(rng.choice([0, 0, 2])), chunk_log2=int(rng.choice([2, 5, 10])), hash_bits=12)
        pairs.append((x, oracle.encode(x, **opts)))
    for x, s in pairs:
        assert np.array_equal(oracle.decode(s), x)
    say(f"[gpu] decode_many {len(pairs)} streams (two launch sequences)")
    res, st = run_batch(pairs)
    assert (st == 0).all()
    for (x, _), got in zip(pairs, res):
        assert np.array_equal(got, x)

    dss = [ax.to_device(s) for _, s in pairs]
    outs = [torch.full((max(d.n, 1),), POISON, dtype=torch.uint8, device="cuda") for d in dss]
    plan = ax.Plan(dss, outs=outs)
    try:
        for graph in (False, True, True):
            say(f"[gpu] plan of {len(dss)} streams, graph={graph}")
            for o in outs:
                o.fill_(POISON)
            plan.statuses.fill_(12345)
            plan.launch(graph=graph)
            torch.cuda.synchronize()
            ax.check_status(plan.statuses)
            for (x, _), o in zip(pairs, outs):
                assert np.array_equal(o[:x.size].cpu().numpy(), x)
    finally:
        plan.close()


def test_decode_on_a_side_stream_without_buffers():
    """decode() and decode_many() allocate their own output, status and
    workspace when none is given; enqueued on a stream that is not the
    current one, those tensors must stay reserved for that stream until the
    decode there has run."""
    import torch

    import paper_2606_04268_amd as ax

    pairs = mixed_streams(6, 31)
    side = torch.cuda.Stream()
    dss = [ax.to_device(s) for _, s in pairs]
    torch.cuda.synchronize()
    results = []
    for d in dss:
        results.append(ax.decode(d, stream=side))
    outs, sts = ax.decode_many(dss, stream=side)
    # allocations on the current stream meanwhile must not reuse those buffers
    junk = [torch.full((1 << 20,), 7, dtype=torch.uint8, device="cuda") for _ in range(16)]
    side.synchronize()
    torch.cuda.synchronize()
    del junk
    for (x, _), (o, st), o2 in zip(pairs, results, outs):
        assert int(st.item()) == 0
        assert np.array_equal(o[:x.size].cpu().numpy(), x)
        assert np.array_equal(o2[:x.size].cpu().numpy(), x)
    assert (sts.cpu().numpy() == 0).all()


@pytest.mark.parametrize("with_tables", [True, False], ids=["batched", "one_by_one"])
def test_batch_with_streams_without_levels(with_tables):
    """Streams in the four-section format (no stored levels) inside a batch:
    they are decoded after the others with their levels derived on the
    device; every stream matches its original and the oracle's decode."""
    pairs = mixed_streams(12, 5)
    for i, kind in enumerate(["wiki", "fastq", "markov", "wiki"]):
        x = synth.make(kind, 200_000 + 77_777 * i, 60 + i)
        pairs.insert(3 * i + 1, (x, oracle.encode(x, block_log2=[12, 16, 20, 14][i], levels=0)))
    say(f"[gpu] decode_many {len(pairs)} streams, 4 without levels, with_tables={with_tables}")
    res, st = run_batch(pairs, with_tables)
    assert (st == 0).all(), st
    for (x, s), got in zip(pairs, res):
        assert np.array_equal(got, x) and np.array_equal(got, oracle.decode(s))
