"""GPU checks of plans (aceapex_plan_*): a batch laid out once decodes
exactly on every launch, eager or through its captured HIP graph, under any
schedule the tuning knobs allow and after autotuning."""
import numpy as np
import pytest

from gpu_util import GUARD, POISON, say
from mixes import mixed_streams

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_04268_amd as ax

    pairs = mixed_streams(16, 41)
    dss = [ax.to_device(s) for _, s in pairs]
    bufs = [torch.full((d.n + 2 * GUARD,), POISON, dtype=torch.uint8, device="cuda") for d in dss]
    outs = [b[GUARD:GUARD + max(d.n, 16)] for b, d in zip(bufs, dss)]
    statuses = torch.full((len(dss),), 12345, dtype=torch.int32, device="cuda")
    return pairs, dss, bufs, outs, statuses


def check(pairs, dss, bufs, statuses, label):
    import torch

    torch.cuda.synchronize()
    st = statuses.cpu().numpy()
    assert (st == 0).all(), (label, st)
    for (x, _), d, b in zip(pairs, dss, bufs):
        h = b.cpu().numpy()
        assert (h[:GUARD] == POISON).all() and (h[GUARD + d.n:] == POISON).all(), label
        assert np.array_equal(h[GUARD:GUARD + d.n], x), label


def poison(bufs, statuses):
    for b in bufs:
        b.fill_(POISON)
    statuses.fill_(12345)


def test_plan_launch_eager_and_graph(batch):
    import torch

    import paper_2606_04268_amd as ax

    pairs, dss, bufs, outs, statuses = batch
    plan = ax.Plan(dss, outs=outs, statuses=statuses)
    try:
        for i in range(3):
            poison(bufs, statuses)
            say(f"[gpu] plan eager launch {i}")
            plan.launch()
            check(pairs, dss, bufs, statuses, f"eager {i}")
        # graph replays, each checked, with eager work and synchronisation between them
        for i in range(4):
            poison(bufs, statuses)
            torch.cuda.synchronize()
            say(f"[gpu] plan graph replay {i}")
            plan.launch(graph=True)
            check(pairs, dss, bufs, statuses, f"graph replay {i}")
    finally:
        plan.close()


@pytest.mark.parametrize("knobs", [dict(xcd_parts=1), dict(long_copy=16), dict(long_copy=1 << 21),
                                   dict(tail_level_max=0), dict(tail_level_max=1 << 20),
                                   dict(level_wg_max=1), dict(level_wg_max=65535)],
                         ids=lambda k: "-".join(f"{a}{b}" for a, b in k.items()))
def test_every_schedule_decodes_the_same(batch, knobs):
    import paper_2606_04268_amd as ax

    pairs, dss, bufs, outs, statuses = batch
    plan = ax.Plan(dss, outs=outs, statuses=statuses, tuning=knobs)
    try:
        assert all(plan.tuning[k] == v for k, v in knobs.items())
        poison(bufs, statuses)
        say(f"[gpu] plan with {knobs}")
        plan.launch()
        check(pairs, dss, bufs, statuses, str(knobs))
        poison(bufs, statuses)
        plan.launch(graph=True)
        check(pairs, dss, bufs, statuses, f"graph {knobs}")
    finally:
        plan.close()


def test_autotune_and_cache(batch, tmp_path):
    import paper_2606_04268_amd as ax

    pairs, dss, bufs, outs, statuses = batch
    cache = str(tmp_path / "tune.json")
    plan = ax.Plan(dss, outs=outs, statuses=statuses)
    try:
        say("[gpu] plan autotune")
        best = plan.tune(reps=1, cache=cache)
        assert plan.tuning == best
        poison(bufs, statuses)
        plan.launch(graph=True)
        check(pairs, dss, bufs, statuses, f"tuned {best}")
    finally:
        plan.close()
    again = ax.Plan(dss, outs=outs, statuses=statuses)
    try:
        assert again.tune(reps=1, cache=cache) == best  # read back, not re-measured
        assert again.tuning == best
    finally:
        again.close()
