#!/usr/bin/env python3
"""Decoded GB/s of the MI355X absolute-offset LZ77 decoder on one GPU.

One step = one full decode of one stream (every stage of the path: chunk
setup, parse + literal scatter, level bucketing and every level of the match
wavefront) from the device-resident compressed stream to the device-resident
output.  Inputs are generated and encoded on the host before timing and stay
in HBM; every timed output is compared byte for byte with the resident
original, and the plain workloads' XXH3-64 with the header's.

Default run (no --mode): ONE JSON line on stdout whose value is the 1 GiB
wiki-markup-like stream encoded without a depth limit (the largest plain
workload), with, in the same line:
  - the same text encoded with depth limit 8 (Sec. 7.4);
  - the 4 MiB Markov text and the 256 MiB FASTQ-like stream;
  - batched: 4,096 independent streams (sizes log-uniform 4 KiB..64 MiB,
    40% Markov text / 40% FASTQ-like / 20% random bytes with 30% repeats)
    decoded as one batch: a plan (autotuned, replayed as a captured HIP
    graph), one aceapex_decode_many call, and a loop of aceapex_decode calls;
  - served: Poisson arrivals at 100 GB/s offered of requests drawn from a pool
    of resident streams (sizes log-uniform 64 KiB..256 MiB, same mix) under a
    200 GB device-memory budget, 300 warm-up then 3,000 measured requests;
    continuous batching against one request at a time;
  - the level-launch floor measured on a one-match-per-level chain, and the
    sync floor it implies for each plain stream ((max_level + 1) launches);
  - the entropy stage: the FASTQ-like stream's literal bytes (its lit[]
    sections, 132 MB, mostly quality strings) tANS-coded on the host and
    decoded on the GPU;
  - roofline (dominant kernel group of the 1 GiB stream), and the CPU oracle
    on a bounded sample of the same text at T = 1, 2, 4, 8, 16 threads with
    the host's memcpy bandwidth at the same T.
Progress goes to stderr.

Other modes (one JSON line each):
  --mode plain    one plain workload (--workload), as the main entry above
  --mode batched  the batched entry alone
  --mode served   the served entry with a sweep of offered loads
  --mode entropy  the entropy stage alone on one workload's literals (--workload)
  --mode derive   one workload (--workload) encoded without stored levels,
                  decoded with levels derived on the device, beside the same
                  text with stored levels
  --mode sweep    depth limit D (1, 2, 10, unlimited) x chain flattening (off,
                  R1, R2) on wiki-like text and FASTQ-like data (32 MiB each):
                  ratio, deepest level and decoded GB/s (Sec. 7.4, Table 5)
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "decoded GB/s at 1 MI355X (bit-exact) vs HBM peak; served p50/p99 latency"
HOST_THREADS = 16  # worker threads of the host encoder and host decoder

WORKLOADS = {
    "wiki1g": dict(kind="wiki", size=1 << 30, seed=0xACE2, enc=dict(),
                   desc="wiki-markup-like 1 GiB (Zipf(1.1) words over a 50k-word vocabulary, sentences of 5-30 "
                        "words, tags every 300-500 bytes, template lines); 1 MiB blocks, min match 4, "
                        "depth unlimited"),
    "wiki1g_d8": dict(kind="wiki", size=1 << 30, seed=0xACE2, enc=dict(max_depth=8),
                      desc="wiki-markup-like 1 GiB; 1 MiB blocks, min match 4, depth limit 8"),
    "fastq256": dict(kind="fastq", size=256 << 20, seed=0xACE1, enc=dict(flatten=1),
                     desc="FASTQ-like 256 MiB: 150 bp reads over ACGT with 1% N, Phred+33 qualities, "
                          "10% near-duplicate reads; 1 MiB blocks, min match 4, chain flattening on"),
    "markov4": dict(kind="markov", size=4 << 20, seed=0xACE0, enc=dict(),
                    desc="order-2 Markov text 4 MiB with 20% copies; 1 MiB blocks, min match 4, no flattening"),
}

# encoder options of the batched / served mixes; chain depth 2 keeps the host
# encode of the ~28 GB batch within a minute on 16 host threads
MIX_ENC = {"markov": dict(), "fastq": dict(flatten=1), "random": dict()}
MIX_CHAIN = 2


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes_per_group(st: dict) -> dict:
    """Bytes each kernel group must move at the least: its share of C + N + M.

    setup reads the stream prefix, block headers and chunk index; parse reads
    cmd/len/lvl/off and the literals and writes the literals; the level
    executor reads every match source and writes every match destination.
    Intermediate match records are not counted: they are this design's cost.
    """
    sec = st["sections"]
    return {
        "setup": sec["header"] + sec["block_headers"] + sec["chunk_index"],
        "parse": sec["cmd"] + sec["len"] + sec["lvl"] + sec["off"] + 2 * st["literal_bytes"],
        "levels": 2 * st["match_bytes"],
    }


def base_line(value, steps, warmup, ms):
    return {"metric": METRIC, "value": round(value, 3), "unit": "GB/s", "n_gpus": 1, "steps": steps,
            "warmup": warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u8", "data": "synthetic"}


def _free_gpu():
    import torch

    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _timed(fn, steps, warmup, stream):
    """Mean ms of fn over `steps` calls after `warmup`, HIP events on `stream`."""
    import torch

    for _ in range(warmup):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


# ------------------------------------------------------------------ plain


def measure_plain(name, args, with_plan=True, x=None):
    """One plain workload: eager aceapex_decode with per-group kernel timing,
    then a plan of the one stream (autotuned, replayed as a captured graph).
    Returns (entry dict, host stream, original bytes)."""
    import torch

    import synth
    import paper_2606_04268_amd as ax
    from paper_2606_04268_amd import _abi
    from paper_2606_04268_amd.profiling import load_traffic
    from paper_2606_04268_amd.stats import stream_stats

    wl = WORKLOADS[name]
    t0 = time.perf_counter()
    if x is None:
        x = synth.make(wl["kind"], wl["size"], wl["seed"])
        log(f"{name}: generated {x.size} bytes in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    s = ax.encode(x, threads=HOST_THREADS, verbose=1 if x.size >= (1 << 30) else 0, **wl["enc"])
    enc_s = time.perf_counter() - t0
    st = stream_stats(s)
    log(f"{name}: encoded to {s.size} bytes in {enc_s:.1f}s; {st['n_seq']} matches, max level {st['max_level']}")

    dev = torch.device("cuda:0")
    ds = ax.to_device(s, dev)
    x_dev = torch.from_numpy(x).to(dev)
    out = torch.empty(ds.n, dtype=torch.uint8, device=dev)
    ws = torch.empty(max(ax.workspace_bytes([ds]), 256), dtype=torch.uint8, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def step():
        ax.decode(ds, out=out, workspace=ws, status=status, stream=stream)

    out.fill_(0xA5)
    step()
    torch.cuda.synchronize()
    ax.check_status(status)
    assert torch.equal(out, x_dev), f"{name}: decode differs from the original bytes"
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    _abi.timing(True)
    ms = _timed(step, args.steps, 0, stream)
    groups = _abi.timing_read()
    _abi.timing(False)
    ax.check_status(status)
    mism, first = ax.compare(out, x_dev, stream=stream)  # k_cmp on the device, outside the timing
    exact = mism == 0
    host_hash = ax.content_hash(out.cpu().numpy())
    hash_ok = host_hash == ds.info.content_hash
    assert exact and hash_ok, f"{name}: decode is not bit-exact ({mism} bytes differ, first at {first})"

    C, N, M = st["comp_bytes"], st["decoded_bytes"], st["match_bytes"]
    roof = HBM_PEAK_GBPS * N / (C + N + M)
    alg = algorithmic_bytes_per_group(st)
    per_group = {k: {"ms_per_launch": v[0] / v[1], "launches": v[1]} for k, v in groups.items() if v[1]}
    dom = max((g for g in per_group if g in alg), key=lambda g: per_group[g]["ms_per_launch"])
    dom_ms = per_group[dom]["ms_per_launch"]
    achieved = alg[dom] / (dom_ms * 1e-3) / 1e9
    rec = load_traffic(os.path.join(ROOT, "profiles", f"traffic_{name}.md"))
    traffic = rec["groups"][dom]["traffic_bytes"] if rec and dom in rec["groups"] else None
    gbps = N / (ms * 1e-3) / 1e9
    entry = {
        "workload": wl["desc"], "gbps": round(gbps, 3), "ms_per_step": round(ms, 4), "path": "aceapex_decode",
        "decoded_bytes": N, "stream_bytes": C, "ratio": round(N / C, 4) if C else None, "blocks": st["n_blocks"],
        "matches": st["n_seq"], "deep_matches": st["n_deep"], "max_level": st["max_level"], "match_bytes": M,
        "literal_bytes": st["literal_bytes"], "chunks": st["n_chunks"], "encode_s": round(enc_s, 1),
        "bit_exact": {"device_compare": exact, "k_cmp_mismatches": mism, "xxh3_64": f"{host_hash:016x}",
                      "xxh3_matches_header": hash_ok},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 5), "traffic": traffic,
                     "algorithmic_bytes_per_launch": alg[dom], "ms_per_launch": round(dom_ms, 5),
                     "launch": "one decode's launches of the group (levels: every k_level and the k_tail)"},
        "decode_roofline": {"algorithmic_bytes": C + N + M, "decoded_roof_gbps": round(roof, 1),
                            "frac_of_decoded_roof": round(gbps / roof, 5)},
        "kernel_groups": {k: {"ms_per_launch": round(v["ms_per_launch"], 5), "launches": v["launches"]}
                          for k, v in per_group.items()},
        "paths": {"aceapex_decode": {"ms_per_step": round(ms, 4), "gbps": round(gbps, 3)}},
    }
    if with_plan:
        pg = plan_graph_leg(ds, out, ws, status, stream, x_dev, args)
        entry["paths"]["plan_graph_tuned"] = pg
        if pg["ms_per_step"] < ms:  # the faster of the two product paths is the entry's figure
            entry.update(gbps=pg["gbps"], ms_per_step=pg["ms_per_step"], path="plan_graph_tuned")
            entry["decode_roofline"]["frac_of_decoded_roof"] = round(pg["gbps"] / roof, 5)
    log(f"{name}: {entry['gbps']:.1f} GB/s ({entry['path']}, {entry['ms_per_step']:.3f} ms)")
    del ds, x_dev, out, ws, status
    _free_gpu()
    return entry, s, x


def plan_graph_leg(ds, out, ws, status, stream, x_dev, args) -> dict:
    """The same decode through a plan (laid out once, schedule autotuned),
    replayed as a captured HIP graph; timed like the eager path and checked."""
    import torch

    import paper_2606_04268_amd as ax

    plan = ax.Plan([ds], outs=[out], statuses=status, workspace=ws, stream=stream)
    try:
        tuned = plan.tune(reps=3, stream=stream)
        out.fill_(0xA5)
        plan.launch(stream=stream, graph=True)
        torch.cuda.synchronize()
        ax.check_status(status)
        assert torch.equal(out, x_dev), "plan decode differs from the original bytes"
        ms = _timed(lambda: plan.launch(stream=stream, graph=True), args.steps, args.warmup, stream)
        ax.check_status(status)
        assert torch.equal(out, x_dev), "plan decode differs from the original bytes"
    finally:
        plan.close()
    log(f"plan + graph, tuned {tuned}: {ms:.4f} ms per decode")
    return {"ms_per_step": round(ms, 4), "gbps": round(ds.n / (ms * 1e-3) / 1e9, 3), "tuning": tuned}


# ------------------------------------------------------------ level floor


def chain_input(levels: int, body: int = 16):
    """Bytes whose parse (most-recent tie-break) is a chain of `levels` levels
    with one match each: segment i is one unique byte then a fixed body, and
    each body is copied from the previous segment's body."""
    import numpy as np

    rng = np.random.default_rng(12345)
    b = rng.integers(0, 256, body, dtype=np.uint8)
    seg = np.empty((levels + 1, body + 4), dtype=np.uint8)
    idx = np.arange(levels + 1, dtype=np.uint32)
    seg[:, :4] = idx.view(np.uint8).reshape(-1, 4) ^ np.uint8(0x80)  # unique 4-byte prefix per segment
    seg[:, 4:] = b
    return seg.reshape(-1)


def level_floor(args):
    """Cost of one level boundary: a chain of one-match levels decoded by a
    plan replayed as a graph, once with every level its own launch (the
    kernel boundary between levels) and once with the levels in the one-
    workgroup tail (a workgroup barrier between levels)."""
    import torch

    import paper_2606_04268_amd as ax

    L = 1024
    x = chain_input(L)
    s = ax.encode(x, tiebreak=1, block_log2=20, hash_bits=16)
    ds = ax.to_device(s)
    levels = int(ds.info.max_level) + 1
    stream = torch.cuda.current_stream()
    x_dev = torch.from_numpy(x).cuda()
    res = {"levels": levels, "matches": int(ds.info.n_seq)}
    for label, tail in (("launch_per_level", 0), ("tail_per_level", 1 << 20)):
        out = torch.empty(ds.n, dtype=torch.uint8, device="cuda")
        plan = ax.Plan([ds], outs=[out], stream=stream, tuning=dict(tail_level_max=tail))
        try:
            plan.launch(stream=stream, graph=True)
            torch.cuda.synchronize()
            ax.check_status(plan.statuses)
            assert torch.equal(out, x_dev), "level-floor chain decodes wrongly"
            ms = _timed(lambda: plan.launch(stream=stream, graph=True), 10, 2, stream)
        finally:
            plan.close()
        res[label + "_us"] = round(ms * 1e3 / levels, 3)
    log(f"level floor: {res}")
    _free_gpu()
    return res


# ----------------------------------------------------------- CPU baseline


def cpu_baseline(x_sample, enc, sample_desc, runs=3) -> dict:
    """The oracle's decoders on the host cores: the sequential decoder, and the
    block-parallel one at T = 1, 2, 4, 8, 16 threads, with the host's memcpy
    bandwidth at the same T; best and median of `runs` runs each."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle
    import paper_2606_04268_amd as ax

    s = ax.encode(x_sample, threads=HOST_THREADS, **enc)
    n = x_sample.size
    out = np.empty(n, dtype=np.uint8)
    out[:] = 0
    visible = len(os.sched_getaffinity(0))
    ts = [t for t in (1, 2, 4, 8, 16) if t <= max(1, visible)]

    def stats(times):
        g = sorted(n / t / 1e9 for t in times)
        return {"best_gbps": round(g[-1], 3), "median_gbps": round(g[len(g) // 2], 3)}

    def timed(fn):
        res = []
        for _ in range(runs):
            t0 = time.perf_counter()
            fn()
            res.append(time.perf_counter() - t0)
        return res

    seq = stats(timed(lambda: oracle.decode_into(s, out, 1)))
    assert np.array_equal(out, x_sample), "oracle decode differs from the original"
    sweep = {}
    src = np.ascontiguousarray(x_sample)
    dst = np.empty_like(src)
    for t in ts:
        d = stats(timed(lambda: oracle.decode_into(s, out, t)))
        assert np.array_equal(out, x_sample), "oracle decode differs from the original"
        parts = np.array_split(np.arange(n), t)
        bounds = [(int(p[0]), int(p[-1]) + 1) for p in parts if p.size]
        with ThreadPoolExecutor(t) as ex:
            def copy_all():
                list(ex.map(lambda ab: np.copyto(dst[ab[0]:ab[1]], src[ab[0]:ab[1]]), bounds))
            copy_all()
            mc = stats(timed(copy_all))
        sweep[str(t)] = {"decode_mt": d, "memcpy": mc,
                         "decode_over_memcpy": round(d["best_gbps"] / mc["best_gbps"], 4)}
        log(f"cpu T={t}: decode_mt {d['best_gbps']:.2f} GB/s, memcpy {mc['best_gbps']:.1f} GB/s")
    log(f"cpu sequential: {seq['best_gbps']:.2f} GB/s")
    best_t = max(sweep, key=lambda k: sweep[k]["decode_mt"]["best_gbps"])
    if sweep[best_t]["decode_mt"]["best_gbps"] > seq["best_gbps"]:
        value, cores, which = sweep[best_t]["decode_mt"]["best_gbps"], int(best_t), f"block-parallel, {best_t} threads"
    else:
        value, cores, which = seq["best_gbps"], 1, "sequential, 1 thread"
    model = "?"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "?")
    except OSError:
        pass
    return {"value": value, "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"{sample_desc} ({n} decoded bytes); best of {runs} runs per decoder and thread count; "
                      f"value = the faster oracle decoder ({which})",
            "sequential": seq, "threads_sweep": sweep, "host_cpu": model, "host_threads_visible": visible}


# ---------------------------------------------------------- pools (mixes)


def build_pool(recipe, chain_depth=MIX_CHAIN):
    """Generate and encode the (kind, size, seed) recipe on the host cores;
    returns [(original, stream)] in recipe order."""
    from concurrent.futures import ThreadPoolExecutor

    import synth
    import paper_2606_04268_amd as ax

    def one(r):
        kind, size, seed = r
        x = synth.make(kind, size, seed)
        return x, ax.encode(x, threads=2, chain_depth=chain_depth, **MIX_ENC[kind])

    t0 = time.perf_counter()
    order = sorted(range(len(recipe)), key=lambda i: -recipe[i][1])
    res = [None] * len(recipe)
    done_bytes, last = 0, time.perf_counter()
    with ThreadPoolExecutor(HOST_THREADS) as ex:
        for i, r in zip(order, ex.map(one, [recipe[i] for i in order])):
            res[i] = r
            done_bytes += recipe[i][1]
            if time.perf_counter() - last > 10:
                last = time.perf_counter()
                log(f"pool: {done_bytes / 1e9:.2f} GB encoded after {last - t0:.0f}s")
    tot = sum(r[1] for r in recipe)
    log(f"pool: {len(recipe)} streams, {tot / 1e9:.2f} GB decoded, generated and encoded in "
        f"{time.perf_counter() - t0:.1f}s on {HOST_THREADS} threads")
    return res


def measure_batched(args):
    """Config 3: independent streams decoded as one batch, three ways."""
    import numpy as np
    import torch

    import synth
    import paper_2606_04268_amd as ax
    from paper_2606_04268_amd import _abi
    from paper_2606_04268_amd.stats import stream_stats

    dev = torch.device("cuda:0")
    recipe = synth.mix_recipe(args.streams, 4 << 10, 64 << 20, 0xACE3)
    pool = build_pool(recipe)
    st = [stream_stats(s) for _, s in pool]
    dss = [ax.to_device(s, dev) for _, s in pool]
    origs = [torch.from_numpy(x).to(dev) for x, _ in pool]
    del pool
    gc.collect()
    sizes = [d.n for d in dss]
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([(n + 255) // 256 * 256 for n in sizes])
    total = int(sum(sizes))
    out = torch.empty(max(int(offs[-1]), 256), dtype=torch.uint8, device=dev)
    outs = [out[int(offs[j]):int(offs[j]) + max(sizes[j], 1)] for j in range(len(sizes))]
    statuses = torch.zeros(len(sizes), dtype=torch.int32, device=dev)
    descs = [_abi.Desc(d.abi(), o.data_ptr(), o.numel(), statuses.data_ptr() + 4 * j)
             for j, (d, o) in enumerate(zip(dss, outs))]
    ws_bytes = _abi.workspace_bytes(descs)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    log(f"batched: {len(descs)} independent streams, {total / 1e9:.2f} GB decoded per call, "
        f"workspace {ws_bytes / 1e9:.2f} GB")
    stream = torch.cuda.current_stream(dev)
    single_ws = torch.empty(max(max(ax.workspace_bytes([d]) for d in dss), 256), dtype=torch.uint8, device=dev)

    def batched():
        rc = _abi.decode_many(descs, ws.data_ptr(), ws.numel(), stream.cuda_stream)
        if rc:
            raise _abi.AceapexError(rc, "decode_many")

    def loop():
        for j, d in enumerate(descs):
            rc = _abi.decode(d.s, outs[j].data_ptr(), outs[j].numel(), single_ws.data_ptr(), single_ws.numel(),
                             statuses.data_ptr() + 4 * j, stream.cuda_stream)
            if rc:
                raise _abi.AceapexError(rc, "decode")

    def verify(label):
        torch.cuda.synchronize()
        ax.check_status(statuses)
        for j in range(len(dss)):
            mism, first = ax.compare(outs[j][:sizes[j]], origs[j], stream=stream)
            if mism:
                raise AssertionError(f"{label}: stream {j} differs from its original ({mism} bytes, first at {first})")

    plan_box = {}

    def plan_graph():
        plan_box["plan"].launch(stream=stream, graph=True)

    res = {}
    steps = max(1, min(args.steps, args.batched_steps))
    for label, fn in (("per_stream_loop", loop), ("decode_many", batched), ("plan_graph_tuned", plan_graph)):
        if label == "plan_graph_tuned":
            plan = ax.Plan(dss, outs=outs, statuses=statuses, workspace=ws, stream=stream)
            t0 = time.perf_counter()
            plan_box.update(plan=plan, tuning=plan.tune(reps=1, stream=stream))
            log(f"autotuned schedule {plan_box['tuning']} in {time.perf_counter() - t0:.1f}s")
        out.fill_(0xA5)
        statuses.fill_(12345)
        fn()
        verify(label)
        _abi.timing(True)
        ms = _timed(fn, steps, 1, stream)
        groups = _abi.timing_read()
        _abi.timing(False)
        verify(label)
        res[label] = {"ms_per_call": round(ms, 3), "gbps": round(total / (ms * 1e-3) / 1e9, 3),
                      "kernel_groups": {k: {"ms_per_call": round(v[0] / (steps + 1), 4),
                                            "launches_per_call": v[1] / (steps + 1)}
                                        for k, v in groups.items() if v[1]}}
        log(f"batched {label}: {ms:.2f} ms per call, {res[label]['gbps']:.1f} GB/s")
    plan_box["plan"].close()
    C = sum(x["comp_bytes"] for x in st)
    M = sum(x["match_bytes"] for x in st)
    roof = HBM_PEAK_GBPS * total / (C + total + M)
    b = res["plan_graph_tuned"]
    entry = {
        "workload": (f"{len(descs)} independent streams, sizes log-uniform 4 KiB..64 MiB, 40% order-2 Markov text "
                     "/ 40% FASTQ-like (flattened) / 20% random bytes with 30% repeats, each stream seeded by "
                     f"SplitMix64(0xACE3 ^ i); encoded with hash-chain depth {MIX_CHAIN}"),
        "gbps": b["gbps"], "ms_per_call": b["ms_per_call"], "path": "plan_graph_tuned",
        "streams": len(descs), "decoded_bytes": total, "stream_bytes": C, "match_bytes": M,
        "matches": int(sum(x["n_seq"] for x in st)), "max_level": int(max(x["max_level"] for x in st)),
        "decode_roofline": {"decoded_roof_gbps": round(roof, 1), "frac_of_decoded_roof": round(b["gbps"] / roof, 5)},
        "bit_exact": {"device_compare": True, "statuses_zero": True},
        "plan_graph_tuned": dict(b, tuning=plan_box["tuning"]), "decode_many": res["decode_many"],
        "per_stream_loop": res["per_stream_loop"],
        "speedup_vs_loop": round(res["per_stream_loop"]["ms_per_call"] / b["ms_per_call"], 3),
    }
    del dss, origs, out, outs, ws, single_ws, statuses, descs
    _free_gpu()
    return entry


def measure_served(args, loads, warm_requests=300, measured_requests=3000, level_us=None):
    """Config 4: Poisson arrivals at each offered load, served three ways:
    continuous batching on the GPU, continuous batching with each request
    routed to the GPU or the host decoder by the cost model (its host rate
    calibrated on the pool, its per-level cost the measured level floor), and
    one request at a time on the GPU."""
    import numpy as np
    import torch

    import synth
    import paper_2606_04268_amd as ax
    from paper_2606_04268_amd.serve import CostModel, Server, poisson_arrivals, summarize

    dev = torch.device("cuda:0")
    recipe = synth.mix_recipe(args.pool, 64 << 10, 256 << 20, 0xACE4)
    pool = build_pool(recipe)
    dss = [ax.to_device(s, dev) for _, s in pool]
    mean = float(np.mean([d.n for d in dss]))
    budget = 200 * 10**9
    cost = CostModel(gpu_level_us=level_us) if level_us else CostModel()
    srv = Server(dss, budget_bytes=budget, lanes=4, max_batch=256, device=dev,
                 host_streams=[s for _, s in pool], cpu_workers=4, cost=cost)
    cpu_gbps = srv.calibrate_cpu()
    log(f"served: pool of {len(dss)} streams, mean {mean / 1e6:.1f} MB; budget {budget / 1e9:.0f} GB, "
        f"lane workspace {srv.lane_ws / 1e9:.1f} GB x {len(srv.lanes)}; host decoder {cpu_gbps:.2f} GB/s")
    # every pool stream once through the server, checked against its original
    warm = srv.run([(0.0, i) for i in range(len(dss))], keep_outputs=True)
    for r in warm:
        if r.status or not np.array_equal(r.result, pool[r.stream][0]):
            raise AssertionError(f"served decode of pool stream {r.stream} is not exact")
    # and once through the host decoder, for the streams the cost model sends there
    cpu_picks = [i for i in range(len(dss)) if srv.route_of(i, "auto") == "cpu"]
    if cpu_picks:
        warm = srv.run([(0.0, i) for i in cpu_picks], keep_outputs=True, route="cpu")
        for r in warm:
            if r.status or not np.array_equal(r.result, pool[r.stream][0]):
                raise AssertionError(f"host-decoded pool stream {r.stream} is not exact")
    del warm, pool
    gc.collect()
    rows = []
    for li, load in enumerate(loads):
        rate = load * 1e9 / mean
        arr = poisson_arrivals(warm_requests + measured_requests, rate, len(dss), seed=0xACE5 + li)
        row = {"offered_gbps": load, "requests": measured_requests, "warmup_requests": warm_requests}
        for mode, route in (("continuous", "gpu"), ("auto", "auto"), ("fifo", "gpu")):
            reqs = srv.run(arr, mode="fifo" if mode == "fifo" else "continuous", timeout_s=300, route=route)
            reqs = sorted(reqs, key=lambda r: r.arrival)[warm_requests:]
            s = summarize(reqs, dss)
            if s["errors"]:
                raise AssertionError(f"{s['errors']} served requests failed at {load} GB/s ({mode})")
            row[mode] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in s.items()}
            log(f"served {load:.0f} GB/s {mode}: p50 {s['p50_ms']:.2f} ms p99 {s['p99_ms']:.2f} ms, "
                f"{s['aggregate_gbps']:.1f} GB/s")
        rows.append(row)
    info = {"workload": (f"Poisson arrivals of requests drawn uniformly from a pool of {len(dss)} resident streams "
                         "(sizes log-uniform 64 KiB..256 MiB, 40% Markov text / 40% FASTQ-like / 20% random with "
                         f"repeats, hash-chain depth {MIX_CHAIN}); 200 GB device-memory budget, inputs and outputs "
                         "resident; continuous batching on 4 HIP streams (GPU only, and with each request routed "
                         "to the GPU or the host decoder by size and deepest level) vs one request at a time"),
            "pool_streams": len(dss), "mean_request_bytes": round(mean), "budget_bytes": budget,
            "cost_model": {"cpu_gbps": round(cost.cpu_gbps, 3), "gpu_gbps": cost.gpu_gbps,
                           "gpu_fixed_us": cost.gpu_fixed_us, "gpu_level_us": cost.gpu_level_us},
            "pool_streams_routed_to_host": len(cpu_picks)}
    del srv, dss
    _free_gpu()
    return info, rows


# ------------------------------------------------------------------ entropy stage


def measure_entropy(stream, name, args):
    """The tANS stage on the literal stream of a workload: host-encoded with
    2^11 table entries and one lane per ~512 literals, decoded on the GPU
    (table build + lane decode), checked byte for byte.  GB/s counts the
    decoded literal bytes."""
    import numpy as np
    import torch

    import paper_2606_04268_amd as ax
    from paper_2606_04268_amd import _abi
    from paper_2606_04268_amd.stats import literals

    lit = literals(stream)
    lanes = int(min(1 << 20, max(1, lit.size // 512)))
    t0 = time.perf_counter()
    c = _abi.tans_encode(lit, 11, lanes)
    enc_s = time.perf_counter() - t0
    p = np.bincount(lit, minlength=256).astype(np.float64) / max(1, lit.size)
    h0 = float(-(p[p > 0] * np.log2(p[p > 0])).sum())
    dev = torch.device("cuda:0")
    d_in = torch.from_numpy(c).to(dev)
    ref = torch.from_numpy(lit).to(dev)
    info = _abi.tans_probe(c)
    out = torch.empty(max(lit.size, 1), dtype=torch.uint8, device=dev)
    ws = torch.empty(max(_abi.tans_workspace_bytes(info), 256), dtype=torch.uint8, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    stream_ = torch.cuda.current_stream(dev)

    def step():
        ax.tans_decode((d_in, c[:544]), out=out, workspace=ws, status=status, stream=stream_)

    step()
    torch.cuda.synchronize()
    ax.check_status(status)
    exact = bool(torch.equal(out[:lit.size], ref))
    assert exact, f"{name}: tANS decode differs from the literals"
    ms = _timed(step, args.steps, 2, stream_)
    ax.check_status(status)
    return {"workload": f"lit[] of the {name} stream", "literal_bytes": int(lit.size), "container_bytes": int(c.size),
            "bits_per_byte": round(8 * c.size / max(1, lit.size), 3), "order0_entropy_bits": round(h0, 3),
            "table_log": 11, "lanes": lanes, "ms_per_decode": round(ms, 4),
            "gbps": round(lit.size / (ms * 1e-3) / 1e9, 2), "bit_exact": exact, "host_encode_s": round(enc_s, 2)}


# ------------------------------------------------------------------ modes


def run_full(args):
    """The default line (see the module text)."""
    t_start = time.perf_counter()
    main_entry, s_main, x_wiki = measure_plain("wiki1g", args)
    floor = level_floor(args)
    d8, _, _ = measure_plain("wiki1g_d8", args, x=x_wiki)
    del s_main
    sample = x_wiki[: args.cpu_sample_mib << 20].copy()
    del x_wiki
    gc.collect()
    others = {}
    for name in ("markov4", "fastq256"):
        others[name], s_other, _ = measure_plain(name, args)
        if name == "fastq256":
            entropy = measure_entropy(s_other, name, args)
        del s_other
    cpu = None if args.no_cpu else cpu_baseline(
        sample, WORKLOADS["wiki1g"]["enc"],
        f"the first {args.cpu_sample_mib} MiB of the same wiki-like text, encoded the same way")
    del sample
    gc.collect()
    batched = None if args.no_batched else measure_batched(args)
    served = None
    if not args.no_served:
        info, rows = measure_served(args, [args.fixed_load], level_us=floor["launch_per_level_us"])
        r = rows[0]
        served = dict(info, offered_gbps=args.fixed_load, p50_ms=r["continuous"]["p50_ms"],
                      p99_ms=r["continuous"]["p99_ms"], aggregate_gbps=r["continuous"]["aggregate_gbps"],
                      auto_p50_ms=r["auto"]["p50_ms"], auto_p99_ms=r["auto"]["p99_ms"],
                      auto_gbps=r["auto"]["aggregate_gbps"], auto_routes=r["auto"]["routes"],
                      fifo_p50_ms=r["fifo"]["p50_ms"], fifo_p99_ms=r["fifo"]["p99_ms"],
                      fifo_gbps=r["fifo"]["aggregate_gbps"], requests=r["requests"],
                      warmup_requests=r["warmup_requests"])

    e = main_entry
    line = base_line(e["gbps"], args.steps, args.warmup, e["ms_per_step"])
    line["config"] = {"workload": e["workload"], "decoded_bytes": e["decoded_bytes"],
                      "stream_bytes": e["stream_bytes"], "blocks": e["blocks"], "matches": e["matches"],
                      "deep_matches": e["deep_matches"], "max_level": e["max_level"],
                      "match_bytes": e["match_bytes"], "literal_bytes": e["literal_bytes"], "chunks": e["chunks"]}
    line["value_path"] = e["path"]
    for k in ("bit_exact", "roofline", "decode_roofline", "kernel_groups", "paths"):
        line[k] = e[k]
    line["sync_floor"] = {
        "level_launch_us": floor["launch_per_level_us"], "tail_level_us": floor["tail_per_level_us"],
        "measured_on": f"a chain of {floor['levels']} levels with one match each, plan replayed as a graph",
        "per_stream_ms": {n: round((v["max_level"] + 1) * floor["launch_per_level_us"] * 1e-3, 3)
                          for n, v in (("wiki1g", e), ("wiki1g_d8", d8), ("markov4", others["markov4"]),
                                       ("fastq256", others["fastq256"]))},
    }
    line["depth_limited"] = d8
    line["configs"] = others
    line["entropy_stage"] = entropy
    if batched:
        line["batched"] = batched
    if served:
        line["served"] = served
    if cpu:
        line["cpu_baseline"] = cpu
    line["host_seconds"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(line), flush=True)


def run_plain(args):
    e, s, x = measure_plain(args.workload, args, with_plan=not args.no_plan)
    line = base_line(e["gbps"], args.steps, args.warmup, e["ms_per_step"])
    line["config"] = {k: e[k] for k in ("workload", "decoded_bytes", "stream_bytes", "blocks", "matches",
                                        "deep_matches", "max_level", "match_bytes", "literal_bytes", "chunks")}
    line["value_path"] = e["path"]
    for k in ("bit_exact", "roofline", "decode_roofline", "kernel_groups", "paths"):
        line[k] = e[k]
    if not args.no_cpu:
        n = min(x.size, args.cpu_sample_mib << 20)
        line["cpu_baseline"] = cpu_baseline(x[:n].copy(), WORKLOADS[args.workload]["enc"],
                                            f"the first {n >> 20} MiB of the same input, encoded the same way")
    print(json.dumps(line), flush=True)


def run_entropy(args):
    import synth
    import paper_2606_04268_amd as ax

    wl = WORKLOADS[args.workload]
    x = synth.make(wl["kind"], wl["size"], wl["seed"])
    s = ax.encode(x, threads=HOST_THREADS, **wl["enc"])
    del x
    e = measure_entropy(s, args.workload, args)
    line = base_line(e["gbps"], args.steps, 2, e["ms_per_decode"])
    line["metric"] = "tANS-decoded literal GB/s"
    line["config"] = {"workload": e["workload"]}
    line["entropy_stage"] = e
    print(json.dumps(line), flush=True)


def run_derive(args):
    """One workload encoded in the four sections of Sec. 3.2 only (no stored
    levels), decoded with aceapex_decode, which derives every match's level
    on the device while the wavefront runs (it reads a counter back every few
    levels, so a decode includes those host round trips); beside it the same
    text with stored levels."""
    import torch

    import synth
    import paper_2606_04268_amd as ax

    wl = WORKLOADS[args.workload]
    x = synth.make(wl["kind"], wl["size"], wl["seed"])
    dev = torch.device("cuda:0")
    x_dev = torch.from_numpy(x).to(dev)
    stream = torch.cuda.current_stream(dev)
    res = {}
    for label, levels in (("derived", 0), ("stored", 1)):
        s = ax.encode(x, threads=HOST_THREADS, levels=levels, **wl["enc"])
        ds = ax.to_device(s, dev)
        out = torch.empty(ds.n, dtype=torch.uint8, device=dev)
        ws = torch.empty(max(ax.workspace_bytes([ds]), 256), dtype=torch.uint8, device=dev)
        status = torch.zeros(1, dtype=torch.int32, device=dev)

        def step():
            ax.decode(ds, out=out, workspace=ws, status=status, stream=stream)

        step()
        torch.cuda.synchronize()
        ax.check_status(status)
        mism, first = ax.compare(out, x_dev, stream=stream)
        assert mism == 0, f"{label}: {mism} bytes differ, first at {first}"
        ms = _timed(step, args.steps, args.warmup, stream)
        ax.check_status(status)
        assert ax.compare(out, x_dev, stream=stream)[0] == 0
        res[label] = {"ms_per_decode": round(ms, 4), "gbps": round(ds.n / (ms * 1e-3) / 1e9, 2),
                      "stream_bytes": int(s.size), "max_level": int(ds.info.max_level)}
        del ds, out, ws
        _free_gpu()
    line = base_line(res["derived"]["gbps"], args.steps, args.warmup, res["derived"]["ms_per_decode"])
    line["metric"] = "decoded GB/s with levels derived on the device (four-section streams)"
    line["config"] = {"workload": wl["desc"] + "; encoded without stored levels"}
    line["derive"] = res
    print(json.dumps(line), flush=True)


def run_batched(args):
    b = measure_batched(args)
    line = base_line(b["gbps"], max(1, min(args.steps, args.batched_steps)), 1, b["ms_per_call"])
    line["config"] = {"workload": "batched: " + b["workload"], "streams": b["streams"],
                      "decoded_bytes": b["decoded_bytes"]}
    line["batched"] = b
    print(json.dumps(line), flush=True)


def run_served(args):
    loads = sorted({float(v) for v in args.loads.split(",")} | {args.fixed_load})
    info, rows = measure_served(args, loads)
    fixed = next(r for r in rows if r["offered_gbps"] == args.fixed_load)
    c = fixed["continuous"]
    line = base_line(c["aggregate_gbps"], len(rows), 1, c["mean_ms"])
    line["config"] = dict(info, workload="served: " + info["workload"] +
                          f"; value = decoded GB/s at {args.fixed_load:.0f} GB/s offered")
    line["served_at_fixed_load"] = {"offered_gbps": args.fixed_load, "p50_ms": c["p50_ms"], "p99_ms": c["p99_ms"],
                                    "auto_p50_ms": fixed["auto"]["p50_ms"], "auto_p99_ms": fixed["auto"]["p99_ms"],
                                    "auto_routes": fixed["auto"]["routes"],
                                    "fifo_p50_ms": fixed["fifo"]["p50_ms"], "fifo_p99_ms": fixed["fifo"]["p99_ms"],
                                    "fifo_gbps": fixed["fifo"]["aggregate_gbps"]}
    line["sweep"] = rows
    line["note"] = "steps = number of offered loads; ms_per_step = mean request latency at the fixed load"
    print(json.dumps(line), flush=True)


def print_algorithmic(args):
    """Algorithmic bytes per kernel group of the workload's stream (JSON), for
    the traffic summaries of the counter runs."""
    import synth
    import paper_2606_04268_amd as ax
    from paper_2606_04268_amd.stats import stream_stats

    wl = WORKLOADS[args.workload]
    s = ax.encode(synth.make(wl["kind"], wl["size"], wl["seed"]), threads=HOST_THREADS, **wl["enc"])
    print(json.dumps(algorithmic_bytes_per_group(stream_stats(s))))


def run_sweep(args):
    """Depth limit D x chain flattening on two content kinds: for each stream,
    the ratio (original / stream bytes), the deepest level and the decoded
    GB/s of a plan replayed as a HIP graph, each decode checked byte for byte."""
    import torch

    import synth
    import paper_2606_04268_amd as ax

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    rows = []
    for kind, seed in (("wiki", 0xACE2), ("fastq", 0xACE1)):
        x = synth.make(kind, args.sweep_mib << 20, seed)
        x_dev = torch.from_numpy(x).to(dev)
        for depth in (1, 2, 10, 0):
            for flatten in (0, 1, 2):
                t0 = time.perf_counter()
                s = ax.encode(x, max_depth=depth, flatten=flatten, threads=HOST_THREADS)
                enc_s = time.perf_counter() - t0
                ds = ax.to_device(s, dev)
                out = torch.empty(ds.n, dtype=torch.uint8, device=dev)
                status = torch.zeros(1, dtype=torch.int32, device=dev)
                plan = ax.Plan([ds], [out], status, stream=stream)
                try:
                    plan.launch(stream=stream, graph=True)
                    torch.cuda.synchronize()
                    ax.check_status(status)
                    if not torch.equal(out, x_dev):
                        raise AssertionError(f"sweep {kind} D={depth} flatten={flatten}: decode differs")
                    ms = _timed(lambda: plan.launch(stream=stream, graph=True), args.steps, max(1, args.warmup),
                                stream)
                    ax.check_status(status)
                    if not torch.equal(out, x_dev):
                        raise AssertionError(f"sweep {kind} D={depth} flatten={flatten}: timed decode differs")
                finally:
                    plan.close()
                row = {"kind": kind, "depth_limit": depth or None, "flatten": ["off", "R1", "R2"][flatten],
                       "ratio": round(x.size / s.size, 4), "max_level": int(ds.info.max_level),
                       "ms": round(ms, 4), "gbps": round(x.size / (ms * 1e-3) / 1e9, 2), "encode_s": round(enc_s, 1)}
                rows.append(row)
                log(f"sweep: {row}")
                del out, ds
    best = max(rows, key=lambda r: r["gbps"])
    line = base_line(best["gbps"], args.steps, args.warmup, best["ms"])
    line["config"] = {"workload": f"sweep: wiki-like text and FASTQ-like data, {args.sweep_mib} MiB each; depth "
                                  "limit 1/2/10/unlimited x flattening off/R1/R2; value = the fastest stream"}
    line["bit_exact"] = {"device_compare": True}
    line["sweep"] = rows
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="full", choices=["full", "plain", "batched", "served", "sweep", "algorithmic", "entropy", "derive"])
    ap.add_argument("--workload", default="wiki1g", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plan", action="store_true", help="plain mode: skip the plan + graph leg")
    ap.add_argument("--no-batched", action="store_true", help="full mode: skip the batched entry")
    ap.add_argument("--no-served", action="store_true", help="full mode: skip the served entry")
    ap.add_argument("--cpu-sample-mib", type=int, default=64, help="MiB of input the CPU oracle decodes")
    ap.add_argument("--sweep-mib", type=int, default=32, help="sweep: MiB per workload")
    ap.add_argument("--streams", type=int, default=4096, help="batched: independent streams")
    ap.add_argument("--batched-steps", type=int, default=3, help="batched: timed calls per path, at most")
    ap.add_argument("--pool", type=int, default=256, help="served: streams in the resident pool")
    ap.add_argument("--loads", default="10,25,50,100,150,200", help="served mode: offered GB/s sweep")
    ap.add_argument("--fixed-load", type=float, default=100.0, help="served: the load the line reports")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "streams are independent, so several GPUs would each decode their own streams "
              "with no communication", file=sys.stderr)
        sys.exit(2)
    {"full": run_full, "plain": run_plain, "batched": run_batched, "served": run_served, "sweep": run_sweep,
     "algorithmic": print_algorithmic, "entropy": run_entropy, "derive": run_derive}[args.mode](args)


if __name__ == "__main__":
    main()
