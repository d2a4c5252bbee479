"""Host-side checks of the profiler summaries that bench.py reads: counter
calibration against a copy of known size, per-decode grouping of kernel
dispatches, the source hash that keeps a stale traffic record out of the
bench line, and kernel labels.  Synthetic CSVs stand in for rocprofv3 output."""
import csv
import json
import os
import types

import pytest

from paper_2606_04268_amd import profiling

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
K = {
    "setup": "(anonymous namespace)::k_setup((anonymous namespace)::Batch)",
    "parse": "void (anonymous namespace)::k_parse<false, 256u, 7680u>((anonymous namespace)::Batch)",
    "level1": "void (anonymous namespace)::k_level<false, 1u>((anonymous namespace)::Batch, unsigned int)",
    "level2": "void (anonymous namespace)::k_level<false, 2u>((anonymous namespace)::Batch, unsigned int)",
    "tail": "void (anonymous namespace)::k_tail<false>((anonymous namespace)::Batch, unsigned int)",
    "count": "(anonymous namespace)::k_count((anonymous namespace)::Batch)",
    "oapply": "(anonymous namespace)::k_oapply((anonymous namespace)::Batch)",
    "parse_ord": "void (anonymous namespace)::k_parse<false, 256u, 7680u, true>((anonymous namespace)::Batch)",
    "copy": "__amd_rocclr_copyBuffer",
    "other": "void at::native::vectorized_elementwise_kernel<16, at::native::FillFunctor<unsigned char>>(int)",
}


def write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=FIELDS)
        w.writeheader()
        for i, (kernel, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": K[kernel], "Counter_Name": counter,
                        "Counter_Value": value})
    return d


def decode_rows(scale):
    # one decode: setup, parse, three level launches of both shapes and the tail
    return [("setup", 10 * scale), ("parse", 1000 * scale), ("level2", 300 * scale), ("level2", 200 * scale),
            ("level1", 50 * scale), ("tail", 5 * scale)]


def test_kernel_names_and_groups():
    assert profiling._short(K["parse"]) == "k_parse"
    assert profiling._short(K["level1"]) == "k_level"
    assert profiling._short(K["setup"]) == "k_setup"
    assert profiling._label(K["level1"]) == "k_level<false, 1u>"
    assert profiling._label(K["tail"]) == "k_tail<false>"
    assert profiling._label(K["setup"]) == "k_setup"
    assert profiling._short(K["copy"]) == "__amd_rocclr_copyBuffer"
    assert {profiling.GROUP_OF[profiling._short(K[k])] for k in ("level1", "level2", "tail")} == {"levels"}


def test_ordered_slot_kernels_count_as_parse(tmp_path):
    """The slot count and scan kernels before an ordered-slot parse belong to
    the parse group of the same decode."""
    assert profiling._label(K["parse_ord"]) == "k_parse<false, 256u, 7680u, true>"
    one = [("setup", 10), ("count", 40), ("oapply", 5), ("parse_ord", 900), ("level2", 300), ("tail", 5)]
    d = write_counters(str(tmp_path / "fetch"), "FETCH_SIZE", one + one)
    r = profiling.per_decode(d, "FETCH_SIZE")
    assert r["decodes"] == 2 and r["dispatches_per_decode"] == 6
    assert r["parse"] == pytest.approx(945) and r["levels"] == pytest.approx(305)


def test_calibration_scales_a_copy_of_one_gib_to_one_gib(tmp_path):
    # the copy kernel reads 1 GiB; a counter that reports half of it in KiB gives factor 2
    d = write_counters(str(tmp_path / "cal"), "FETCH_SIZE",
                       [("other", 7), ("copy", (1 << 20) / 2), ("copy", (1 << 20) / 2 - 3)])
    f = profiling.calibration(d, "FETCH_SIZE")
    assert f == pytest.approx(2.0 * 1024)  # bytes per KiB unit read
    with pytest.raises(SystemExit):
        profiling.calibration(write_counters(str(tmp_path / "none"), "FETCH_SIZE", [("other", 1)]), "FETCH_SIZE")


def test_per_decode_groups_every_dispatch_of_each_decode(tmp_path):
    rows = [("other", 99)] + decode_rows(1) + [("other", 99)] + decode_rows(3)
    d = write_counters(str(tmp_path / "fetch"), "FETCH_SIZE", rows)
    r = profiling.per_decode(d, "FETCH_SIZE")
    assert r["decodes"] == 2
    assert r["dispatches_per_decode"] == 6
    # the mean of the two decodes, kernels outside the decode path ignored
    assert r["setup"] == pytest.approx(20)
    assert r["parse"] == pytest.approx(2000)
    assert r["levels"] == pytest.approx(555 * 2)


def test_summary_round_trip_and_stale_source(tmp_path, monkeypatch):
    cal = write_counters(str(tmp_path / "calf"), "FETCH_SIZE", [("copy", 1 << 20)])
    calw = write_counters(str(tmp_path / "calw"), "WRITE_SIZE", [("copy", 1 << 20)])
    fetch = write_counters(str(tmp_path / "f"), "FETCH_SIZE", decode_rows(1))
    write = write_counters(str(tmp_path / "w"), "WRITE_SIZE", decode_rows(2))
    out = str(tmp_path / "traffic.md")
    args = types.SimpleNamespace(cal_fetch=cal, cal_write=calw, fetch=fetch, write=write,
                                 algorithmic=json.dumps({"setup": 1000, "parse": 2000, "levels": 4000}),
                                 title="t", workload="w", key="k", command=["cmd"], out=out)
    profiling.summarize(args)
    rec = profiling.load_traffic(out)
    assert rec is not None and rec["workload"] == "k"
    lv = rec["groups"]["levels"]
    # counters in KiB with a factor of 1: bytes = KiB * 1024
    assert lv["fetch_bytes"] == 555 * 1024 and lv["write_bytes"] == 1110 * 1024
    assert lv["traffic_bytes"] == lv["fetch_bytes"] + lv["write_bytes"]
    assert lv["traffic_over_algorithmic"] == pytest.approx(round(1665 * 1024 / 4000, 3))
    # a record taken on another version of the kernel source is not returned
    monkeypatch.setattr(profiling, "source_sha256", lambda: "0" * 64)
    assert profiling.load_traffic(out) is None
    assert profiling.load_traffic(str(tmp_path / "missing.md")) is None


def test_committed_summary_parses():
    path = os.path.join(os.path.dirname(profiling.HERE), "profiles", "traffic_fastq256.md")
    with open(path) as f:
        text = f.read()
    assert "<!-- traffic: " in text
    rec = json.loads(text.split("<!-- traffic: ", 1)[1].split(" -->", 1)[0])
    assert set(rec["groups"]) == {"setup", "parse", "levels"}
    assert len(rec["source_sha256"]) == 64
