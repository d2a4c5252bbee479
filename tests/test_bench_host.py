"""Host-side checks of bench.py's contract (no GPU): more than one GPU is
refused with a message, and the algorithmic bytes the roofline divides by
split C + N + M (stream sections without padding, decoded bytes, match bytes
read once more) exactly between the kernel groups."""
import json
import os
import subprocess
import sys

import bench
import synth
import paper_2606_04268_amd as ax
from paper_2606_04268_amd.stats import stream_stats

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_stream_sections_add_up_to_the_stream():
    x = synth.markov(1 << 20, 3)
    s = ax.encode(x)
    st = stream_stats(s)
    assert sum(st["sections"].values()) == s.size == st["comp_bytes"]
    assert st["literal_bytes"] + st["match_bytes"] == x.size == st["decoded_bytes"]
    assert sum(st["level_counts"]) == st["n_seq"]
    assert sum(st["level_bytes"]) == st["match_bytes"]


def test_algorithmic_bytes_split_c_plus_n_plus_m():
    for kind, opts in (("markov", {}), ("fastq", {"flatten": 1})):
        x = synth.make(kind, 3 << 19, 11)
        s = ax.encode(x, block_log2=18, **opts)
        st = stream_stats(s)
        g = bench.algorithmic_bytes_per_group(st)
        c = st["comp_bytes"] - st["sections"]["padding"]
        assert g["setup"] + g["parse"] + g["levels"] == c + st["decoded_bytes"] + st["match_bytes"]
        assert g["levels"] == 2 * st["match_bytes"]
        assert g["parse"] >= 2 * st["literal_bytes"]


def test_algorithmic_mode_prints_one_json_line():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--mode", "algorithmic", "--workload",
                        "markov4"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    lines = [line for line in r.stdout.splitlines() if line.strip()]
    assert len(lines) == 1
    g = json.loads(lines[0])
    assert set(g) == {"setup", "parse", "levels"} and all(v > 0 for v in g.values())
