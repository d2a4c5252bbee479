"""Host code under the compiler's sanitizers (CPU only, gcc/g++):
  - the oracle (C) under AddressSanitizer + UBSan: encode, sequential and
    block-parallel decode, level recomputation, damaged streams, the tANS
    coder and damaged tANS containers;
  - the oracle's block-parallel decoder under ThreadSanitizer;
  - the library's host decoder (format.cpp + hostdec.cpp, which need no GPU
    toolchain) under AddressSanitizer + UBSan and under ThreadSanitizer, on
    streams of every configuration's kind, the four-stream format and
    damaged copies.
Skipped where gcc cannot build sanitized programs."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2606_04268_amd", "csrc")
ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
TSAN = ["-fsanitize=thread"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
           TSAN_OPTIONS="halt_on_error=1")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None, reason="no gcc")


def build(tmp, name, cc, flags, srcs, extra=()):
    exe = os.path.join(tmp, name)
    cmd = [cc, "-O1", "-g", *flags, "-o", exe, *srcs, *extra]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        if "cannot find" in r.stderr or "unrecognized" in r.stderr:
            pytest.skip(f"sanitizer runtime unavailable: {r.stderr[:200]}")
        raise AssertionError(r.stderr)
    return exe


def run(exe, args, timeout=600):
    r = subprocess.run([exe, *args], capture_output=True, text=True, env=ENV, timeout=timeout)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


@pytest.fixture(scope="module")
def inputs(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    files = []
    for kind, n, seed in [("markov", 150_000, 1), ("fastq", 120_000, 2), ("wiki", 200_000, 3),
                          ("random", 40_000, 4), ("wiki", 0, 5), ("markov", 1, 6), ("wiki", 70_001, 7)]:
        p = d / f"{kind}_{n}.bin"
        p.write_bytes(synth.make(kind, n, seed).tobytes())
        files.append(str(p))
    return d, files


ORACLE_SRCS = [os.path.join(ROOT, "oracle", "aceapex_oracle.c"), os.path.join(ROOT, "oracle", "tans_oracle.c"),
               os.path.join(SAN, "oracle_driver.c")]


def test_oracle_asan_ubsan(inputs):
    d, files = inputs
    exe = build(str(d), "oracle_asan", "gcc", ["-std=c11"] + ASAN, ORACLE_SRCS, ["-lpthread"])
    out = run(exe, files)
    assert out.count("ok ") == len(files)


def test_oracle_decode_mt_tsan(inputs):
    d, files = inputs
    exe = build(str(d), "oracle_tsan", "gcc", ["-std=c11"] + TSAN, ORACLE_SRCS, ["-lpthread"])
    out = run(exe, ["--mt-only"] + files)
    assert out.count("ok ") == len(files)


@pytest.fixture(scope="module")
def streams(inputs):
    d, files = inputs
    args = []
    for i, f in enumerate(files):
        x = np.fromfile(f, dtype=np.uint8)
        for j, opts in enumerate([dict(block_log2=12), dict(block_log2=14, flatten=1, max_depth=4),
                                  dict(block_log2=10, levels=0, chunk_log2=3)]):
            p = d / f"s{i}_{j}.acx"
            p.write_bytes(oracle.encode(x, **opts).tobytes())
            args += [str(p), f]
    return d, args


HOSTDEC_SRCS = [os.path.join(CSRC, "hostdec.cpp"), os.path.join(CSRC, "format.cpp"),
                os.path.join(SAN, "hostdec_driver.cpp")]


def test_host_decoder_asan_ubsan(streams):
    d, args = streams
    exe = build(str(d), "hostdec_asan", "g++", ["-std=c++17", "-I", os.path.join(ROOT, "include")] + ASAN,
                HOSTDEC_SRCS, ["-lpthread"])
    out = run(exe, args)
    assert out.count("ok ") == len(args) // 2


def test_host_decoder_tsan(streams):
    d, args = streams
    exe = build(str(d), "hostdec_tsan", "g++", ["-std=c++17", "-I", os.path.join(ROOT, "include")] + TSAN,
                HOSTDEC_SRCS, ["-lpthread"])
    out = run(exe, ["--few"] + args)
    assert out.count("ok ") == len(args) // 2
