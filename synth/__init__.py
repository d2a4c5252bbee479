"""Seeded synthetic inputs (raw bytes only) shared by the oracle tests and the GPU path.

The module wraps ``synth.c`` (compiled to ``libsynth.so`` next to this file by
``__graft_entry__.build()``).  It contains no part of the codec: no match
finder, no offsets, no levels.  The paper's corpora (Sec. 4.2: enwik9, FASTQ
NA12878, silesia, nci) are not available; these generators are stand-ins with
the same kind of structure, and no item of those corpora is reproduced.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

MiB = 1 << 20
GiB = 1 << 30


def build(verbose: bool = False) -> str:
    """Compile synth.c into libsynth.so (plain gcc, host code only)."""
    import subprocess

    src = os.path.join(_HERE, "synth.c")
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u64 = ctypes.c_uint64
        for name, extra in (("synth_markov", [ctypes.c_double]), ("synth_fastq", []),
                            ("synth_wiki", []), ("synth_random", [ctypes.c_double])):
            fn = getattr(lib, name)
            fn.argtypes = [u8p, u64, u64] + extra
            fn.restype = ctypes.c_int
        lib.synth_splitmix64.argtypes = [u64]
        lib.synth_splitmix64.restype = u64
        lib.synth_uniform.argtypes = [ctypes.POINTER(ctypes.c_double), u64, u64]
        lib.synth_uniform.restype = None
        lib.synth_raw.argtypes = [ctypes.POINTER(ctypes.c_uint64), u64, u64]
        lib.synth_raw.restype = None
        lib.synth_raw_state.argtypes = [ctypes.POINTER(ctypes.c_uint64), u64, ctypes.POINTER(ctypes.c_uint64)]
        lib.synth_raw_state.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _call(name: str, n: int, seed: int, *extra) -> np.ndarray:
    out = np.empty(n, dtype=np.uint8)
    rc = getattr(_load(), name)(_ptr(out), n, seed & (2**64 - 1), *extra)
    if rc != 0:
        raise MemoryError(f"{name}({n}) failed")
    return out


def markov(n: int, seed: int, copy_frac: float = 0.20) -> np.ndarray:
    """Order-2 Markov text over 64 printable symbols with a copy overlay."""
    return _call("synth_markov", n, seed, copy_frac)


def fastq(n: int, seed: int) -> np.ndarray:
    """FASTQ-like records (150 bp reads, Phred+33 qualities, 10% near-duplicate reads)."""
    return _call("synth_fastq", n, seed)


def wiki(n: int, seed: int) -> np.ndarray:
    """Wiki-markup-like text: Zipf(1.1) words, sentences, tags, template lines."""
    return _call("synth_wiki", n, seed)


def random_repeats(n: int, seed: int, copy_frac: float = 0.30) -> np.ndarray:
    """Uniform random bytes with a copy overlay of earlier substrings."""
    return _call("synth_random", n, seed, copy_frac)


def splitmix64(x: int) -> int:
    """One SplitMix64 output for state ``x`` (used to derive per-stream seeds)."""
    return int(_load().synth_splitmix64(x & (2**64 - 1)))


def uniform(n: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    _load().synth_uniform(out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n, seed)
    return out


def raw64_state(n: int, state) -> np.ndarray:
    """n raw xoshiro256** outputs from the given 4-word state (for reference vectors)."""
    st = np.ascontiguousarray(np.asarray(state, dtype=np.uint64))
    out = np.empty(n, dtype=np.uint64)
    _load().synth_raw_state(out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n,
                            st.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out


def raw64(n: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _load().synth_raw(out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n, seed)
    return out


# --------------------------------------------------------------------------
# Workload recipes: (kind, size, seed) for every configuration.  Only shapes
# and seeds live here; how a stream is encoded is the caller's business.

CFG_SEEDS = {0: 0xACE0, 1: 0xACE1, 2: 0xACE2, 3: 0xACE3, 4: 0xACE4}


def make(kind: str, n: int, seed: int) -> np.ndarray:
    if kind == "markov":
        return markov(n, seed)
    if kind == "fastq":
        return fastq(n, seed)
    if kind == "wiki":
        return wiki(n, seed)
    if kind == "random":
        return random_repeats(n, seed)
    raise ValueError(kind)


def mix_recipe(count: int, lo: int, hi: int, seed: int):
    """Per-stream (kind, size, seed) of the batched / served mixes.

    Stream i draws from a generator seeded with SplitMix64(seed ^ i): a kind
    (40% markov text, 40% FASTQ-like, 20% random+repeats) and a size
    log-uniform in [lo, hi].
    """
    out = []
    for i in range(count):
        s = splitmix64(seed ^ i)
        u = uniform(2, s)
        kind = "markov" if u[0] < 0.4 else ("fastq" if u[0] < 0.8 else "random")
        size = int(round(math.exp(math.log(lo) + u[1] * (math.log(hi) - math.log(lo)))))
        out.append((kind, size, s))
    return out
