"""Writes tests/golden/synth_hashes.json: XXH3-64 digests that pin the
determinism of the seeded input generators and of the oracle's encoder on
each configuration's input (the encoder is not unique, so these pin this
build's own choices only; decoded bytes are the parity target).  Calls only
synth/ and oracle/.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

CASES = {
    "markov_4MiB_0xACE0": ("markov", 4 << 20, 0xACE0, {}),
    "fastq_1MiB_0xACE1": ("fastq", 1 << 20, 0xACE1, {"flatten": 1}),
    "wiki_1MiB_0xACE2": ("wiki", 1 << 20, 0xACE2, {}),
    "wiki_1MiB_0xACE2_d8": ("wiki", 1 << 20, 0xACE2, {"max_depth": 8}),
    "random_1MiB_0xACE3": ("random", 1 << 20, 0xACE3, {}),
}


def digests():
    out = {}
    for name, (kind, n, seed, opts) in CASES.items():
        x = synth.make(kind, n, seed)
        s = oracle.encode(x, **opts)
        out[name] = {"input_xxh3": f"{oracle.content_hash(x):016x}", "stream_xxh3": f"{oracle.content_hash(s):016x}",
                     "stream_bytes": int(s.size)}
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "synth_hashes.json"), "w") as f:
        json.dump(digests(), f, indent=1, sort_keys=True)
        f.write("\n")
    print("wrote", os.path.join(HERE, "synth_hashes.json"))
