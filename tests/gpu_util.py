"""Shared helpers of the GPU tests: decode through the C ABI into a buffer
with guard bands on both sides, and report what came back."""
from __future__ import annotations

import sys

import numpy as np

GUARD = 4096
POISON = 0xA5


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_decode(stream, poison=POISON, check_guards=True):
    """Decode a host stream on cuda:0; returns (bytes, status)."""
    import torch

    import paper_2606_04268_amd as ax

    ds = ax.to_device(stream)
    n = ds.n
    buf = torch.full((n + 2 * GUARD,), poison, dtype=torch.uint8, device="cuda")
    out = buf[GUARD:GUARD + n] if n else buf[GUARD:GUARD + 16]
    _, st = ax.decode(ds, out=out)
    torch.cuda.synchronize()
    status = int(st.cpu().item())
    host = buf.cpu().numpy()
    if check_guards:
        assert (host[:GUARD] == poison).all(), "write below the output buffer"
        assert (host[GUARD + n:] == poison).all(), "write above the output buffer"
    return host[GUARD:GUARD + n].copy(), status
