"""Helpers of the GPU tests: numpy <-> torch device copies and oracle/GPU parameter pairs."""
from __future__ import annotations

import sys

import numpy as np

_VIEW = {np.dtype(np.uint64): np.int64, np.dtype(np.uint32): np.int32, np.dtype(np.uint16): np.int16,
         np.dtype(np.int8): np.int8, np.dtype(np.int32): np.int32, np.dtype(np.int64): np.int64}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def to_dev(a: np.ndarray):
    import torch
    a = np.ascontiguousarray(a)
    return torch.from_numpy(a.view(_VIEW[a.dtype]).copy()).cuda()


def to_host(t, dtype) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(dtype)


def empty(shape, dtype):
    import torch
    tdt = {np.uint64: torch.int64, np.uint32: torch.int32, np.uint16: torch.int16,
           np.int8: torch.int8, np.int32: torch.int32}[dtype]
    return torch.zeros(shape, dtype=tdt, device="cuda")


def pair(log_n: int, L: int, h: int = 2, item_bits: int = 16, mu: int = 4):
    """GPU parameters and the oracle context over the same ciphertext primes."""
    import paper_2310_14565_amd as pk
    from oracle.core import Context
    gp = pk.Params(log_n, L, h, item_bits, mu)
    ctx = Context(gp.n, gp.q_primes)
    return gp, ctx
