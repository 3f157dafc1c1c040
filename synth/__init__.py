"""Seeded synthetic inputs for the collective workloads.

This module is shared by the CPU oracle side (tests, baselines) and by the
device-side runs. It holds random-number recipes only: no collective
arithmetic, no factorization, no quantization.

Recipe (host generator):
  * every (workload, request, rank, block) draws from its own PCG64 stream
    seeded with ``SeedSequence([240805962, workload, request, rank, block])``;
  * a rank buffer of ``n`` elements is the concatenation of blocks of
    ``BLOCK`` elements, so any block can be regenerated on its own;
  * ``int32``: uniform integers in [-1000, 1000] (both ends inclusive);
  * ``float32``: standard normal N(0, 1);
  * ``float32_outliers``: standard normal, then a Bernoulli(0.01) mask of
    entries multiplied by 1e3 (drawn from the same block stream).

Device generator (for buffers too large to draw on the host in a test run):
  torch's seeded device generator, normal or integer, same distributions.
  The host copy of such a buffer is read back before any collective runs.
"""
from __future__ import annotations

import math

import numpy as np

ROOT_SEED = 240805962
BLOCK = 1 << 20

KINDS = ("int32", "float32", "float32_outliers")


def _stream(workload: int, request: int, rank: int, block: int) -> np.random.Generator:
    ss = np.random.SeedSequence([ROOT_SEED, int(workload), int(request), int(rank), int(block)])
    return np.random.Generator(np.random.PCG64(ss))


def _draw_block(kind: str, workload: int, request: int, rank: int, block: int, n: int) -> np.ndarray:
    g = _stream(workload, request, rank, block)
    if kind == "int32":
        return g.integers(-1000, 1001, size=n, dtype=np.int32)
    if kind == "float32":
        return g.standard_normal(n, dtype=np.float32)
    if kind == "float32_outliers":
        x = g.standard_normal(n, dtype=np.float32)
        mask = g.random(n) < 0.01
        x[mask] *= np.float32(1e3)
        return x
    raise ValueError(f"unknown input kind {kind!r}")


def rank_buffer(kind: str, workload: int, request: int, rank: int, n: int) -> np.ndarray:
    """The whole ``n``-element input of one virtual rank (host, numpy)."""
    if n <= 0:
        return np.zeros(0, dtype=np.int32 if kind == "int32" else np.float32)
    parts = []
    for b in range(math.ceil(n / BLOCK)):
        m = min(BLOCK, n - b * BLOCK)
        parts.append(_draw_block(kind, workload, request, rank, b, m))
    return np.concatenate(parts)


def rank_block(kind: str, workload: int, request: int, rank: int, n: int, block: int) -> np.ndarray:
    """Block ``block`` of rank ``rank``'s ``n``-element input, drawn on its own."""
    m = min(BLOCK, n - block * BLOCK)
    return _draw_block(kind, workload, request, rank, block, m)


def rank_buffers(kind: str, workload: int, request: int, nranks: int, n: int) -> list[np.ndarray]:
    """Inputs of all virtual ranks, one numpy array each."""
    return [rank_buffer(kind, workload, request, r, n) for r in range(nranks)]


def device_buffers(kind: str, seed: int, nranks: int, n: int, device: str = "cuda"):
    """Inputs of all ranks drawn on the device with torch's seeded generator.

    Returns one 2-D tensor of shape (nranks, n); row r is rank r's buffer.
    """
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(ROOT_SEED) * 1000003 + int(seed))
    if kind == "int32":
        return torch.randint(-1000, 1001, (nranks, n), generator=gen, device=device, dtype=torch.int32)
    x = torch.randn((nranks, n), generator=gen, device=device, dtype=torch.float32)
    if kind == "float32_outliers":
        mask = torch.rand((nranks, n), generator=gen, device=device) < 0.01
        x = torch.where(mask, x * 1e3, x)
    return x


def log_uniform_sizes(seed: int, count: int, lo: int, hi: int, multiple: int) -> list[int]:
    """Sizes drawn log-uniformly in [lo, hi], rounded down to ``multiple`` (>= multiple)."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, 77, int(seed)])))
    u = g.uniform(math.log(lo), math.log(hi), size=count)
    out = []
    for v in u:
        s = int(math.exp(v)) // multiple * multiple
        out.append(max(multiple, s))
    return out


def choice_stream(seed: int, tag: int) -> np.random.Generator:
    """A PCG64 stream for workload-mix draws (types, dtypes, arrival times)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, 99, int(tag), int(seed)])))
