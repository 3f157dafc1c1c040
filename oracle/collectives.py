"""Direct definitions of the eight collectives — test oracle.

Follows the collectives listed in the paper's Background (Table 1) with their textbook (MPI)
meaning, and the buffer convention of Sec. 3.2:
the largest per-rank buffer holds ``d * p`` elements and chunk ``q`` is
elements ``[q*d, (q+1)*d)``.

Every function takes a list of per-rank 1-D numpy arrays (``sends[r]`` is
rank r's send buffer) and returns new arrays; inputs are never modified.

Arithmetic: floating-point reductions are carried out in float64 and the
float64 result is returned (the exact reference the executor is scored
against); integer reductions are carried out in int64 and wrapped to int32
two's complement. ``max`` and ``min`` are exact in any precision.

Parity: pinned by tests/test_oracle_collectives.py (hand-computed values,
brute force on tiny P, algebraic invariants).
"""
from __future__ import annotations

import numpy as np

OPS = ("sum", "max", "min")


def wide(a: np.ndarray) -> np.ndarray:
    """The accumulation type of the oracle: float64 for floats, int64 for ints."""
    a = np.asarray(a)
    if a.dtype.kind == "f":
        return a.astype(np.float64)
    if a.dtype.kind in "iu":
        return a.astype(np.int64)
    raise TypeError(f"unsupported dtype {a.dtype}")


def wrap_int32(x: np.ndarray) -> np.ndarray:
    """Two's-complement wrap of an int64 array to int32 (addition modulo 2**32)."""
    return ((x.astype(np.int64) + (1 << 31)) % (1 << 32) - (1 << 31)).astype(np.int32)


def finish(acc: np.ndarray, like: np.dtype) -> np.ndarray:
    """Convert a wide accumulator back: ints wrap to int32, floats stay float64."""
    if np.dtype(like).kind in "iu":
        return wrap_int32(acc)
    return acc


def combine(arrays: list[np.ndarray], op: str) -> np.ndarray:
    """Elementwise ``op`` over a list of equal-length arrays, in rank order, wide precision."""
    if op not in OPS:
        raise ValueError(op)
    if not arrays:
        raise ValueError("combine needs at least one operand")
    acc = wide(arrays[0]).copy()
    for a in arrays[1:]:
        b = wide(a)
        if op == "sum":
            acc = acc + b
        elif op == "max":
            acc = np.maximum(acc, b)
        else:
            acc = np.minimum(acc, b)
    return finish(acc, np.asarray(arrays[0]).dtype)


def abs_sum(arrays: list[np.ndarray]) -> np.ndarray:
    """Elementwise sum of absolute values over ranks (float64): the condition scale of a sum."""
    acc = np.zeros(len(arrays[0]), dtype=np.float64)
    for a in arrays:
        acc += np.abs(np.asarray(a, dtype=np.float64))
    return acc


def _chunk(a: np.ndarray, q: int, d: int) -> np.ndarray:
    return a[q * d:(q + 1) * d]


def broadcast(sends: list[np.ndarray], root: int) -> list[np.ndarray]:
    """Every rank receives the root's buffer: ``y_r = s_root``."""
    return [np.array(sends[root], copy=True) for _ in sends]


def reduce(sends: list[np.ndarray], root: int, op: str = "sum") -> np.ndarray:
    """The root receives the elementwise ``op`` over all ranks' buffers (other ranks receive nothing)."""
    del root  # the value does not depend on which rank receives it
    return combine(sends, op)


def scatter(send_root: np.ndarray, p: int) -> list[np.ndarray]:
    """Rank r receives chunk r of the root's buffer (``d = len / p``)."""
    n = len(send_root)
    if n % p:
        raise ValueError("scatter buffer must hold p equal chunks")
    d = n // p
    return [np.array(_chunk(send_root, r, d), copy=True) for r in range(p)]


def gather(sends: list[np.ndarray]) -> np.ndarray:
    """The root receives the concatenation of all ranks' buffers, chunk r = ``s_r``."""
    return np.concatenate([np.asarray(s) for s in sends])


def all_gather(sends: list[np.ndarray]) -> list[np.ndarray]:
    """Every rank receives the concatenation: chunk q of ``y_r`` is ``s_q``."""
    g = gather(sends)
    return [g.copy() for _ in sends]


def reduce_scatter(sends: list[np.ndarray], op: str = "sum") -> list[np.ndarray]:
    """Rank r receives chunk r of the elementwise ``op`` over all ranks' buffers."""
    p = len(sends)
    n = len(sends[0])
    if n % p:
        raise ValueError("reduce-scatter buffers must hold p equal chunks")
    d = n // p
    full = combine(sends, op)
    return [full[r * d:(r + 1) * d].copy() for r in range(p)]


def all_reduce(sends: list[np.ndarray], op: str = "sum") -> list[np.ndarray]:
    """Every rank receives the elementwise ``op`` over all ranks' buffers."""
    full = combine(sends, op)
    return [full.copy() for _ in sends]


def all_to_all(sends: list[np.ndarray]) -> list[np.ndarray]:
    """Chunk i of rank j's output is chunk j of rank i's input."""
    p = len(sends)
    n = len(sends[0])
    if n % p:
        raise ValueError("all-to-all buffers must hold p equal chunks")
    d = n // p
    out = []
    for j in range(p):
        out.append(np.concatenate([np.asarray(_chunk(sends[i], j, d)) for i in range(p)]))
    return out


# ---------------------------------------------------------------- scoring
def scaled_error(got: np.ndarray, exact: np.ndarray, scale: np.ndarray) -> float:
    """Largest elementwise ``|got - exact| / max(|exact|, scale)``.

    ``scale`` is the elementwise sum of absolute inputs. This is the
    condition-scaled relative error of a computed sum: the textbook bound for
    any summation order in precision u is ``h * u * sum|a|`` with ``h`` the
    longest chain of additions, so this quantity is what that bound limits.
    """
    got = np.asarray(got, dtype=np.float64)
    exact = np.asarray(exact, dtype=np.float64)
    den = np.maximum(np.abs(exact), np.asarray(scale, dtype=np.float64))
    den = np.where(den == 0, 1.0, den)
    if got.size == 0:
        return 0.0
    return float(np.max(np.abs(got - exact) / den))


def error_report(got: np.ndarray, exact: np.ndarray, scale: np.ndarray) -> dict:
    """Max absolute, condition-scaled, plain relative (where well conditioned) and normwise errors."""
    got = np.asarray(got, dtype=np.float64)
    exact = np.asarray(exact, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    if got.size == 0:
        return {"max_abs": 0.0, "scaled": 0.0, "rel_well_conditioned": 0.0, "normwise": 0.0}
    diff = np.abs(got - exact)
    well = np.abs(exact) >= 1e-3 * scale
    rel = diff[well] / np.abs(exact[well]) if np.any(well) else np.zeros(1)
    nrm = float(np.linalg.norm(exact))
    return {
        "max_abs": float(diff.max()),
        "scaled": scaled_error(got, exact, scale),
        "rel_well_conditioned": float(rel.max()) if rel.size else 0.0,
        "normwise": float(np.linalg.norm(got - exact) / nrm) if nrm > 0 else float(np.linalg.norm(got - exact)),
    }
