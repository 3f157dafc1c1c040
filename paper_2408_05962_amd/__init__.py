"""Hierarchical collective executor for one MI355X (HiCCL, arXiv 2408.05962).

The native library ``libhiccl.so`` (C ABI in include/hiccl.h) holds the
planner and the gfx950 kernels; this package is its Python binding and the
composition helpers of Table 2 / Listing 2.
"""
from .hiccl import (BATCH, DTYPES, ELEM_SIZE, EXEC, OPS, ORDER, Batch, Comm, HicclError, Server, addr, autotune, autotune_batch,
                    autotune_model,
                    check, from_payload, lib, run_batch, to_payload)
from . import collectives

__all__ = ["Comm", "Batch", "Server", "HicclError", "autotune", "autotune_batch", "autotune_model", "to_payload", "from_payload", "collectives", "lib", "run_batch",
           "check", "addr", "DTYPES", "ELEM_SIZE", "OPS", "EXEC", "ORDER", "BATCH"]
