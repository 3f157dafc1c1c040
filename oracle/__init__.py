"""CPU oracle for the hierarchical collective executor — TEST INFRASTRUCTURE.

Plain, slow, obviously correct implementations of what the executor must
compute, written from the paper (HiCCL, arXiv 2408.05962):

  collectives  direct definitions of the eight collectives (float64 / int64)
  steps        a fence-delimited primitive-step interpreter (multicast,
               reduction, fence as defined in Sec. 3.1
               and Sec. 3.3)
  tree         the hierarchical tree factorization, striping and per-level
               byte accounting of Sec. 4 (Optimizations), and the minimum
               top-level volumes implied by Table 3; also the summation order of a factorized
               reduction, for order-exact float32 / bf16 / fp8 expectations
  quant        bf16 and OCP fp8-e4m3 (with power-of-two per-256-element
               scales) encoders and decoders, from the format definitions

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU
baseline may import this package. It shares no code with the executor
library and imports nothing from it.
"""
