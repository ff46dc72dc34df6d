"""MI355X-native multi-RHS AMG-Krylov solve phase (paper arXiv 2103.07329).

Submodules:
  inputs    -- seeded synthetic problems (matrices, right-hand sides)
  xamg      -- thin ctypes binding over the C-ABI library libxamg.so (device
               solver, batched solves, the host hierarchy build, the CNN)
  warmstart -- training data, training loop and comparison of the learned
               warm start (every numeric step runs in libxamg)
  build     -- compiles libxamg.so for gfx950

Nothing is loaded at import time; the HIP library is opened on first use and
its absence is an error (there is no CPU fallback).
"""
__all__ = ["inputs"]
