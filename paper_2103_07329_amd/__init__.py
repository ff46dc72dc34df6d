"""MI355X-native multi-RHS AMG-Krylov solve phase (paper arXiv 2103.07329).

Submodules:
  inputs  -- seeded synthetic problems (matrices, right-hand sides)
  xamg    -- thin ctypes binding over the C-ABI library libxamg.so
  hier    -- host-side hierarchy construction (binding to the library's setup)

Nothing is loaded at import time; the HIP library is opened on first use and
its absence is an error (there is no CPU fallback).
"""
__all__ = ["inputs"]
