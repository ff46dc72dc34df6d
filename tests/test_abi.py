"""The C-ABI library loads and exports every symbol include/xamg.h declares
(CPU only: no compute calls that need a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names += re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(xamg_\w+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_library_exports_declared_symbols():
    from paper_2103_07329_amd import xamg
    L = xamg.lib()
    decl = _declared()
    assert len(decl) >= 15
    missing = [n for n in decl if not hasattr(L, n)]
    assert not missing, missing
    assert set(xamg.EXPORTS) <= set(decl)


def test_error_strings_and_defaults():
    import ctypes
    from paper_2103_07329_amd import xamg
    L = xamg.lib()
    for code in (0, 1, -1, -2, -3, -4, -5):
        assert L.xamg_strerror(code)
    o = xamg.default_options()
    assert o.method == xamg.CG and o.smoother == xamg.JACOBI
    assert abs(o.omega - 2.0 / 3.0) < 1e-15 and o.cheby_degree == 2 and o.max_iters == 1000
    assert o.gs_block == 8
    p = xamg.SetupParamsT()
    L.xamg_default_setup_params(ctypes.byref(p))
    assert p.theta == 0.25 and p.max_coarse == 64


def test_setup_argument_errors_without_device():
    """xamg_setup validates its arguments before touching a device."""
    import ctypes
    import numpy as np
    from paper_2103_07329_amd import inputs, xamg
    L = xamg.lib()
    h = ctypes.c_void_p()
    assert L.xamg_setup(None, None, ctypes.byref(h)) == xamg.EINVAL
    prob = inputs.poisson7(4)
    keep = []
    a = xamg._csr_struct(*prob.csr(), keep=keep)
    H = xamg.HierT(1, ctypes.pointer(a), None, None, None)
    bad = xamg.default_options(method=7)
    assert L.xamg_setup(ctypes.byref(H), ctypes.byref(bad), ctypes.byref(h)) == xamg.EINVAL
    bad = xamg.default_options(index_bits=16)      # 16-bit needs MIXED
    assert L.xamg_setup(ctypes.byref(H), ctypes.byref(bad), ctypes.byref(h)) == xamg.EINVAL
    for blk in (0, 5, 32):                          # Gauss-Seidel blocks: 4, 8 or 16 rows
        bad = xamg.default_options(smoother=xamg.GAUSS_SEIDEL, gs_block=blk)
        assert L.xamg_setup(ctypes.byref(H), ctypes.byref(bad), ctypes.byref(h)) == xamg.EINVAL
    bad = xamg.default_options(smoother=3)
    assert L.xamg_setup(ctypes.byref(H), ctypes.byref(bad), ctypes.byref(h)) == xamg.EINVAL
    # pipelined BiCGStab needs a linear preconditioner: not the FP32 cycle
    bad = xamg.default_options(method=xamg.PBICGSTAB, precision=xamg.MIXED)
    assert L.xamg_setup(ctypes.byref(H), ctypes.byref(bad), ctypes.byref(h)) == xamg.EINVAL
    assert b"linear" in L.xamg_last_error()
    big = inputs.poisson7(11)                       # 1331 rows > 1024 on the coarsest level
    b = xamg._csr_struct(*big.csr(), keep=keep)
    H2 = xamg.HierT(1, ctypes.pointer(b), None, None, None)
    assert L.xamg_setup(ctypes.byref(H2), None, ctypes.byref(h)) == xamg.EINVAL
    rp, ci, v = prob.csr()
    ci2 = ci.copy(); ci2[0] = 999
    c = xamg._csr_struct(rp, ci2, v, keep=keep)
    H3 = xamg.HierT(1, ctypes.pointer(c), None, None, None)
    assert L.xamg_setup(ctypes.byref(H3), None, ctypes.byref(h)) == xamg.EINVAL
    assert L.xamg_solve(None, None, None, 1, 1e-8, None) == xamg.EINVAL
