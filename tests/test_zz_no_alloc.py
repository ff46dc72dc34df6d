"""GPU: xamg_solve_noalloc (every work buffer in the library's static
scratch array) against xamg_solve on the same handle and inputs.

Same kernels and launch shapes on both paths, so results agree to FP64
rounding of identical operations (in practice bitwise); the bar is the FP64
solve parity bar: identical iteration counts and return codes, per-column
relative difference <= 1e-13.  Two no-allocation calls run back to back, the
second with a smaller input, so stale scratch contents from the first would
show.
"""
import sys

import numpy as np
import pytest

from paper_2103_07329_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def xm():
    from paper_2103_07329_amd import xamg
    xamg.lib()
    return xamg


def _run(torch, fn, B, tol):
    Bd = torch.from_numpy(np.ascontiguousarray(B)).cuda()
    Xd = torch.zeros_like(Bd)
    rc, st = fn(Bd, Xd, tol=tol, check=False)
    torch.cuda.synchronize()
    return Xd.cpu().numpy(), st, rc


def _compare(X, st, rc, Xr, sr, rcr):
    assert rc == rcr
    assert np.array_equal(st["iters"], sr["iters"])
    assert np.array_equal(st["restarts"], sr["restarts"])
    d = np.linalg.norm(X - Xr, axis=0) / np.linalg.norm(Xr, axis=0)
    assert d.max() <= 1e-13, d
    return bool(np.array_equal(X, Xr))


def test_noalloc_matches_solve_twice_smaller_second(torch, xm):
    p = inputs.poisson7(24)
    H = xm.HostHierarchy(*p.csr())
    S = xm.Solver(H, smoother=xm.CHEBYSHEV)
    B8 = inputs.uniform_rhs(p.n, 8, 41)
    B3 = inputs.uniform_rhs(p.n, 3, 42)
    # reference: the allocating entry point (tunes the launch shapes first)
    _say("[noalloc] poisson24 CG Chebyshev: xamg_solve m=8, m=3")
    Xr8, sr8, rcr8 = _run(torch, S.solve, B8, 1e-10)
    Xr3, sr3, rcr3 = _run(torch, S.solve, B3, 1e-10)
    _say("[noalloc] xamg_solve_noalloc m=8 then m=3")
    X8, s8, rc8 = _run(torch, S.solve_noalloc, B8, 1e-10)
    X3, s3, rc3 = _run(torch, S.solve_noalloc, B3, 1e-10)
    b8 = _compare(X8, s8, rc8, Xr8, sr8, rcr8)
    b3 = _compare(X3, s3, rc3, Xr3, sr3, rcr3)
    _say(f"  iters {s8['iters'].tolist()} / {s3['iters'].tolist()}, bitwise {b8} {b3}")
    # the allocating path is unchanged afterwards
    Xa, sa, rca = _run(torch, S.solve, B8, 1e-10)
    assert rca == rcr8 and np.array_equal(Xa, Xr8)
    S.close()


def test_noalloc_bicgstab_mixed_smaller_system(torch, xm):
    p = inputs.poisson7(12)
    H = xm.HostHierarchy(*p.csr())
    S = xm.Solver(H, method=xm.BICGSTAB, precision=xm.MIXED)
    B = inputs.uniform_rhs(p.n, 5, 43)
    _say("[noalloc] poisson12 BiCGStab mixed m=5")
    Xr, sr, rcr = _run(torch, S.solve, B, 1e-9)
    X, st, rc = _run(torch, S.solve_noalloc, B, 1e-9)
    X2, st2, rc2 = _run(torch, S.solve_noalloc, B[:, :2].copy(), 1e-9)
    Xr2, sr2, rcr2 = _run(torch, S.solve, B[:, :2].copy(), 1e-9)
    _compare(X, st, rc, Xr, sr, rcr)
    _compare(X2, st2, rc2, Xr2, sr2, rcr2)
    S.close()


def test_noalloc_rejects_work_beyond_the_scratch(torch, xm):
    p = inputs.poisson7(64)
    H = xm.HostHierarchy(*p.csr())
    S = xm.Solver(H)
    B = np.zeros((p.n, 32))
    B[0, :] = 1.0
    _say("[noalloc] poisson64 m=32: over the scratch size")
    Bd = torch.from_numpy(B).cuda()
    Xd = torch.zeros_like(Bd)
    rc, _ = S.solve_noalloc(Bd, Xd, check=False)
    assert rc == xm.EINVAL
    assert b"scratch" in xm.lib().xamg_last_error()
    S.close()


def test_noalloc_on_a_fresh_handle_takes_the_cached_shapes(torch, xm):
    # a handle never tuned takes the shapes the tuning cache holds for its
    # operators (tuned here by another handle's first solve): no timing, no
    # allocation, and the other handle's solution bit for bit
    p = inputs.poisson7(20)
    H = xm.HostHierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, 16, 44)
    _say("[noalloc] poisson20 m=16: fresh handle after another handle's tuning")
    S1 = xm.Solver(H, smoother=xm.CHEBYSHEV)
    Xr, sr, rcr = _run(torch, S1.solve, B, 1e-10)
    S2 = xm.Solver(H, smoother=xm.CHEBYSHEV)
    X, st, rc = _run(torch, S2.solve_noalloc, B, 1e-10)
    assert S2.tuning(16) == S1.tuning(16)
    assert _compare(X, st, rc, Xr, sr, rcr)
    S1.close()
    S2.close()
