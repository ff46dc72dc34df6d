"""GPU: pipelined BiCGStab (method XAMG_PBICGSTAB) against the oracle's.

The k-step iterates and full solves match the oracle's pipelined form (and
so, to rounding, BiCGStab's) with equal iteration counts; the breakdown case
stops the column as the oracle does; a true-residual restart from a far
initial guess converges; and the allocation-free entry point gives the same
bits.  (The mixed-precision cycle is refused at setup: the recurrences carry
images under the preconditioner and need it linear, which the FP32 cycle is
only to FP32 accuracy; tests/test_abi.py checks the refusal.)
"""
import sys

import numpy as np
import pytest

import krylov_cases as kc
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


@pytest.fixture(scope="module")
def jump20(orc):
    p = inputs.jump7(20, inputs.jump_kappa(20, np.random.default_rng(31)))
    return p, orc.Hierarchy(*p.csr())


def _solve(torch, S, B, X0=None, tol=1e-8, noalloc=False):
    B = np.ascontiguousarray(B.reshape(B.shape[0], -1))
    Bd = torch.from_numpy(B).cuda()
    Xd = torch.zeros_like(Bd) if X0 is None else torch.from_numpy(np.ascontiguousarray(X0)).cuda()
    f = S.solve_noalloc if noalloc else S.solve
    rc, st = f(Bd, Xd, tol=tol, check=False)
    torch.cuda.synchronize()
    return Xd.cpu().numpy(), st, rc


@pytest.mark.parametrize("smoother", [0, 1, 2])
@pytest.mark.parametrize("m", [1, 8, 16])
def test_pbicgstab_matches_oracle(orc, torch, xm, jump20, smoother, m):
    p, H = jump20
    _say(f"[pbicgstab] jump20 smoother={smoother} m={m}")
    B = inputs.uniform_rhs(p.n, m, 60 + m)
    Xo, so, rco = H.solve(B, method=orc.PBICGSTAB, smoother=smoother, tol=1e-9)
    S = xm.Solver(H.export(), method=xm.PBICGSTAB, smoother=smoother)
    X, st, rc = _solve(torch, S, B, tol=1e-9)
    S.close()
    _say(f"  oracle iters {so['iters'].tolist()}; gpu iters {st['iters'].tolist()}")
    assert rc == rco == xm.OK
    assert np.array_equal(st["iters"], so["iters"])
    err = np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
    assert err.max() <= 1e-7, err
    tr = np.linalg.norm(B - orc.spmm(*p.csr(), X), axis=0) / np.linalg.norm(B, axis=0)
    assert np.all(tr <= 1e-9)


def test_pbicgstab_iterates(orc, torch, xm, jump20):
    p, H = jump20
    _say("[pbicgstab] k-step iterates")
    B = inputs.uniform_rhs(p.n, 4, 64)
    for k in (1, 2, 3, 5):
        Xo, so, _ = H.solve(B, method=orc.PBICGSTAB, smoother=1, max_iters=k, tol=1e-30)
        Xs, ss, _ = H.solve(B, method=orc.BICGSTAB, smoother=1, max_iters=k, tol=1e-30)
        S = xm.Solver(H.export(), method=xm.PBICGSTAB, smoother=1, max_iters=k)
        X, st, rc = _solve(torch, S, B, tol=1e-30)
        S.close()
        assert rc == xm.NOT_CONVERGED
        assert np.array_equal(st["iters"], so["iters"])
        err = np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
        assert err.max() <= 1e-11, (k, err)
        err = np.linalg.norm(X - Xs, axis=0) / np.linalg.norm(Xs, axis=0)
        assert err.max() <= 1e-11, (k, err)


def test_pbicgstab_breakdown_stops_column(orc, torch, xm):
    _say("[pbicgstab] rho breakdown")
    A, b = kc.rho_breakdown()
    rp, ci, v = kc.csr(A)
    B = np.stack([b, np.random.default_rng(9).uniform(-1, 1, len(b))], axis=1)
    Xo, so, rco = orc.Hierarchy(rp, ci, v).solve(B, method=orc.PBICGSTAB, precond=False,
                                                 tol=1e-12)
    S = xm.Solver({"A": [(rp, ci, v)], "P": [], "R": [], "lmax": [0.0]},
                  method=xm.PBICGSTAB, precond=0)
    X, st, rc = _solve(torch, S, B, tol=1e-12)
    S.close()
    assert rc == rco == xm.EBREAKDOWN
    assert np.array_equal(st["iters"], so["iters"])
    assert np.array_equal(st["converged"], so["converged"])
    assert np.allclose(X, Xo, rtol=0, atol=1e-12 * max(1.0, np.abs(Xo).max()))


def test_pbicgstab_true_residual_restart(orc, torch, xm):
    _say("[pbicgstab] true-residual restart")
    p = inputs.poisson7(10)
    Ho = orc.Hierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, 4, 3)
    X0 = 1e3 * inputs.uniform_rhs(p.n, 4, 4)
    S = xm.Solver(Ho.export(), method=xm.PBICGSTAB, x0_mode=xm.X0_GIVEN)
    X, st, rc = _solve(torch, S, B, X0=X0, tol=1e-11)
    S.close()
    _say(f"  iters {st['iters'].tolist()} restarts {st['restarts'].tolist()}")
    assert rc == xm.OK
    tr = np.linalg.norm(B - orc.spmm(*p.csr(), X), axis=0) / np.linalg.norm(B, axis=0)
    assert np.all(tr <= 1e-11), tr
    assert np.all(st["restarts"] >= 1)


def test_pbicgstab_noalloc(orc, torch, xm, jump20):
    p, H = jump20
    _say("[pbicgstab] allocation-free entry point")
    B = inputs.uniform_rhs(p.n, 8, 66)
    S = xm.Solver(H.export(), method=xm.PBICGSTAB, smoother=1)
    X1, s1, rc1 = _solve(torch, S, B)
    X2, s2, rc2 = _solve(torch, S, B, noalloc=True)
    S.close()
    assert rc1 == rc2 == xm.OK
    assert np.array_equal(X1, X2) and np.array_equal(s1["iters"], s2["iters"])
