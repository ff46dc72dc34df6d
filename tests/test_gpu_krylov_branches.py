"""GPU: the Krylov branches a solve rarely takes, against the oracle.

Breakdowns and restarts are driven from the host with inputs built for them
(tests/krylov_cases.py): the quantities that must vanish are exactly zero in
floating point on both sides, so return codes, iteration counts and restart
counts must agree exactly.  The true-residual restart comes from a huge
initial guess whose rounding the recurrence residual does not see; there the
two sides round differently (order of the dot sums), so the restart itself
is required on both and the iteration counts may differ by one.
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


def _one_level(A):
    rp, ci, v = kc.csr(A)
    return {"A": [(rp, ci, v)], "P": [], "R": [], "lmax": [0.0]}


def _solve(torch, S, B, X0=None, tol=1e-12):
    B = np.ascontiguousarray(B.reshape(B.shape[0], -1))
    Bd = torch.from_numpy(B).cuda()
    Xd = torch.zeros_like(Bd) if X0 is None else torch.from_numpy(np.ascontiguousarray(X0)).cuda()
    rc, st = S.solve(Bd, Xd, tol=tol, check=False)
    torch.cuda.synchronize()
    return Xd.cpu().numpy(), st, rc


@pytest.mark.parametrize("case", ["rho_breakdown", "rhv_breakdown", "omega_breakdown"])
def test_bicgstab_breakdowns_match_oracle(orc, torch, xm, case):
    _say(f"[branches] BiCGStab {case}")
    A, b = getattr(kc, case)()
    rng = np.random.default_rng(9)
    # a second, ordinary column rides along: columns are independent
    B = np.stack([b, rng.uniform(-1, 1, len(b))], axis=1)
    Ho = orc.Hierarchy(*kc.csr(A))
    Xo, so, rco = Ho.solve(B, method=orc.BICGSTAB, precond=False, tol=1e-12)
    S = xm.Solver(_one_level(A), method=xm.BICGSTAB, precond=0)
    X, st, rc = _solve(torch, S, B)
    S.close()
    _say(f"  oracle rc {rco} iters {so['iters']} restarts {so['restarts']}; "
         f"gpu rc {rc} iters {st['iters']} restarts {st['restarts']}")
    assert rc == rco
    assert np.array_equal(st["iters"], so["iters"])
    assert np.array_equal(st["restarts"], so["restarts"])
    assert np.array_equal(st["converged"], so["converged"])
    assert np.allclose(X, Xo, rtol=0, atol=1e-12 * max(1.0, np.abs(Xo).max()))


def test_cg_indefinite_breakdown(orc, torch, xm):
    _say("[branches] CG indefinite one-level")
    A, B = kc.indefinite()
    Ho = orc.Hierarchy(*kc.csr(A))
    Xo, so, rco = Ho.solve(B, tol=1e-12)
    S = xm.Solver(_one_level(A))
    X, st, rc = _solve(torch, S, B)
    S.close()
    assert rc == rco == xm.EBREAKDOWN
    assert np.array_equal(st["iters"], so["iters"])
    assert np.array_equal(st["converged"], so["converged"])
    assert np.allclose(X, Xo, rtol=0, atol=1e-13)


@pytest.mark.parametrize("method", [0, 1])
def test_unpreconditioned_matches_oracle(orc, torch, xm, method):
    _say(f"[branches] no preconditioner, method {method}")
    p = inputs.poisson7(12)
    Ho = orc.Hierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, 4, 31)
    S = xm.Solver(Ho.export(), method=method, precond=0)
    # the first iterates agree up to rounding
    for k in (1, 2, 3, 6):
        S2 = xm.Solver(Ho.export(), method=method, precond=0, max_iters=k)
        X, st, rc = _solve(torch, S2, B, tol=1e-30)
        S2.close()
        Xo, so, _ = Ho.solve(B, method=method, precond=False, max_iters=k, tol=1e-30)
        assert np.array_equal(st["iters"], so["iters"])
        err = np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
        assert err.max() <= 1e-11, (k, err)
    Xo, so, rco = Ho.solve(B, method=method, precond=False, tol=1e-8)
    X, st, rc = _solve(torch, S, B, tol=1e-8)
    S.close()
    _say(f"  oracle iters {so['iters']}; gpu iters {st['iters']}")
    assert rc == rco == xm.OK
    if method == 0:
        assert np.array_equal(st["iters"], so["iters"])
    else:
        # unpreconditioned BiCGStab converges erratically over ~40 iterations:
        # the order of the dot sums shifts the stopping step by a few
        assert np.all(np.abs(st["iters"] - so["iters"]) <= 3)
    err = np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
    assert err.max() <= 1e-7, err


@pytest.mark.parametrize("method,precision", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_true_residual_restart(orc, torch, xm, method, precision):
    _say(f"[branches] true-residual restart, method {method} precision {precision}")
    p = inputs.poisson7(10)
    Ho = orc.Hierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, 4, 3)
    X0 = 1e6 * inputs.uniform_rhs(p.n, 4, 4)
    Xo, so, rco = Ho.solve(B, X0=X0, method=method, tol=1e-11)
    S = xm.Solver(Ho.export(), method=method, precision=precision, x0_mode=xm.X0_GIVEN)
    X, st, rc = _solve(torch, S, B, X0=X0, tol=1e-11)
    S.close()
    _say(f"  oracle iters {so['iters']} restarts {so['restarts']}; "
         f"gpu iters {st['iters']} restarts {st['restarts']}")
    assert rc == rco == xm.OK
    assert np.all(so["restarts"] >= 1) and np.all(st["restarts"] >= 1)
    if precision == 0:
        assert np.all(np.abs(st["iters"] - so["iters"]) <= 1)
    A = orc.spmm(*p.csr(), X)
    tr = np.linalg.norm(B - A, axis=0) / np.linalg.norm(B, axis=0)
    assert np.all(tr <= 1e-11), tr
    Xref, _, _ = Ho.solve(B, method=method, tol=1e-13)
    err = np.linalg.norm(X - Xref, axis=0) / np.linalg.norm(Xref, axis=0)
    assert err.max() <= 1e-7, err
