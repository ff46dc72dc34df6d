"""GPU: CG's merged forms (options.merged = 1, 2) against the standard form
(merged = 0) and the oracle's merged form.

The merged forms move x's update (form 1: into the next p = z + beta p pass;
form 2: that pass into the SpMM, which gathers z + beta p) but change no
operation on an element: the same fused multiply-adds, and the SpMM's rows
summed in the same order.  So every form's solution must equal the standard
form's bit for bit on the GPU, and the oracle's merged form (bitwise the
oracle's standard form) to the usual parity bound with identical iteration
counts.  The cases reach each place where a deferred update is applied:
convergence, iteration caps, true-residual restarts, a breakdown, frozen
columns beside active ones, replays of the batched solver's captured graph
(form 2's buffer parity is kept on the device) and the allocation-free entry
point.
"""
import sys

import numpy as np
import pytest

import krylov_cases as kc
from paper_2103_07329_amd import inputs

pytestmark = pytest.mark.gpu

FORMS = (0, 1, 2)


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


def _solve(torch, S, B, X0=None, tol=1e-8, noalloc=False):
    B = np.ascontiguousarray(B.reshape(B.shape[0], -1))
    Bd = torch.from_numpy(B).cuda()
    Xd = torch.zeros_like(Bd) if X0 is None else torch.from_numpy(np.ascontiguousarray(X0)).cuda()
    f = S.solve_noalloc if noalloc else S.solve
    rc, st = f(Bd, Xd, tol=tol, check=False)
    torch.cuda.synchronize()
    return Xd.cpu().numpy(), st, rc


def _padded(m):
    return 1 << (int(m) - 1).bit_length()


def _forms(torch, xm, hier, B, X0=None, tol=1e-8, **opts):
    """Every form on the launch shapes the standard form's autotuner chose
    (a lane split changes the order of a row's sum, so separately tuned
    solvers need not agree bit for bit)."""
    out, tun = {}, None
    mp = _padded(B.shape[1] if B.ndim == 2 else 1)
    for f in FORMS:
        S = xm.Solver(hier, merged=f, **opts)
        if tun is not None:
            S.set_tuning(mp, tun)
        out[f] = _solve(torch, S, B, X0=X0, tol=tol)
        if tun is None:
            tun = S.tuning(mp)
        S.close()
    return out


def _bitwise(out):
    X0, s0, rc0 = out[0]
    for f in FORMS[1:]:
        X, st, rc = out[f]
        assert rc == rc0, f
        assert np.array_equal(X, X0), f
        for key in ("iters", "converged", "restarts", "relres", "true_relres"):
            assert np.array_equal(st[key], s0[key]), (f, key)


@pytest.mark.parametrize("smoother", [0, 1])
@pytest.mark.parametrize("m", [1, 5, 16])
def test_merged_forms_match(orc, torch, xm, smoother, m):
    _say(f"[merged] poisson 26^3 smoother={smoother} m={m}")
    p = inputs.poisson7(26)
    Ho = orc.Hierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, m, 40 + m)
    out = _forms(torch, xm, Ho.export(), B, smoother=smoother)
    _bitwise(out)
    Xo, so, rco = Ho.solve(B, smoother=smoother, merged=True, tol=1e-8)
    X, st, rc = out[2]
    assert rc == rco == xm.OK
    assert np.array_equal(st["iters"], so["iters"])
    err = np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
    assert err.max() <= 1e-7, err


def test_merged_forms_match_occupancy_capped_sweep(torch, xm):
    # 48^3 rows make 3456 tiles of 32 rows, more than a sweeping launch's
    # blocks, so the Krylov SpMM grids are capped by the kernels' occupancy;
    # form 2's SpMM holds more registers than the standard one, and both
    # must still run on one grid for the dots to agree bit for bit
    _say("[merged] poisson 48^3 m=16 (sweeps capped by occupancy)")
    p = inputs.poisson7(48)
    H = xm.HostHierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, 16, 47)
    out = _forms(torch, xm, H, B, smoother=1)
    _bitwise(out)
    assert out[0][2] == xm.OK


@pytest.mark.parametrize("smoother", [0, 1])
def test_merged_mixed_precision(orc, torch, xm, smoother):
    _say(f"[merged] jump 20^3 mixed precision smoother={smoother}")
    p = inputs.jump7(20, inputs.jump_kappa(20, np.random.default_rng(3)))
    Ho = orc.Hierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, 8, 44)
    out = _forms(torch, xm, Ho.export(), B, smoother=smoother, precision=xm.MIXED)
    _bitwise(out)
    assert out[2][2] == xm.OK


def test_merged_iteration_caps(orc, torch, xm):
    # a cap stops the solve with x's last update still pending: the flush
    # before the true residual applies it, so x_k is the k-th CG iterate
    _say("[merged] iteration caps 1..4")
    p = inputs.jump7(12, inputs.jump_kappa(12, np.random.default_rng(5), block=3))
    Ho = orc.Hierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, 4, 45)
    for k in (1, 2, 3, 4):
        out = _forms(torch, xm, Ho.export(), B, tol=1e-30, max_iters=k)
        _bitwise(out)
        Xo, so, _ = Ho.solve(B, merged=True, max_iters=k, tol=1e-30)
        X, st, rc = out[2]
        assert rc == xm.NOT_CONVERGED
        assert np.array_equal(st["iters"], so["iters"])
        err = np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
        assert err.max() <= 1e-11, (k, err)


@pytest.mark.parametrize("precision", [0, 1])
def test_merged_true_residual_restart(orc, torch, xm, precision):
    _say(f"[merged] true-residual restart precision={precision}")
    p = inputs.poisson7(10)
    Ho = orc.Hierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, 4, 3)
    X0 = 1e6 * inputs.uniform_rhs(p.n, 4, 4)
    out = _forms(torch, xm, Ho.export(), B, X0=X0, tol=1e-11, precision=precision,
                 x0_mode=xm.X0_GIVEN)
    _bitwise(out)
    X, st, rc = out[2]
    assert rc == xm.OK and np.all(st["restarts"] >= 1)
    tr = np.linalg.norm(B - orc.spmm(*p.csr(), X), axis=0) / np.linalg.norm(B, axis=0)
    assert np.all(tr <= 1e-11), tr


def test_merged_breakdown(orc, torch, xm):
    _say("[merged] CG indefinite one-level")
    A, B = kc.indefinite()
    rp, ci, v = kc.csr(A)
    one = {"A": [(rp, ci, v)], "P": [], "R": [], "lmax": [0.0]}
    out = _forms(torch, xm, one, B, tol=1e-12)
    _bitwise(out)
    Xo, so, rco = orc.Hierarchy(rp, ci, v).solve(B, merged=True, tol=1e-12)
    X, st, rc = out[2]
    assert rc == rco == xm.EBREAKDOWN
    assert np.array_equal(st["iters"], so["iters"])
    assert np.allclose(X, Xo, rtol=0, atol=1e-13)


def test_merged_frozen_and_active_columns(orc, torch, xm):
    # column 0 is a Laplacian eigenvector: unpreconditioned CG is done with
    # it after one iteration while the other columns go on
    _say("[merged] frozen column beside active ones")
    N = 12
    p = inputs.poisson7(N)
    Ho = orc.Hierarchy(*p.csr())
    g = np.arange(1, N + 1) / (N + 1)
    mode = np.einsum("i,j,k->ijk", np.sin(np.pi * g), np.sin(2 * np.pi * g),
                     np.sin(3 * np.pi * g)).reshape(-1)
    B = np.column_stack([mode, inputs.uniform_rhs(p.n, 3, 46)])
    out = _forms(torch, xm, Ho.export(), B, tol=1e-10, precond=0)
    _bitwise(out)
    Xo, so, _ = Ho.solve(B, precond=False, merged=True, tol=1e-10)
    X, st, rc = out[2]
    assert st["iters"][0] == 1 and st["iters"][1:].min() > 10
    assert np.array_equal(st["iters"], so["iters"])
    err = np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
    assert err.max() <= 1e-9, err


@pytest.mark.parametrize("ipl", [3, 4])
def test_merged_batched_replays(orc, torch, xm, ipl):
    """Form 2 under the batched solver: graphs of an odd and an even number
    of iterations, replayed with eager work between the replays, must give
    the eager per-system result of the standard form exactly."""
    _say(f"[merged] batched form 2, {ipl} iterations per launch")
    systems = inputs.batched_systems(seed=1004, count=4, max_side=20)
    Bs, ref, solvers = [], [], []
    for prob, B in systems:
        Hh = xm.HostHierarchy(*prob.csr())
        S0 = xm.Solver(Hh, merged=0)
        Bd = torch.from_numpy(np.ascontiguousarray(B)).cuda()
        X = torch.zeros_like(Bd)
        rc, st = S0.solve(Bd, X)
        assert rc == xm.OK
        ref.append((X.cpu().numpy(), st["iters"]))
        mp = _padded(B.shape[1])
        tun = S0.tuning(mp)
        S0.close()
        S2 = xm.Solver(Hh, merged=2)
        S2.set_tuning(mp, tun)
        solvers.append(S2)
        Bs.append(Bd)
    batch = xm.Batch(solvers, iters_per_launch=ipl)
    for rep in range(3):
        Xs = [torch.full_like(Bd, 7.0) for Bd in Bs]
        rc, sts = batch.solve(Bs, Xs)
        assert rc == xm.OK
        for (Xr, itr), X, st in zip(ref, Xs, sts):
            assert np.array_equal(st["iters"], itr)
            assert np.array_equal(X.cpu().numpy(), Xr)
        torch.cuda.synchronize()
    batch.close()
    for S in solvers:
        S.close()


def test_merged_noalloc(orc, torch, xm):
    _say("[merged] allocation-free entry point, form 2")
    p = inputs.poisson7(24)
    Ho = orc.Hierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, 8, 47)
    S = xm.Solver(Ho.export(), merged=2)
    X1, s1, rc1 = _solve(torch, S, B)
    X2, s2, rc2 = _solve(torch, S, B, noalloc=True)
    X3, s3, rc3 = _solve(torch, S, B[:, :3].copy(), noalloc=True)
    tun4 = S.tuning(4)
    S.close()
    assert rc1 == rc2 == rc3 == xm.OK
    assert np.array_equal(X1, X2) and np.array_equal(s1["iters"], s2["iters"])
    S0 = xm.Solver(Ho.export(), merged=0)
    S0.set_tuning(4, tun4)
    X4, s4, _ = _solve(torch, S0, B[:, :3].copy())
    S0.close()
    assert np.array_equal(X3, X4) and np.array_equal(s3["iters"], s4["iters"])
