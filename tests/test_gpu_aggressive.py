"""GPU: hierarchies with aggressive coarsening and multipass interpolation
(the first levels coarsened by a second RS pass on the distance-two
strength), handed to the device as data, against the oracle: one V-cycle
element-wise within 1e-12 (FP64), PCG with the oracle's iteration counts and
error <= 1e-7, the mixed-precision solve to the true residual."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

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


CASES = [("poisson", 1, 1), ("poisson", 2, 2), ("jump", 1, 2), ("jump", 2, 1)]


def _problem(kind):
    if kind == "poisson":
        return inputs.poisson7(24)
    return inputs.jump7(23, inputs.jump_kappa(23, np.random.default_rng(8)))


@pytest.mark.parametrize("case", range(len(CASES)))
def test_aggressive_hierarchy_vcycle_and_pcg(orc, torch, xm, case):
    kind, agg, paths = CASES[case]
    p = _problem(kind)
    H = orc.Hierarchy(*p.csr(), agg_levels=agg, num_paths=paths)
    _say(f"[aggressive] {kind} n={p.n} agg={agg} paths={paths} sizes {H.sizes()}")
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n, p.n))
    B = inputs.uniform_rhs(p.n, 8, 500 + case)
    Bd = torch.from_numpy(B).cuda()
    for smoother in (0, 1):
        S = xm.Solver(H.export(), smoother=smoother)
        Zref = H.vcycle(B, smoother=smoother)
        Zd = torch.full_like(Bd, float("nan"))
        S.vcycle(Bd, Zd)
        torch.cuda.synchronize()
        Z = Zd.cpu().numpy()
        assert np.abs(Z - Zref).max() <= 1e-12 * np.abs(Zref).max()
        Xo, so, rco = H.solve(B, smoother=smoother, tol=1e-8)
        Xd = torch.zeros_like(Bd)
        rc, st = S.solve(Bd, Xd, tol=1e-8)
        S.close()
        X = Xd.cpu().numpy()
        err = np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
        _say(f"   smoother {smoother}: iters gpu {st['iters'].max()} oracle {so['iters'].max()}, "
             f"err {err.max():.1e}")
        assert rc == rco == xm.OK
        assert np.array_equal(st["iters"], so["iters"])
        assert err.max() <= 1e-7
    Sm = xm.Solver(H.export(), smoother=1, precision=xm.MIXED, index_bits=16)
    Xd = torch.zeros_like(Bd)
    rc, st = Sm.solve(Bd, Xd, tol=1e-8)
    Sm.close()
    X = Xd.cpu().numpy()
    tr = np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)
    assert rc == xm.OK and np.all(tr <= 1e-8)


def test_library_setup_aggressive_equals_oracle_solution(orc, torch, xm):
    p = inputs.poisson7(20)
    Hl = xm.HostHierarchy(*p.csr(), agg_levels=1, num_paths=1)
    Ho = orc.Hierarchy(*p.csr(), agg_levels=1, num_paths=1)
    assert Hl.sizes() == Ho.sizes()
    B = inputs.uniform_rhs(p.n, 4, 77)
    S = xm.Solver(Hl, smoother=1)
    Bd = torch.from_numpy(B).cuda()
    Xd = torch.zeros_like(Bd)
    rc, st = S.solve(Bd, Xd, tol=1e-8)
    S.close()
    Xo, so, _ = Ho.solve(B, smoother=1, tol=1e-8)
    assert rc == xm.OK and np.array_equal(st["iters"], so["iters"])
    err = np.linalg.norm(Xd.cpu().numpy() - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
    assert err.max() <= 1e-7


def test_paper_parameter_example(orc, torch, xm):
    """The configuration of the paper's parameter example (Section 2.4):
    pipelined BiCGStab, at most 20 iterations, AMG with two aggressive
    levels and two paths, coarsening to at most 500 rows, Chebyshev degree 2
    smoothing.  The library's own setup against the oracle's: the same
    hierarchy sizes, the oracle's iteration counts, error <= 1e-7."""
    p = inputs.poisson7(32)
    kw = dict(max_coarse=500, agg_levels=2, num_paths=2)
    Hl = xm.HostHierarchy(*p.csr(), **kw)
    Ho = orc.Hierarchy(*p.csr(), **kw)
    _say(f"[paper example] poisson32 levels {Hl.sizes()}")
    assert Hl.sizes() == Ho.sizes()
    assert Hl.sizes()[-1] <= 500
    B = inputs.uniform_rhs(p.n, 8, 78)
    Xo, so, rco = Ho.solve(B, method=orc.PBICGSTAB, smoother=orc.CHEBYSHEV, max_iters=20,
                           tol=1e-8)
    S = xm.Solver(Hl, method=xm.PBICGSTAB, smoother=xm.CHEBYSHEV, max_iters=20)
    Bd = torch.from_numpy(B).cuda()
    Xd = torch.zeros_like(Bd)
    rc, st = S.solve(Bd, Xd, tol=1e-8)
    S.close()
    X = Xd.cpu().numpy()
    err = np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(p.n, p.n))
    tr = np.linalg.norm(B - A @ X, axis=0) / np.linalg.norm(B, axis=0)
    _say(f"   iters gpu {st['iters'].tolist()} oracle {so['iters'].tolist()}, err {err.max():.1e}, "
         f"true relres {tr.max():.1e}")
    assert rc == rco == xm.OK
    assert np.array_equal(st["iters"], so["iters"])
    assert err.max() <= 1e-7 and np.all(tr <= 1e-8)
