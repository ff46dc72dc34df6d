"""Pins of the oracle's merged CG form (CPU only).

The merged form regroups CG's vector updates: x's update of iteration k is
applied in the pass of iteration k + 1 that forms p = z + beta p (which reads
the old p anyway), and a pending update is applied before a column's true
residual is formed.  No operation on an element changes, so its
results must equal the standard form's bit for bit; the standard form is
pinned on its own by the Galerkin property of its iterates
(test_oracle_krylov_pins).  The cases reach every place where a deferred
update is applied: ordinary convergence, iteration caps (the solve stops
right after the last iteration's application), true-residual restarts (the
application before the true residual),
breakdowns, frozen columns next to active ones, and each preconditioner
variant.
"""
import numpy as np
import pytest

import krylov_cases as kc
from paper_2103_07329_amd import inputs
from test_oracle_krylov_pins import dense, pcg_iterates, _rel


def _same(a, b):
    Xa, sa, rca = a
    Xb, sb, rcb = b
    assert rca == rcb
    assert np.array_equal(Xa, Xb)
    for key in ("iters", "relres", "true_relres", "converged", "restarts"):
        assert np.array_equal(sa[key], sb[key]), key


@pytest.mark.parametrize("smoother", [0, 1, 2])
@pytest.mark.parametrize("flexible", [False, True])
def test_merged_equals_standard(orc, smoother, flexible):
    p = inputs.jump7(9, inputs.jump_kappa(9, np.random.default_rng(8), block=3))
    H = orc.Hierarchy(*p.csr(), max_coarse=20)
    B = inputs.uniform_rhs(p.n, 5, 11)
    kw = dict(smoother=smoother, flexible=flexible, tol=1e-10)
    std = H.solve(B, **kw)
    assert std[2] == orc.OK and std[1]["iters"].min() > 3
    _same(H.solve(B, merged=True, **kw), std)


def test_merged_unpreconditioned(orc):
    p = inputs.poisson7(8)
    H = orc.Hierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, 3, 12)
    _same(H.solve(B, precond=False, merged=True, tol=1e-10),
          H.solve(B, precond=False, tol=1e-10))


def test_merged_iterates_at_caps(orc):
    # x_k after a cap of k iterations holds the k-th update only through the
    # application in the last iteration's p pass: it is the Galerkin iterate
    p = inputs.jump7(7, inputs.jump_kappa(7, np.random.default_rng(5), block=2))
    A = dense(*p.csr())
    H = orc.Hierarchy(*p.csr(), max_coarse=20)
    M = H.vcycle(np.eye(p.n))
    b = inputs.uniform_rhs(p.n, 1, 6)[:, 0]
    expected = pcg_iterates(A, M, b, 5)
    for k in range(1, 6):
        got = H.solve(b, merged=True, max_iters=k, tol=1e-300)
        _same(got, H.solve(b, max_iters=k, tol=1e-300))
        assert got[2] == orc.NOT_CONVERGED
        assert _rel(got[0], expected[k - 1]) <= 1e-9, k


def test_merged_frozen_and_active_columns(orc):
    # column 0 is an eigenvector of the 7-point Laplacian: unpreconditioned
    # CG converges on it in one iteration, then it stays frozen while the
    # other columns keep iterating (and keep applying their own updates)
    N = 8
    p = inputs.poisson7(N)
    H = orc.Hierarchy(*p.csr())
    g = np.arange(1, N + 1) / (N + 1)
    mode = np.einsum("i,j,k->ijk", np.sin(np.pi * g), np.sin(2 * np.pi * g),
                     np.sin(np.pi * g)).reshape(-1)
    B = np.column_stack([mode, inputs.uniform_rhs(p.n, 2, 13)])
    got = H.solve(B, precond=False, merged=True, tol=1e-10)
    _same(got, H.solve(B, precond=False, tol=1e-10))
    assert got[1]["iters"][0] == 1 and got[1]["iters"][1:].min() > 10


@pytest.mark.parametrize("flexible", [False, True])
def test_merged_true_residual_restart(orc, flexible):
    # the restart case of the standard form: the recurrence passes tol while
    # b - A x does not, which is judged on x after its pending update
    p = inputs.poisson7(10)
    H = orc.Hierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, 4, 3)
    X0 = 1e6 * inputs.uniform_rhs(p.n, 4, 4)
    got = H.solve(B, X0=X0, flexible=flexible, merged=True, tol=1e-11)
    _same(got, H.solve(B, X0=X0, flexible=flexible, tol=1e-11))
    assert got[2] == orc.OK and np.all(got[1]["restarts"] >= 1)


def test_merged_breakdown(orc):
    A, B = kc.indefinite()
    H = orc.Hierarchy(*kc.csr(A))
    got = H.solve(B, merged=True, tol=1e-12)
    _same(got, H.solve(B, tol=1e-12))
    assert got[2] == orc.EBREAKDOWN
