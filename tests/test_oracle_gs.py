"""Pins of the oracle's l1-hybrid Gauss-Seidel sweep (the GPU form of the
symmetric Gauss-Seidel smoother) against dense triangular solves written
from the splitting's definition, and the special cases that reduce to
textbook methods: one block = plain Gauss-Seidel, blocks of one row =
l1-Jacobi."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.linalg import solve_triangular

from paper_2103_07329_amd import inputs

from test_oracle_pins import _hgs_splitting, dense


def _random_spd(n, seed):
    rng = np.random.default_rng(seed)
    W = sp.random(n, n, density=0.3, random_state=rng).toarray()
    W = np.triu(W, 1)
    W = W + W.T
    A = np.diag(W.sum(axis=1) + 0.5) - W
    S = sp.csr_matrix(A)
    S.sort_indices()
    return A, (S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(np.float64))


def test_one_block_is_gauss_seidel(orc):
    p = inputs.jump7(5, inputs.jump_kappa(5, np.random.default_rng(2), block=2))
    A = dense(*p.csr())
    rng = np.random.default_rng(1)
    b = rng.standard_normal((p.n, 3))
    xo = rng.standard_normal((p.n, 3))
    L, U, D = np.tril(A, -1), np.triu(A, 1), np.diag(np.diag(A))
    xf = orc.hgs_sweep(*p.csr(), p.n, 0, b, xo)
    assert np.allclose(xf, solve_triangular(D + L, b - U @ xo, lower=True), rtol=1e-12, atol=1e-12)
    xb = orc.hgs_sweep(*p.csr(), p.n, 1, b, xo)
    assert np.allclose(xb, solve_triangular(D + U, b - L @ xo, lower=False), rtol=1e-12,
                       atol=1e-12)


def test_single_row_blocks_are_l1_jacobi(orc):
    A, csr = _random_spd(30, 4)
    rng = np.random.default_rng(5)
    b = rng.standard_normal((30, 2))
    xo = rng.standard_normal((30, 2))
    dl1 = np.diag(A) + (np.abs(A).sum(axis=1) - np.abs(np.diag(A)))
    expect = xo + (b - A @ xo) / dl1[:, None]
    for backward in (0, 1):
        assert np.allclose(orc.hgs_sweep(*csr, 1, backward, b, xo), expect, rtol=1e-12,
                           atol=1e-12)


@pytest.mark.parametrize("B", [2, 3, 8])
@pytest.mark.parametrize("backward", [0, 1])
def test_sweep_equals_splitting(orc, B, backward):
    # n = 31 leaves a ragged last block for every B
    A, csr = _random_spd(31, 10 + B)
    rng = np.random.default_rng(B)
    b = rng.standard_normal((31, 4))
    xo = rng.standard_normal((31, 4))
    Mf, Mb = _hgs_splitting(A, B)
    M = Mb if backward else Mf
    expect = xo + solve_triangular(M, b - A @ xo, lower=not backward)
    got = orc.hgs_sweep(*csr, B, backward, b, xo)
    assert np.allclose(got, expect, rtol=1e-12, atol=1e-12)


def test_symmetric_sweep_is_a_self_adjoint_contraction(orc):
    """S = (I - Mb^-1 A)(I - Mf^-1 A) with Mb = Mf^T for symmetric A: A S is
    symmetric and ||S||_A < 1 (the l1 diagonal makes each sweep convergent)."""
    A, csr = _random_spd(24, 7)
    n = 24
    I = np.eye(n)
    Z = np.zeros((n, n))
    # error propagation: sweep the identity columns with b = 0
    Ef = orc.hgs_sweep(*csr, 5, 0, Z, I)
    S = orc.hgs_sweep(*csr, 5, 1, Z, Ef)
    AS = A @ S
    assert np.allclose(AS, AS.T, rtol=0, atol=1e-12 * np.abs(AS).max())
    Lc = np.linalg.cholesky(A)
    assert np.linalg.norm(Lc.T @ S @ np.linalg.inv(Lc.T), 2) < 1.0
