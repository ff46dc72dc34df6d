"""Pins of the oracle's FP32 V-cycle (the reduced-precision preconditioner),
CPU only.

* It is an FP32 computation of the FP64 cycle: the two agree to a bound
  derived from FP32 rounding (unit roundoff u = 2^-24; each pass rounds every
  stored operand and every multiply-add once, a row sum of k terms costs at
  most k u; with row lengths <= 27 on these problems, two smoothing passes,
  a residual and two transfers per level, and a contraction of the error by
  the cycle itself, 64 u bounds the max-norm relative difference with
  room), and they do differ by more than FP64 rounding.
* A dense float32 computation with NumPy of the same cycle (two and three
  levels, every smoother written as its dense splitting) agrees with it
  within FP32 rounding of differently ordered sums.
* The FP32 cycle is symmetric to FP32 accuracy.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2103_07329_amd import inputs

U32 = 2.0 ** -24


def dense(rp, ci, v, shape):
    return sp.csr_matrix((v, ci, rp), shape=shape).toarray()


def _relmax(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _problem(k):
    rng = np.random.default_rng(77)
    return [inputs.poisson7(12), inputs.jump7(16, inputs.jump_kappa(16, rng, block=4)),
            inputs.anisotropic7(10)][k]


@pytest.mark.parametrize("smoother", [0, 1, 2])
@pytest.mark.parametrize("k", [0, 1, 2])
def test_vcycle32_is_an_fp32_computation_of_the_cycle(orc, smoother, k):
    p = _problem(k)
    H = orc.Hierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, 3, 8)
    z64 = H.vcycle(B, smoother=smoother)
    z32 = H.vcycle32(B, smoother=smoother)
    d = _relmax(z32, z64)
    assert 1e-10 < d <= 64 * U32, d
    # the result is a float32 value widened to float64
    assert np.array_equal(z32, z32.astype(np.float32).astype(np.float64))


def _dense_cycle32(H, b, smoother, omega=2.0 / 3.0, degree=2, lo_frac=0.3, hi_frac=1.1,
                   gs_block=8):
    """The V(1,1) cycle from zero with dense float32 NumPy operations; the
    Gauss-Seidel sweeps as their dense splittings x + M^-1 (b - A x)."""
    f = np.float32
    L = H.nlev
    A = [dense(*H.A(l)[:3], H.A(l)[3]) for l in range(L)]
    P = [dense(*H.P(l)[:3], H.P(l)[3]) for l in range(L - 1)]
    R = [dense(*H.R(l)[:3], H.R(l)[3]) for l in range(L - 1)]

    def smooth(l, bl, x):
        Al = A[l].astype(f)
        dinv = (1.0 / np.diag(A[l])).astype(f)
        if smoother == 0:
            return x + f(omega) * dinv[:, None] * (bl - Al @ x)
        if smoother == 1:
            hi = hi_frac * H.lmax(l)
            lo = lo_frac * hi
            theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
            sigma = theta / delta
            rho = 1.0 / sigma
            r = dinv[:, None] * (bl - Al @ x)
            d = r / f(theta)
            for kk in range(1, degree + 1):
                x = x + d
                if kk < degree:
                    rn = 1.0 / (2.0 * sigma - rho)
                    r = r - dinv[:, None] * (Al @ d)
                    d = f(rn * rho) * d + f(2.0 * rn / delta) * r
                    rho = rn
            return x
        n = A[l].shape[0]
        blk = np.arange(n) // gs_block
        same = blk[:, None] == blk[None, :]
        dl1 = np.diag(A[l]) + np.where(~same, np.abs(A[l]), 0.0).sum(axis=1)
        low = np.where(same & (np.arange(n)[:, None] > np.arange(n)[None, :]), A[l], 0.0)
        Mf = (np.diag(dl1) + low).astype(f)
        Mb = (np.diag(dl1) + low.T).astype(f)
        x = x + np.linalg.solve(Mf, bl - Al @ x)
        return x + np.linalg.solve(Mb, bl - Al @ x)

    def cycle(l, bl):
        if l == L - 1:
            inv = np.linalg.inv(A[l]).astype(f)
            return inv @ bl
        x = np.zeros_like(bl)
        x = smooth(l, bl, x)
        r = bl - A[l].astype(f) @ x
        xc = cycle(l + 1, R[l].astype(f) @ r)
        x = x + P[l].astype(f) @ xc
        return smooth(l, bl, x)

    return cycle(0, b.astype(f)).astype(np.float64)


@pytest.mark.parametrize("smoother", [0, 1, 2])
@pytest.mark.parametrize("N,coarse", [(6, 60), (7, 20)])
def test_vcycle32_matches_dense_float32(orc, smoother, N, coarse):
    p = inputs.jump7(N, inputs.jump_kappa(N, np.random.default_rng(3), block=2))
    H = orc.Hierarchy(*p.csr(), max_coarse=coarse)
    assert H.nlev >= 2
    B = inputs.uniform_rhs(p.n, 2, 4)
    z32 = H.vcycle32(B, smoother=smoother)
    zd = _dense_cycle32(H, B, smoother)
    z64 = H.vcycle(B, smoother=smoother)
    # both are FP32 computations of the same cycle: each within 64 u of FP64,
    # so within 128 u of each other; and the dense one is no FP64 result
    assert _relmax(z32, zd) <= 128 * U32
    assert _relmax(zd, z64) > 1e-10


def test_vcycle32_symmetric_to_fp32_accuracy(orc):
    p = _problem(1)
    H = orc.Hierarchy(*p.csr())
    U = np.random.default_rng(9).standard_normal((p.n, 5))
    for smoother in (0, 1, 2):
        G = U.T @ H.vcycle32(U, smoother=smoother)
        assert np.abs(G - G.T).max() <= 64 * U32 * np.abs(G).max()
