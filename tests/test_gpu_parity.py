"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Both sides take the same seeded inputs and the same hierarchy (the oracle's,
handed to the device as plain arrays), so FP64 results differ only by the
rounding of fused multiply-adds and the order of dot-product sums.
Tolerances (FP64): element-wise relative 1e-12 for single operators and one
V-cycle; for full solves, equal iteration counts and per-column relative
error <= 1e-7 against the oracle at the same tolerance (expected ~1e-11),
and a true relative residual <= tol recomputed on the CPU.
"""
import sys

import numpy as np
import pytest

from paper_2103_07329_amd import inputs

pytestmark = pytest.mark.gpu

MS = [1, 2, 4, 8, 16, 32]


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


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.fixture(scope="module")
def jump24(orc):
    rng = np.random.default_rng(77)
    p = inputs.jump7(24, inputs.jump_kappa(24, rng))
    return p, orc.Hierarchy(*p.csr())


@pytest.fixture(scope="module")
def poisson32(orc):
    p = inputs.poisson7(32)
    return p, orc.Hierarchy(*p.csr())


@pytest.mark.parametrize("m", MS)
def test_spmm_all_levels(orc, torch, xm, jump24, m):
    p, H = jump24
    _say(f"[spmm] jump24 m={m}")
    S = xm.Solver(H.export())
    rng = np.random.default_rng(m)
    for l in range(H.nlev):
        ops = [(xm.OP_A, H.A(l))]
        if l + 1 < H.nlev:
            ops += [(xm.OP_P, H.P(l)), (xm.OP_R, H.R(l))]
        for op, (rp, ci, v, (nr, nc)) in ops:
            X = rng.uniform(-1, 1, (nc, m))
            Yref = orc.spmm(rp, ci, v, X, ncols=nc)
            Xd = _dev(torch, X)
            Yd = torch.full((nr, m), np.nan, dtype=torch.float64, device="cuda")
            S.spmm(op, l, Xd, Yd)
            torch.cuda.synchronize()
            Y = Yd.cpu().numpy()
            assert np.isfinite(Y).all()
            assert _relmax(Y, Yref) <= 1e-13, (l, op)
    S.close()


@pytest.mark.parametrize("smoother", [0, 1])
@pytest.mark.parametrize("m", [1, 8, 32])
def test_vcycle_fp64(orc, torch, xm, jump24, smoother, m):
    p, H = jump24
    _say(f"[vcycle] jump24 smoother={smoother} m={m}")
    S = xm.Solver(H.export(), smoother=smoother)
    B = inputs.uniform_rhs(p.n, m, 5)
    Zref = H.vcycle(B, smoother=smoother)
    Bd = _dev(torch, B)
    Zd = torch.full_like(Bd, np.nan)
    S.vcycle(Bd, Zd)
    torch.cuda.synchronize()
    assert _relmax(Zd.cpu().numpy(), Zref) <= 1e-12
    S.close()


@pytest.mark.parametrize("smoother", [0, 1])
@pytest.mark.parametrize("m", [1, 3, 8])
def test_pcg_fp64_poisson32(orc, torch, xm, poisson32, smoother, m):
    p, H = poisson32
    _say(f"[pcg] poisson32 smoother={smoother} m={m}")
    B = inputs.uniform_rhs(p.n, 8, 1001)[:, :m].copy()
    Xo, so, rco = H.solve(B, smoother=smoother, tol=1e-8)
    assert rco == 0
    S = xm.Solver(H.export(), smoother=smoother)
    Bd = _dev(torch, B)
    Xd = torch.zeros_like(Bd)
    rc, st = S.solve(Bd, Xd, tol=1e-8)
    assert rc == xm.OK
    X = Xd.cpu().numpy()
    assert np.array_equal(st["iters"], so["iters"])
    for j in range(m):
        err = np.linalg.norm(X[:, j] - Xo[:, j]) / np.linalg.norm(Xo[:, j])
        assert err <= 1e-7, (j, err)
    # true residual recomputed on the CPU in FP64
    R = B - orc.spmm(*p.csr(), X)
    tr = np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)
    assert np.all(tr <= 1e-8)
    assert np.allclose(st["true_relres"], tr, rtol=1e-6, atol=1e-14)
    assert st["converged"].all()
    assert st["ms"] > 0.0          # the solve's wall time
    S.close()


def test_pcg_jump_vs_tight_reference(orc, torch, xm, jump24):
    p, H = jump24
    _say("[pcg] jump24 m=4 vs tight reference")
    B = inputs.uniform_rhs(p.n, 4, 3)
    Xref, _, _ = H.solve(B, tol=1e-12)
    Xalg, so, _ = H.solve(B, tol=1e-8)
    S = xm.Solver(H.export())
    Bd = _dev(torch, B)
    Xd = torch.zeros_like(Bd)
    rc, st = S.solve(Bd, Xd, tol=1e-8)
    assert rc == xm.OK
    X = Xd.cpu().numpy()
    assert np.array_equal(st["iters"], so["iters"])
    e_alg = np.linalg.norm(X - Xalg, axis=0) / np.linalg.norm(Xalg, axis=0)
    assert e_alg.max() <= 1e-7
    e_ref = np.linalg.norm(X - Xref, axis=0) / np.linalg.norm(Xref, axis=0)
    e_ref_oracle = np.linalg.norm(Xalg - Xref, axis=0) / np.linalg.norm(Xref, axis=0)
    # the device iterate is as close to the exact solution as the oracle's
    assert np.all(e_ref <= 1.01 * e_ref_oracle + 1e-13)
    S.close()


def test_solve_edge_cases(orc, torch, xm, poisson32):
    p, H = poisson32
    _say("[edge] zero column, iteration cap, NaN, x0 given, bad m")
    S = xm.Solver(H.export())
    B = inputs.uniform_rhs(p.n, 4, 1)
    B[:, 2] = 0.0
    Bd = _dev(torch, B)
    Xd = torch.full_like(Bd, 3.0)
    rc, st = S.solve(Bd, Xd)
    assert rc == xm.OK
    X = Xd.cpu().numpy()
    assert np.all(X[:, 2] == 0.0) and st["iters"][2] == 0 and st["converged"][2]
    # iteration cap
    S2 = xm.Solver(H.export(), max_iters=1)
    Xd = torch.zeros_like(Bd)
    rc, st = S2.solve(Bd, Xd)
    assert rc == xm.NOT_CONVERGED
    Xo, so, rco = H.solve(B, max_iters=1)
    assert rco == 1
    assert np.array_equal(st["iters"], so["iters"])
    assert np.allclose(Xd.cpu().numpy(), Xo, rtol=0, atol=1e-12 * np.abs(Xo).max())
    # NaN in B
    Bn = B.copy(); Bn[7, 1] = np.nan
    rc, _ = S.solve(_dev(torch, Bn), torch.zeros_like(Bd), check=False)
    assert rc == xm.EINVAL
    # m out of range
    B33 = _dev(torch, np.ones((p.n, 33)))
    rc, _ = S.solve(B33, torch.zeros_like(B33), check=False)
    assert rc == xm.EINVAL
    # initial guess = solution: 0 iterations
    Xs, _, _ = H.solve(B, tol=1e-12)
    S3 = xm.Solver(H.export(), x0_mode=xm.X0_GIVEN)
    Xd = _dev(torch, Xs)
    rc, st = S3.solve(Bd, Xd, tol=1e-10)
    assert rc == xm.OK and np.all(st["iters"] == 0)
    for s in (S, S2, S3):
        s.close()


def test_one_level_hierarchy(orc, torch, xm):
    p = inputs.poisson7(4)
    H = orc.Hierarchy(*p.csr())
    assert H.nlev == 1
    _say("[one-level] poisson4")
    B = inputs.uniform_rhs(p.n, 2, 4)
    S = xm.Solver(H.export())
    Bd = _dev(torch, B)
    Xd = torch.zeros_like(Bd)
    rc, st = S.solve(Bd, Xd, tol=1e-12)
    assert rc == xm.OK and np.all(st["iters"] == 1)
    Xo, so, _ = H.solve(B, tol=1e-12)
    assert _relmax(Xd.cpu().numpy(), Xo) <= 1e-12
    S.close()


def test_coarsest_level_beyond_lds(orc, torch, xm):
    """A coarsest level of more than 64 rows has its inverse applied from
    global memory: a one-level hierarchy of 216 rows (CG converges in one
    step) and a V-cycle coarsened to at most 500 rows (128 here), FP64
    against the oracle and the FP32 cycle within its rounding bounds."""
    p = inputs.poisson7(6)
    H = orc.Hierarchy(*p.csr(), max_coarse=500)
    assert H.nlev == 1 and p.n == 216
    _say("[coarse] one level of 216 rows")
    B = inputs.uniform_rhs(p.n, 3, 14)
    S = xm.Solver(H.export())
    Bd = _dev(torch, B)
    Xd = torch.zeros_like(Bd)
    rc, st = S.solve(Bd, Xd, tol=1e-12)
    S.close()
    Xo, so, _ = H.solve(B, tol=1e-12)
    assert rc == xm.OK and np.all(st["iters"] == 1)
    assert _relmax(Xd.cpu().numpy(), Xo) <= 1e-12
    p = inputs.jump7(24, inputs.jump_kappa(24, np.random.default_rng(15)))
    H = orc.Hierarchy(*p.csr(), max_coarse=500)
    nL = H.sizes()[-1]
    _say(f"[coarse] jump24 levels {H.sizes()}")
    assert 64 < nL <= 500
    for m in (1, 16):
        B = inputs.uniform_rhs(p.n, m, 15 + m)
        Bd = _dev(torch, B)
        for smoother in (0, 1):
            Zref = H.vcycle(B, smoother=smoother)
            S = xm.Solver(H.export(), smoother=smoother)
            Zd = torch.full_like(Bd, np.nan)
            S.vcycle(Bd, Zd)
            torch.cuda.synchronize()
            S.close()
            assert _relmax(Zd.cpu().numpy(), Zref) <= 1e-12, (m, smoother)
        Z32 = H.vcycle32(B, smoother=1)
        Sm = xm.Solver(H.export(), smoother=1, precision=xm.MIXED)
        Zd = torch.full_like(Bd, np.nan)
        Sm.vcycle(Bd, Zd)
        torch.cuda.synchronize()
        Sm.close()
        assert _relmax(Zd.cpu().numpy(), Z32) <= 128 * 2.0 ** -24, m


def test_device_setup_matches_host_setup_solution(orc, torch, xm):
    """The library's own host setup feeds the device solver: the solution
    must match the oracle (own setup) to the same bar."""
    p = inputs.poisson7(24)
    _say("[own-setup] poisson24 m=8 chebyshev")
    Hp = xm.HostHierarchy(*p.csr())
    Ho = orc.Hierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, 8, 12)
    Xo, so, _ = Ho.solve(B, smoother=1)
    S = xm.Solver(Hp, smoother=1)
    Bd = _dev(torch, B)
    Xd = torch.zeros_like(Bd)
    rc, st = S.solve(Bd, Xd)
    assert rc == xm.OK
    assert np.array_equal(st["iters"], so["iters"])
    e = np.linalg.norm(Xd.cpu().numpy() - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
    assert e.max() <= 1e-7
    S.close()


# --------------------------------------------------------------------------
# BiCGStab (FP64)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("smoother", [0, 1])
@pytest.mark.parametrize("m", [1, 8])
def test_bicgstab_fp64(orc, torch, xm, jump24, smoother, m):
    p, H = jump24
    _say(f"[bicgstab] jump24 smoother={smoother} m={m}")
    B = inputs.uniform_rhs(p.n, m, 31)
    Xo, so, rco = H.solve(B, method=orc.BICGSTAB, smoother=smoother, tol=1e-8)
    assert rco == 0
    S = xm.Solver(H.export(), method=xm.BICGSTAB, smoother=smoother)
    Bd = _dev(torch, B)
    Xd = torch.zeros_like(Bd)
    rc, st = S.solve(Bd, Xd, tol=1e-8)
    assert rc == xm.OK
    assert np.array_equal(st["iters"], so["iters"])
    X = Xd.cpu().numpy()
    e = np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
    assert e.max() <= 1e-7, e
    tr = np.linalg.norm(B - orc.spmm(*p.csr(), X), axis=0) / np.linalg.norm(B, axis=0)
    assert np.all(tr <= 1e-8)
    S.close()


def test_bicgstab_edge_cases(orc, torch, xm, poisson32):
    p, H = poisson32
    _say("[bicgstab-edge] zero column, cap, one-level")
    B = inputs.uniform_rhs(p.n, 4, 7)
    B[:, 1] = 0.0
    S = xm.Solver(H.export(), method=xm.BICGSTAB)
    Bd = _dev(torch, B)
    Xd = torch.zeros_like(Bd)
    rc, st = S.solve(Bd, Xd)
    assert rc == xm.OK and st["iters"][1] == 0 and np.all(Xd.cpu().numpy()[:, 1] == 0)
    S2 = xm.Solver(H.export(), method=xm.BICGSTAB, max_iters=1)
    rc, st = S2.solve(Bd, torch.zeros_like(Bd))
    Xo, so, rco = H.solve(B, method=orc.BICGSTAB, max_iters=1)
    assert rc == xm.NOT_CONVERGED and rco == orc.NOT_CONVERGED
    assert np.array_equal(st["iters"], so["iters"])
    p4 = inputs.poisson7(4)
    H4 = orc.Hierarchy(*p4.csr())
    S3 = xm.Solver(H4.export(), method=xm.BICGSTAB)
    B4 = inputs.uniform_rhs(p4.n, 2, 2)
    X4 = torch.zeros((p4.n, 2), dtype=torch.float64, device="cuda")
    rc, st = S3.solve(_dev(torch, B4), X4, tol=1e-12)
    assert rc == xm.OK and np.all(st["iters"] == 1)
    for s in (S, S2, S3):
        s.close()


# --------------------------------------------------------------------------
# mixed precision (FP32 V-cycle, FP64 Krylov) and 16-bit indices
# --------------------------------------------------------------------------
# An FP32 V-cycle differs from the FP64 one by the rounding of every stored
# operand and every operation.  The oracle's own FP32 cycle is pinned within
# 64 u (u = 2^-24) of the FP64 cycle (tests/test_oracle_fp32.py, where the
# bound is derived); the device's FP32 cycle must meet the same bound against
# the FP64 oracle, and so lie within 128 u of the oracle's FP32 cycle.
U32 = 2.0 ** -24


@pytest.mark.parametrize("smoother", [0, 1, 2])
@pytest.mark.parametrize("m", [1, 16])
def test_vcycle_mixed_vs_fp32_oracle(orc, torch, xm, jump24, smoother, m):
    p, H = jump24
    _say(f"[vcycle-mixed] jump24 smoother={smoother} m={m}")
    B = inputs.uniform_rhs(p.n, m, 6)
    Z64 = H.vcycle(B, smoother=smoother)
    Z32 = H.vcycle32(B, smoother=smoother)
    S = xm.Solver(H.export(), smoother=smoother, precision=xm.MIXED)
    Bd = _dev(torch, B)
    Zd = torch.full_like(Bd, np.nan)
    S.vcycle(Bd, Zd)
    torch.cuda.synchronize()
    Z = Zd.cpu().numpy()
    e64, e32, eo = _relmax(Z, Z64), _relmax(Z, Z32), _relmax(Z32, Z64)
    _say(f"  |gpu - fp64| {e64:.2e}, |gpu - fp32 oracle| {e32:.2e}, |fp32 oracle - fp64| {eo:.2e}")
    assert e64 <= 64 * U32, e64
    assert e32 <= 128 * U32, e32
    assert e64 > 1e-12          # really computed in reduced precision
    S.close()


@pytest.mark.parametrize("smoother", [0, 1])
def test_index16_bitwise_equal_index32(orc, torch, xm, smoother):
    """16-bit column offsets decode to the same columns in the same order,
    so the FP32 V-cycle must be bit-identical to the 32-bit-index one.
    At 136^3 the z-neighbours lie N^2 = 18496 > 2^14 rows away, so level-0
    row blocks need three index windows."""
    p = inputs.anisotropic7(136)
    _say(f"[index16] aniso136 smoother={smoother}")
    Hh = xm.HostHierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, 2, 9)
    Bd = _dev(torch, B)
    outs = []
    for bits in (32, 16):
        S = xm.Solver(Hh, smoother=smoother, precision=xm.MIXED, index_bits=bits)
        S.autotune(2, enable=False)     # same row splits for both index widths
        if bits == 16:
            fr = [S.index16_fraction(l) for l in range(S.nlev - 1)]
            _say("   16-bit fraction per level (A, P, R):", [tuple(round(x, 3) for x in f) for f in fr])
            assert fr[0][0] == 1.0
        Zd = torch.full_like(Bd, np.nan)
        S.vcycle(Bd, Zd)
        torch.cuda.synchronize()
        outs.append(Zd.cpu().numpy())
        S.close()
    assert np.isfinite(outs[0]).all()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("method,smoother,m", [(0, 0, 8), (1, 0, 8), (0, 1, 16), (1, 1, 16),
                                                (1, 2, 4)])
def test_mixed_solve_accuracy(orc, torch, xm, jump24, method, smoother, m):
    """FP64 Krylov with an FP32 preconditioner reaches the same tolerance;
    its error against a tight FP64 reference is no worse than twice the
    FP64 oracle's own error at the same tolerance (or 1e-7)."""
    p, H = jump24
    _say(f"[mixed-solve] jump24 method={method} smoother={smoother} m={m}")
    B = inputs.uniform_rhs(p.n, m, 44)
    Xref, _, _ = H.solve(B, method=method, smoother=smoother, tol=1e-12)
    Xalg, so, _ = H.solve(B, method=method, smoother=smoother, tol=1e-8)
    S = xm.Solver(H.export(), method=method, smoother=smoother, precision=xm.MIXED,
                  index_bits=16)
    Bd = _dev(torch, B)
    Xd = torch.zeros_like(Bd)
    rc, st = S.solve(Bd, Xd, tol=1e-8)
    assert rc == xm.OK
    X = Xd.cpu().numpy()
    tr = np.linalg.norm(B - orc.spmm(*p.csr(), X), axis=0) / np.linalg.norm(B, axis=0)
    assert np.all(tr <= 1e-8)
    e_mix = np.linalg.norm(X - Xref, axis=0) / np.linalg.norm(Xref, axis=0)
    e_alg = np.linalg.norm(Xalg - Xref, axis=0) / np.linalg.norm(Xref, axis=0)
    assert np.all(e_mix <= np.maximum(1e-7, 2 * e_alg)), (e_mix, e_alg)
    # the FP32 preconditioner costs at most a couple of iterations
    assert np.all(st["iters"] <= so["iters"] + 2)
    _say(f"   iters mixed {st['iters'].tolist()} fp64 {so['iters'].tolist()} "
         f"err {e_mix.max():.2e} (fp64 oracle {e_alg.max():.2e})")
    S.close()


def _poisson_with_far_couplings(N, seed, w=0.01):
    """7-point Poisson plus symmetric weak couplings from every row of the
    first quarter to a random column in the second half (M-matrix kept: each
    added -w is matched by +w on both diagonals).  Row blocks of the first
    quarter then touch at least five 2^14-wide column windows, which forces
    the 32-bit fallback of the 16-bit index encoding there; the other blocks
    stay compressed."""
    import scipy.sparse as sp
    p = inputs.poisson7(N)
    n = p.n
    rng = np.random.default_rng(seed)
    i = np.arange(n // 4)
    j = rng.integers(n // 2, n, i.size)
    E = sp.coo_matrix((np.full(i.size, -w), (i, j)), shape=(n, n)).tocsr()
    E = E + E.T
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(n, n)) + E
    A = A + sp.diags(-np.asarray(E.sum(axis=1)).ravel())
    A = sp.csr_matrix(A)
    A.sum_duplicates()
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64)


def test_index16_wide_fallback_bitwise(orc, torch, xm):
    rp, ci, v = _poisson_with_far_couplings(48, 3)
    _say("[index16-wide] poisson48 + far couplings")
    Hh = xm.HostHierarchy(rp, ci, v)
    B = inputs.uniform_rhs(len(rp) - 1, 4, 10)
    Bd = _dev(torch, B)
    outs = []
    for bits in (32, 16):
        S = xm.Solver(Hh, precision=xm.MIXED, index_bits=bits)
        S.autotune(4, enable=False)     # same row splits for both index widths
        if bits == 16:
            fr = S.index16_fraction(0)
            _say("   level-0 16-bit fraction (A, P, R):", fr)
            assert 0.0 < fr[0] < 1.0
        Zd = torch.full_like(Bd, np.nan)
        S.vcycle(Bd, Zd)
        torch.cuda.synchronize()
        outs.append(Zd.cpu().numpy())
        S.close()
    assert np.isfinite(outs[0]).all()
    assert np.array_equal(outs[0], outs[1])


def test_autotune_choices_and_invariance(orc, torch, xm, jump24):
    """The autotuner only changes how a row's nonzeros are split over lanes
    (the order of additions inside a row), so solves with and without it
    agree to rounding and take the same iterations."""
    p, H = jump24
    _say("[autotune] jump24 m=16")
    B = inputs.uniform_rhs(p.n, 16, 71)
    Bd = _dev(torch, B)
    S = xm.Solver(H.export(), smoother=xm.CHEBYSHEV)
    S.autotune(16, enable=False)
    X0 = torch.zeros_like(Bd)
    rc0, st0 = S.solve(Bd, X0)
    S.autotune(16, enable=True)
    tun = S.tuning(16)
    _say("   splits (A, A pre-smoothing, P, R) per level:", tun)
    # lane groups plus any of the flags sweep 16, 512-thread blocks 32,
    # 32-bit indices 64, twice the columns per lane 128, banded walk 256..768
    ok = {s | f for s in (1, 2, 4, 8) for f in range(0, 1024, 16)}
    for l, t in enumerate(tun[:-1]):
        assert t[0] in ok
        if l + 1 < S.nlev:
            assert t[1] in ok and t[2] in ok and t[3] in ok
    assert tun[-1][0] in ok
    X1 = torch.zeros_like(Bd)
    rc1, st1 = S.solve(Bd, X1)
    assert rc0 == rc1 == xm.OK
    assert np.array_equal(st0["iters"], st1["iters"])
    assert _relmax(X1.cpu().numpy(), X0.cpu().numpy()) <= 1e-11
    S.close()


def test_tuning_cache_shared_across_handles(orc, torch, xm, jump24):
    """The autotuner's choices are cached per operator key: a second handle
    on the same hierarchy takes the first one's launch shapes without timing,
    so the two solve bit for bit alike; a re-tune on one handle times afresh
    and replaces the cached choices, which a third handle then takes."""
    p, H = jump24
    _say("[autotune] tuning cache, jump24 m=8")
    B = inputs.uniform_rhs(p.n, 8, 72)
    Bd = _dev(torch, B)
    out = []

    def solve_new():
        S = xm.Solver(H.export(), smoother=xm.CHEBYSHEV)
        X = torch.zeros_like(Bd)
        rc, _ = S.solve(Bd, X)
        assert rc == xm.OK
        out.append((S, X))
        return S, X

    S1, X1 = solve_new()
    S2, X2 = solve_new()
    assert S2.tuning(8) == S1.tuning(8)
    assert torch.equal(X1, X2)
    S2.autotune(8, enable=True)
    S3, X3 = solve_new()
    assert S3.tuning(8) == S2.tuning(8)
    X2b = torch.zeros_like(Bd)
    S2.solve(Bd, X2b)
    assert torch.equal(X3, X2b)
    for S, _ in out:
        S.close()


# --------------------------------------------------------------------------
# batched uneven systems (one captured graph)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("precision", [0, 1])
def test_batched_equals_individual(orc, torch, xm, precision):
    """Every replay of the captured graph (with eager checks between
    replays) must give exactly the eager per-system result."""
    _say(f"[batched] 5 jump systems, precision={precision}")
    systems = inputs.batched_systems(seed=1004, count=5, max_side=24)
    solvers, Bs = [], []
    for prob, B in systems:
        Hh = xm.HostHierarchy(*prob.csr())
        solvers.append(xm.Solver(Hh, precision=precision))
        Bs.append(_dev(torch, B))
    ref = []
    for S, Bd in zip(solvers, Bs):
        X = torch.zeros_like(Bd)
        rc, st = S.solve(Bd, X)
        assert rc == xm.OK
        ref.append((X.cpu().numpy(), st["iters"]))
    batch = xm.Batch(solvers, iters_per_launch=3)
    for rep in range(2):
        Xs = [torch.full_like(Bd, 7.0) for Bd in Bs]
        rc, sts = batch.solve(Bs, Xs)
        assert rc == xm.OK
        for (Xr, itr), X, st in zip(ref, Xs, sts):
            assert np.array_equal(st["iters"], itr)
            assert np.array_equal(X.cpu().numpy(), Xr)
            assert st["converged"].all()
            assert st["ms"] == sts[0]["ms"] > 0.0   # the whole batch's wall time
    batch.close()
    for S in solvers:
        S.close()


def test_batched_vs_oracle_and_cap(orc, torch, xm):
    _say("[batched] 3 systems vs oracle, iteration cap")
    systems = inputs.batched_systems(seed=7, count=3, max_side=16)
    solvers, Bs, orcs = [], [], []
    for prob, B in systems:
        Ho = orc.Hierarchy(*prob.csr())
        solvers.append(xm.Solver(Ho.export()))
        orcs.append((Ho, B))
        Bs.append(_dev(torch, B))
    batch = xm.Batch(solvers)
    Xs = [torch.zeros_like(b) for b in Bs]
    rc, sts = batch.solve(Bs, Xs)
    assert rc == xm.OK
    for (Ho, B), X, st in zip(orcs, Xs, sts):
        Xo, so, _ = Ho.solve(B)
        assert np.array_equal(st["iters"], so["iters"])
        e = np.linalg.norm(X.cpu().numpy() - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
        assert e.max() <= 1e-7
    batch.close()
    capped = [xm.Solver(Ho.export(), max_iters=2) for Ho, _ in orcs]
    b2 = xm.Batch(capped, iters_per_launch=4)
    Xs = [torch.zeros_like(b) for b in Bs]
    rc, sts = b2.solve(Bs, Xs)
    assert rc == xm.NOT_CONVERGED
    for st in sts:
        assert st["iters"].max() <= 2
    b2.close()
    for S in solvers + capped:
        S.close()
