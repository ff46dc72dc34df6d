"""GPU parity at the full sizes of the benchmark workloads, in the launch
configuration the bench times: the library's own host setup, and the launch
shapes its autotuner picks on the first solve of the handle.

* Poisson 128^3, Chebyshev-2 V(1,1) PCG (Section 3's 7-point Poisson
  problems): the oracle's V-cycle and whole solve finish in seconds at this
  size, so they are compared element by element.  The FP64 V-cycle must be
  within 1e-12 of the oracle's.  The FP64 solve (m = 16 and m = 1) must take
  the oracle's iteration counts, lie within 1e-7 of its solution, and pass
  1e-8 in the true residual recomputed on the CPU.  The FP32 V-cycle with
  16-bit offsets must meet the bounds of the small mixed-precision tests
  against the oracle's FP64 and FP32 cycles, and the mixed solve the same
  solution and residual bounds as the FP64 one.
* Every FP64 operator of that hierarchy (A_l, P_l, R_l) at m = 16: sampled
  rows of Y = Op X against the row sums formed on the CPU one row at a time.
* Anisotropic 256^3, BiCGStab with the FP32 V-cycle and 16-bit offsets
  (m = 16): the oracle's whole solve takes minutes here, so properties that
  hold at any size.  The true residual (the oracle's SpMM) must be <= 1e-8,
  the FP64 solve on the same hierarchy must agree within 1e-7, and sampled
  rows of A_0 must match.
* The warm-start network at 128^3 (m = 32 Gaussian-source columns).  An
  output voxel depends only on the 9^3 inputs around it: four 3^3 layers,
  no bias, zero padding.  So sampled voxels (interior, on faces and edges,
  at corners) are compared with the oracle's forward over a 9^3 patch
  aligned to the volume's faces where the voxel is near them.
"""
import sys

import numpy as np
import pytest
from scipy.sparse import csr_matrix

import oracle
from paper_2103_07329_amd import inputs

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


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


def _relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _relcols(a, b):
    return float((np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max())


def _true_relres(orc, csr, B, X):
    R = B - orc.spmm(*csr, X)
    return float((np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)).max())


def _tuned_solver(torch, xm, H, Bd, **opts):
    """A handle whose first solve has tuned its launch shapes (as the
    bench's warm-up does)."""
    S = xm.Solver(H, **opts)
    X = torch.zeros_like(Bd)
    rc, _ = S.solve(Bd, X, tol=1e-8)
    assert rc == xm.OK
    return S


def _solve(torch, S, Bd):
    X = torch.zeros_like(Bd)
    rc, st = S.solve(Bd, X, tol=1e-8)
    torch.cuda.synchronize()
    return X.cpu().numpy(), st, rc


def _check_sampled_rows(torch, S, op, level, csr, m, rng, what):
    """Y = Op X on the device against sampled rows summed on the CPU: the
    first and last 64 rows and 4096 random ones.  Both sides round a row sum
    of k terms by at most k u sum |a x| each (FP64), so |dev - ref| <=
    2 (k + 1) 2^-53 sum |a x| per row."""
    rp, ci, v, (nr, nc) = csr
    X = rng.uniform(-1.0, 1.0, (nc, m))
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.full((nr, m), float("nan"), dtype=torch.float64, device="cuda")
    S.spmm(op, level, Xd, Yd)
    torch.cuda.synchronize()
    Y = Yd.cpu().numpy()
    assert np.isfinite(Y).all(), what          # every row written
    rows = np.unique(np.concatenate([np.arange(min(nr, 64)), np.arange(max(0, nr - 64), nr),
                                     rng.integers(0, nr, min(nr, 4096))]))
    A = csr_matrix((v, ci, rp), shape=(nr, nc))[rows]
    ref = A @ X
    mag = abs(A) @ np.abs(X)
    k = np.diff(A.indptr)[:, None]
    bound = 2.0 * (k + 1) * 2.0 ** -53 * mag + 1e-300
    worst = float((np.abs(Y[rows] - ref) / bound).max())
    _say(f"  {what}: {nr} x {nc}, {len(rows)} rows sampled, worst err/bound {worst:.3f}")
    assert worst <= 1.0, what


# --------------------------------------------------------------------------
# Poisson 128^3 (the bench's default workload)
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def p128(orc, torch, xm):
    _say("[full] poisson 128^3: library and oracle setups")
    p = inputs.poisson7(128)
    H = xm.HostHierarchy(*p.csr())
    Ho = orc.Hierarchy(*p.csr())
    assert H.sizes() == Ho.sizes()
    B = inputs.uniform_rhs(p.n, 16, 1002)       # the bench's right-hand sides
    Bd = torch.from_numpy(B).cuda()
    return p, H, Ho, B, Bd


@pytest.fixture(scope="module")
def oracle128(orc, p128):
    p, H, Ho, B, Bd = p128
    _say("[full] poisson 128^3: oracle solve, m = 16")
    Xo, so, rco = Ho.solve(B, smoother=orc.CHEBYSHEV, tol=1e-8)
    assert rco == 0
    return Xo, so


def test_poisson128_fp64_vcycle_and_operators(orc, torch, xm, p128):
    p, H, Ho, B, Bd = p128
    S = _tuned_solver(torch, xm, H, Bd, smoother=xm.CHEBYSHEV, method=xm.CG)
    _say(f"[full] poisson 128^3 FP64: launch shapes {S.tuning(16)}")
    Zo = Ho.vcycle(B, smoother=orc.CHEBYSHEV)
    Zd = torch.full_like(Bd, float("nan"))
    S.vcycle(Bd, Zd)
    torch.cuda.synchronize()
    e = _relmax(Zd.cpu().numpy(), Zo)
    _say(f"  V-cycle: max rel err vs oracle {e:.2e}")
    assert e <= 1e-12
    rng = np.random.default_rng(128)
    for l in range(S.nlev):
        _check_sampled_rows(torch, S, xm.OP_A, l, H.A(l), 16, rng, f"A_{l}")
        if l < S.nlev - 1:
            _check_sampled_rows(torch, S, xm.OP_P, l, H.P(l), 16, rng, f"P_{l}")
            _check_sampled_rows(torch, S, xm.OP_R, l, H.R(l), 16, rng, f"R_{l}")
    S.close()


def test_poisson128_fp64_solve_against_oracle(orc, torch, xm, p128, oracle128):
    p, H, Ho, B, Bd = p128
    Xo, so = oracle128
    S = _tuned_solver(torch, xm, H, Bd, smoother=xm.CHEBYSHEV, method=xm.CG)
    X, st, rc = _solve(torch, S, Bd)
    err, tr = _relcols(X, Xo), _true_relres(orc, p.csr(), B, X)
    _say(f"[full] poisson 128^3 FP64 m=16: iters {st['iters'].tolist()} (oracle "
         f"{so['iters'].tolist()}), err vs oracle {err:.2e}, true relres {tr:.2e}")
    assert rc == xm.OK
    assert np.array_equal(st["iters"], so["iters"])
    assert err <= 1e-7 and tr <= 1e-8
    S.close()
    # one right-hand side alone (m = 1, its own launch shapes)
    B1d = Bd[:, :1].contiguous()
    S1 = _tuned_solver(torch, xm, H, B1d, smoother=xm.CHEBYSHEV, method=xm.CG)
    X1, st1, rc1 = _solve(torch, S1, B1d)
    Xo1, so1, _ = Ho.solve(B[:, :1].copy(), smoother=orc.CHEBYSHEV, tol=1e-8)
    err1 = _relcols(X1, Xo1)
    _say(f"  m=1: iters {st1['iters'].tolist()} (oracle {so1['iters'].tolist()}), err {err1:.2e}")
    assert rc1 == xm.OK and np.array_equal(st1["iters"], so1["iters"]) and err1 <= 1e-7
    S1.close()


def test_poisson128_mixed_against_oracle(orc, torch, xm, p128, oracle128):
    p, H, Ho, B, Bd = p128
    Xo, so = oracle128
    S = _tuned_solver(torch, xm, H, Bd, smoother=xm.CHEBYSHEV, method=xm.CG,
                      precision=xm.MIXED, index_bits=16)
    _say(f"[full] poisson 128^3 mixed: launch shapes {S.tuning(16)}")
    Z64 = Ho.vcycle(B, smoother=orc.CHEBYSHEV)
    Z32 = Ho.vcycle32(B, smoother=orc.CHEBYSHEV)
    Zd = torch.full_like(Bd, float("nan"))
    S.vcycle(Bd, Zd)
    torch.cuda.synchronize()
    Z = Zd.cpu().numpy()
    e64, e32 = _relmax(Z, Z64), _relmax(Z, Z32)
    _say(f"  FP32 V-cycle: |gpu - fp64| {e64:.2e} ({e64 / U32:.1f} u), "
         f"|gpu - fp32 oracle| {e32:.2e} ({e32 / U32:.1f} u)")
    assert e64 <= 64 * U32 and e32 <= 128 * U32
    assert e64 > 1e-12
    X, st, rc = _solve(torch, S, Bd)
    err, tr = _relcols(X, Xo), _true_relres(orc, p.csr(), B, X)
    _say(f"  mixed solve: iters {st['iters'].tolist()}, err vs FP64 oracle {err:.2e}, "
         f"true relres {tr:.2e}")
    assert rc == xm.OK and err <= 1e-7 and tr <= 1e-8
    S.close()


# --------------------------------------------------------------------------
# anisotropic 256^3, BiCGStab with the FP32 V-cycle and 16-bit offsets
# --------------------------------------------------------------------------
def test_aniso256_mixed_bicgstab_properties(orc, torch, xm):
    _say("[full] aniso 256^3: library setup")
    p = inputs.anisotropic7(256)
    H = xm.HostHierarchy(*p.csr())
    B = inputs.uniform_rhs(p.n, 16, 1003)       # the bench's right-hand sides
    Bd = torch.from_numpy(B).cuda()
    opts = dict(smoother=xm.JACOBI, method=xm.BICGSTAB)
    Sm = _tuned_solver(torch, xm, H, Bd, precision=xm.MIXED, index_bits=16, **opts)
    Xm, stm, rcm = _solve(torch, Sm, Bd)
    Sm.close()
    trm = _true_relres(orc, p.csr(), B, Xm)
    S64 = _tuned_solver(torch, xm, H, Bd, **opts)
    X64, st64, rc64 = _solve(torch, S64, Bd)
    tr64 = _true_relres(orc, p.csr(), B, X64)
    d = _relcols(Xm, X64)
    _say(f"  mixed: iters {stm['iters'].max()}, true relres {trm:.2e}; FP64: iters "
         f"{st64['iters'].max()}, true relres {tr64:.2e}; mixed vs FP64 {d:.2e}")
    assert rcm == rc64 == xm.OK
    assert trm <= 1e-8 and tr64 <= 1e-8 and d <= 1e-7
    _check_sampled_rows(torch, S64, xm.OP_A, 0, H.A(0), 16, np.random.default_rng(256), "A_0")
    S64.close()


# --------------------------------------------------------------------------
# the warm-start network at 128^3
# --------------------------------------------------------------------------
def _patch_forward(Wq, xin, pt, N):
    """The network's output at voxel pt = (k, j, i) of an N^3 volume, from the
    9^3 input patch that holds its receptive field, aligned to the volume's
    faces where pt lies within 4 voxels of them (so the oracle's zero padding
    falls where the volume's does)."""
    lo = [min(max(c - 4, 0), N - 9) for c in pt]
    patch = xin[lo[0]:lo[0] + 9, lo[1]:lo[1] + 9, lo[2]:lo[2] + 9]
    y = oracle.cnn_forward(9, Wq, np.ascontiguousarray(patch).reshape(-1), quantize=True)[-1]
    return float(y.reshape(9, 9, 9)[pt[0] - lo[0], pt[1] - lo[1], pt[2] - lo[2]])


def test_warmstart_network_full_size_sampled_voxels(torch, xm):
    N, m = 128, 32
    n = N ** 3
    _say(f"[full] warm-start network {N}^3, m={m}")
    rng = np.random.default_rng(555)
    Ws = [(2.0 * rng.standard_normal((co, ci, 27)) / np.sqrt(27 * ci)).astype(np.float32)
          for ci, co in oracle.CNN_LAYERS]
    net = xm.Cnn(N, xm.join_weights(Ws))
    B = inputs.gaussian_rhs(N, m, 5005)
    Bd = torch.from_numpy(B).cuda()
    X0d = torch.zeros((n, m), dtype=torch.float64, device="cuda")
    fb = net.warmstart(Bd, X0d, None)
    torch.cuda.synchronize()
    net.close()
    assert np.all(fb == 0)
    X0 = X0d.cpu().numpy().reshape(N, N, N, m)
    Wq = [oracle.bf16(W) for W in Ws]
    E, H_ = 0, N - 1
    pts = [(a, b, c) for a in (E, H_) for b in (E, H_) for c in (E, H_)]          # corners
    pts += [(E, 64, 64), (H_, 64, 64), (64, E, 64), (64, H_, 64), (64, 64, E), (64, 64, H_)]
    pts += [(E, E, 37), (H_, 70, E), (2, 3, 90), (125, 126, 1)]                    # edges, near faces
    pts += [tuple(int(t) for t in rng.integers(0, N, 3)) for _ in range(24)]
    for j in range(0, m, 4):
        s = np.sqrt(B[:, j] @ B[:, j] / n)
        xin = (B[:, j] / s).astype(np.float32).reshape(N, N, N)
        ref = np.array([s * _patch_forward(Wq, xin, pt, N) for pt in pts])
        got = np.array([X0[pt[0], pt[1], pt[2], j] for pt in pts])
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        worst = np.abs(got - ref).max() / np.abs(ref).max()
        _say(f"  column {j}: {len(pts)} voxels, rel err {rel:.2e}, max err / max |ref| {worst:.2e}")
        # stored activations are BF16 on both sides; a rounding that goes the
        # other way moves a value by one BF16 unit downstream (see
        # tests/test_gpu_cnn.py), far below a wrong tap, channel or index
        assert rel <= 2e-3 and worst <= 2.0 ** -6
