"""CPU oracle for the multi-RHS AMG-Krylov solve (TEST INFRASTRUCTURE ONLY).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.  The arithmetic lives in ``oracle.c`` (plain FP64 C,
see its header for the definitions followed); this module is argument
marshalling through ctypes plus small NumPy helpers.

Functions with no independent pin: none in the solve path; the Chebyshev
interval constants and the Lanczos start vector are readings (not fixed by
the paper) and are checked only for their stated properties.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, EINVAL, ENOMEM, EBREAKDOWN = 0, 1, -1, -2, -5
CG, BICGSTAB, MG, PBICGSTAB = 0, 1, 2, 3
JACOBI, CHEBYSHEV, GAUSS_SEIDEL = 0, 1, 2
A_, P_, R_ = 0, 1, 2


def build(force=True):
    """Compile oracle.c into liboracle.so (gcc -O3 for x86-64-v3, i.e. AVX2
    and FMA, which every host of this GPU generation has; OpenMP over row
    loops and dot-product chunks)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_c_int, _c_dbl, _vp = ctypes.c_int, ctypes.c_double, ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_build.argtypes = [_c_int, _i32p, _i32p, _f64p, _c_dbl, _c_int,
                                _c_int, _c_int, _c_int, _c_int, ctypes.POINTER(_vp)]
        L.orc_hier_free.argtypes = [_vp]
        L.orc_hier_nlev.argtypes = [_vp]
        L.orc_hier_info.argtypes = [_vp, _c_int, _c_int, _i32p]
        L.orc_hier_copy.argtypes = [_vp, _c_int, _c_int, _i32p, _i32p, _f64p]
        L.orc_hier_cf.argtypes = [_vp, _c_int, _i32p]
        L.orc_hier_lmax.argtypes = [_vp, _c_int]
        L.orc_hier_lmax.restype = _c_dbl
        L.orc_vcycle.argtypes = [_vp, _c_int, _c_dbl, _c_int, _c_dbl, _c_dbl,
                                 _c_int, _c_int, _f64p, _f64p]
        L.orc_vcycle32.argtypes = [_vp, _c_int, _c_dbl, _c_int, _c_dbl, _c_dbl,
                                   _c_int, _c_int, _f64p, _f64p]
        L.orc_solve.argtypes = [_vp, _c_int, _c_int, _c_dbl, _c_int, _c_dbl,
                                _c_dbl, _c_int, _c_int, _c_int, _c_int, _c_int, _c_dbl,
                                _c_int, _c_int, _f64p, _f64p, _i32p, _f64p, _f64p,
                                _i32p, _i32p]
        L.orc_hgs_sweep.argtypes = [_c_int, _i32p, _i32p, _f64p, _c_int, _c_int,
                                    _c_int, _f64p, _f64p, _f64p]
        L.orc_hgs_sweep.restype = None
        L.orc_spmm.argtypes = [_c_int, _c_int, _i32p, _i32p, _f64p, _c_int,
                               _f64p, _f64p]
        L.orc_jacobi.argtypes = [_c_int, _i32p, _i32p, _f64p, _f64p, _c_dbl,
                                 _c_int, _f64p, _f64p]
        L.orc_chebyshev.argtypes = [_c_int, _i32p, _i32p, _f64p, _f64p, _c_dbl,
                                    _c_dbl, _c_int, _c_int, _f64p, _f64p]
        L.orc_lanczos.argtypes = [_c_int, _i32p, _i32p, _f64p, _c_int,
                                  ctypes.c_ulonglong]
        L.orc_lanczos.restype = _c_dbl
        L.orc_sm64_uniform.argtypes = [ctypes.c_ulonglong, ctypes.c_ulonglong]
        L.orc_sm64_uniform.restype = _c_dbl
        L.orc_dense_solve.argtypes = [_c_int, _f64p, _c_int, _f64p]
        L.orc_rs_split.argtypes = [_c_int, _i32p, _i32p, _f64p, _c_dbl, _i32p]
        L.orc_agg_split.argtypes = [_c_int, _i32p, _i32p, _f64p, _c_dbl, _c_int, _i32p]
        L.orc_strength_count.argtypes = [_c_int, _i32p, _i32p, _f64p, _c_dbl,
                                         _i32p]
        L.orc_conv3d_fwd.argtypes = [_c_int, _c_int, _c_int, _f64p, _f64p, _f64p]
        L.orc_conv3d_fwd.restype = None
        L.orc_conv3d_dgrad.argtypes = [_c_int, _c_int, _c_int, _f64p, _f64p, _f64p]
        L.orc_conv3d_dgrad.restype = None
        L.orc_conv3d_wgrad.argtypes = [_c_int, _c_int, _c_int, _f64p, _f64p, _f64p]
        L.orc_conv3d_wgrad.restype = None
        L.orc_bf16_round.argtypes = [_c_dbl]
        L.orc_bf16_round.restype = _c_dbl
        L.orc_set_verbose.argtypes = [_c_int]
        L.orc_set_verbose.restype = None
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = _c_int
        _lib = L
    return _lib


def num_threads():
    return lib().orc_num_threads()


def set_verbose(on=True):
    """One progress line per Krylov iteration on stderr."""
    lib().orc_set_verbose(1 if on else 0)


def _csr(rp, ci, v):
    return (np.ascontiguousarray(rp, np.int32), np.ascontiguousarray(ci, np.int32),
            np.ascontiguousarray(v, np.float64))


# --------------------------------------------------------------------------
# single operations
# --------------------------------------------------------------------------
def spmm(rp, ci, v, X, ncols=None):
    rp, ci, v = _csr(rp, ci, v)
    X = np.ascontiguousarray(X, np.float64)
    n = rp.size - 1
    m = 1 if X.ndim == 1 else X.shape[1]
    Y = np.empty((n, m))
    lib().orc_spmm(n, ncols if ncols is not None else X.shape[0], rp, ci, v, m,
                   X.reshape(-1, m), Y)
    return Y if X.ndim > 1 else Y[:, 0]


def jacobi(rp, ci, v, dinv, omega, B, X):
    rp, ci, v = _csr(rp, ci, v)
    X = np.array(X, np.float64, order="C", copy=True)
    B = np.ascontiguousarray(B, np.float64)
    m = X.shape[1]
    lib().orc_jacobi(rp.size - 1, rp, ci, v, np.ascontiguousarray(dinv, np.float64),
                     omega, m, B, X)
    return X


def chebyshev(rp, ci, v, dinv, lo, hi, degree, B, X):
    rp, ci, v = _csr(rp, ci, v)
    X = np.array(X, np.float64, order="C", copy=True)
    B = np.ascontiguousarray(B, np.float64)
    lib().orc_chebyshev(rp.size - 1, rp, ci, v, np.ascontiguousarray(dinv, np.float64),
                        lo, hi, degree, X.shape[1], B, X)
    return X


def lanczos_lmax(rp, ci, v, steps=10, key=7 << 32):
    rp, ci, v = _csr(rp, ci, v)
    return lib().orc_lanczos(rp.size - 1, rp, ci, v, steps, key)


def sm64_uniform(key, i):
    return lib().orc_sm64_uniform(key, i)


def dense_solve(A, B):
    A = np.ascontiguousarray(A, np.float64)
    B = np.array(B, np.float64, order="C", copy=True)
    vec = B.ndim == 1
    if vec:
        B = B[:, None].copy()
    rc = lib().orc_dense_solve(A.shape[0], A, B.shape[1], B)
    if rc:
        raise np.linalg.LinAlgError("singular")
    return B[:, 0] if vec else B


def rs_split(rp, ci, v, theta=0.25):
    """C/F split of the first Ruge-Stueben pass: 1 = C, 2 = F."""
    rp, ci, v = _csr(rp, ci, v)
    st = np.empty(rp.size - 1, np.int32)
    rc = lib().orc_rs_split(rp.size - 1, rp, ci, v, theta, st)
    assert rc == 0
    return st


def agg_split(rp, ci, v, theta=0.25, num_paths=1):
    """C/F split of aggressive coarsening (first RS pass, then a second pass
    over its C points on their distance-two strength): 1 = C, 2 = F."""
    rp, ci, v = _csr(rp, ci, v)
    st = np.empty(rp.size - 1, np.int32)
    rc = lib().orc_agg_split(rp.size - 1, rp, ci, v, theta, num_paths, st)
    assert rc == 0
    return st


def strength_counts(rp, ci, v, theta=0.25):
    rp, ci, v = _csr(rp, ci, v)
    c = np.empty(rp.size - 1, np.int32)
    lib().orc_strength_count(rp.size - 1, rp, ci, v, theta, c)
    return c


# --------------------------------------------------------------------------
# hierarchy + solve
# --------------------------------------------------------------------------
class Hierarchy:
    """Owns an oracle hierarchy handle; exports its arrays as NumPy."""

    def __init__(self, rp, ci, v, theta=0.25, max_coarse=64, max_levels=40,
                 lanczos_steps=10, agg_levels=0, num_paths=1):
        rp, ci, v = _csr(rp, ci, v)
        h = _vp()
        rc = lib().orc_build(rp.size - 1, rp, ci, v, theta, max_coarse,
                             max_levels, lanczos_steps, agg_levels, num_paths,
                             ctypes.byref(h))
        if rc != 0:
            raise RuntimeError(f"oracle hierarchy build failed: {rc}")
        self._h = h
        self.nlev = lib().orc_hier_nlev(h)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_hier_free(self._h)
            self._h = None

    def csr(self, which, level):
        info = np.empty(3, np.int32)
        rc = lib().orc_hier_info(self._h, which, level, info)
        if rc:
            raise IndexError(level)
        nr, nc, nnz = (int(x) for x in info)
        rp = np.empty(nr + 1, np.int32)
        ci = np.empty(max(nnz, 1), np.int32)
        v = np.empty(max(nnz, 1), np.float64)
        lib().orc_hier_copy(self._h, which, level, rp, ci, v)
        return rp, ci[:nnz], v[:nnz], (nr, nc)

    def A(self, l):
        return self.csr(A_, l)

    def P(self, l):
        return self.csr(P_, l)

    def R(self, l):
        return self.csr(R_, l)

    def cf(self, l):
        n = self.A(l)[3][0]
        out = np.empty(n, np.int32)
        lib().orc_hier_cf(self._h, l, out)
        return out

    def lmax(self, l):
        return lib().orc_hier_lmax(self._h, l)

    def sizes(self):
        return [self.A(l)[3][0] for l in range(self.nlev)]

    def export(self):
        """Plain-array form {A: [...], P: [...], R: [...], lmax: [...]} used to
        hand the same hierarchy to another implementation."""
        return {
            "A": [self.A(l)[:3] for l in range(self.nlev)],
            "P": [self.P(l)[:3] + (self.P(l)[3][1],) for l in range(self.nlev - 1)],
            "R": [self.R(l)[:3] for l in range(self.nlev - 1)],
            "lmax": [self.lmax(l) for l in range(self.nlev)],
        }

    def vcycle(self, B, smoother=JACOBI, omega=2.0 / 3.0, degree=2,
               lo_frac=0.3, hi_frac=1.1, gs_block=8):
        B = np.ascontiguousarray(B, np.float64)
        vec = B.ndim == 1
        if vec:
            B = B[:, None].copy()
        X = np.zeros_like(B)
        lib().orc_vcycle(self._h, smoother, omega, degree, lo_frac, hi_frac,
                         gs_block, B.shape[1], B, X)
        return X[:, 0] if vec else X

    def vcycle32(self, B, smoother=JACOBI, omega=2.0 / 3.0, degree=2,
                 lo_frac=0.3, hi_frac=1.1, gs_block=8):
        """The V(1,1) cycle carried out in FP32 (level matrices, D^-1, the
        coarsest inverse and all vectors rounded to float, float sums); B is
        rounded to float, the result is returned as float64."""
        B = np.ascontiguousarray(B, np.float64)
        vec = B.ndim == 1
        if vec:
            B = B[:, None].copy()
        X = np.zeros_like(B)
        lib().orc_vcycle32(self._h, smoother, omega, degree, lo_frac, hi_frac,
                           gs_block, B.shape[1], B, X)
        return X[:, 0] if vec else X

    def solve(self, B, X0=None, method=CG, smoother=JACOBI, omega=2.0 / 3.0,
              degree=2, lo_frac=0.3, hi_frac=1.1, flexible=False, precond=True,
              max_iters=1000, tol=1e-8, gs_block=8, merged=False):
        """Returns (X, stats dict, return code).  precond=False solves without
        a preconditioner (M = I); merged=True runs CG in its merged form
        (x's update deferred into the next p update).  stats: iters, relres, true_relres,
        converged, restarts (breakdown plus true-residual restarts) per
        column."""
        B = np.ascontiguousarray(B, np.float64)
        vec = B.ndim == 1
        if vec:
            B = B[:, None].copy()
        n, m = B.shape
        if X0 is None:
            X = np.zeros_like(B)
            given = 0
        else:
            X = np.array(X0, np.float64, order="C", copy=True).reshape(n, m)
            given = 1
        it = np.zeros(m, np.int32)
        rr = np.zeros(m)
        tr = np.zeros(m)
        cv = np.zeros(m, np.int32)
        rs = np.zeros(m, np.int32)
        rc = lib().orc_solve(self._h, method, smoother, omega, degree, lo_frac,
                             hi_frac, gs_block, int(flexible), int(precond), int(merged),
                             max_iters,
                             tol, given, m, B, X, it, rr, tr, cv, rs)
        st = {"iters": it, "relres": rr, "true_relres": tr,
              "converged": cv.astype(bool), "restarts": rs}
        return (X[:, 0] if vec else X), st, rc


# --------------------------------------------------------------------------
# bias-free 3D CNN (learned warm start)
# --------------------------------------------------------------------------
CNN_LAYERS = ((1, 16), (16, 16), (16, 16), (16, 1))   # (cin, cout); ReLU after 1-3


def hgs_sweep(rp, ci, v, B, backward, b, xo):
    """One l1-hybrid Gauss-Seidel sweep (blocks of B rows) from xo: returns xn."""
    rp, ci, v = _csr(rp, ci, v)
    b = np.ascontiguousarray(b, np.float64)
    vec = b.ndim == 1
    b2 = b[:, None] if vec else b
    xo2 = np.ascontiguousarray(np.asarray(xo, np.float64).reshape(b2.shape))
    xn = np.empty_like(b2)
    lib().orc_hgs_sweep(rp.size - 1, rp, ci, v, int(B), int(backward), b2.shape[1],
                        np.ascontiguousarray(b2), xo2, xn)
    return xn[:, 0] if vec else xn


def conv3d_fwd(N, W, x):
    """x: (n, cin) -> (n, cout); W: (cout, cin, 27)."""
    W = np.ascontiguousarray(W, np.float64)
    cout, cin = W.shape[:2]
    x = np.ascontiguousarray(x, np.float64).reshape(N ** 3, cin)
    y = np.empty((N ** 3, cout))
    lib().orc_conv3d_fwd(N, cin, cout, x, W, y)
    return y


def conv3d_dgrad(N, W, g):
    W = np.ascontiguousarray(W, np.float64)
    cout, cin = W.shape[:2]
    g = np.ascontiguousarray(g, np.float64).reshape(N ** 3, cout)
    d = np.empty((N ** 3, cin))
    lib().orc_conv3d_dgrad(N, cin, cout, g, W, d)
    return d


def conv3d_wgrad(N, g, x, cin, cout):
    g = np.ascontiguousarray(g, np.float64).reshape(N ** 3, cout)
    x = np.ascontiguousarray(x, np.float64).reshape(N ** 3, cin)
    dW = np.empty((cout, cin, 27))
    lib().orc_conv3d_wgrad(N, cin, cout, g, x, dW)
    return dW


def bf16(a):
    """Round-to-nearest-even to bfloat16 (element-wise), as float64."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    u = np.where(finite, u + 0x7FFF + ((u >> 16) & 1), u) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def cnn_forward(N, Ws, x, quantize=False):
    """Forward of the 4-layer network on one normalised sample x (n,).
    Returns the list of layer outputs [a1, a2, a3, y] (a1..a3 after ReLU).
    quantize=True rounds weights and stored activations to BF16 as the
    device path does (the final output stays in higher precision)."""
    q = bf16 if quantize else (lambda a: np.asarray(a, np.float64))
    a = q(np.asarray(x, np.float64).reshape(N ** 3, 1))
    outs = []
    for l, W in enumerate(Ws):
        z = conv3d_fwd(N, q(W), a)
        if l < 3:
            a = q(np.maximum(z, 0.0))
            outs.append(a)
        else:
            outs.append(z)
    return outs


def cnn_loss_and_grads(N, Ws, xs, ts, quantize=False):
    """Mean over samples of ||f(x) - t||^2 / ||t||^2 and its gradient
    with respect to each layer's weights (backpropagation through the
    oracle's forward, dgrad and wgrad)."""
    q = bf16 if quantize else (lambda a: np.asarray(a, np.float64))
    grads = [np.zeros_like(np.asarray(W, np.float64)) for W in Ws]
    loss = 0.0
    S = len(xs)
    for x, t in zip(xs, ts):
        t = np.asarray(t, np.float64).reshape(-1)
        a0 = q(np.asarray(x, np.float64).reshape(N ** 3, 1))
        a1, a2, a3, y = cnn_forward(N, Ws, x, quantize)
        y = y.reshape(-1)
        tt = float(t @ t)
        e = y - t
        loss += float(e @ e) / tt / S
        g = (2.0 * e / tt / S).reshape(-1, 1)
        acts = [a0, a1, a2, a3]
        for l in (3, 2, 1, 0):
            grads[l] += conv3d_wgrad(N, g, acts[l], Ws[l].shape[1], Ws[l].shape[0])
            if l > 0:
                d = conv3d_dgrad(N, q(Ws[l]), g)
                g = d * (acts[l] > 0)
                if quantize:
                    g = q(g)
    return loss, grads


def cnn_residual_loss_and_grads(N, Ws, xs, A, quantize=False):
    """Residual loss of the network as a solver's initial guess: the mean
    over samples of ||x - A f(x)||^2 / ||x||^2 (x a normalised right-hand
    side, A = (rp, ci, v) the operator on the N^3 grid), and its gradient
    with respect to each layer's weights.  dL/dy = -2 A^T (x - A y) /
    (||x||^2 S), then backpropagation as in cnn_loss_and_grads."""
    import scipy.sparse as sp
    rp, ci, v = _csr(*A)
    n = N ** 3
    At = sp.csr_matrix((v, ci, rp), shape=(n, n)).T.tocsr()   # A^T, a library transpose
    q = bf16 if quantize else (lambda a: np.asarray(a, np.float64))
    grads = [np.zeros_like(np.asarray(W, np.float64)) for W in Ws]
    loss = 0.0
    S = len(xs)
    for x in xs:
        b = np.asarray(x, np.float64).reshape(-1)
        a0 = q(b.reshape(n, 1))
        a1, a2, a3, y = cnn_forward(N, Ws, x, quantize)
        y = y.reshape(-1)
        r = b - spmm(rp, ci, v, y[:, None])[:, 0]
        bb = float(b @ b)
        loss += float(r @ r) / bb / S
        g = (-2.0 / (bb * S) * spmm(At.indptr, At.indices, At.data, r[:, None])[:, 0]).reshape(-1, 1)
        acts = [a0, a1, a2, a3]
        for l in (3, 2, 1, 0):
            grads[l] += conv3d_wgrad(N, g, acts[l], Ws[l].shape[1], Ws[l].shape[0])
            if l > 0:
                d = conv3d_dgrad(N, q(Ws[l]), g)
                g = d * (acts[l] > 0)
                if quantize:
                    g = q(g)
    return loss, grads


def adam_step(w, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, ICLR 2015, Algorithm 1) in float64:
    moments m, v updated in place, bias-corrected with step count t >= 1,
    w <- w - lr * mhat / (sqrt(vhat) + eps).  Returns the new w."""
    m[...] = beta1 * m + (1.0 - beta1) * g
    v[...] = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps)
