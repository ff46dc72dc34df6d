"""Thin ctypes binding of libxamg.so (include/xamg.h).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  Device buffers are torch tensors on the current HIP device
(float64, contiguous, row-major n x m); the stream is torch's current stream
unless one is given.  If the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxamg.so")

OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, ENODEV, EBREAKDOWN = 0, 1, -1, -2, -3, -4, -5
CG, BICGSTAB, MG, PBICGSTAB = 0, 1, 2, 3
JACOBI, CHEBYSHEV, GAUSS_SEIDEL = 0, 1, 2
FP64, MIXED = 0, 1
X0_ZERO, X0_GIVEN = 0, 1
OP_A, OP_P, OP_R = 0, 1, 2
TIMER_OFF, TIMER_KRYLOV_SPMM, TIMER_PRESMOOTH = 0, 1, 2
CNN_TIMER_OFF, CNN_TIMER_CONV16, CNN_TIMER_WGRAD16 = 0, 1, 2


class XamgError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib().xamg_strerror(code).decode()
        detail = lib().xamg_last_error().decode()
        super().__init__(f"{where}: {msg} ({code}) {detail}")


class CsrT(ctypes.Structure):
    _fields_ = [("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class HierT(ctypes.Structure):
    _fields_ = [("nlevels", ctypes.c_int32), ("A", ctypes.POINTER(CsrT)),
                ("P", ctypes.POINTER(CsrT)), ("R", ctypes.POINTER(CsrT)),
                ("lmax", ctypes.POINTER(ctypes.c_double))]


class SetupParamsT(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("max_coarse", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("lanczos_steps", ctypes.c_int32),
                ("agg_levels", ctypes.c_int32), ("num_paths", ctypes.c_int32)]


class OptionsT(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("smoother", ctypes.c_int32),
                ("omega", ctypes.c_double), ("cheby_degree", ctypes.c_int32),
                ("cheby_lo_frac", ctypes.c_double), ("cheby_hi_frac", ctypes.c_double),
                ("precision", ctypes.c_int32), ("index_bits", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("x0_mode", ctypes.c_int32),
                ("flexible", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("gs_block", ctypes.c_int32), ("precond", ctypes.c_int32),
                ("merged", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class StatsT(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("relres", ctypes.c_double), ("true_relres", ctypes.c_double),
                ("restarts", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("ms", ctypes.c_double)]


_lib = None

EXPORTS = [
    "xamg_default_setup_params", "xamg_hierarchy_build", "xamg_hierarchy_view",
    "xamg_hierarchy_cf", "xamg_hierarchy_free", "xamg_default_options", "xamg_setup",
    "xamg_solve", "xamg_solve_noalloc", "xamg_vcycle", "xamg_spmm", "xamg_info", "xamg_index16_fraction",
    "xamg_batch_create", "xamg_solve_batched", "xamg_batch_destroy",
    "xamg_autotune", "xamg_tuning", "xamg_set_tuning", "xamg_timer_enable", "xamg_timer_read", "xamg_destroy",
    "xamg_strerror", "xamg_last_error",
    "xamg_cnn_create", "xamg_cnn_get_weights", "xamg_cnn_set_weights", "xamg_cnn_pass",
    "xamg_cnn_pass_residual", "xamg_cnn_get_grads", "xamg_cnn_adam", "xamg_cnn_layer", "xamg_warmstart",
    "xamg_cnn_timer_enable", "xamg_cnn_timer_read", "xamg_cnn_destroy",
]

CNN_PARAMS = 14688
CNN_LAYERS = ((1, 16), (16, 16), (16, 16), (16, 1))   # (cin, cout) per layer


def lib():
    """Load libxamg.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError(f"{LIB_PATH} not built; run python -m paper_2103_07329_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.xamg_default_setup_params.argtypes = [ctypes.POINTER(SetupParamsT)]
        L.xamg_default_setup_params.restype = None
        L.xamg_hierarchy_build.argtypes = [ctypes.POINTER(CsrT), ctypes.POINTER(SetupParamsT),
                                           ctypes.POINTER(vp)]
        L.xamg_hierarchy_view.argtypes = [vp, ctypes.POINTER(HierT)]
        L.xamg_hierarchy_cf.argtypes = [vp, i32, vp]
        L.xamg_hierarchy_free.argtypes = [vp]
        L.xamg_hierarchy_free.restype = None
        L.xamg_default_options.argtypes = [ctypes.POINTER(OptionsT)]
        L.xamg_default_options.restype = None
        L.xamg_setup.argtypes = [ctypes.POINTER(HierT), ctypes.POINTER(OptionsT),
                                 ctypes.POINTER(vp)]
        L.xamg_solve.argtypes = [vp, vp, vp, i32, dbl, ctypes.POINTER(StatsT)]
        L.xamg_solve_noalloc.argtypes = [vp, vp, vp, i32, dbl, ctypes.POINTER(StatsT)]
        L.xamg_vcycle.argtypes = [vp, vp, vp, i32]
        L.xamg_spmm.argtypes = [vp, i32, i32, i32, vp, vp]
        L.xamg_info.argtypes = [vp, ctypes.POINTER(i64), i32]
        L.xamg_index16_fraction.argtypes = [vp, i32, ctypes.POINTER(dbl)]
        L.xamg_batch_create.argtypes = [ctypes.POINTER(vp), i32, i32, ctypes.POINTER(vp)]
        L.xamg_solve_batched.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.POINTER(i32), dbl, ctypes.POINTER(vp)]
        L.xamg_batch_destroy.argtypes = [vp]
        L.xamg_autotune.argtypes = [vp, i32, i32]
        L.xamg_tuning.argtypes = [vp, i32, ctypes.POINTER(i32), i32]
        L.xamg_set_tuning.argtypes = [vp, i32, ctypes.POINTER(i32), i32]
        L.xamg_timer_enable.argtypes = [vp, i32]
        L.xamg_timer_read.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
        L.xamg_destroy.argtypes = [vp]
        L.xamg_strerror.argtypes = [ctypes.c_int]
        L.xamg_strerror.restype = ctypes.c_char_p
        L.xamg_last_error.argtypes = []
        L.xamg_last_error.restype = ctypes.c_char_p
        f32p = ctypes.POINTER(ctypes.c_float)
        L.xamg_cnn_create.argtypes = [i32, f32p, vp, ctypes.POINTER(vp)]
        L.xamg_cnn_get_weights.argtypes = [vp, f32p]
        L.xamg_cnn_set_weights.argtypes = [vp, f32p]
        L.xamg_cnn_pass.argtypes = [vp, vp, vp, i32, vp, ctypes.POINTER(dbl)]
        L.xamg_cnn_pass_residual.argtypes = [vp, vp, vp, i32, ctypes.POINTER(dbl)]
        L.xamg_cnn_get_grads.argtypes = [vp, f32p]
        L.xamg_cnn_adam.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_float]
        L.xamg_cnn_layer.argtypes = [vp, i32, i32, vp, vp, vp]
        L.xamg_warmstart.argtypes = [vp, vp, vp, vp, i32, ctypes.POINTER(i32)]
        L.xamg_cnn_timer_enable.argtypes = [vp, i32]
        L.xamg_cnn_timer_read.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
        L.xamg_cnn_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _check(rc, where, allow=(OK,)):
    if rc not in allow:
        raise XamgError(rc, where)
    return rc


def _csr_struct(rp, ci, v, ncols=None, keep=None):
    rp = np.ascontiguousarray(rp, np.int32)
    ci = np.ascontiguousarray(ci, np.int32)
    v = np.ascontiguousarray(v, np.float64)
    if keep is not None:
        keep.extend([rp, ci, v])
    n = rp.size - 1
    return CsrT(n, n if ncols is None else int(ncols), int(rp[-1]),
                rp.ctypes.data, ci.ctypes.data, v.ctypes.data)


# ---------------------------------------------------------------------------
# host hierarchy (the library's own classical AMG setup)
# ---------------------------------------------------------------------------
class HostHierarchy:
    def __init__(self, rp, ci, v, theta=0.25, max_coarse=64, max_levels=40,
                 lanczos_steps=10, agg_levels=0, num_paths=1):
        keep = []
        a = _csr_struct(rp, ci, v, keep=keep)
        prm = SetupParamsT(theta, max_coarse, max_levels, lanczos_steps, agg_levels, num_paths)
        h = ctypes.c_void_p()
        _check(lib().xamg_hierarchy_build(ctypes.byref(a), ctypes.byref(prm), ctypes.byref(h)),
               "xamg_hierarchy_build")
        self._h = h
        self._view = HierT()
        _check(lib().xamg_hierarchy_view(h, ctypes.byref(self._view)), "xamg_hierarchy_view")
        self.nlev = self._view.nlevels

    def close(self):
        if getattr(self, "_h", None):
            lib().xamg_hierarchy_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def view(self):
        return self._view

    @staticmethod
    def _arrays(c):
        n, nnz = c.nrows, c.nnz
        rp = np.ctypeslib.as_array(ctypes.cast(c.row_ptr, ctypes.POINTER(ctypes.c_int32)),
                                   (n + 1,)).copy()
        if nnz:
            ci = np.ctypeslib.as_array(ctypes.cast(c.col, ctypes.POINTER(ctypes.c_int32)),
                                       (nnz,)).copy()
            v = np.ctypeslib.as_array(ctypes.cast(c.val, ctypes.POINTER(ctypes.c_double)),
                                      (nnz,)).copy()
        else:
            ci = np.zeros(0, np.int32)
            v = np.zeros(0)
        return rp, ci, v, (n, c.ncols)

    def A(self, l):
        return self._arrays(self._view.A[l])

    def P(self, l):
        return self._arrays(self._view.P[l])

    def R(self, l):
        return self._arrays(self._view.R[l])

    def lmax(self, l):
        return self._view.lmax[l]

    def cf(self, l):
        n = self._view.A[l].nrows
        out = np.empty(n, np.int8)
        _check(lib().xamg_hierarchy_cf(self._h, l, out.ctypes.data), "xamg_hierarchy_cf")
        return out

    def sizes(self):
        return [self._view.A[l].nrows for l in range(self.nlev)]

    def export(self):
        return {
            "A": [self.A(l)[:3] for l in range(self.nlev)],
            "P": [self.P(l)[:3] + (self.P(l)[3][1],) for l in range(self.nlev - 1)],
            "R": [self.R(l)[:3] for l in range(self.nlev - 1)],
            "lmax": [self.lmax(l) for l in range(self.nlev)],
        }


def hierarchy_struct(h):
    """HierT for a HostHierarchy or for an exported dict of arrays; returns
    (struct, keepalive)."""
    if isinstance(h, HostHierarchy):
        return h.view(), [h]
    keep = []
    nl = len(h["A"])
    A = (CsrT * nl)()
    P = (CsrT * max(nl - 1, 1))()
    R = (CsrT * max(nl - 1, 1))()
    for l in range(nl):
        rp, ci, v = h["A"][l][:3]
        A[l] = _csr_struct(rp, ci, v, keep=keep)
    for l in range(nl - 1):
        rp, ci, v, nc = h["P"][l]
        P[l] = _csr_struct(rp, ci, v, ncols=nc, keep=keep)
        rp, ci, v = h["R"][l][:3]
        R[l] = _csr_struct(rp, ci, v, ncols=len(h["A"][l][0]) - 1, keep=keep)
    lm = (ctypes.c_double * nl)(*[float(x) for x in h["lmax"]])
    keep += [A, P, R, lm]
    s = HierT(nl, A, P, R, lm)
    return s, keep


# ---------------------------------------------------------------------------
# device solver
# ---------------------------------------------------------------------------
def default_options(**kw):
    o = OptionsT()
    lib().xamg_default_options(ctypes.byref(o))
    for k, val in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, val)
    return o


def _ptr(t, dtype="float64"):
    import torch
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if str(t.dtype) != f"torch.{dtype}":
        raise ValueError(f"tensor must be {dtype}")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """Device solver over a hierarchy (HostHierarchy or exported arrays)."""

    def __init__(self, hierarchy, stream=None, **options):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        opts = default_options(**options)
        opts.stream = stream
        self.options = opts
        s, keep = hierarchy_struct(hierarchy)
        h = ctypes.c_void_p()
        _check(lib().xamg_setup(ctypes.byref(s), ctypes.byref(opts), ctypes.byref(h)),
               "xamg_setup")
        del keep
        self._h = h
        info = (ctypes.c_int64 * (1 + 3 * 64))()
        _check(lib().xamg_info(h, info, len(info)), "xamg_info")
        self.nlev = int(info[0])
        self.sizes = [int(info[1 + 3 * l]) for l in range(self.nlev)]
        self.nnzA = [int(info[2 + 3 * l]) for l in range(self.nlev)]
        self.nnzP = [int(info[3 + 3 * l]) for l in range(self.nlev)]
        self.n = self.sizes[0]

    def close(self):
        if getattr(self, "_h", None):
            lib().xamg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, B, X, tol=1e-8, check=True):
        """B, X: (n, m) float64 CUDA tensors; X is in/out.  Returns
        (return code, stats dict)."""
        m = B.shape[1] if B.dim() == 2 else 1
        st = (StatsT * m)()
        rc = lib().xamg_solve(self._h, _ptr(B), _ptr(X), m, tol, st)
        if check:
            _check(rc, "xamg_solve", allow=(OK, NOT_CONVERGED))
        stats = {
            "iters": np.array([s.iters for s in st], np.int32),
            "converged": np.array([bool(s.converged) for s in st]),
            "relres": np.array([s.relres for s in st]),
            "true_relres": np.array([s.true_relres for s in st]),
            "restarts": np.array([s.restarts for s in st], np.int32),
            "ms": float(st[0].ms) if len(st) else 0.0,
        }
        return rc, stats

    def solve_noalloc(self, B, X, tol=1e-8, check=True):
        """xamg_solve_noalloc: as solve(), with every work buffer in the
        library's static scratch array (no device allocation in the call)."""
        m = B.shape[1] if B.dim() == 2 else 1
        st = (StatsT * m)()
        rc = lib().xamg_solve_noalloc(self._h, _ptr(B), _ptr(X), m, tol, st)
        if check:
            _check(rc, "xamg_solve_noalloc", allow=(OK, NOT_CONVERGED))
        return rc, self._stats(st)

    @staticmethod
    def _stats(st):
        return {
            "iters": np.array([s.iters for s in st], np.int32),
            "converged": np.array([bool(s.converged) for s in st]),
            "relres": np.array([s.relres for s in st]),
            "true_relres": np.array([s.true_relres for s in st]),
            "restarts": np.array([s.restarts for s in st], np.int32),
            "ms": float(st[0].ms) if len(st) else 0.0,
        }

    def vcycle(self, B, X):
        m = B.shape[1]
        _check(lib().xamg_vcycle(self._h, _ptr(B), _ptr(X), m), "xamg_vcycle")

    def autotune(self, m, enable=True):
        _check(lib().xamg_autotune(self._h, m, 1 if enable else 0), "xamg_autotune")

    def tuning(self, m):
        """Per level (A, A pre-smoothing, P, R) row splits, then a last
        1-tuple: the Krylov operator's (FP64 A_0) split (see xamg_tuning)."""
        out = (ctypes.c_int32 * (4 * self.nlev + 1))()
        _check(lib().xamg_tuning(self._h, m, out, len(out)), "xamg_tuning")
        return [tuple(out[4 * l:4 * l + 4]) for l in range(self.nlev)] + [(out[4 * self.nlev],)]

    def set_tuning(self, m, splits):
        """Force the row splits for m columns: one (A, A pre-smoothing, P, R)
        tuple per level and the Krylov operator's 1-tuple, as tuning()
        returns (see xamg_set_tuning)."""
        flat = [int(v) for t in splits for v in t]
        arr = (ctypes.c_int32 * len(flat))(*flat)
        _check(lib().xamg_set_tuning(self._h, m, arr, len(flat)), "xamg_set_tuning")

    def timer_enable(self, kind):
        _check(lib().xamg_timer_enable(self._h, kind), "xamg_timer_enable")

    def timer_read(self):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check(lib().xamg_timer_read(self._h, ctypes.byref(ms), ctypes.byref(cnt)), "xamg_timer_read")
        return ms.value, cnt.value

    def index16_fraction(self, level):
        out = (ctypes.c_double * 3)()
        _check(lib().xamg_index16_fraction(self._h, level, out), "xamg_index16_fraction")
        return tuple(out)

    def spmm(self, op, level, X, Y):
        m = X.shape[1]
        _check(lib().xamg_spmm(self._h, op, level, m, _ptr(X), _ptr(Y)), "xamg_spmm")


class Batch:
    """Batched solves over several CG Solvers (one captured graph)."""

    def __init__(self, solvers, iters_per_launch=0):
        self.solvers = list(solvers)
        hs = (ctypes.c_void_p * len(self.solvers))(*[s._h.value for s in self.solvers])
        b = ctypes.c_void_p()
        _check(lib().xamg_batch_create(hs, len(self.solvers), iters_per_launch, ctypes.byref(b)),
               "xamg_batch_create")
        self._b = b

    def close(self):
        if getattr(self, "_b", None):
            lib().xamg_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, Bs, Xs, tol=1e-8, check=True):
        ns = len(self.solvers)
        Bp = (ctypes.c_void_p * ns)(*[_ptr(b).value for b in Bs])
        Xp = (ctypes.c_void_p * ns)(*[_ptr(x).value for x in Xs])
        ms = [b.shape[1] for b in Bs]
        mm = (ctypes.c_int32 * ns)(*ms)
        sts = [(StatsT * m)() for m in ms]
        sp = (ctypes.c_void_p * ns)(*[ctypes.addressof(s) for s in sts])
        rc = lib().xamg_solve_batched(self._b, Bp, Xp, mm, tol, sp)
        if check:
            _check(rc, "xamg_solve_batched", allow=(OK, NOT_CONVERGED))
        out = []
        for st in sts:
            out.append({
                "iters": np.array([s.iters for s in st], np.int32),
                "converged": np.array([bool(s.converged) for s in st]),
                "relres": np.array([s.relres for s in st]),
                "true_relres": np.array([s.true_relres for s in st]),
                "restarts": np.array([s.restarts for s in st], np.int32),
                "ms": float(st[0].ms) if len(st) else 0.0,
            })
        return rc, out


def _f32_host(a, count):
    a = np.ascontiguousarray(a, np.float32).reshape(-1)
    if a.size != count:
        raise ValueError(f"expected {count} values, got {a.size}")
    return a


def split_weights(flat):
    """Flat XAMG_CNN_PARAMS array -> [W1, W2, W3, W4], W_l of shape (cout, cin, 27)."""
    flat = np.asarray(flat).reshape(-1)
    out, k = [], 0
    for cin, cout in CNN_LAYERS:
        size = cout * cin * 27
        out.append(flat[k:k + size].reshape(cout, cin, 27))
        k += size
    return out


def join_weights(Ws):
    return np.concatenate([np.asarray(W, np.float32).reshape(-1) for W in Ws])


class Cnn:
    """Warm-start network on an N^3 grid (device weights, Adam state)."""

    def __init__(self, N, weights, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        w = _f32_host(weights, CNN_PARAMS)
        h = ctypes.c_void_p()
        _check(lib().xamg_cnn_create(N, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), stream,
                                     ctypes.byref(h)), "xamg_cnn_create")
        self._h = h
        self.N = N
        self.n = N ** 3

    def close(self):
        if getattr(self, "_h", None):
            lib().xamg_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def weights(self):
        w = np.empty(CNN_PARAMS, np.float32)
        _check(lib().xamg_cnn_get_weights(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "xamg_cnn_get_weights")
        return w

    def set_weights(self, weights):
        w = _f32_host(weights, CNN_PARAMS)
        _check(lib().xamg_cnn_set_weights(self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "xamg_cnn_set_weights")

    def grads(self):
        g = np.empty(CNN_PARAMS, np.float32)
        _check(lib().xamg_cnn_get_grads(self._h, g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "xamg_cnn_get_grads")
        return g

    def forward(self, x, y=None):
        """x: (S, n) float32 device tensor of normalised samples -> y (S, n)."""
        import torch
        S = x.shape[0]
        if y is None:
            y = torch.empty_like(x)
        _check(lib().xamg_cnn_pass(self._h, _ptr(x, "float32"), None, S, _ptr(y, "float32"), None),
               "xamg_cnn_pass")
        return y

    def loss_and_grads(self, x, t):
        """One forward + backward over the samples; returns the loss (the
        gradients stay on the device for adam(); grads() copies them)."""
        S = x.shape[0]
        loss = ctypes.c_double()
        _check(lib().xamg_cnn_pass(self._h, _ptr(x, "float32"), _ptr(t, "float32"), S, None,
                                   ctypes.byref(loss)), "xamg_cnn_pass")
        return loss.value

    def residual_loss_and_grads(self, x, solver):
        """One forward + backward over the samples with the residual loss
        ||x - A f(x)||^2 / ||x||^2 (A = the solver's finest operator);
        returns the loss (see xamg_cnn_pass_residual)."""
        S = x.shape[0]
        loss = ctypes.c_double()
        _check(lib().xamg_cnn_pass_residual(self._h, solver._h, _ptr(x, "float32"), S,
                                            ctypes.byref(loss)), "xamg_cnn_pass_residual")
        return loss.value

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(lib().xamg_cnn_adam(self._h, lr, beta1, beta2, eps), "xamg_cnn_adam")

    def layer(self, layer, mode, inp, mask, out):
        """Single-layer kernel (see xamg_cnn_layer); BF16 tensors are
        torch.bfloat16, FP32 tensors torch.float32."""
        def p(t):
            if t is None:
                return None
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("tensor must be a contiguous GPU tensor")
            return ctypes.c_void_p(t.data_ptr())
        _check(lib().xamg_cnn_layer(self._h, layer, mode, p(inp), p(mask), p(out)), "xamg_cnn_layer")

    def timer_enable(self, kind):
        _check(lib().xamg_cnn_timer_enable(self._h, kind), "xamg_cnn_timer_enable")

    def timer_read(self):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check(lib().xamg_cnn_timer_read(self._h, ctypes.byref(ms), ctypes.byref(cnt)),
               "xamg_cnn_timer_read")
        return ms.value, cnt.value

    def warmstart(self, B, X0, solver=None):
        """X0 (n, m) from B (n, m), float64 device tensors.  With a solver,
        columns whose initial residual is not below ||b|| are reset to zero;
        returns the per-column fallback flags."""
        m = B.shape[1]
        fb = (ctypes.c_int32 * m)()
        _check(lib().xamg_warmstart(self._h, solver._h if solver is not None else None, _ptr(B),
                                    _ptr(X0), m, fb), "xamg_warmstart")
        return np.array(list(fb), np.int32)
