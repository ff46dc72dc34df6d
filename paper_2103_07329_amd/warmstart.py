"""Learned warm start: training data from the library's own FP64 solver,
training with the library's CNN kernels, and the comparison of warm-started
solves with zero-guess solves.

Everything numeric runs in libxamg through the ``xamg`` binding: the solves
(AMG-preconditioned CG), the network's forward and backward passes, Adam,
and the warm start with its per-column fallback.  torch holds device
memory and prepares the training set (generation of the right-hand sides,
their normalisation, mini-batch gathers); it also times with events and
computes the reported norms.

Recipe (extension of the method, not in the paper):
  * samples: Gaussian-source right-hand sides (``inputs.gaussian_params``),
    solved to relative residual 1e-8; a pair is (b / s, x / s) with
    s = ||b|| / sqrt(n), in FP32;
  * loss ("solution"): mean over the mini-batch of ||f(b/s) - x/s||^2 /
    ||x/s||^2; or ("residual") the quantity the zero-guess fallback judges,
    ||b/s - A f(b/s)||^2 / ||b/s||^2, which needs no solved targets;
  * Adam, lr 1e-3, betas (0.9, 0.999), eps 1e-8, FP32 master weights;
  * He-normal initial weights (std sqrt(2 / fan_in); the output layer
    sqrt(1 / fan_in)), fixed seed;
  * train / validation split of the generated pairs by a seeded permutation.
"""
from __future__ import annotations

import sys
import time

import numpy as np

from . import inputs, xamg


def log(*a):
    print(*a, file=sys.stderr, flush=True)
    sys.stdout.flush()


def he_init(seed):
    rng = np.random.default_rng(seed)
    Ws = []
    for l, (cin, cout) in enumerate(xamg.CNN_LAYERS):
        fan_in = 27 * cin
        std = np.sqrt((1.0 if l == 3 else 2.0) / fan_in)
        Ws.append((std * rng.standard_normal((cout, cin, 27))).astype(np.float32))
    return xamg.join_weights(Ws)


def make_pairs(solver, N, count, seed, torch, chunk=32, tol=1e-8):
    """Generate ``count`` normalised (input, target) pairs on the device.
    Returns (xs, ts, iters): FP32 tensors (count, n) and the solver's
    iteration count per sample."""
    n = N ** 3
    params = inputs.gaussian_params(N, count, seed)
    xs = torch.empty((count, n), dtype=torch.float32, device="cuda")
    ts = torch.empty((count, n), dtype=torch.float32, device="cuda")
    iters = np.zeros(count, np.int32)
    t0 = time.time()
    for k0 in range(0, count, chunk):
        cols = list(range(k0, min(count, k0 + chunk)))
        B = inputs.gaussian_rhs_torch(N, params, cols, torch, "cuda")
        X = torch.zeros_like(B)
        rc, st = solver.solve(B, X, tol)
        if not st["converged"].all():
            raise RuntimeError("training solve did not converge")
        iters[cols] = st["iters"]
        s = torch.sqrt((B * B).sum(0) / n)
        xs[cols] = (B / s).t().float()
        ts[cols] = (X / s).t().float()
        if (k0 // chunk) % 8 == 7 or k0 + chunk >= count:
            log(f"[warmstart] pairs {cols[-1] + 1}/{count} ({time.time() - t0:.1f} s)")
    return xs, ts, iters


def train(net, xs, ts, train_idx, val_idx, torch, epochs=20, batch=8, lr=1e-3, seed=5,
          max_seconds=None, objective="solution", solver=None):
    """Mini-batch Adam over ``train_idx``; validation loss after each epoch.
    objective "residual" trains on ||x - A f(x)||^2 / ||x||^2 with A the
    finest operator of ``solver`` (``ts`` unused).  Returns the history
    [(epoch, train_loss, val_loss, seconds)]."""
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.time()
    vi = torch.as_tensor(val_idx, device="cuda")
    if objective == "residual":
        def step(idx):
            return net.residual_loss_and_grads(xs.index_select(0, idx).contiguous(), solver)
    elif objective == "solution":
        def step(idx):
            return net.loss_and_grads(xs.index_select(0, idx).contiguous(),
                                      ts.index_select(0, idx).contiguous())
    else:
        raise ValueError(objective)
    for ep in range(1, epochs + 1):
        order = rng.permutation(train_idx)
        tot, nb = 0.0, 0
        for k in range(0, len(order) - batch + 1, batch):
            idx = torch.as_tensor(order[k:k + batch], device="cuda")
            loss = step(idx)
            net.adam(lr)
            tot += loss
            nb += 1
        vl = 0.0
        for k in range(0, len(val_idx), 32):
            sl = vi[k:k + 32]
            vl += step(sl) * len(sl)
        vl /= len(val_idx)
        el = time.time() - t0
        hist.append((ep, tot / max(nb, 1), vl, el))
        log(f"[warmstart] epoch {ep}/{epochs}: train loss {tot / max(nb, 1):.4f}, "
            f"validation loss {vl:.4f} ({el:.1f} s)")
        if max_seconds is not None and el > max_seconds:
            log(f"[warmstart] stopping after {ep} epochs (time limit {max_seconds} s)")
            break
    return hist


def compare(s_zero, s_given, net, B, tol, torch, reps=3):
    """Solve B from X0 = 0 and from the warm start (CNN + fallback).
    Returns a dict of per-column iterations, fallbacks, the initial
    relative residuals and median times (ms) over ``reps`` runs."""
    m = B.shape[1]
    out = {}
    X = torch.zeros_like(B)
    times = []
    for _ in range(reps):
        X.zero_()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        rc, st0 = s_zero.solve(B, X, tol)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    out["zero"] = {"iters": st0["iters"].tolist(), "true_relres": st0["true_relres"].tolist(),
                   "ms": float(np.median(times))}
    Xz = X.clone()
    X0 = torch.zeros_like(B)
    times, tcnn = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        fb = net.warmstart(B, X0, s_given)
        e1.record()
        X.copy_(X0)
        rc, st1 = s_given.solve(B, X, tol)
        e2.record()
        torch.cuda.synchronize()
        tcnn.append(e0.elapsed_time(e1))
        times.append(e0.elapsed_time(e2))
    # initial residuals of the warm start, for the record
    R = torch.empty_like(B)
    s_given.spmm(xamg.OP_A, 0, X0, R)
    r0 = (torch.linalg.vector_norm(B - R, dim=0) / torch.linalg.vector_norm(B, dim=0)).cpu().numpy()
    out["warm"] = {"iters": st1["iters"].tolist(), "true_relres": st1["true_relres"].tolist(),
                   "ms": float(np.median(times)), "cnn_ms": float(np.median(tcnn)),
                   "fallback": fb.tolist(), "initial_relres": r0.tolist()}
    out["solution_rel_diff"] = float(
        (torch.linalg.vector_norm(X - Xz) / torch.linalg.vector_norm(Xz)).item())
    out["m"] = m
    return out
