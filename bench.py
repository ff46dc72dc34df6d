#!/usr/bin/env python3
"""Benchmark: ms per right-hand side of the multi-RHS AMG-Krylov solve phase.

Default workload (one "step" = one complete solve of an n x m block from
X0 = 0 to relative residual 1e-8): 3D Poisson, 7-point stencil, 128^3
unknowns (n = 2,097,152, nnz = 14,581,760), m = 16 uniform[-1, 1] right-hand
sides (seed 1002), classical AMG V(1,1) with a degree-2 Chebyshev smoother
preconditioning CG, FP64 throughout.  The hierarchy is built once on the
host by the library's own setup and uploaded before timing; B and X are
resident in HBM when the timed region starts.

Other workloads (--workload): poisson32 (32^3, Jacobi, m = 8), aniso256
(anisotropic 256^3, BiCGStab, m = 16, FP32 preconditioner with 16-bit
offsets vs FP64), gs150 (150^3, BiCGStab with symmetric Gauss-Seidel
smoothing -- the configuration of the paper's single-node runs -- m = 16,
with P_m for m = 1..16), batched, warmstart.

One JSON line on stdout: value = ms per RHS (lower is better); roofline of
the dominant fine-level kernel from HIP events recorded by the library
around that kernel's launches inside the timed solves; the CPU oracle timed
on the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2103_07329_amd/csrc/kernels.hpp", "paper_2103_07329_amd/csrc/ops.hpp",
                  "paper_2103_07329_amd/csrc/solver.hpp", "paper_2103_07329_amd/csrc/cycle.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def spmm_bytes(n, nnz, m, vb=8, ib=4, xb=8):
    """Y = A X: every nonzero (value + index) and row pointer read once,
    X read once, Y written once."""
    return nnz * (vb + ib) + 4 * (n + 1) + 2 * n * m * xb


def presmooth_bytes(n, nnz, m, vb=8, ib=4, bb=8, xb=8, jacobi=False):
    """Pre-smoothing from zero in one pass (Chebyshev: x = p(D^-1 A) D^-1 b;
    Jacobi: x = w D^-1 b fused with r = b - A x): matrix and row pointers
    once, b read once, D^-1 read once, x written (Jacobi: r written too)."""
    return (nnz * (vb + ib) + 4 * (n + 1) + n * m * bb + n * vb + n * m * xb
            + (n * m * xb if jacobi else 0))


def pcg_iteration_bytes(S, m, chebyshev, mixed, flexible, idx16=None, merged=1):
    """Algorithmic bytes of one PCG iteration: every array each kernel of
    the iteration reads or writes, counted once per kernel.  The V-cycle is
    Jacobi or Chebyshev-2 V(1,1) (FP32 vectors and values when mixed; its
    level-0 input r and output z are FP64), then the Krylov passes of the
    CG form: merged = 0: q = A p with its dot, x += a p and r -= a q with
    (r, r), p = z + b p; 1: q = A p, r -= a q, then x += a p_old with
    p = z + b p in one pass; 2: q = A (z + b p) writing the new p and
    updating x in the SpMM, then r -= a q.  Mixed: r -= a q also writes the
    FP32 copy of r.  idx16[l] = fraction of 16-bit column indices of
    (A_l, P_l, R_l)."""
    n, nnzA, nnzP, L = S.sizes, S.nnzA, S.nnzP, S.nlev
    vb = 4 if mixed else 8
    tot = 0.0
    for l in range(L):
        V = n[l] * m * vb
        if l == L - 1:
            tot += n[l] * n[l] * vb + 2 * V        # dense inverse, b in, x out
            continue
        ibA, ibP, ibR = ((2 * f + 4 * (1 - f)) for f in idx16[l]) if idx16 else (4, 4, 4)
        MA = nnzA[l] * (vb + ibA) + 4 * (n[l] + 1)
        MP = nnzP[l] * (vb + ibP) + 4 * (n[l] + 1)
        MR = nnzP[l] * (vb + ibR) + 4 * (n[l + 1] + 1)
        Vc = n[l + 1] * m * vb
        d = n[l] * vb                              # D^-1
        io = n[l] * m * 8 if l == 0 else V         # level-0 input r / output z (FP64)
        if chebyshev:
            tot += MA + io + d + V                 # pre: gather b (A D^-1), D^-1, write x
            tot += MA + V + io + V                 # residual
        else:
            tot += MA + io + d + 2 * V             # pre: gather b, D^-1, write x and r
        tot += MR + V + Vc                         # restriction
        tot += MP + Vc + 2 * V                     # prolongation add
        if chebyshev:
            tot += MA + V + io + d + V             # post 1: gather x, b, D^-1, write r0
            tot += MA + V + V + d + io             # post 2: gather r0, x, D^-1, write z
        else:
            tot += MA + V + io + d + io            # post: gather x, b, D^-1, write z
        if l == 0:
            tot += n[0] * m * 8 * (1 if flexible else 0) + (0 if not chebyshev else n[0] * m * 8)
    V0 = n[0] * m * 8
    A0 = nnzA[0] * 12 + 4 * (n[0] + 1)
    r32 = n[0] * m * 4 if mixed else 0
    if merged == 2:
        tot += A0 + 6 * V0                         # gather z, p; write p', q; x read, write
        tot += 3 * V0 + r32                        # r update
    elif merged == 1:
        tot += A0 + 2 * V0                         # q = A p
        tot += 3 * V0 + r32                        # r update
        tot += 5 * V0                              # x += a p_old, p = z + b p
    else:
        tot += A0 + 2 * V0                         # q = A p
        tot += 6 * V0 + r32 + 3 * V0               # x, r update; p update
    return tot


def stored_traffic(workload, kernel):
    """HBM bytes per launch from the committed PMC summary of this
    workload/kernel, if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"pmc_{workload}_{kernel}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha") != kernel_source_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _best_ms(torch, fn, reps):
    fn()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return best


def stream_bandwidth(torch, nbytes=1 << 30, reps=5):
    """Streaming rates of this device (GB/s of bytes read + written), timed
    with events on the current stream, best of reps: a plain torch copy of
    nbytes (a blit of 256 workgroups) and the elementwise sum c = a + b over
    three arrays of nbytes/2 (torch's vectorised elementwise kernel, every
    CU busy).  The larger is the practical ceiling of a streaming kernel."""
    n = nbytes // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    copy_gbs = 2.0 * n * 8 / (_best_ms(torch, lambda: b.copy_(a), reps) * 1e-3) / 1e9
    del a, b
    h = n // 2
    x = torch.ones(h, dtype=torch.float64, device="cuda")
    y = torch.ones(h, dtype=torch.float64, device="cuda")
    z = torch.empty_like(x)
    add_gbs = 3.0 * h * 8 / (_best_ms(torch, lambda: torch.add(x, y, out=z), reps) * 1e-3) / 1e9
    del x, y, z
    torch.cuda.empty_cache()
    return {"copy_gbs": copy_gbs, "add_gbs": add_gbs, "ceiling_gbs": max(copy_gbs, add_gbs)}


def timed_solves(S, Bd, Xd, steps, tol, stream, torch):
    rcs, iters, tr = [], None, 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rc, st = S.solve(Bd, Xd, tol=tol)
        rcs.append(rc)
        iters = st["iters"]
        tr = max(tr, float(st["true_relres"].max()))
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, iters, tr, rcs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="poisson128",
                    choices=["poisson128", "poisson32", "aniso256", "gs150", "batched",
                             "warmstart"])
    ap.add_argument("--ws-pairs", type=int, default=2048,
                    help="warmstart: (B, X) training pairs generated by the FP64 solver")
    ap.add_argument("--krylov-split", type=int, default=0,
                    help="after tuning, force this launch shape on the FP64 A_0 (the Krylov "
                         "SpMM; on an FP64 handle also the finest residual and post-smoothing "
                         "passes), e.g. 513 for the banded XCD walk (see xamg_tuning)")
    ap.add_argument("--fine-pre-split", type=int, default=0,
                    help="after tuning, force this launch shape on the finest pre-smoothing pass")
    ap.add_argument("--ws-epochs", type=int, default=20)
    ap.add_argument("--ws-objective", choices=["residual", "solution"], default="residual",
                    help="warmstart: train on ||b - A f(b)||^2/||b||^2 (the quantity the "
                         "fallback judges) or on ||f(b) - x||^2/||x||^2")
    ap.add_argument("--ws-weights", default=None,
                    help="warmstart: load trained weights (.npy) instead of training")
    ap.add_argument("--ws-save", default=None,
                    help="warmstart: save the trained weights (.npy) here")
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP64-vs-mixed and multi-RHS-gain extras")
    ap.add_argument("--cpu-iters", type=int, default=0,
                    help="oracle sample: this many iterations, scaled to the solve")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 512 MiB device copy (PMC byte-counter calibration)")
    ap.add_argument("--print-source-hash", action="store_true")
    ap.add_argument("--cpu-full", action="store_true",
                    help="full oracle solve; per-column error of the GPU result against it")
    args = ap.parse_args()

    if args.print_source_hash:
        print(kernel_source_hash())
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; run with --gpus 1 "
                                   "(sharding across GPUs is a design note only)"}))
        sys.exit(2)

    import torch

    from paper_2103_07329_amd import inputs, xamg

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    wl = args.workload
    if wl == "batched":
        return bench_batched(args, torch, inputs, xamg)
    if wl == "warmstart":
        return bench_warmstart(args, torch, inputs, xamg)
    if args.calibrate_copy:
        # a plain copy of known size: 512 MiB read + 512 MiB written
        xc = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device=dev)
        yc = torch.empty_like(xc)
        yc.copy_(xc)
        torch.cuda.synchronize()
        del xc, yc
    if wl == "poisson128":
        N, m = 128, args.m or 16
        prob = inputs.poisson7(N)
        B = inputs.uniform_rhs(prob.n, 16, 1002)[:, :m].copy()
        opts = dict(smoother=xamg.CHEBYSHEV, method=xamg.CG)
        desc = f"poisson{N}_chebyshev2_vcycle11_pcg_fp64"
    elif wl == "poisson32":
        N, m = 32, args.m or 8
        prob = inputs.poisson7(N)
        B = inputs.uniform_rhs(prob.n, 8, 1001)[:, :m].copy()
        opts = dict(smoother=xamg.JACOBI, method=xamg.CG)
        desc = f"poisson{N}_jacobi_vcycle11_pcg_fp64"
    elif wl == "gs150":
        # the configuration of the paper's single-node runs (Section 3.1):
        # BiCGStab, classical AMG, symmetric Gauss-Seidel smoothing, 150^3
        N, m = 150, args.m or 16
        prob = inputs.poisson7(N)
        B = inputs.uniform_rhs(prob.n, 16, 1007)[:, :m].copy()
        opts = dict(smoother=xamg.GAUSS_SEIDEL, method=xamg.BICGSTAB, gs_block=8)
        desc = f"poisson{N}_sgs_l1hybrid8_vcycle11_bicgstab_fp64"
    else:
        N, m = 256, args.m or 16
        prob = inputs.anisotropic7(N)
        B = inputs.uniform_rhs(prob.n, m, 1003)
        opts = dict(smoother=xamg.JACOBI, method=xamg.BICGSTAB, precision=xamg.MIXED,
                    index_bits=16)
        desc = f"aniso{N}_jacobi_vcycle11_bicgstab_fp32precond_idx16"
    log(f"[bench] workload {desc}: {prob}, m={m}")
    t0 = time.time()
    Hh = xamg.HostHierarchy(*prob.csr())
    t_setup = time.time() - t0
    log(f"[bench] host AMG setup {t_setup:.1f}s, levels {Hh.sizes()}")
    stream = torch.cuda.current_stream()
    S = xamg.Solver(Hh, stream=stream.cuda_stream, **opts)
    nnzA = S.nnzA
    Bd = torch.from_numpy(B).to(dev)
    Xd = torch.zeros_like(Bd)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        rc, st = S.solve(Bd, Xd, tol=1e-8)
        assert rc == xamg.OK, rc
    mp = m if m in (1, 2, 4, 8, 16, 32) else 1 << (m - 1).bit_length()
    if args.krylov_split or args.fine_pre_split:
        # the tuned shapes, with the FP64 A_0's and/or the finest pre-smoothing
        # pass's replaced (for profiling a shape)
        tun = S.tuning(mp)
        if args.krylov_split:
            tun[-1] = (args.krylov_split,)
        if args.fine_pre_split:
            tun[0] = (tun[0][0], args.fine_pre_split) + tuple(tun[0][2:])
        S.set_tuning(mp, tun)
        S.solve(Bd, Xd, tol=1e-8)

    log(f"[bench] launch shapes (A, A pre-smoothing, P, R per level; Krylov A_0): "
        f"{S.tuning(mp)}")
    # timed region: K complete solves, with the library's event timer on the
    # fine-level pre-smoothing pass (kernel A) -- then on the Krylov SpMM
    # (kernel B) in an identical second pass
    precision = opts.get("precision", xamg.FP64)
    mixed = precision == xamg.MIXED
    vb32 = 4 if mixed else 8
    ib32 = 2 if opts.get("index_bits", 32) == 16 else 4
    kernels = {}
    ms_step = None
    for kind, name in ((xamg.TIMER_PRESMOOTH, "fine_presmooth"),
                       (xamg.TIMER_KRYLOV_SPMM, "fine_krylov_spmm")):
        if kind == xamg.TIMER_KRYLOV_SPMM and opts["method"] != xamg.CG:
            continue
        S.timer_enable(kind)
        ms, iters, trmax, rcs = timed_solves(S, Bd, Xd, args.steps, 1e-8, stream, torch)
        tms, cnt = S.timer_read()
        S.timer_enable(xamg.TIMER_OFF)
        assert all(r == xamg.OK for r in rcs), rcs
        if ms_step is None:
            ms_step, iters0, tr0 = ms, iters, trmax
        if cnt == 0:
            continue
        avg_ms = tms / cnt
        if kind == xamg.TIMER_PRESMOOTH:
            # (the Gauss-Seidel sweeps always read 32-bit column indices; with
            # the Jacobi or Chebyshev smoother a mixed cycle gathers the FP32
            # copy of its FP64 input that the Krylov step writes)
            gsw = opts["smoother"] == xamg.GAUSS_SEIDEL
            nbytes = presmooth_bytes(prob.n, prob.nnz, m, vb=vb32,
                                     ib=ib32 if mixed and not gsw else 4,
                                     bb=4 if mixed and not gsw else 8, xb=vb32,
                                     jacobi=opts["smoother"] == xamg.JACOBI)
            what = {xamg.CHEBYSHEV: "Chebyshev", xamg.JACOBI: "Jacobi",
                    xamg.GAUSS_SEIDEL: "Gauss-Seidel forward sweep"}[opts["smoother"]]
            kdesc = (f"rows_kernel<{m}> {what} pre-smoothing pass from zero, finest level "
                     f"({'FP32 values' if mixed else 'FP64'})")
        else:
            nbytes = spmm_bytes(prob.n, prob.nnz, m)
            kdesc = f"rows_kernel<{m}> finest-level q = A p with fused (p, q) dot (FP64 CSR)"
        gbs = nbytes / (avg_ms * 1e-3) / 1e9
        kernels[name] = {"kernel": kdesc, "launches": cnt, "avg_us": avg_ms * 1e3,
                         "total_ms_per_step": tms / args.steps, "algorithmic_bytes": nbytes,
                         "achieved_gbs": gbs}
        log(f"[bench] {name}: {cnt} launches, avg {avg_ms * 1e3:.1f} us, "
            f"{nbytes / 1e6:.1f} MB, {gbs:.0f} GB/s ({gbs / HBM_PEAK_GBS:.1%})")
    log(f"[bench] {args.steps} solves: {ms_step:.3f} ms/solve, {ms_step / m:.3f} ms/RHS, "
        f"iters {iters0.tolist()}, max true relres {tr0:.2e}")

    iteration = None
    smo = opts["smoother"]
    if opts["method"] == xamg.CG and smo in (xamg.JACOBI, xamg.CHEBYSHEV):
        idx16 = None
        if mixed and opts.get("index_bits", 32) == 16:
            import ctypes
            idx16 = []
            for l in range(S.nlev - 1):
                fr = (ctypes.c_double * 3)()
                xamg.lib().xamg_index16_fraction(S._h, l, fr)
                idx16.append(tuple(fr))
        ib = pcg_iteration_bytes(S, m, smo == xamg.CHEBYSHEV, mixed,
                                 flexible=mixed, idx16=idx16, merged=S.options.merged)
        it = int(iters0.max())
        gbs_it = ib * it / (ms_step * 1e-3) / 1e9
        iteration = {"bytes": ib, "iters": it, "ms_per_iteration": ms_step / it,
                     "achieved_gbs": gbs_it, "frac": gbs_it / HBM_PEAK_GBS}
        log(f"[bench] whole PCG iteration: {ib / 1e6:.0f} MB algorithmic, "
            f"{ms_step / it:.3f} ms -> {gbs_it:.0f} GB/s ({gbs_it / HBM_PEAK_GBS:.1%} of peak; "
            f"start and final residual check included in the time)")

    dom = max(kernels, key=lambda k: kernels[k]["total_ms_per_step"])
    K = kernels[dom]
    traffic = stored_traffic(wl, dom)
    sb = stream_bandwidth(torch)
    cgbs = sb["ceiling_gbs"]
    log(f"[bench] device copy {sb['copy_gbs']:.0f} GB/s, elementwise a + b {sb['add_gbs']:.0f} GB/s; "
        f"roofline kernel {K['achieved_gbs'] / cgbs:.1%} of the faster")
    roofline = {"kernel": K["kernel"], "bound": "hbm", "achieved": K["achieved_gbs"],
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": K["achieved_gbs"] / HBM_PEAK_GBS,
                "traffic": traffic, "algorithmic_bytes": K["algorithmic_bytes"],
                "avg_us": K["avg_us"], "launches_timed": K["launches"],
                "measured_copy_gbs": sb["copy_gbs"], "measured_add_gbs": sb["add_gbs"],
                "stream_ceiling_gbs": cgbs, "frac_of_stream": K["achieved_gbs"] / cgbs}

    extras = {}
    if not args.no_extras:
        # FP64 vs mixed precision (FP32 V-cycle, 16-bit offsets) on the same workload
        oo = dict(opts)
        if mixed:
            oo.update(precision=xamg.FP64, index_bits=32)
        else:
            oo.update(precision=xamg.MIXED, index_bits=16)
        Sm = xamg.Solver(Hh, stream=stream.cuda_stream, **oo)
        Xm = torch.zeros_like(Bd)
        Sm.solve(Bd, Xm, tol=1e-8)
        msm, itm, trm, rcm = timed_solves(Sm, Bd, Xm, args.steps, 1e-8, stream, torch)
        dx = (torch.linalg.norm(Xm - Xd, dim=0) / torch.linalg.norm(Xd, dim=0)).max().item()
        other = "fp64" if mixed else "mixed_precision"
        extras[other] = {"ms_per_rhs": msm / m, "iters": int(itm.max()),
                         "max_true_relres": trm, "max_rel_diff": dx}
        log(f"[bench] {other}: {msm / m:.3f} ms/RHS, iters {int(itm.max())}, "
            f"rel diff {dx:.2e}")
        Sm.close()
        # the CG forms (standard, x's update in the p pass, p pass in the
        # SpMM) on the launch shapes tuned for this solve: bitwise the same
        # iterates, different passes over the vectors
        if opts["method"] == xamg.CG and wl == "poisson128":
            forms = {}
            mp = 1 << (m - 1).bit_length()
            tun = S.tuning(mp)
            for f in (0, 1, 2):
                Sf = xamg.Solver(Hh, stream=stream.cuda_stream, **dict(opts, merged=f))
                Sf.set_tuning(mp, tun)
                Xf = torch.zeros_like(Bd)
                Sf.solve(Bd, Xf, tol=1e-8)
                msf, itf, trf, rcf = timed_solves(Sf, Bd, Xf, args.steps, 1e-8, stream, torch)
                forms[f"merged{f}"] = {
                    "ms_per_rhs": msf / m, "iters": int(itf.max()),
                    "bitwise_equal_to_default": bool(torch.equal(Xf, Xd)),
                    "bytes_per_iteration": pcg_iteration_bytes(
                        Sf, m, smo == xamg.CHEBYSHEV, mixed, flexible=mixed, merged=f)}
                log(f"[bench] CG form merged={f}: {msf / m:.4f} ms/RHS, iters {int(itf.max())}, "
                    f"{forms[f'merged{f}']['bytes_per_iteration'] / 1e9:.2f} GB/iteration, "
                    f"bitwise equal {forms[f'merged{f}']['bitwise_equal_to_default']}")
                Sf.close()
            extras["cg_forms"] = forms
        # pipelined BiCGStab beside BiCGStab (FP64 cycle only: its recurrences
        # need a linear preconditioner)
        if opts["method"] == xamg.BICGSTAB and not mixed:
            Sp = xamg.Solver(Hh, stream=stream.cuda_stream, **dict(opts, method=xamg.PBICGSTAB))
            Xp = torch.zeros_like(Bd)
            Sp.solve(Bd, Xp, tol=1e-8)
            msp, itp, trp, rcp = timed_solves(Sp, Bd, Xp, args.steps, 1e-8, stream, torch)
            dxp = (torch.linalg.norm(Xp - Xd, dim=0) / torch.linalg.norm(Xd, dim=0)).max().item()
            extras["pipelined_bicgstab"] = {"ms_per_rhs": msp / m, "iters": int(itp.max()),
                                            "max_true_relres": trp, "max_rel_diff": dxp}
            log(f"[bench] pipelined BiCGStab: {msp / m:.3f} ms/RHS, iters {int(itp.max())}, "
                f"rel diff {dxp:.2e}")
            Sp.close()
        # multigrid as the solver (no Krylov acceleration), same smoother
        if wl == "poisson128":
            Sg = xamg.Solver(Hh, stream=stream.cuda_stream, **dict(opts, method=xamg.MG))
            Xg = torch.zeros_like(Bd)
            Sg.solve(Bd, Xg, tol=1e-8)
            msg, itg, trg, rcg = timed_solves(Sg, Bd, Xg, args.steps, 1e-8, stream, torch)
            extras["mg_solver"] = {"ms_per_rhs": msg / m, "iters": int(itg.max()),
                                   "max_true_relres": trg}
            log(f"[bench] MG as solver: {msg / m:.3f} ms/RHS, iters {int(itg.max())}")
            Sg.close()
        # aggressive coarsening of the finest level (a second RS pass on the
        # distance-two strength, one path; multipass interpolation): smaller
        # operator complexity, more iterations
        if wl in ("poisson128", "aniso256"):
            t0 = time.time()
            Ha = xamg.HostHierarchy(*prob.csr(), agg_levels=1, num_paths=1)
            t_agg = time.time() - t0
            Sa = xamg.Solver(Ha, stream=stream.cuda_stream, **opts)
            Xa = torch.zeros_like(Bd)
            Sa.solve(Bd, Xa, tol=1e-8)
            msa, ita, tra, rca = timed_solves(Sa, Bd, Xa, args.steps, 1e-8, stream, torch)
            agg = {"agg_levels": 1, "num_paths": 1, "levels": Ha.sizes(),
                   "operator_complexity": sum(Sa.nnzA) / Sa.nnzA[0],
                   "grid_complexity": sum(Sa.sizes) / Sa.sizes[0],
                   "ms_per_rhs": msa / m, "iters": int(ita.max()), "max_true_relres": tra,
                   "host_setup_s": round(t_agg, 1)}
            if opts["method"] == xamg.CG and opts["smoother"] in (xamg.JACOBI, xamg.CHEBYSHEV):
                agg["bytes_per_iteration"] = pcg_iteration_bytes(
                    Sa, m, opts["smoother"] == xamg.CHEBYSHEV, mixed, flexible=mixed,
                    merged=Sa.options.merged)
            extras["aggressive"] = agg
            log(f"[bench] aggressive level 0: levels {Ha.sizes()}, C_A "
                f"{agg['operator_complexity']:.3f}, C_G {agg['grid_complexity']:.3f}, "
                f"{msa / m:.3f} ms/RHS, iters {int(ita.max())}")
            Sa.close()
            del Ha
        # the configuration of the paper's parameter example (Section 2.4):
        # pipelined BiCGStab, AMG with two aggressive levels and two paths,
        # coarsening to 500 rows, Chebyshev degree 2 smoothing (FP64)
        if wl == "poisson128":
            t0 = time.time()
            He = xamg.HostHierarchy(*prob.csr(), max_coarse=500, agg_levels=2, num_paths=2)
            t_ex = time.time() - t0
            Se = xamg.Solver(He, stream=stream.cuda_stream, method=xamg.PBICGSTAB,
                             smoother=xamg.CHEBYSHEV)
            Xe = torch.zeros_like(Bd)
            Se.solve(Bd, Xe, tol=1e-8)
            mse, ite, tre, rce = timed_solves(Se, Bd, Xe, args.steps, 1e-8, stream, torch)
            extras["paper_example"] = {
                "method": "pipelined BiCGStab", "agg_levels": 2, "num_paths": 2,
                "max_coarse": 500, "smoother": "chebyshev2", "levels": He.sizes(),
                "operator_complexity": sum(Se.nnzA) / Se.nnzA[0],
                "ms_per_rhs": mse / m, "iters": int(ite.max()), "max_true_relres": tre,
                "host_setup_s": round(t_ex, 1)}
            log(f"[bench] paper example (PBiCGStab, 2 aggressive levels, 2 paths): levels "
                f"{He.sizes()}, {mse / m:.3f} ms/RHS, iters {int(ite.max())}")
            Se.close()
            del He
        # multi-RHS gain P_m = m T_1 / T_m
        if wl in ("poisson128", "gs150"):
            res = {}
            for mm in (1, 2, 4, 8):
                Bm = Bd[:, :mm].contiguous()
                Xmm = torch.zeros_like(Bm)
                S.solve(Bm, Xmm, tol=1e-8)
                t, _, _, _ = timed_solves(S, Bm, Xmm, max(2, args.steps // 2), 1e-8, stream, torch)
                res[mm] = t
            res[m] = ms_step
            ms_list = sorted(res)
            extras["multi_rhs_gain"] = {
                "m": ms_list, "ms_per_solve": [res[k] for k in ms_list],
                "P_m": [k * res[1] / res[k] for k in ms_list]}
            log(f"[bench] P_m: " + ", ".join(f"m={k}: {k * res[1] / res[k]:.2f}" for k in ms_list))

    cpu = None
    if not args.no_cpu:
        import oracle
        t0 = time.time()
        Ho = oracle.Hierarchy(*prob.csr())
        log(f"[bench] oracle setup {time.time() - t0:.1f}s (not timed)")
        kw = dict(smoother={xamg.CHEBYSHEV: oracle.CHEBYSHEV, xamg.JACOBI: oracle.JACOBI,
                            xamg.GAUSS_SEIDEL: oracle.GAUSS_SEIDEL}[opts["smoother"]],
                  method=oracle.BICGSTAB if opts["method"] == xamg.BICGSTAB else oracle.CG,
                  gs_block=opts.get("gs_block", 8))
        sample_iters = args.cpu_iters if args.cpu_iters > 0 else (
            2 if wl == "aniso256" and not args.cpu_full else 0)
        oracle.set_verbose(True)
        t0 = time.perf_counter()
        if sample_iters:
            Xo, so, rco = Ho.solve(B, max_iters=sample_iters, tol=1e-8, **kw)
        else:
            Xo, so, rco = Ho.solve(B, tol=1e-8, **kw)
        tcpu = time.perf_counter() - t0
        gpu_it = int(iters0.max())
        if sample_iters:
            tcpu = tcpu / sample_iters * gpu_it
            sample = (f"{sample_iters} FP64 oracle iterations on the same workload, "
                      f"scaled to the {gpu_it} iterations of the GPU solve (setup excluded)")
        else:
            sample = (f"full FP64 oracle solve of the same workload ({int(so['iters'].max())} "
                      f"iterations, setup excluded)")
            err = np.linalg.norm(Xd.cpu().numpy() - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
            log(f"[bench] GPU vs oracle max rel err {err.max():.2e}")
            extras["per_column_rel_err_vs_oracle"] = [float(e) for e in err]
            extras["oracle_iters"] = [int(i) for i in so["iters"]]
        cpu = {"value": tcpu * 1e3 / m, "unit": "ms/RHS", "cores": oracle.num_threads(),
               "kind": "oracle", "sample": sample}
        log(f"[bench] oracle {tcpu:.1f}s -> {cpu['value']:.1f} ms/RHS on {cpu['cores']} threads")

    out = {
        "metric": "ms per RHS to rel. residual 1e-8 (AMG-PCG), FP64 vs mixed; SpMM HBM GB/s",
        "value": ms_step / m,
        "unit": "ms/RHS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64/f32" if mixed else "f64",
        "data": "synthetic",
        "config": {
            "workload": desc, "n": prob.n, "nnz": prob.nnz, "m": m, "tol": 1e-8,
            "iters": int(iters0.max()), "levels": S.nlev,
            "operator_complexity": round(sum(nnzA) / nnzA[0], 3),
            "grid_complexity": round(sum(S.sizes) / S.sizes[0], 3),
            "host_setup_s": round(t_setup, 2),
            "cg_form": f"merged{S.options.merged}" if opts.get("method", xamg.CG) == xamg.CG
            else None,
            "launch_shapes": [list(t) for t in S.tuning(mp)],
        },
        "roofline": roofline,
        "kernels": kernels,
        "iteration": iteration,
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)
    S.close()


def bench_warmstart(args, torch, inputs, xamg):
    """Learned warm start on 3D Poisson 128^3, m = 32 Gaussian-source
    right-hand sides (seed 1006).  The network is trained first (untimed)
    on pairs solved by the library's FP64 AMG-PCG (seed 1005; 1792 training
    / 256 validation, seeded split), unless weights are given.  One step =
    warm start (CNN forward per column + zero-guess fallback) + PCG solve
    from it, against the same solve from X0 = 0."""
    from paper_2103_07329_amd import warmstart as W
    N, m, tol = 128, 32, 1e-8
    n = N ** 3
    prob = inputs.poisson7(N)
    log(f"[bench] workload warmstart: {prob}, m={m}")
    t0 = time.time()
    Hh = xamg.HostHierarchy(*prob.csr())
    t_setup = time.time() - t0
    stream = torch.cuda.current_stream()
    opts = dict(smoother=xamg.CHEBYSHEV, method=xamg.CG)
    S0 = xamg.Solver(Hh, stream=stream.cuda_stream, **opts)
    S1 = xamg.Solver(Hh, stream=stream.cuda_stream, x0_mode=xamg.X0_GIVEN, **opts)
    net = xamg.Cnn(N, W.he_init(7), stream=stream.cuda_stream)
    train_info = None
    if args.ws_weights:
        net.set_weights(np.load(args.ws_weights))
        train_info = {"weights": os.path.basename(args.ws_weights)}
    else:
        t0 = time.time()
        xs, ts, it = W.make_pairs(S0, N, args.ws_pairs, 1005, torch)
        t_pairs = time.time() - t0
        perm = np.random.default_rng(5).permutation(args.ws_pairs)
        nval = args.ws_pairs // 8
        t0 = time.time()
        hist = W.train(net, xs, ts, perm[nval:], perm[:nval], torch, epochs=args.ws_epochs,
                       batch=8, lr=1e-3, seed=5, objective=args.ws_objective, solver=S0)
        t_train = time.time() - t0
        train_info = {"objective": args.ws_objective,
                      "pairs": args.ws_pairs, "train": int(args.ws_pairs - nval),
                      "validation": int(nval), "epochs": len(hist), "batch": 8, "lr": 1e-3,
                      "pair_solve_iters": float(it.mean()), "pairs_s": round(t_pairs, 1),
                      "train_s": round(t_train, 1), "final_train_loss": hist[-1][1],
                      "final_validation_loss": hist[-1][2],
                      "validation_loss_by_epoch": [round(h[2], 5) for h in hist]}
        del xs, ts
        torch.cuda.empty_cache()
        if args.ws_save:
            np.save(args.ws_save, net.weights())
    params = inputs.gaussian_params(N, m, 1006)
    Bd = inputs.gaussian_rhs_torch(N, params, list(range(m)), torch, "cuda")
    # quality of the raw network guess (no fallback) against the converged solution
    Xref = torch.zeros_like(Bd)
    S0.solve(Bd, Xref, tol)
    X0raw = torch.zeros_like(Bd)
    net.warmstart(Bd, X0raw, None)
    R = torch.empty_like(Bd)
    S0.spmm(xamg.OP_A, 0, X0raw, R)
    bn = torch.linalg.vector_norm(Bd, dim=0)
    raw_res = (torch.linalg.vector_norm(Bd - R, dim=0) / bn).cpu().numpy()
    raw_err = (torch.linalg.vector_norm(Xref - X0raw, dim=0)
               / torch.linalg.vector_norm(Xref, dim=0)).cpu().numpy()
    log(f"[bench] raw CNN guess: median rel error {np.median(raw_err):.3f}, "
        f"median initial rel residual {np.median(raw_res):.3f}")
    # also: PCG from the raw guess, no fallback (for the record)
    Xr = X0raw.clone()
    _, st_raw = S1.solve(Bd, Xr, tol)
    X = torch.zeros_like(Bd)
    X0 = torch.zeros_like(Bd)

    def zero_step():
        X.zero_()
        return S0.solve(Bd, X, tol)

    def warm_step():
        fb = net.warmstart(Bd, X0, S1)
        X.copy_(X0)
        rc, st = S1.solve(Bd, X, tol)
        return rc, st, fb

    for _ in range(args.warmup):
        zero_step()
        warm_step()

    def timed(fn):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        outs = [fn() for _ in range(args.steps)]
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps, outs[-1]

    ms_zero, (rcz, stz) = timed(zero_step)
    Xz = X.clone()
    net.timer_enable(xamg.CNN_TIMER_CONV16)
    ms_warm, (rcw, stw, fb) = timed(warm_step)
    tms, cnt = net.timer_read()
    net.timer_enable(xamg.CNN_TIMER_OFF)
    assert rcz == xamg.OK and rcw == xamg.OK, (rcz, rcw)
    diff = (torch.linalg.vector_norm(X - Xz, dim=0) / torch.linalg.vector_norm(Xz, dim=0)).max().item()
    # CNN inference alone
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        net.warmstart(Bd, X0, S1)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_cnn = e0.elapsed_time(e1) / args.steps
    log(f"[bench] zero guess: {ms_zero:.2f} ms/solve, iters {stz['iters'].tolist()}")
    log(f"[bench] warm start: {ms_warm:.2f} ms/solve (CNN + fallback {ms_cnn:.2f} ms), "
        f"iters {stw['iters'].tolist()}, fallbacks {int(fb.sum())}/{m}, max rel diff {diff:.1e}")
    # one 16 -> 16 layer over one sample: 27 * 16 * 16 multiply-adds per voxel
    # against 64 bytes per voxel (16 BF16 channels read, 16 written): 216
    # flop/B, below the BF16 ridge of 2.5 PFLOP/s / 8 TB/s = 312 flop/B, so the
    # layer is bound by HBM (16.8 us at 128^3) before the MFMA (11.6 us)
    flops = 2.0 * n * 27 * 16 * 16
    cbytes = 2.0 * n * 16 * 2
    avg_ms = tms / max(cnt, 1)
    tfs = flops / (avg_ms * 1e-3) / 1e12
    gbs = cbytes / (avg_ms * 1e-3) / 1e9
    log(f"[bench] conv16: {cnt} launches, avg {avg_ms * 1e3:.1f} us, {gbs:.0f} GB/s "
        f"({gbs / 8000.0:.2%} of 8 TB/s), {tfs:.1f} TFLOP/s ({tfs / 2500.0:.2%} of 2.5 PFLOP/s)")
    roofline = {"kernel": "conv16_lds (16 -> 16 channel 3x3x3 convolution, BF16 MFMA, FP32 "
                          "accumulation), CNN forward", "bound": "hbm", "achieved": gbs,
                "peak": 8000.0, "unit": "GB/s", "frac": gbs / 8000.0, "traffic": None,
                "algorithmic_bytes": cbytes, "algorithmic_flops": flops,
                "mfma_tflops": tfs, "mfma_frac": tfs / 2500.0,
                "avg_us": avg_ms * 1e3, "launches_timed": cnt}
    cpu = None
    if not args.no_cpu:
        import oracle
        t0 = time.time()
        Ho = oracle.Hierarchy(*prob.csr())
        log(f"[bench] oracle setup {time.time() - t0:.1f}s (not timed)")
        Bh = Bd[:, :1].cpu().numpy()
        Ws = [oracle.bf16(w) for w in xamg.split_weights(net.weights().astype(np.float64))]
        oracle.set_verbose(True)
        t0 = time.perf_counter()
        b = Bh[:, 0]
        s = np.sqrt(b @ b / n)
        x0 = s * oracle.cnn_forward(N, Ws, (b / s).astype(np.float32), quantize=True)[-1].reshape(-1)
        r0 = b - oracle.spmm(*Ho.A(0)[:3], x0[:, None], ncols=n)[:, 0]
        if not np.linalg.norm(r0) < np.linalg.norm(b):
            x0[:] = 0.0
        Xo, so, rco = Ho.solve(Bh, X0=x0[:, None], method=oracle.CG, smoother=oracle.CHEBYSHEV,
                               tol=tol)
        tcpu = time.perf_counter() - t0
        cpu = {"value": tcpu * 1e3, "unit": "ms/RHS", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "one right-hand side of the same workload: FP64 CNN forward on "
                         "BF16-rounded operands, fallback test, FP64 PCG solve"}
        log(f"[bench] oracle {tcpu:.1f}s per RHS on {cpu['cores']} threads")
    out = {
        "metric": "ms per RHS to rel. residual 1e-8 (AMG-PCG), FP64 vs mixed; SpMM HBM GB/s",
        "value": ms_warm / m,
        "unit": "ms/RHS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_warm,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 solve, bf16/f32 CNN", "data": "synthetic",
        "config": {"workload": "poisson128_gaussian_m32_cnn_warmstart_pcg_chebyshev2_fp64",
                   "n": n, "m": m, "tol": tol, "host_setup_s": round(t_setup, 2)},
        "zero_guess": {"ms_per_rhs": ms_zero / m, "iters": stz["iters"].tolist()},
        "warm_start": {"ms_per_rhs": ms_warm / m, "iters": stw["iters"].tolist(),
                       "cnn_and_fallback_ms": ms_cnn, "fallbacks": int(fb.sum()),
                       "max_rel_diff_vs_zero_guess_solution": diff},
        "raw_guess": {"median_rel_error": float(np.median(raw_err)),
                      "median_initial_relres": float(np.median(raw_res)),
                      "max_initial_relres": float(raw_res.max()),
                      "iters_without_fallback": st_raw["iters"].tolist()},
        "training": train_info,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    for o in (S0, S1, net):
        o.close()


def batched_cpu_baseline(systems, sts, Xs, nrhs):
    """The oracle (FP64 CG, Jacobi V(1,1)) on a bounded sample of the batch:
    full solves of the systems in increasing order of n x m until about 10 s
    of oracle time (setup excluded), then scaled to the whole batch by work
    n x m x iterations (the GPU's per-system iteration counts for the
    systems not sampled).  Also returns the sampled systems' error of the
    batched solution against the oracle's."""
    import oracle
    work = [p.n * B.shape[1] * int(st["iters"].max()) for (p, B), st in zip(systems, sts)]
    order = sorted(range(len(systems)), key=lambda s: systems[s][0].n * systems[s][1].shape[1])
    t_s, w_s, errs, done = 0.0, 0, [], []
    for s in order:
        if t_s >= 10.0:
            break
        done.append(s)
        prob, B = systems[s]
        Ho = oracle.Hierarchy(*prob.csr())
        t0 = time.perf_counter()
        Xo, so, rco = Ho.solve(B, method=oracle.CG, smoother=oracle.JACOBI, tol=1e-8)
        t_s += time.perf_counter() - t0
        w_s += prob.n * B.shape[1] * int(so["iters"].max())
        X = Xs[s].cpu().numpy()
        errs.append(float((np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)).max()))
    t_all = t_s * sum(work) / w_s
    log(f"[bench] oracle sample (systems {done}): {t_s:.1f}s -> whole batch {t_all:.1f}s, "
        f"batched vs oracle max rel err {max(errs):.2e}")
    return {"value": t_all * 1e3 / nrhs, "unit": "ms/RHS", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": (f"full FP64 oracle solves of systems {done} of the batch (least "
                       f"n x m first, about 10 s; setup excluded), scaled to all 12 by "
                       f"n x m x iterations"),
            "sample_rel_err_vs_batched": max(errs)}


def bench_batched(args, torch, inputs, xamg):
    """12 jump-coefficient systems of uneven size and column count (seed
    1004), AMG-PCG with an FP32 preconditioner and 16-bit offsets, all
    iterations from one captured HIP graph; compared with 12 separate FP64
    solves and 12 separate mixed solves."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    systems = inputs.batched_systems(seed=1004, count=12)
    t0 = time.time()
    hier, Bs = [], []
    for prob, B in systems:
        hier.append(xamg.HostHierarchy(*prob.csr()))
        Bs.append(torch.from_numpy(B).to(dev))
    t_setup = time.time() - t0
    sides = [p.N for p, _ in systems]
    ms = [B.shape[1] for _, B in systems]
    nrhs = sum(ms)
    log(f"[bench] batched: sides {sides}, m {ms}, host setup {t_setup:.1f}s")
    mixed = [xamg.Solver(H, stream=stream.cuda_stream, precision=xamg.MIXED, index_bits=16)
             for H in hier]
    batch = xamg.Batch(mixed)
    Xs = [torch.zeros_like(B) for B in Bs]
    for _ in range(args.warmup):
        rc, _ = batch.solve(Bs, Xs)
        assert rc == xamg.OK, rc
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rc, sts = batch.solve(Bs, Xs)
        assert rc == xamg.OK, rc
    torch.cuda.synchronize()
    ms_batched = (time.perf_counter() - t0) * 1e3 / args.steps
    iters = [int(st["iters"].max()) for st in sts]
    tr = max(float(st["true_relres"].max()) for st in sts)
    log(f"[bench] batched graph: {ms_batched:.2f} ms per batch, {ms_batched / nrhs:.4f} ms/RHS, "
        f"iters {iters}, max true relres {tr:.2e}")

    def separate(solvers):
        Xl = [torch.zeros_like(B) for B in Bs]
        for S, B, X in zip(solvers, Bs, Xl):
            S.solve(B, X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for S, B, X in zip(solvers, Bs, Xl):
                rc, _ = S.solve(B, X)
                assert rc == xamg.OK, rc
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps, Xl

    ms_sep_mixed, _ = separate(mixed)
    fp64 = [xamg.Solver(H, stream=stream.cuda_stream) for H in hier]
    ms_sep_fp64, X64 = separate(fp64)
    err = max(float((torch.linalg.norm(X - Y, dim=0) / torch.linalg.norm(Y, dim=0)).max())
              for X, Y in zip(Xs, X64))
    log(f"[bench] separate mixed: {ms_sep_mixed:.2f} ms, separate FP64: {ms_sep_fp64:.2f} ms, "
        f"batched vs FP64 max rel diff {err:.2e}")
    big = int(np.argmax([p.n for p, _ in systems]))
    S = mixed[big]
    S.timer_enable(xamg.TIMER_PRESMOOTH)
    Xb = torch.zeros_like(Bs[big])
    S.solve(Bs[big], Xb)
    tms, cnt = S.timer_read()
    S.timer_enable(xamg.TIMER_OFF)
    pb, mb = systems[big][0], ms[big]
    nbytes = presmooth_bytes(pb.n, pb.nnz, mb, vb=4, ib=2, bb=8, xb=4, jacobi=True)
    gbs = nbytes / (tms / cnt * 1e-3) / 1e9
    out = {
        "metric": "ms per RHS to rel. residual 1e-8 (AMG-PCG), FP64 vs mixed; SpMM HBM GB/s",
        "value": ms_batched / nrhs, "unit": "ms/RHS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_batched, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64/f32", "data": "synthetic",
        "config": {"workload": "batched12_jump_pcg_fp32precond_idx16_graph", "sides": sides,
                   "m": ms, "total_rhs": nrhs, "tol": 1e-8, "iters": iters,
                   "host_setup_s": round(t_setup, 1)},
        "roofline": {"kernel": f"rows_kernel<{mb}> Jacobi pre-smoothing pass, FP32 values, "
                               f"16-bit offsets, largest system (n={pb.n})",
                     "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes": nbytes,
                     "avg_us": tms / cnt * 1e3},
        "separate_solves": {"mixed_ms": ms_sep_mixed, "fp64_ms": ms_sep_fp64,
                            "fp64_ms_per_rhs": ms_sep_fp64 / nrhs,
                            "max_rel_diff_batched_vs_fp64": err},
        "cpu_baseline": None if args.no_cpu else batched_cpu_baseline(systems, sts, Xs, nrhs),
    }
    print(json.dumps(out), flush=True)
    batch.close()
    for S in mixed + fp64:
        S.close()


if __name__ == "__main__":
    main()
