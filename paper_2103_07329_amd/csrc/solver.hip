// solver.hip -- device setup, V-cycle, Krylov drivers and the C ABI of
// libxamg (declared in include/xamg.h).
//
// The solve follows the paper's solver structure (Section 2.3: solver
// objects with setup() and solve(); Section 2.4: construct the hierarchy,
// then solve for NV right-hand sides at once):
//   xamg_setup  uploads the hierarchy (A_l, P_l, R_l) in FP64, and in FP32
//               (optionally with 16-bit indices) for a mixed-precision
//               preconditioner (Section 2.3, "data compression"), computes
//               D_l^-1 and the inverse of the coarsest matrix;
//   xamg_solve  runs preconditioned CG (or BiCGStab, bicgstab.hip) with one
//               set of scalars per column; every vector operation and dot
//               is a device kernel, the scalars stay on the device, and the
//               host only polls the number of still-active columns.
#include <chrono>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"
#include "kernels.hpp"
#include "ops.hpp"
#include "solver.hpp"

namespace xamg {

using namespace dev;

// ---------------------------------------------------------------------------
// device memory helpers
// ---------------------------------------------------------------------------
void Handle::check(hipError_t e, const char* what)
{
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory) {
            set_error("device allocation failed (%s)", what);
            throw DevFail{XAMG_ENOMEM};
        }
        set_error("HIP error %d (%s) in %s", int(e), hipGetErrorString(e), what);
        throw DevFail{XAMG_EHIP};
    }
}

void* Handle::alloc_bytes(size_t bytes)
{
    void* p = nullptr;
    check(hipMalloc(&p, std::max<size_t>(bytes, 256)), "hipMalloc");
    allocs.push_back(p);
    return p;
}

void Handle::release(void* p)
{
    if (!p) return;
    auto it = std::find(allocs.begin(), allocs.end(), p);
    if (it != allocs.end()) {
        hipFree(p);
        allocs.erase(it);
    }
}

Handle::~Handle()
{
    for (void* p : allocs) hipFree(p);
    if (st_host) hipHostFree(st_host);
    for (hipEvent_t e : ev_pool) hipEventDestroy(e);
}

// kernel timer: an event pair around each launch of the selected kind
void Handle::timer_begin(int kind)
{
    if (timer_kind == 0 || kind != timer_kind) return;
    if (ev_used + 2 > ev_pool.size()) {
        for (int k = 0; k < 64; ++k) {
            hipEvent_t e;
            check(hipEventCreate(&e), "hipEventCreate");
            ev_pool.push_back(e);
        }
    }
    check(hipEventRecord(ev_pool[ev_used], stream), "hipEventRecord");
}

void Handle::timer_end(int kind)
{
    if (timer_kind == 0 || kind != timer_kind) return;
    check(hipEventRecord(ev_pool[ev_used + 1], stream), "hipEventRecord");
    ev_used += 2;
}

// add up the recorded pairs (after the stream has been synchronised)
void Handle::timer_collect()
{
    for (size_t k = 0; k + 1 < ev_used; k += 2) {
        float ms = 0.0f;
        check(hipEventElapsedTime(&ms, ev_pool[k], ev_pool[k + 1]), "hipEventElapsedTime");
        timer_ms += ms;
        timer_count += 1;
    }
    ev_used = 0;
}

template <typename T>
static T* upload(Handle& h, const T* src, size_t n)
{
    T* d = h.alloc<T>(n);
    if (n) h.check(hipMemcpy(d, src, n * sizeof(T), hipMemcpyHostToDevice), "upload");
    return d;
}

static DCsr upload_csr(Handle& h, const xamg_csr_t& c, bool fp32)
{
    DCsr d;
    d.nr = int(c.nrows);
    d.nc = int(c.ncols);
    d.nnz = c.nnz;
    for (int k = 0; k < 6; ++k) d.split[k] = d.split_pre[k] = split_for(c.nnz, int(c.nrows));
    d.rp = upload(h, c.row_ptr, size_t(c.nrows) + 1);
    d.ci = upload(h, c.col, size_t(c.nnz));
    if (c.nrows == c.ncols)
        for (int64_t i = 0; i < c.nrows; ++i)
            for (int64_t k = c.row_ptr[i]; k < c.row_ptr[i + 1]; ++k)
                d.bw = std::max<int64_t>(d.bw, c.col[k] > i ? c.col[k] - i : i - c.col[k]);
    if (fp32) {
        std::vector<float> v(c.val, c.val + c.nnz);
        d.v = upload(h, v.data(), v.size());
        d.fp32 = true;
    } else {
        d.v = upload(h, c.val, size_t(c.nnz));
    }
    return d;
}

// A square operator whose rows are (nearly) all of one length, with the
// shorter rows padded to that length by explicit zeros at columns the row
// does not hold (the nearest ones, i +- 1, i +- 2, ...), in sorted order.
// The zeros add exact zeros to every row sum, so results are unchanged.
// Padded only when the maximum row length is at most 32, the padding adds
// at most 15% entries and the padded count fits 32-bit offsets.
bool pad_uniform(const xamg_csr_t& c, UniformCsr& u)
{
    if (c.nrows != c.ncols || c.nrows < 1) return false;
    const int n = int(c.nrows);
    int w = 0;
    for (int i = 0; i < n; ++i) w = std::max(w, c.row_ptr[i + 1] - c.row_ptr[i]);
    if (w < 1 || w > 32 || double(n) * w > 1.15 * double(c.nnz) || w > n) return false;
    // entry offsets i * rowlen are 32-bit, like the CSR row pointers
    if (int64_t(n) * w > int64_t(INT32_MAX)) return false;
    u.rowlen = w;
    u.rp.resize(size_t(n) + 1);
    u.ci.resize(size_t(n) * w);
    u.v.resize(size_t(n) * w);
    std::vector<int32_t> cols;
    for (int i = 0; i < n; ++i) {
        const int b = c.row_ptr[i], e = c.row_ptr[i + 1];
        cols.assign(c.col + b, c.col + e);
        for (int dist = 1; int(cols.size()) < w; ++dist)
            for (int cand : {i - dist, i + dist})
                if (int(cols.size()) < w && cand >= 0 && cand < n &&
                    !std::binary_search(c.col + b, c.col + e, cand))
                    cols.push_back(cand);
        std::sort(cols.begin(), cols.end());
        int k = b;
        for (int q = 0; q < w; ++q) {
            const size_t o = size_t(i) * w + q;
            u.ci[o] = cols[q];
            if (k < e && c.col[k] == cols[q]) u.v[o] = c.val[k++];
            else u.v[o] = 0.0;
        }
        u.rp[i] = i * w;
    }
    u.rp[n] = n * w;
    u.view.nrows = c.nrows;
    u.view.ncols = c.ncols;
    u.view.nnz = int64_t(n) * w;
    u.view.row_ptr = u.rp.data();
    u.view.col = u.ci.data();
    u.view.val = u.v.data();
    return true;
}

// 16-bit index encoding of a CSR pattern (see Idx16 in kernels.hpp): per
// block of kIdxRows rows, up to 4 windows with an int32 base each; an entry
// is (window << 14) | (col - base).  Windows are formed greedily over the
// block's sorted distinct columns; a block needing more than 4 windows stays
// in 32 bits (base.w = -1).  Returns the fraction of nonzeros encoded.
static double encode16(Handle& h, const xamg_csr_t& c, DCsr& d)
{
    const int n = int(c.nrows);
    const int nblk = (n + kIdxRows - 1) / kIdxRows;
    std::vector<uint16_t> off(size_t(std::max<int64_t>(c.nnz, 1)), 0);
    std::vector<int4> base(std::max(nblk, 1));
    int64_t enc = 0;
    std::vector<int> cols;
    for (int b = 0; b < nblk; ++b) {
        const int r0 = b * kIdxRows, r1 = std::min(n, r0 + kIdxRows);
        cols.assign(c.col + c.row_ptr[r0], c.col + c.row_ptr[r1]);
        std::sort(cols.begin(), cols.end());
        int bases[4] = {0, 0, 0, 0};
        int nw = 0;
        bool ok = true;
        for (int col : cols) {
            if (nw > 0 && col - bases[nw - 1] < (1 << 14)) continue;
            if (nw == 4) { ok = false; break; }
            bases[nw++] = col;
        }
        if (!ok) {
            base[b] = make_int4(0, 0, 0, -1);
            continue;
        }
        for (int w = nw; w < 4; ++w) bases[w] = bases[nw > 0 ? nw - 1 : 0];
        base[b] = make_int4(bases[0], bases[1], bases[2], bases[3]);
        for (int64_t k = c.row_ptr[r0]; k < c.row_ptr[r1]; ++k) {
            const int col = c.col[k];
            int w = nw - 1;
            while (w > 0 && col < bases[w]) --w;
            off[k] = uint16_t((w << 14) | (col - bases[w]));
        }
        enc += c.row_ptr[r1] - c.row_ptr[r0];
    }
    d.off = upload(h, off.data(), off.size());
    d.base = upload(h, base.data(), base.size());
    return c.nnz > 0 ? double(enc) / double(c.nnz) : 1.0;
}

// ---------------------------------------------------------------------------
// work buffers
// ---------------------------------------------------------------------------
// The work buffers of a solve for mc columns, in one fixed order: `get`
// supplies the memory of each (a device allocation, or a slice of a region
// the caller owns).  w.lev must already hold h.nlev entries.
template <class Get>
static void layout_work(const Handle& h, int mc, bool bicg, bool pad, Work& w, Get&& get)
{
    w.mcap = mc;
    const size_t es = h.opt.precision == XAMG_MIXED ? sizeof(float) : sizeof(double);
    for (int l = 0; l < h.nlev; ++l) {
        const size_t n = size_t(h.lev[l].n) * mc;
        auto& W = w.lev[l];
        W = LevelWork{};
        const size_t esl = (h.nlev == 1) ? sizeof(double) : es;
        if (l > 0) W.B = get(n * esl);
        if (l + 1 < h.nlev) {
            W.X = get(n * esl);
            W.R = get(n * esl);
            W.T = get(n * esl);
        }
        if (l > 0) W.X2 = get(n * esl);
    }
    const size_t n0 = size_t(h.lev[0].n) * mc;
    w.r = static_cast<double*>(get(n0 * sizeof(double)));
    w.z = static_cast<double*>(get(n0 * sizeof(double)));
    w.p = static_cast<double*>(get(n0 * sizeof(double)));
    w.q = static_cast<double*>(get(n0 * sizeof(double)));
    w.t = static_cast<double*>(get(n0 * sizeof(double)));
    w.p2 = nullptr;
    if (h.opt.method == XAMG_CG && h.opt.merged == 2)
        w.p2 = static_cast<double*>(get(n0 * sizeof(double)));
    w.r32 = w.p32 = w.s32 = nullptr;
    w.rh = w.v = w.s = w.ph = w.sh = nullptr;
    w.bpad = w.xpad = nullptr;
    if (h.opt.precision == XAMG_MIXED && h.opt.method == XAMG_CG &&
        h.opt.smoother != XAMG_GAUSS_SEIDEL && h.nlev > 1)
        w.r32 = static_cast<float*>(get(n0 * sizeof(float)));
    if (bicg && h.opt.precision == XAMG_MIXED && h.opt.smoother != XAMG_GAUSS_SEIDEL &&
        h.nlev > 1) {
        w.p32 = static_cast<float*>(get(n0 * sizeof(float)));
        w.s32 = static_cast<float*>(get(n0 * sizeof(float)));
    }
    if (bicg) {
        w.rh = static_cast<double*>(get(n0 * sizeof(double)));
        w.v = static_cast<double*>(get(n0 * sizeof(double)));
        w.s = static_cast<double*>(get(n0 * sizeof(double)));
        w.ph = static_cast<double*>(get(n0 * sizeof(double)));
        w.sh = static_cast<double*>(get(n0 * sizeof(double)));
    }
    w.rt = w.pw = w.wh = w.y = w.zh = w.qh = nullptr;
    if (bicg && h.opt.method == XAMG_PBICGSTAB)
        for (double** q : {&w.rt, &w.pw, &w.wh, &w.y, &w.zh, &w.qh})
            *q = static_cast<double*>(get(n0 * sizeof(double)));
    if (pad) {
        w.bpad = static_cast<double*>(get(n0 * sizeof(double)));
        w.xpad = static_cast<double*>(get(n0 * sizeof(double)));
    }
}

void ensure_work(Handle& h, int mp, bool bicg)
{
    const bool pipe = h.opt.method == XAMG_PBICGSTAB;
    if (h.w.mcap >= mp && (!bicg || h.w.rh) && (!pipe || h.w.rt)) return;
    // free old
    for (auto& W : h.w.lev) {
        h.release(W.B); h.release(W.X); h.release(W.X2); h.release(W.R); h.release(W.T);
    }
    for (double* p : {h.w.r, h.w.z, h.w.p, h.w.p2, h.w.q, h.w.t, h.w.rh, h.w.v, h.w.s, h.w.ph,
                      h.w.sh, h.w.xpad, h.w.bpad, h.w.rt, h.w.pw, h.w.wh, h.w.y, h.w.zh, h.w.qh})
        h.release(p);
    h.release(h.w.r32);
    h.release(h.w.p32);
    h.release(h.w.s32);
    const int mc = std::max(mp, h.w.mcap);
    h.w = Work{};
    h.w.lev.resize(h.nlev);
    layout_work(h, mc, bicg, false, h.w, [&](size_t bytes) { return h.alloc_bytes(bytes); });
}

size_t carve_work(const Handle& h, int mp, bool bicg, bool pad, Work& w, char* base,
                  size_t cap)
{
    size_t used = 0;
    bool fits = true;
    layout_work(h, mp, bicg, pad, w, [&](size_t bytes) -> void* {
        const size_t at = used;
        used += (bytes + 255) & ~size_t(255);
        fits = fits && used <= cap;
        return (base && fits) ? static_cast<void*>(base + at) : nullptr;
    });
    return used;
}

void sync_state(Handle& h)
{
    h.check(hipMemcpyAsync(h.st_host, h.st, sizeof(ColState), hipMemcpyDeviceToHost, h.stream),
            "state copy");
    h.check(hipStreamSynchronize(h.stream), "stream sync");
}

void poll_state(Handle& h)
{
    static_assert(offsetof(ColState, bn2) == 16, "the polled fields lead the column state");
    h.check(hipMemcpyAsync(h.st_host, h.st, 16, hipMemcpyDeviceToHost, h.stream), "poll copy");
    h.check(hipStreamSynchronize(h.stream), "stream sync");
}

template <class F>
static int dispatch_m(int mp, F&& f)
{
    switch (mp) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 16: return f(std::integral_constant<int, 16>{});
    case 32: return f(std::integral_constant<int, 32>{});
    default: return XAMG_EINVAL;
    }
}

int padded_m(int m)
{
    int mp = 1;
    while (mp < m) mp <<= 1;
    return mp;
}

static void fill_stats(const Handle& h, int m, xamg_stats_t* stats, double ms)
{
    if (!stats) return;
    const ColState& s = *h.st_host;
    for (int j = 0; j < m; ++j) {
        stats[j].iters = s.iters[j];
        stats[j].converged = (s.conv[j] && !(s.true_relres[j] > s.tol)) ? 1 : 0;
        stats[j].relres = s.relres[j];
        stats[j].true_relres = s.true_relres[j];
        stats[j].restarts = s.nrst[j];
        stats[j].reserved = 0;
        stats[j].ms = ms;
    }
}

// The solve proper, on buffers that are already in place: h.w for mp =
// padded(m) columns (with w.bpad / w.xpad when m is not a power of two),
// h.st and h.part.  Launches, copies and synchronisations only.
int solve_run(Handle& h, const double* B, double* X, int m, double tol, xamg_stats_t* stats)
{
    const auto t0 = std::chrono::steady_clock::now();
    const int mp = padded_m(m);
    const int n = h.lev[0].n;
    const double* Bs = B;
    double* Xs = X;
    if (mp != m) {
        hipLaunchKernelGGL((copy_cols_kernel<double, double>), dim3(2048), dim3(256), 0, h.stream,
                           B, m, h.w.bpad, mp, n, m);
        hipLaunchKernelGGL((copy_cols_kernel<double, double>), dim3(2048), dim3(256), 0, h.stream,
                           X, m, h.w.xpad, mp, n, m);
        Bs = h.w.bpad;
        Xs = h.w.xpad;
    }
    int rc = dispatch_m(mp, [&](auto mc) {
        constexpr int M = decltype(mc)::value;
        if (h.opt.method == XAMG_BICGSTAB) return bicgstab<M>(h, Bs, Xs, tol);
        if (h.opt.method == XAMG_PBICGSTAB) return pbicgstab<M>(h, Bs, Xs, tol);
        if (h.opt.method == XAMG_MG) return mg_solve<M>(h, Bs, Xs, tol);
        return pcg<M>(h, Bs, Xs, tol);
    });
    if (mp != m)
        hipLaunchKernelGGL((copy_cols_kernel<double, double>), dim3(2048), dim3(256), 0, h.stream,
                           h.w.xpad, mp, X, m, n, m);
    h.check(hipStreamSynchronize(h.stream), "solve sync");
    h.timer_collect();
    if (rc != XAMG_OK) return rc;
    fill_stats(h, m, stats,
               std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                   .count());
    const ColState& s = *h.st_host;
    bool failed = false, notconv = false;
    for (int j = 0; j < m; ++j) {
        failed |= s.failed[j] != 0;
        notconv |= !(s.conv[j] && !(s.true_relres[j] > s.tol));
    }
    if (failed) {
        set_error("Krylov breakdown: a column stopped (BiCGStab: a breakdown persisted after "
                  "its restart; pipelined BiCGStab: any breakdown)");
        return XAMG_EBREAKDOWN;
    }
    return notconv ? XAMG_NOT_CONVERGED : XAMG_OK;
}

int solve_impl(Handle& h, const double* B, double* X, int m, double tol, xamg_stats_t* stats)
{
    const int mp = padded_m(m);
    const int n = h.lev[0].n;
    ensure_work(h, mp, bicg_like(h.opt));
    if (h.autotune)
        dispatch_m(mp, [&](auto mc) {
            autotune<decltype(mc)::value>(h);
            return 0;
        });
    if (mp != m && !h.w.bpad) {
        h.w.bpad = h.alloc<double>(size_t(n) * h.w.mcap);
        h.w.xpad = h.alloc<double>(size_t(n) * h.w.mcap);
    }
    return solve_run(h, B, X, m, tol, stats);
}

}  // namespace xamg

// ===========================================================================
// C ABI
// ===========================================================================
using xamg::Handle;

extern "C" {

void xamg_default_options(xamg_options_t* o)
{
    o->method = XAMG_CG;
    o->smoother = XAMG_JACOBI;
    o->omega = 2.0 / 3.0;
    o->cheby_degree = 2;
    o->cheby_lo_frac = 0.3;
    o->cheby_hi_frac = 1.1;
    o->precision = XAMG_FP64;
    o->index_bits = 32;
    o->max_iters = 1000;
    o->x0_mode = XAMG_X0_ZERO;
    o->flexible = 0;
    o->check_every = 0;
    o->gs_block = 8;
    o->precond = 1;
    o->merged = 1;
    o->stream = nullptr;
}

static int device_ok()
{
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0)
        return xamg::fail(XAMG_ENODEV, "no HIP device");
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess)
        return xamg::fail(XAMG_ENODEV, "cannot query device");
    if (std::strncmp(p.gcnArchName, "gfx950", 6) != 0) {
        xamg::set_error("device %d is %s, not gfx950", dev, p.gcnArchName);
        return XAMG_ENODEV;
    }
    return XAMG_OK;
}

int xamg_setup(const xamg_hierarchy_t* H, const xamg_options_t* opt, xamg_handle_t** out)
{
    xamg::clear_error();
    if (!H || !out) return xamg::fail(XAMG_EINVAL, "null argument");
    *out = nullptr;
    xamg_options_t o;
    if (opt) o = *opt; else xamg_default_options(&o);
    if (o.method != XAMG_CG && o.method != XAMG_BICGSTAB && o.method != XAMG_MG &&
        o.method != XAMG_PBICGSTAB)
        return xamg::fail(XAMG_EINVAL, "method");
    if (o.smoother != XAMG_JACOBI && o.smoother != XAMG_CHEBYSHEV &&
        o.smoother != XAMG_GAUSS_SEIDEL)
        return xamg::fail(XAMG_EINVAL, "smoother");
    if (o.smoother == XAMG_GAUSS_SEIDEL && o.gs_block != 4 && o.gs_block != 8 && o.gs_block != 16)
        return xamg::fail(XAMG_EINVAL, "gs_block must be 4, 8 or 16");
    if (o.smoother == XAMG_CHEBYSHEV && (o.cheby_degree < 1 || o.cheby_degree > 2))
        return xamg::fail(XAMG_EINVAL, "cheby_degree must be 1 or 2");
    if (o.smoother == XAMG_CHEBYSHEV &&
        !(o.cheby_hi_frac > 0.0 && o.cheby_lo_frac > 0.0 && o.cheby_lo_frac < 1.0))
        return xamg::fail(XAMG_EINVAL, "Chebyshev interval fractions");
    if (o.precision != XAMG_FP64 && o.precision != XAMG_MIXED) return xamg::fail(XAMG_EINVAL, "precision");
    if (o.index_bits != 32 && o.index_bits != 16) return xamg::fail(XAMG_EINVAL, "index_bits");
    if (o.index_bits == 16 && o.precision != XAMG_MIXED)
        return xamg::fail(XAMG_EINVAL, "16-bit indices apply to the mixed-precision preconditioner");
    if (o.max_iters < 0) return xamg::fail(XAMG_EINVAL, "max_iters");
    if (o.precond != 0 && o.precond != 1) return xamg::fail(XAMG_EINVAL, "precond must be 0 or 1");
    if (o.precond == 0 && o.method == XAMG_MG)
        return xamg::fail(XAMG_EINVAL, "multigrid as the solver needs the V-cycle");
    if (o.merged < 0 || o.merged > 2) return xamg::fail(XAMG_EINVAL, "merged must be 0, 1 or 2");
    if (o.method == XAMG_PBICGSTAB && o.precision == XAMG_MIXED)
        return xamg::fail(XAMG_EINVAL,
                          "pipelined BiCGStab needs the FP64 V-cycle: its recurrences assume a "
                          "linear preconditioner, and the FP32 cycle is linear only to FP32 "
                          "accuracy");
    if (H->nlevels < 1 || H->nlevels > XAMG_MAX_LEVELS || !H->A)
        return xamg::fail(XAMG_EINVAL, "nlevels");
    if (H->nlevels > 1 && (!H->P || !H->R)) return xamg::fail(XAMG_EINVAL, "P/R missing");
    if (o.smoother == XAMG_CHEBYSHEV && H->nlevels > 1 && !H->lmax)
        return xamg::fail(XAMG_EINVAL, "lmax missing");
    for (int l = 0; l < H->nlevels; ++l) {
        int rc = xamg::validate_csr(&H->A[l], true, "A[l]");
        if (rc) return rc;
        if (l + 1 < H->nlevels) {
            rc = xamg::validate_csr(&H->P[l], false, "P[l]");
            if (rc) return rc;
            rc = xamg::validate_csr(&H->R[l], false, "R[l]");
            if (rc) return rc;
            if (H->P[l].nrows != H->A[l].nrows || H->P[l].ncols != H->A[l + 1].nrows ||
                H->R[l].nrows != H->A[l + 1].nrows || H->R[l].ncols != H->A[l].nrows)
                return xamg::fail(XAMG_EINVAL, "inconsistent level sizes");
            if (o.smoother == XAMG_CHEBYSHEV && !(H->lmax[l] > 0.0 && std::isfinite(H->lmax[l])))
                return xamg::fail(XAMG_EINVAL, "lmax must be positive");
        }
    }
    const int nL = int(H->A[H->nlevels - 1].nrows);
    if (nL > xamg::kMaxCoarse)
        return xamg::fail(XAMG_EINVAL, "coarsest level must have <= 1024 rows");
    int rc = device_ok();
    if (rc) return rc;

    Handle* h = new (std::nothrow) Handle;
    if (!h) return xamg::fail(XAMG_ENOMEM, "host allocation");
    try {
        h->opt = o;
        h->stream = static_cast<hipStream_t>(o.stream);
        {
            int dev = 0, ncu = 0;
            if (hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) ==
                    hipSuccess &&
                ncu > 0)
                h->num_cu = ncu;
            h->device = dev;
        }
        h->nlev = H->nlevels;
        h->lev.resize(h->nlev);
        h->w_na.lev.resize(h->nlev);
        const bool mixed = o.precision == XAMG_MIXED;
        for (int l = 0; l < h->nlev; ++l) {
            auto& L = h->lev[l];
            // rows of (nearly) uniform length are stored padded to exactly
            // that length, so the row kernels need no row pointers
            xamg::UniformCsr pad;
            const bool padded = l + 1 < h->nlev && xamg::pad_uniform(H->A[l], pad);
            const xamg_csr_t& a = padded ? pad.view : H->A[l];
            L.n = int(a.nrows);
            L.lmax = H->lmax ? H->lmax[l] : 0.0;
            L.A64 = xamg::upload_csr(*h, a, false);
            if (padded) L.A64.rowlen = pad.rowlen, L.A64.nnz = H->A[l].nnz;
            std::vector<double> d(L.n);
            for (int i = 0; i < L.n; ++i)
                for (int k = a.row_ptr[i]; k < a.row_ptr[i + 1]; ++k)
                    if (a.col[k] == i) d[i] = 1.0 / a.val[k];
            L.dinv64 = xamg::upload(*h, d.data(), d.size());
            if (l + 1 < h->nlev) {
                L.P64 = xamg::upload_csr(*h, H->P[l], false);
                L.R64 = xamg::upload_csr(*h, H->R[l], false);
            }
            if (mixed && l + 1 < h->nlev) {
                L.A32 = xamg::upload_csr(*h, a, true);
                if (padded) L.A32.rowlen = pad.rowlen, L.A32.nnz = H->A[l].nnz;
                L.P32 = xamg::upload_csr(*h, H->P[l], true);
                L.R32 = xamg::upload_csr(*h, H->R[l], true);
                if (o.index_bits == 16) {
                    L.frac16[0] = xamg::encode16(*h, a, L.A32);
                    L.frac16[1] = xamg::encode16(*h, H->P[l], L.P32);
                    L.frac16[2] = xamg::encode16(*h, H->R[l], L.R32);
                }
                std::vector<float> df(d.begin(), d.end());
                L.dinv32 = xamg::upload(*h, df.data(), df.size());
            }
            if (o.smoother != XAMG_GAUSS_SEIDEL && l + 1 < h->nlev) {
                // A D^-1 for the pre-smoothing pass from zero (which gathers
                // b_j d_j), in the precision the V-cycle runs in
                std::vector<double> vd(size_t(a.nnz));
                for (int64_t k = 0; k < a.nnz; ++k) vd[k] = a.val[k] * d[a.col[k]];
                if (mixed) {
                    std::vector<float> vf(vd.begin(), vd.end());
                    L.A32.vd = xamg::upload(*h, vf.data(), vf.size());
                } else {
                    L.A64.vd = xamg::upload(*h, vd.data(), vd.size());
                }
            }
            if (o.smoother == XAMG_GAUSS_SEIDEL && l + 1 < h->nlev) {
                // l1 diagonal of the Gauss-Seidel blocks: a_ii plus the
                // absolute couplings to rows outside the row's block
                std::vector<double> e(L.n, 0.0);
                const int B = o.gs_block;
                for (int i = 0; i < L.n; ++i) {
                    const int lo = (i / B) * B, hi = lo + B;
                    double di = 0.0;
                    for (int k = a.row_ptr[i]; k < a.row_ptr[i + 1]; ++k) {
                        const int c = a.col[k];
                        if (c == i) di += a.val[k];
                        else if (c < lo || c >= hi) di += std::fabs(a.val[k]);
                    }
                    e[i] = 1.0 / di;
                }
                L.dl1inv64 = xamg::upload(*h, e.data(), e.size());
                if (mixed) {
                    std::vector<float> ef(e.begin(), e.end());
                    L.dl1inv32 = xamg::upload(*h, ef.data(), ef.size());
                }
            }
        }
        // coarsest level inverse (FP64 LU with partial pivoting on the host)
        {
            const xamg_csr_t& a = H->A[h->nlev - 1];
            std::vector<double> dense(size_t(nL) * nL, 0.0), inv(size_t(nL) * nL);
            for (int i = 0; i < nL; ++i)
                for (int k = a.row_ptr[i]; k < a.row_ptr[i + 1]; ++k)
                    dense[size_t(i) * nL + a.col[k]] = a.val[k];
            if (xamg::dense_inverse(nL, dense.data(), inv.data()) != XAMG_OK) {
                delete h;
                return xamg::fail(XAMG_EBREAKDOWN, "singular coarsest matrix");
            }
            h->inv64 = xamg::upload(*h, inv.data(), inv.size());
            std::vector<float> invf(inv.begin(), inv.end());
            h->inv32 = xamg::upload(*h, invf.data(), invf.size());
        }
        h->st = h->alloc<xamg::dev::ColState>(1);
        h->check(hipHostMalloc(&h->st_host, sizeof(xamg::dev::ColState), hipHostMallocDefault),
                 "hipHostMalloc");
        std::memset(h->st_host, 0, sizeof(xamg::dev::ColState));
        h->check(hipMemcpy(h->st, h->st_host, sizeof(xamg::dev::ColState), hipMemcpyHostToDevice),
                 "state init");
        h->nb_cap = 2048;
        h->part = h->alloc<double>(size_t(h->nb_cap) * xamg::dev::kMaxDots * XAMG_MAX_M);
    } catch (const xamg::DevFail& f) {
        delete h;
        return f.code;
    } catch (const std::bad_alloc&) {
        delete h;
        return xamg::fail(XAMG_ENOMEM, "host allocation");
    }
    *out = static_cast<xamg_handle_t*>(h);
    return XAMG_OK;
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int xamg_solve(xamg_handle_t* hh, const double* B, double* X, int32_t m, double tol,
               xamg_stats_t* stats)
{
    xamg::clear_error();
    Handle* h = static_cast<Handle*>(hh);
    if (!h || !B || !X) return xamg::fail(XAMG_EINVAL, "null argument");
    if (m < 1 || m > XAMG_MAX_M) return xamg::fail(XAMG_EINVAL, "m must be in 1..32");
    if (!(tol > 0.0) || !std::isfinite(tol)) return xamg::fail(XAMG_EINVAL, "tol must be positive");
    if (!aligned16(B) || !aligned16(X)) return xamg::fail(XAMG_EINVAL, "B and X must be 16-byte aligned");
    try {
        int rc = xamg::solve_impl(*h, B, X, m, tol, stats);
        if (rc == XAMG_EINVAL && xamg::last_error()[0] == '\0')
            xamg::set_error("B contains NaN or Inf");
        return rc;
    } catch (const xamg::DevFail& f) {
        return f.code;
    } catch (const std::bad_alloc&) {
        return xamg::fail(XAMG_ENOMEM, "host allocation");
    }
}

int xamg_vcycle(xamg_handle_t* hh, const double* B, double* X, int32_t m)
{
    xamg::clear_error();
    Handle* h = static_cast<Handle*>(hh);
    if (!h || !B || !X) return xamg::fail(XAMG_EINVAL, "null argument");
    if (m < 1 || m > XAMG_MAX_M || (m & (m - 1)) != 0)
        return xamg::fail(XAMG_EINVAL, "m must be a power of two in 1..32");
    try {
        xamg::ensure_work(*h, m, false);
        // every column counts as active for a stand-alone cycle
        h->st_host->nactive = m;
        h->check(hipMemcpyAsync(&h->st->nactive, &h->st_host->nactive, sizeof(int),
                                hipMemcpyHostToDevice, h->stream), "state");
        xamg::dispatch_m(m, [&](auto mc) {
            constexpr int M = decltype(mc)::value;
            if (h->autotune) xamg::autotune<M>(*h);
            xamg::vcycle<M>(*h, B, X, 0, nullptr);
            return 0;
        });
        h->check(hipStreamSynchronize(h->stream), "vcycle sync");
        h->timer_collect();
    } catch (const xamg::DevFail& f) {
        return f.code;
    }
    return XAMG_OK;
}

int xamg_spmm(xamg_handle_t* hh, int32_t op, int32_t level, int32_t m, const double* X, double* Y)
{
    xamg::clear_error();
    Handle* h = static_cast<Handle*>(hh);
    if (!h || !X || !Y) return xamg::fail(XAMG_EINVAL, "null argument");
    if (level < 0 || level >= h->nlev) return xamg::fail(XAMG_EINVAL, "level");
    if (op != XAMG_OP_A && level == h->nlev - 1) return xamg::fail(XAMG_EINVAL, "no P/R on the coarsest level");
    if (m < 1 || m > XAMG_MAX_M || (m & (m - 1)) != 0)
        return xamg::fail(XAMG_EINVAL, "m must be a power of two in 1..32");
    const xamg::DCsr& d = op == XAMG_OP_A ? h->lev[level].A64
                        : op == XAMG_OP_P ? h->lev[level].P64 : h->lev[level].R64;
    try {
        xamg::dispatch_m(m, [&](auto mc) {
            constexpr int M = decltype(mc)::value;
            xamg::spmm64<M>(*h, d, X, Y);
            return 0;
        });
        h->check(hipGetLastError(), "spmm launch");
    } catch (const xamg::DevFail& f) {
        return f.code;
    }
    return XAMG_OK;
}

int xamg_info(const xamg_handle_t* hh, int64_t* out, int32_t cap)
{
    const Handle* h = static_cast<const Handle*>(hh);
    if (!h || !out) return xamg::fail(XAMG_EINVAL, "null argument");
    if (cap < 1 + 3 * h->nlev) return xamg::fail(XAMG_EINVAL, "output too short");
    out[0] = h->nlev;
    for (int l = 0; l < h->nlev; ++l) {
        out[1 + 3 * l] = h->lev[l].n;
        out[2 + 3 * l] = h->lev[l].A64.nnz;
        out[3 + 3 * l] = l + 1 < h->nlev ? h->lev[l].P64.nnz : 0;
    }
    return XAMG_OK;
}

int xamg_index16_fraction(const xamg_handle_t* hh, int32_t level, double* out)
{
    const Handle* h = static_cast<const Handle*>(hh);
    if (!h || !out) return xamg::fail(XAMG_EINVAL, "null argument");
    if (level < 0 || level >= h->nlev - 1) return xamg::fail(XAMG_EINVAL, "level");
    for (int k = 0; k < 3; ++k) out[k] = h->lev[level].frac16[k];
    return XAMG_OK;
}

int xamg_timer_enable(xamg_handle_t* hh, int32_t kind)
{
    Handle* h = static_cast<Handle*>(hh);
    if (!h) return xamg::fail(XAMG_EINVAL, "null argument");
    if (kind < XAMG_TIMER_OFF || kind > XAMG_TIMER_PRESMOOTH) return xamg::fail(XAMG_EINVAL, "timer kind");
    h->timer_kind = kind;
    h->timer_ms = 0.0;
    h->timer_count = 0;
    h->ev_used = 0;
    return XAMG_OK;
}

int xamg_timer_read(xamg_handle_t* hh, double* ms, int64_t* count)
{
    Handle* h = static_cast<Handle*>(hh);
    if (!h || !ms || !count) return xamg::fail(XAMG_EINVAL, "null argument");
    *ms = h->timer_ms;
    *count = h->timer_count;
    return XAMG_OK;
}

int xamg_autotune(xamg_handle_t* hh, int32_t m, int32_t enable)
{
    xamg::clear_error();
    Handle* h = static_cast<Handle*>(hh);
    if (!h) return xamg::fail(XAMG_EINVAL, "null argument");
    if (m < 1 || m > XAMG_MAX_M || (m & (m - 1)) != 0)
        return xamg::fail(XAMG_EINVAL, "m must be a power of two in 1..32");
    h->autotune = enable ? 1 : 0;
    if (!enable) return XAMG_OK;
    try {
        xamg::ensure_work(*h, m, xamg::bicg_like(h->opt));
        int k = 0;
        while ((1 << k) < m) ++k;
        h->tuned_mask &= ~(1u << k);
        h->tune_fresh = true;   // a request times afresh and replaces cached choices
        try {
            xamg::dispatch_m(m, [&](auto mc) {
                xamg::autotune<decltype(mc)::value>(*h);
                return 0;
            });
        } catch (...) {
            h->tune_fresh = false;
            throw;
        }
        h->tune_fresh = false;
    } catch (const xamg::DevFail& f) {
        return f.code;
    }
    return XAMG_OK;
}

int xamg_tuning(const xamg_handle_t* hh, int32_t m, int32_t* out, int32_t cap)
{
    const Handle* h = static_cast<const Handle*>(hh);
    if (!h || !out) return xamg::fail(XAMG_EINVAL, "null argument");
    if (m < 1 || m > XAMG_MAX_M || (m & (m - 1)) != 0)
        return xamg::fail(XAMG_EINVAL, "m must be a power of two in 1..32");
    if (cap < 4 * h->nlev + 1) return xamg::fail(XAMG_EINVAL, "output too short");
    int k = 0;
    while ((1 << k) < m) ++k;
    const bool mixed = h->opt.precision == XAMG_MIXED;
    for (int l = 0; l < h->nlev; ++l) {
        const auto& L = h->lev[l];
        const bool last = l + 1 == h->nlev;
        const xamg::DCsr& A = (mixed && !last) ? L.A32 : L.A64;
        out[4 * l] = A.split[k];
        out[4 * l + 1] = last ? 0 : A.split_pre[k];
        out[4 * l + 2] = last ? 0 : (mixed ? L.P32 : L.P64).split[k];
        out[4 * l + 3] = last ? 0 : (mixed ? L.R32 : L.R64).split[k];
    }
    out[4 * h->nlev] = h->lev[0].A64.split[k];   // the Krylov operator (FP64 A_0)
    return XAMG_OK;
}

int xamg_set_tuning(xamg_handle_t* hh, int32_t m, const int32_t* in, int32_t count)
{
    xamg::clear_error();
    Handle* h = static_cast<Handle*>(hh);
    if (!h || !in) return xamg::fail(XAMG_EINVAL, "null argument");
    if (m < 1 || m > XAMG_MAX_M || (m & (m - 1)) != 0)
        return xamg::fail(XAMG_EINVAL, "m must be a power of two in 1..32");
    if (count < 4 * h->nlev + 1) return xamg::fail(XAMG_EINVAL, "input too short");
    const int flags = xamg::kShapeFlags;
    const auto valid = [flags](int v) {
        const int s = v & 15;
        return (v & ~(flags | 15)) == 0 && (s == 1 || s == 2 || s == 4 || s == 8);
    };
    for (int l = 0; l < h->nlev; ++l) {
        const bool last = l + 1 == h->nlev;
        for (int e = 0; e < (last ? 1 : 4); ++e)
            if (!valid(in[4 * l + e])) {
                xamg::set_error("split %d (level %d, entry %d) is not 1, 2, 4 or 8 plus flags "
                                "16, 32, 64, 128, 256, 512", in[4 * l + e], l, e);
                return XAMG_EINVAL;
            }
    }
    if (!valid(in[4 * h->nlev])) {
        xamg::set_error("split %d of the Krylov operator is not 1, 2, 4 or 8 plus flags",
                        in[4 * h->nlev]);
        return XAMG_EINVAL;
    }
    int k = 0;
    while ((1 << k) < m) ++k;
    for (int l = 0; l < h->nlev; ++l) {
        auto& L = h->lev[l];
        const bool last = l + 1 == h->nlev;
        for (xamg::DCsr* A : {&L.A64, &L.A32}) {
            A->split[k] = in[4 * l];
            if (!last) A->split_pre[k] = in[4 * l + 1];
        }
        if (last) continue;
        L.P64.split[k] = L.P32.split[k] = in[4 * l + 2];
        L.R64.split[k] = L.R32.split[k] = in[4 * l + 3];
    }
    h->lev[0].A64.split[k] = in[4 * h->nlev];
    h->tuned_mask |= 1u << k;
    h->tune_epoch += 1;
    return XAMG_OK;
}

int xamg_destroy(xamg_handle_t* hh)
{
    Handle* h = static_cast<Handle*>(hh);
    if (!h) return XAMG_OK;
    if (h->stream) hipStreamSynchronize(h->stream);
    else hipDeviceSynchronize();
    delete h;
    return XAMG_OK;
}

}  // extern "C"
