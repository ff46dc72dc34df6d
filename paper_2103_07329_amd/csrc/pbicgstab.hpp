// pbicgstab.hpp -- pipelined BiCGStab (Cools and Vanroose 2017; the paper's
// Section 2.1 lists it), right-preconditioned, for m interleaved columns
// with one set of scalars per column.
//
// BiCGStab on K = A M (M the V-cycle) with the auxiliary vectors
// s = K p, z = K s, v = K z, w = K r, t = K w, q = r - alpha s, y = K q, so
// that neither product with K in an iteration waits for a dot product:
//   pass A:  p = r + beta (p - omega s),  s = w + beta (s - omega z),
//            z = t + beta (z - omega v),  ph = rt + beta (ph - omega sh),
//            sh = wh + beta (sh - omega zh),  q = r - alpha s,  y = w - alpha z,
//            qh = rt - alpha sh;  dots (q,q), (q,y), (y,y), (rh,s), (rh,z)
//   omega = (q,y)/(y,y); a column with ||q|| <= tol ||b|| stops at the half step
//   zh = M z, v = A zh
//   pass B:  x += alpha ph + omega qh,  r = q - omega y,
//            w = y - omega (t - alpha v),  rt = qh - omega (wh - alpha zh)
//            (half step: x += alpha ph, r = q);  dots (rh,r), (rh,w), (r,r)
//   wh = M w, t = A wh
//   beta' = (alpha/omega) (rh,r)/rho,  alpha' = (rh,r) / ((rh,w) + beta' (rh,s)
//            - beta' omega (rh,z)),  rho = (rh,r).
// rt = M r, wh = M w, zh = M z, ph = M p, sh = M s, qh = M q: x follows the
// M-images, which the V-cycle of each product with K already supplies for z
// and w.  Start, and restart of a column from its iterate: rh = r, rt = M r,
// w = A rt, wh = M w, t = A wh, alpha = (rh,r)/(rh,w), beta = 0.  A
// breakdown (|(rh,r)| or the denominator of alpha <= 1e-300 ||b||^2, or
// omega = 0) stops the column.  On one GPU the products do not overlap the
// reductions (each is one finalize kernel); the form's value is across GPUs.
#pragma once

#include "bicgstab.hpp"

namespace xamg {

using namespace dev;

namespace pbicg {

// per-column coefficients of the pipelined passes, loaded once per thread
template <int CPT>
struct PbCoef {
    double al[CPT] = {}, be[CPT] = {}, om[CPT] = {};
    int ac[CPT] = {}, hf[CPT] = {};
    __device__ __forceinline__ void load(const ColState* st, int j0)
    {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int j = j0 + c;
            ac[c] = st->active[j];
            hf[c] = st->half[j];
            al[c] = st->alpha[j];
            be[c] = st->beta[j];
            om[c] = st->omega[j];
        }
    }
};

// pass A (see the header); dots (q,q), (q,y), (y,y), (rh,s), (rh,z)
template <int M, int CPT>
struct OpPbA {
    using AT = double;
    static constexpr bool kMatrix = false;
    static constexpr int kDots = 5;
    const int* rp = nullptr;
    const double* val = nullptr;
    Idx32 idx{nullptr};
    const ColState* st;
    const double *r, *w, *t, *rt, *wh, *v, *zh, *rh;
    double *p, *s, *z, *ph, *sh, *q, *y, *qh;
    __device__ __forceinline__ bool active_any() const { return st->nactive > 0; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int, int) const { return Pack<AT, CPT>{}; }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&)[CPT], double (&d)[ND][CPT]) const
    {
        const size_t o = size_t(i) * M + j0;
        auto pi = load_pack<double, CPT>(p + o);
        auto si = load_pack<double, CPT>(s + o);
        auto zi = load_pack<double, CPT>(z + o);
        auto phi = load_pack<double, CPT>(ph + o);
        auto shi = load_pack<double, CPT>(sh + o);
        const auto ri = load_pack<double, CPT>(r + o);
        const auto wi = load_pack<double, CPT>(w + o);
        const auto ti = load_pack<double, CPT>(t + o);
        const auto rti = load_pack<double, CPT>(rt + o);
        const auto whi = load_pack<double, CPT>(wh + o);
        const auto vi = load_pack<double, CPT>(v + o);
        const auto zhi = load_pack<double, CPT>(zh + o);
        const auto hi = load_pack<double, CPT>(rh + o);
        Pack<double, CPT> qo, yo, qho;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            if (cf_.ac[c]) {
                const double b = cf_.be[c], w0 = cf_.om[c], a = cf_.al[c];
                const double po = pi.v[c], so = si.v[c], zo = zi.v[c];
                const double pho = phi.v[c], sho = shi.v[c];
                pi.v[c] = ri.v[c] + b * (po - w0 * so);
                si.v[c] = wi.v[c] + b * (so - w0 * zo);
                zi.v[c] = ti.v[c] + b * (zo - w0 * vi.v[c]);
                phi.v[c] = rti.v[c] + b * (pho - w0 * sho);
                shi.v[c] = whi.v[c] + b * (sho - w0 * zhi.v[c]);
                qo.v[c] = ri.v[c] - a * si.v[c];
                yo.v[c] = wi.v[c] - a * zi.v[c];
                qho.v[c] = rti.v[c] - a * shi.v[c];
            } else {
                qo.v[c] = yo.v[c] = qho.v[c] = 0.0;
            }
            d[0][c] += qo.v[c] * qo.v[c];
            d[1][c] += qo.v[c] * yo.v[c];
            d[2][c] += yo.v[c] * yo.v[c];
            d[3][c] += hi.v[c] * si.v[c];
            d[4][c] += hi.v[c] * zi.v[c];
        }
        store_pack<double, CPT>(p + o, pi);
        store_pack<double, CPT>(s + o, si);
        store_pack<double, CPT>(z + o, zi);
        store_pack<double, CPT>(ph + o, phi);
        store_pack<double, CPT>(sh + o, shi);
        store_pack<double, CPT>(q + o, qo);
        store_pack<double, CPT>(y + o, yo);
        store_pack<double, CPT>(qh + o, qho);
    }
    static constexpr bool kBegin = true;
    PbCoef<CPT> cf_;
    __device__ __forceinline__ void begin(int j0) { cf_.load(st, j0); }
};

// pass B (see the header); dots (rh,r), (rh,w), (r,r)
template <int M, int CPT>
struct OpPbB {
    using AT = double;
    static constexpr bool kMatrix = false;
    static constexpr int kDots = 3;
    const int* rp = nullptr;
    const double* val = nullptr;
    Idx32 idx{nullptr};
    const ColState* st;
    double *x, *r, *w, *rt;
    const double *ph, *qh, *q, *y, *t, *v, *wh, *zh, *rh;
    __device__ __forceinline__ bool active_any() const { return st->nactive > 0; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int, int) const { return Pack<AT, CPT>{}; }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&)[CPT], double (&d)[ND][CPT]) const
    {
        const size_t o = size_t(i) * M + j0;
        auto xi = load_pack<double, CPT>(x + o);
        auto ri = load_pack<double, CPT>(r + o);
        auto wi = load_pack<double, CPT>(w + o);
        auto rti = load_pack<double, CPT>(rt + o);
        const auto phi = load_pack<double, CPT>(ph + o);
        const auto qhi = load_pack<double, CPT>(qh + o);
        const auto qi = load_pack<double, CPT>(q + o);
        const auto yi = load_pack<double, CPT>(y + o);
        const auto ti = load_pack<double, CPT>(t + o);
        const auto vi = load_pack<double, CPT>(v + o);
        const auto whi = load_pack<double, CPT>(wh + o);
        const auto zhi = load_pack<double, CPT>(zh + o);
        const auto hi = load_pack<double, CPT>(rh + o);
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            if (cf_.ac[c]) {
                const double a = cf_.al[c], w0 = cf_.om[c];
                if (cf_.hf[c]) {
                    xi.v[c] += a * phi.v[c];
                    ri.v[c] = qi.v[c];
                } else {
                    xi.v[c] += a * phi.v[c] + w0 * qhi.v[c];
                    ri.v[c] = qi.v[c] - w0 * yi.v[c];
                    wi.v[c] = yi.v[c] - w0 * (ti.v[c] - a * vi.v[c]);
                    rti.v[c] = qhi.v[c] - w0 * (whi.v[c] - a * zhi.v[c]);
                }
            }
            d[0][c] += hi.v[c] * ri.v[c];
            d[1][c] += hi.v[c] * wi.v[c];
            d[2][c] += ri.v[c] * ri.v[c];
        }
        store_pack<double, CPT>(x + o, xi);
        store_pack<double, CPT>(r + o, ri);
        store_pack<double, CPT>(w + o, wi);
        store_pack<double, CPT>(rt + o, rti);
    }
    static constexpr bool kBegin = true;
    PbCoef<CPT> cf_;
    __device__ __forceinline__ void begin(int j0) { cf_.load(st, j0); }
};

// start or restart: on the columns with rst set, rh = r and the recurrence
// vectors zero (beta = 0 then makes p = r, s = w, z = t, ph = rt, sh = wh)
template <int M, int CPT>
struct OpPbSeed {
    using AT = double;
    static constexpr bool kMatrix = false;
    static constexpr int kDots = 0;
    const int* rp = nullptr;
    const double* val = nullptr;
    Idx32 idx{nullptr};
    const ColState* st;
    const double* r;
    double *rh, *p, *s, *z, *v, *ph, *sh, *zh;
    __device__ __forceinline__ bool active_any() const { return true; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int, int) const { return Pack<AT, CPT>{}; }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&)[CPT], double (&)[ND][CPT]) const
    {
        bool any = false;
#pragma unroll
        for (int c = 0; c < CPT; ++c) any |= rs_[c] != 0;
        if (!any) return;
        const size_t o = size_t(i) * M + j0;
        const auto ri = load_pack<double, CPT>(r + o);
        auto hi = load_pack<double, CPT>(rh + o);
#pragma unroll
        for (int c = 0; c < CPT; ++c)
            if (rs_[c]) hi.v[c] = ri.v[c];
        store_pack<double, CPT>(rh + o, hi);
        double* const us[7] = {p, s, z, v, ph, sh, zh};
        for (int k = 0; k < 7; ++k) {
            auto ui = load_pack<double, CPT>(us[k] + o);
#pragma unroll
            for (int c = 0; c < CPT; ++c)
                if (rs_[c]) ui.v[c] = 0.0;
            store_pack<double, CPT>(us[k] + o, ui);
        }
    }
    static constexpr bool kBegin = true;
    int rs_[CPT] = {};
    __device__ __forceinline__ void begin(int j0)
    {
#pragma unroll
        for (int c = 0; c < CPT; ++c) rs_[c] = st->rst[j0 + c] && st->active[j0 + c];
    }
};

// dots (rh, r), (rh, w) of a (re)start
template <int M, int CPT>
struct OpPbStartDots {
    using AT = double;
    static constexpr bool kMatrix = false;
    static constexpr int kDots = 2;
    const int* rp = nullptr;
    const double* val = nullptr;
    Idx32 idx{nullptr};
    const double *rh, *r, *w;
    __device__ __forceinline__ bool active_any() const { return true; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int, int) const { return Pack<AT, CPT>{}; }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&)[CPT], double (&d)[ND][CPT]) const
    {
        const size_t o = size_t(i) * M + j0;
        const auto hi = load_pack<double, CPT>(rh + o);
        const auto ri = load_pack<double, CPT>(r + o);
        const auto wi = load_pack<double, CPT>(w + o);
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            d[0][c] += hi.v[c] * ri.v[c];
            d[1][c] += hi.v[c] * wi.v[c];
        }
    }
};

__device__ __forceinline__ void stop(ColState* st, int j)
{
    st->active[j] = 0;
    st->failed[j] = 1;
}

struct FinPbStart {   // tot: (rh, r)[M], (rh, w)[M]; the columns with rst set
    ColState* st;
    int M;
    __device__ void operator()(const double* tot) const
    {
        const int j = threadIdx.x;
        if (j < M && st->rst[j]) {
            st->rst[j] = 0;
            if (st->active[j]) {
                const double rr = tot[j], rw = tot[M + j];
                const double tiny = 1e-300 * st->bn2[j];
                if (fabs(rr) <= tiny || fabs(rw) <= tiny) {
                    stop(st, j);
                } else {
                    st->rz[j] = rr;
                    st->alpha[j] = rr / rw;
                    st->beta[j] = 0.0;
                    st->omega[j] = 1.0;
                }
            }
        }
        recount_active(st, M);
    }
};

struct FinPbA {   // tot: (q,q), (q,y), (y,y), (rh,s), (rh,z), each [M]
    ColState* st;
    int M;
    __device__ void operator()(const double* tot) const
    {
        const int j = threadIdx.x;
        if (j < M && st->active[j]) {
            st->iters[j] += 1;
            st->rhs[j] = tot[3 * M + j];
            st->rhz[j] = tot[4 * M + j];
            st->half[j] = sqrt(tot[j]) / sqrt(st->bn2[j]) <= st->tol;
            if (!st->half[j]) {
                const double qy = tot[M + j], yy = tot[2 * M + j];
                const double w = yy > 0.0 ? qy / yy : 0.0;
                st->omega[j] = w;
                if (w == 0.0) stop(st, j);
            }
        }
        recount_active(st, M);
    }
};

struct FinPbB {   // tot: (rh,r), (rh,w), (r,r), each [M]
    ColState* st;
    int M;
    __device__ void operator()(const double* tot) const
    {
        const int j = threadIdx.x;
        if (j < M && st->active[j]) {
            const double rhr = tot[j], rhw = tot[M + j], rr = tot[2 * M + j];
            st->rr[j] = rr;
            const double rel = sqrt(rr) / sqrt(st->bn2[j]);
            st->relres[j] = rel;
            if (st->half[j] || rel <= st->tol) {
                st->active[j] = 0;
                st->conv[j] = 1;
                st->half[j] = 0;
            } else {
                const double tiny = 1e-300 * st->bn2[j];
                const double a = st->alpha[j], w = st->omega[j];
                const double b = (a / w) * (rhr / st->rz[j]);
                const double del = rhw + b * st->rhs[j] - b * w * st->rhz[j];
                if (fabs(rhr) <= tiny || fabs(del) <= tiny) {
                    stop(st, j);
                } else {
                    st->beta[j] = b;
                    st->alpha[j] = rhr / del;
                    st->rz[j] = rhr;
                }
            }
        }
        recount_active(st, M);
    }
};

// the columns a true-residual check restarted (cp) start again from r = t
struct FinPbRestart {
    ColState* st;
    int M;
    __device__ void operator()(const double*) const
    {
        const int j = threadIdx.x;
        if (j < M && st->cp[j]) st->rst[j] = 1;
    }
};

}  // namespace pbicg

// rh = r, rt = M r, w = A rt, wh = M w, t = A wh and the scalars, on the
// columns with rst set (the products run over every column: the others are
// fresh at the start, and inactive at a restart)
template <int M>
void pb_start(Handle& h)
{
    using namespace pbicg;
    constexpr int CPT = cpt_for<double, M>();
    const int n = h.lev[0].n;
    const DCsr& A = h.lev[0].A64;
    const double* av = static_cast<const double*>(A.v);
    auto& w = h.w;
    const int cap = h.nb_cap;
    const int* na = &h.st->nactive;
    OpPbSeed<M, CPT> seed{nullptr, nullptr, Idx32{nullptr}, h.st, w.r,
                          w.rh,    w.p,     w.s,           w.z,  w.v,
                          w.ph,    w.sh,    w.zh};
    launch_rows<M, CPT>(h, seed, n, cap);
    auto product = [&](const double* in, double* mid, double* out) {
        apply_prec<M>(h, in, mid, 0, nullptr);
        launch_op<M, double, double>(h, A, A.template split_of<M>(), n, cap, [&](auto cpt, auto ix) {
            return OpAx<M, decltype(cpt)::value, double, double, decltype(ix), 0>{A.rp, av, ix, mid,
                                                                                  out, na};
        });
    };
    product(w.r, w.rt, w.pw);    // rt = M r, w = A rt
    product(w.pw, w.wh, w.t);    // wh = M w, t = A wh
    OpPbStartDots<M, CPT> dots{nullptr, nullptr, Idx32{nullptr}, w.rh, w.r, w.pw};
    const int nb = launch_rows<M, CPT>(h, dots, n, cap);
    launch_fin(h, nb, 2 * M, FinPbStart{h.st, M});
}

template <int M>
int pbicgstab(Handle& h, const double* B, double* X, double tol)
{
    using namespace pbicg;
    constexpr int CPT = cpt_for<double, M>();
    const int n = h.lev[0].n;
    const DCsr& A = h.lev[0].A64;
    const double* av = static_cast<const double*>(A.v);
    auto& w = h.w;
    ColState* st = h.st;
    const int cap = h.nb_cap;
    const int* na = &st->nactive;

    if (h.opt.x0_mode == XAMG_X0_ZERO)
        hipLaunchKernelGGL((copy_cols_kernel<double, double>), dim3(1024), dim3(256), 0, h.stream,
                           nullptr, M, X, M, n, 0);
    {
        const int nb = launch_op<M, double, double>(
            h, A, A.template split_of<M>(), n, cap, [&](auto cpt, auto ix) {
                return OpResid<M, decltype(cpt)::value, double, double, double, decltype(ix), 2>{
                    A.rp, av, ix, X, B, w.r, nullptr};
            });
        // the CG start: column state, rst = 1 on every column (the pipelined
        // start below consumes it)
        launch_fin(h, nb, 2 * M, FinInit{st, tol, M, h.opt.max_iters});
    }
    if (h.opt.x0_mode == XAMG_X0_GIVEN) {
        OpFixCols<M, CPT> op{nullptr, nullptr, Idx32{nullptr}, st, nullptr, nullptr, X};
        launch_rows<M, CPT>(h, op, n, cap);
    }
    // every recurrence vector finite before its first (masked) update
    for (double* u : {w.p, w.s, w.z, w.v, w.ph, w.sh, w.zh, w.q, w.y, w.qh, w.rt, w.pw, w.wh, w.t})
        hipLaunchKernelGGL((copy_cols_kernel<double, double>), dim3(1024), dim3(256), 0, h.stream,
                           nullptr, M, u, M, n, 0);
    poll_state(h);
    if (h.st_host->nrestart < 0) return XAMG_EINVAL;
    pb_start<M>(h);
    poll_state(h);

    int it = 0;
    PollPlan plan{h.opt.check_every};
    int next = plan.next_after(0, h.st_host->worst, tol);
    for (;;) {
        if (h.st_host->nactive == 0 || it >= h.opt.max_iters) {
            const int nb = launch_op<M, double, double>(
                h, A, A.template split_of<M>(), n, cap, [&](auto cpt, auto ix) {
                    return OpResid<M, decltype(cpt)::value, double, double, double, decltype(ix),
                                   2>{A.rp, av, ix, X, B, w.t, nullptr};
                });
            launch_fin(h, nb, 2 * M, FinTrueB{st, M, it < h.opt.max_iters ? 1 : 0});
            sync_state(h);
            if (h.st_host->nrestart == 0 || it >= h.opt.max_iters) break;
            // restarted columns: r = b - A x (in t), then the start sequence
            OpFixCols<M, CPT> cp{nullptr, nullptr, Idx32{nullptr}, st, w.r, w.t, nullptr};
            launch_rows<M, CPT>(h, cp, n, cap);
            launch_fin(h, 0, 0, FinPbRestart{st, M});
            pb_start<M>(h);
            poll_state(h);
            plan = PollPlan{h.opt.check_every};
            next = plan.next_after(it, h.st_host->worst, tol);
            continue;
        }
        ++it;
        {
            OpPbA<M, CPT> op{nullptr, nullptr, Idx32{nullptr}, st, w.r, w.pw, w.t, w.rt, w.wh, w.v,
                             w.zh, w.rh, w.p, w.s, w.z, w.ph, w.sh, w.q, w.y, w.qh};
            const int nb = launch_rows<M, CPT>(h, op, n, cap);
            launch_fin(h, nb, 5 * M, FinPbA{st, M});
        }
        // v = K z
        apply_prec<M>(h, w.z, w.zh, 0, nullptr);
        launch_op<M, double, double>(h, A, A.template split_of<M>(), n, cap, [&](auto cpt, auto ix) {
            return OpAx<M, decltype(cpt)::value, double, double, decltype(ix), 0>{A.rp, av, ix, w.zh,
                                                                                  w.v, na};
        });
        {
            OpPbB<M, CPT> op{nullptr, nullptr, Idx32{nullptr}, st, X, w.r, w.pw, w.rt, w.ph, w.qh,
                             w.q, w.y, w.t, w.v, w.wh, w.zh, w.rh};
            const int nb = launch_rows<M, CPT>(h, op, n, cap);
            launch_fin(h, nb, 3 * M, FinPbB{st, M});
        }
        // t = K w (skipped once every column has stopped)
        apply_prec<M>(h, w.pw, w.wh, 0, nullptr);
        launch_op<M, double, double>(h, A, A.template split_of<M>(), n, cap, [&](auto cpt, auto ix) {
            return OpAx<M, decltype(cpt)::value, double, double, decltype(ix), 0>{A.rp, av, ix, w.wh,
                                                                                  w.t, na};
        });
        if (it >= next || it >= h.opt.max_iters) {
            poll_state(h);
            next = plan.next_after(it, h.st_host->worst, tol);
        }
    }
    return XAMG_OK;
}

}  // namespace xamg
