// bicgstab.hpp -- right-preconditioned BiCGStab (van der Vorst 1992; the
// paper's Section 2.1 lists BiCGStab among its Krylov solvers) for m
// interleaved columns with one set of scalars per column:
//
//   r = b - A x, rh = r, rho = alpha = omega = 1, v = p = 0;
//   loop: rho' = (rh, r); beta = (rho'/rho)(alpha/omega);
//         p = r + beta (p - omega v); ph = M p; v = A ph;
//         alpha = rho' / (rh, v); s = r - alpha v;
//         if ||s||/||b|| <= tol: x += alpha ph, stop;
//         sh = M s; t = A sh; omega = (t, s)/(t, t);
//         x += alpha ph + omega sh; r = s - omega t; rho = rho'.
//
// A breakdown (|rho'| or |(rh, v)| <= 1e-300 ||b||^2, or omega = 0)
// restarts the column with rh = r, rho = alpha = omega = 1, p = v = 0; two
// breakdowns in a row stop it (reported as XAMG_EBREAKDOWN).  The scalar
// recurrences run in one-block finalize kernels on the device; every
// vector operation is a fused row pass (ops.hpp / below).
#pragma once

#include "cycle.hpp"

namespace xamg {

using namespace dev;

namespace bicg {

// y = A x with dots of y against w (and against y)
template <int M, int CPT, typename MT, class IdxT, int KIND>
struct OpAxW {   // KIND 1: (w, y); KIND 2: (w, y), (y, y)
    using AT = MT;
    static constexpr bool kMatrix = true;
    static constexpr int kDots = KIND;
    const int* rp;
    const MT* val;
    IdxT idx;
    const double* x;
    double* y;
    const double* w;
    const int* nactive;
    __device__ __forceinline__ bool active_any() const { return *nactive > 0; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int c, int j0) const
    {
        const auto v = load_pack<double, CPT>(x + size_t(c) * M + j0);
        Pack<AT, CPT> r;
#pragma unroll
        for (int t = 0; t < CPT; ++t) r.v[t] = AT(v.v[t]);
        return r;
    }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&acc)[CPT], double (&d)[ND][CPT]) const
    {
        const size_t o = size_t(i) * M + j0;
        Pack<double, CPT> yo;
#pragma unroll
        for (int t = 0; t < CPT; ++t) yo.v[t] = double(acc[t]);
        store_pack<double, CPT>(y + o, yo);
        const auto wi = load_pack<double, CPT>(w + o);
#pragma unroll
        for (int t = 0; t < CPT; ++t) {
            d[0][t] += wi.v[t] * yo.v[t];
            if constexpr (KIND == 2) d[1][t] += yo.v[t] * yo.v[t];
        }
    }
    // > 0: every row holds exactly rowlen entries, row i at i * rowlen (no row
    // pointers are read); 0: CSR row pointers
    int rowlen = 0;
};

// p = r + beta (p - omega v); on a reset column: rh = r, p = r, v = 0
template <int M, int CPT>
struct OpBicgP {
    using AT = double;
    static constexpr bool kMatrix = false;
    static constexpr int kDots = 0;
    const int* rp = nullptr;
    const double* val = nullptr;
    Idx32 idx{nullptr};
    const ColState* st;
    const double* r;
    double *p, *v, *rh;
    float* p32 = nullptr;   // optional FP32 copy of p (input of a mixed V-cycle)
    __device__ __forceinline__ bool active_any() const { return st->nactive > 0; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int, int) const { return Pack<AT, CPT>{}; }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&)[CPT], double (&)[ND][CPT]) const
    {
        const size_t o = size_t(i) * M + j0;
        const auto ri = load_pack<double, CPT>(r + o);
        auto pi = load_pack<double, CPT>(p + o);
        auto vi = load_pack<double, CPT>(v + o);
        auto hi = load_pack<double, CPT>(rh + o);
        bool reset = false;
#pragma unroll
        for (int t = 0; t < CPT; ++t) {
            if (!ac_[t]) continue;
            if (pz_[t]) {
                hi.v[t] = ri.v[t];
                pi.v[t] = ri.v[t];
                vi.v[t] = 0.0;
                reset = true;
            } else {
                pi.v[t] = ri.v[t] + be_[t] * (pi.v[t] - om_[t] * vi.v[t]);
            }
        }
        store_pack<double, CPT>(p + o, pi);
        if (p32) {
            Pack<float, CPT> pf;
#pragma unroll
            for (int t = 0; t < CPT; ++t) pf.v[t] = float(pi.v[t]);
            store_pack<float, CPT>(p32 + o, pf);
        }
        if (reset) {
            store_pack<double, CPT>(v + o, vi);
            store_pack<double, CPT>(rh + o, hi);
        }
    }
    // the lane's columns' coefficients and flags, loaded once per thread
    static constexpr bool kBegin = true;
    double be_[CPT] = {}, om_[CPT] = {};
    int ac_[CPT] = {}, pz_[CPT] = {};
    __device__ __forceinline__ void begin(int j0)
    {
#pragma unroll
        for (int t = 0; t < CPT; ++t) {
            ac_[t] = st->active[j0 + t];
            pz_[t] = st->pz[j0 + t];
            be_[t] = st->beta[j0 + t];
            om_[t] = st->omega[j0 + t];
        }
    }
};

// s = r - alpha v; dot (s, s)
template <int M, int CPT>
struct OpBicgS {
    using AT = double;
    static constexpr bool kMatrix = false;
    static constexpr int kDots = 1;
    const int* rp = nullptr;
    const double* val = nullptr;
    Idx32 idx{nullptr};
    const ColState* st;
    const double *r, *v;
    double* s;
    float* s32 = nullptr;   // optional FP32 copy of s (input of a mixed V-cycle)
    __device__ __forceinline__ bool active_any() const { return st->nactive > 0; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int, int) const { return Pack<AT, CPT>{}; }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&)[CPT], double (&d)[ND][CPT]) const
    {
        const size_t o = size_t(i) * M + j0;
        const auto ri = load_pack<double, CPT>(r + o);
        const auto vi = load_pack<double, CPT>(v + o);
        Pack<double, CPT> so;
#pragma unroll
        for (int t = 0; t < CPT; ++t) {
            so.v[t] = ri.v[t] - al_[t] * vi.v[t];
            d[0][t] += so.v[t] * so.v[t];
        }
        store_pack<double, CPT>(s + o, so);
        if (s32) {
            Pack<float, CPT> sf;
#pragma unroll
            for (int t = 0; t < CPT; ++t) sf.v[t] = float(so.v[t]);
            store_pack<float, CPT>(s32 + o, sf);
        }
    }
    static constexpr bool kBegin = true;
    double al_[CPT] = {};
    __device__ __forceinline__ void begin(int j0)
    {
#pragma unroll
        for (int t = 0; t < CPT; ++t) al_[t] = st->alpha[j0 + t];
    }
};

// x += alpha ph + omega sh; r = s - omega t (active columns);
// dots (rh, r) and (r, r)
template <int M, int CPT>
struct OpBicgXR {
    using AT = double;
    static constexpr bool kMatrix = false;
    static constexpr int kDots = 2;
    const int* rp = nullptr;
    const double* val = nullptr;
    Idx32 idx{nullptr};
    const ColState* st;
    double *x, *r;
    const double *ph, *sh, *s, *t, *rh;
    __device__ __forceinline__ bool active_any() const { return st->nactive > 0; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int, int) const { return Pack<AT, CPT>{}; }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&)[CPT], double (&d)[ND][CPT]) const
    {
        const size_t o = size_t(i) * M + j0;
        auto xi = load_pack<double, CPT>(x + o);
        auto ri = load_pack<double, CPT>(r + o);
        const auto pi = load_pack<double, CPT>(ph + o);
        const auto qi = load_pack<double, CPT>(sh + o);
        const auto si = load_pack<double, CPT>(s + o);
        const auto ti = load_pack<double, CPT>(t + o);
        const auto hi = load_pack<double, CPT>(rh + o);
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            if (go_[c]) {
                xi.v[c] += al_[c] * pi.v[c] + om_[c] * qi.v[c];
                ri.v[c] = si.v[c] - om_[c] * ti.v[c];
            }
            d[0][c] += hi.v[c] * ri.v[c];
            d[1][c] += ri.v[c] * ri.v[c];
        }
        store_pack<double, CPT>(x + o, xi);
        store_pack<double, CPT>(r + o, ri);
    }
    static constexpr bool kBegin = true;
    double al_[CPT] = {}, om_[CPT] = {};
    int go_[CPT] = {};
    __device__ __forceinline__ void begin(int j0)
    {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int j = j0 + c;
            go_[c] = st->active[j] && !st->skip[j];
            al_[c] = st->alpha[j];
            om_[c] = st->omega[j];
        }
    }
};

// ---- scalar steps (one block) ----------------------------------------------
__device__ __forceinline__ double tiny_of(const ColState* st, int j)
{
    return 1e-300 * st->bn2[j];
}

// Prepare column j for the next iteration from rho' = (rh, r):
// beta and rho, or a restart (p = r, rh = r, v = 0) when one is pending or
// rho' breaks down; a second breakdown in a row stops the column.
__device__ __forceinline__ void prep_next(ColState* st, int j, double rhr, double rr)
{
    if (!st->active[j]) return;
    st->pz[j] = 0;
    if (!st->rst[j] && fabs(rhr) <= tiny_of(st, j)) {
        if (++st->brk[j] >= 2) {
            st->active[j] = 0;
            st->failed[j] = 1;
            return;
        }
        st->rst[j] = 1;
        st->nrst[j] += 1;
    }
    if (st->rst[j]) {
        // rh := r, rho = alpha = omega = 1: rho' = (r, r), beta = rho', p = r
        st->rst[j] = 0;
        st->pz[j] = 1;
        st->alpha[j] = st->omega[j] = 1.0;
        st->rz[j] = rr;
        st->beta[j] = 0.0;
        return;
    }
    st->beta[j] = (rhr / st->rz[j]) * (st->alpha[j] / st->omega[j]);
    st->rz[j] = rhr;
}

struct FinInitB {   // tot: (b,b)[M], (r,r)[M]
    ColState* st;
    double tol;
    int M;
    __device__ void operator()(const double* tot) const
    {
        const int j = threadIdx.x;
        if (j < M) {
            const double bb = tot[j], rr = tot[M + j];
            st->bn2[j] = bb;
            st->rr[j] = rr;
            const double rel = bb > 0.0 ? sqrt(rr) / sqrt(bb) : 0.0;
            st->relres[j] = rel;
            st->true_relres[j] = rel;
            const int act = (bb > 0.0) && !(rel <= tol);
            st->active[j] = act;
            st->conv[j] = !act;
            st->iters[j] = 0;
            st->brk[j] = st->skip[j] = st->half[j] = st->failed[j] = st->cp[j] = 0;
            st->nrst[j] = 0;
            st->rst[j] = 1;   // first iteration: rh = r, p = r, v = 0
            st->alpha[j] = st->omega[j] = st->rz[j] = 1.0;
            st->beta[j] = 0.0;
            prep_next(st, j, rr, rr);
        }
        if (j == 0) {
            st->tol = tol;
            st->max_iters = 1 << 30;   // the host loop enforces the cap
            int bad = 0;
            for (int q = 0; q < M; ++q) bad |= !isfinite(tot[q]);
            st->nrestart = bad ? -1 : 0;
        }
        recount_active(st, M);
    }
};

struct FinAlphaB {   // tot: (rh, v)[M]
    ColState* st;
    int M;
    __device__ void operator()(const double* tot) const
    {
        const int j = threadIdx.x;
        if (j < M) {
            st->skip[j] = 0;
            st->half[j] = 0;
            if (st->active[j]) {
                st->iters[j] += 1;
                const double rv = tot[j];
                if (fabs(rv) <= tiny_of(st, j)) {
                    if (++st->brk[j] >= 2) {
                        st->active[j] = 0;
                        st->failed[j] = 1;
                    } else {
                        st->rst[j] = 1;
                        st->skip[j] = 1;
                        st->nrst[j] += 1;
                    }
                    st->alpha[j] = 0.0;
                } else {
                    st->alpha[j] = st->rz[j] / rv;
                }
            } else {
                st->alpha[j] = 0.0;
            }
        }
        recount_active(st, M);
    }
};

struct FinHalf {   // tot: (s, s)[M]
    ColState* st;
    int M;
    __device__ void operator()(const double* tot) const
    {
        const int j = threadIdx.x;
        if (j < M && st->active[j] && !st->skip[j])
            st->half[j] = sqrt(tot[j]) / sqrt(st->bn2[j]) <= st->tol;
    }
};

struct FinOmega {   // tot: (t, s)[M], (t, t)[M]
    ColState* st;
    int M;
    __device__ void operator()(const double* tot) const
    {
        const int j = threadIdx.x;
        if (j < M && st->active[j]) {
            if (st->skip[j] || st->half[j]) {
                st->omega[j] = st->skip[j] ? st->omega[j] : 0.0;
            } else {
                const double ts = tot[j], tt = tot[M + j];
                const double w = tt > 0.0 ? ts / tt : 0.0;
                st->omega[j] = w;
                if (w == 0.0) {
                    if (++st->brk[j] >= 2) {
                        // the update below still applies (x += alpha ph)
                        st->failed[j] = 1;
                    } else {
                        st->nrst[j] += 1;
                    }
                    st->rst[j] = 1;
                } else {
                    st->brk[j] = 0;
                }
            }
        }
    }
};

struct FinRRB {   // tot: (rh, r)[M], (r, r)[M]
    ColState* st;
    int M;
    __device__ void operator()(const double* tot) const
    {
        const int j = threadIdx.x;
        if (j < M && st->active[j]) {
            const double rhr = tot[j], rr = tot[M + j];
            if (st->failed[j]) {
                st->active[j] = 0;
            } else if (st->skip[j]) {
                st->skip[j] = 0;
                prep_next(st, j, rhr, rr);
            } else {
                st->rr[j] = rr;
                const double rel = sqrt(rr) / sqrt(st->bn2[j]);
                st->relres[j] = rel;
                if (st->half[j] || rel <= st->tol) {
                    st->active[j] = 0;
                    st->conv[j] = 1;
                    st->half[j] = 0;
                } else {
                    prep_next(st, j, rhr, rr);
                }
            }
        }
        recount_active(st, M);
    }
};

// after a true-residual restart: r = t was copied for the flagged columns
struct FinRestartB {
    ColState* st;
    int M;
    __device__ void operator()(const double* tot) const   // tot: (b,b)[M], (t,t)[M]
    {
        const int j = threadIdx.x;
        if (j < M && st->cp[j]) {
            st->rr[j] = tot[M + j];
            st->brk[j] = 0;
            st->rst[j] = 1;
            prep_next(st, j, tot[M + j], tot[M + j]);
        }
    }
};

// FinTrue of the CG driver, reused: true residual, restart decisions
struct FinTrueB {
    ColState* st;
    int M;
    int allow_restart;
    __device__ void operator()(const double* tot) const
    {
        const int j = threadIdx.x;
        __shared__ int nr;
        if (j == 0) nr = 0;
        __syncthreads();
        if (j < M) {
            const double bb = tot[j], tt = tot[M + j];
            const double tr = bb > 0.0 ? sqrt(tt) / sqrt(bb) : 0.0;
            st->true_relres[j] = tr;
            st->cp[j] = 0;
            if (allow_restart && st->conv[j] && bb > 0.0 && !(tr <= st->tol) && !st->failed[j]) {
                st->conv[j] = 0;
                st->active[j] = 1;
                st->cp[j] = 1;
                st->relres[j] = tr;
                st->nrst[j] += 1;
                atomicAdd(&nr, 1);
            }
        }
        __syncthreads();
        if (j == 0) st->nrestart = nr;
        recount_active(st, M);
    }
};

}  // namespace bicg

using namespace bicg;

template <int M>
int bicgstab(Handle& h, const double* B, double* X, double tol)
{
    constexpr int CPT = cpt_for<double, M>();
    const int n = h.lev[0].n;
    const DCsr& A = h.lev[0].A64;
    const double* av = static_cast<const double*>(A.v);
    auto& w = h.w;
    ColState* st = h.st;
    const int cap = h.nb_cap;
    const int* na = &st->nactive;
    double *r = w.r, *rh = w.rh, *p = w.p, *v = w.v, *s = w.s, *t = w.t, *ph = w.ph, *sh = w.sh;

    if (h.opt.x0_mode == XAMG_X0_ZERO)
        hipLaunchKernelGGL((copy_cols_kernel<double, double>), dim3(1024), dim3(256), 0, h.stream,
                           nullptr, M, X, M, n, 0);
    // p, v, s must hold finite values before their first masked update
    for (double* z : {p, v, s})
        hipLaunchKernelGGL((copy_cols_kernel<double, double>), dim3(1024), dim3(256), 0, h.stream,
                           nullptr, M, z, M, n, 0);
    {
        const int nb = launch_op<M, double, double>(
            h, A, A.template split_of<M>(), n, cap, [&](auto cpt, auto ix) {
                return OpResid<M, decltype(cpt)::value, double, double, double, decltype(ix), 2>{
                    A.rp, av, ix, X, B, r, nullptr};
            });
        launch_fin(h, nb, 2 * M, FinInitB{st, tol, M});
    }
    if (h.opt.x0_mode == XAMG_X0_GIVEN) {
        OpFixCols<M, CPT> op{nullptr, nullptr, Idx32{nullptr}, st, nullptr, nullptr, X};
        launch_rows<M, CPT>(h, op, n, cap);
    }
    poll_state(h);
    if (h.st_host->nrestart < 0) return XAMG_EINVAL;

    int it = 0;
    PollPlan plan{h.opt.check_every};
    int next = plan.next_after(0, h.st_host->worst, tol);
    for (;;) {
        if (h.st_host->nactive == 0 || it >= h.opt.max_iters) {
            const int nb = launch_op<M, double, double>(
                h, A, A.template split_of<M>(), n, cap, [&](auto cpt, auto ix) {
                    return OpResid<M, decltype(cpt)::value, double, double, double, decltype(ix),
                                   2>{A.rp, av, ix, X, B, t, nullptr};
                });
            launch_fin(h, nb, 2 * M, FinTrueB{st, M, it < h.opt.max_iters ? 1 : 0});
            sync_state(h);
            if (h.st_host->nrestart == 0 || it >= h.opt.max_iters) break;
            OpFixCols<M, CPT> cp{nullptr, nullptr, Idx32{nullptr}, st, r, t, nullptr};
            launch_rows<M, CPT>(h, cp, n, cap);
            launch_fin(h, nb, 2 * M, FinRestartB{st, M});   // partials of (b,b),(t,t) still valid
            poll_state(h);
            plan = PollPlan{h.opt.check_every};
            next = plan.next_after(it, h.st_host->worst, tol);
            continue;
        }
        ++it;
        {
            OpBicgP<M, CPT> op{nullptr, nullptr, Idx32{nullptr}, st, r, p, v, rh, h.w.p32};
            launch_rows<M, CPT>(h, op, n, cap);
        }
        apply_prec<M>(h, p, ph, 0, nullptr, h.w.p32);
        {
            const int nb = launch_op<M, double, double>(
                h, A, A.template split_of<M>(), n, cap, [&](auto cpt, auto ix) {
                    return OpAxW<M, decltype(cpt)::value, double, decltype(ix), 1>{
                        A.rp, av, ix, ph, v, rh, na};
                });
            launch_fin(h, nb, M, FinAlphaB{st, M});
        }
        {
            OpBicgS<M, CPT> op{nullptr, nullptr, Idx32{nullptr}, st, r, v, s, h.w.s32};
            const int nb = launch_rows<M, CPT>(h, op, n, cap);
            launch_fin(h, nb, M, FinHalf{st, M});
        }
        apply_prec<M>(h, s, sh, 0, nullptr, h.w.s32);
        {
            const int nb = launch_op<M, double, double>(
                h, A, A.template split_of<M>(), n, cap, [&](auto cpt, auto ix) {
                    return OpAxW<M, decltype(cpt)::value, double, decltype(ix), 2>{
                        A.rp, av, ix, sh, t, s, na};
                });
            launch_fin(h, nb, 2 * M, FinOmega{st, M});
        }
        {
            OpBicgXR<M, CPT> op{nullptr, nullptr, Idx32{nullptr}, st, X, r, ph, sh, s, t, rh};
            const int nb = launch_rows<M, CPT>(h, op, n, cap);
            launch_fin(h, nb, 2 * M, FinRRB{st, M});
        }
        if (it >= next || it >= h.opt.max_iters) {
            poll_state(h);
            next = plan.next_after(it, h.st_host->worst, tol);
        }
    }
    return XAMG_OK;
}

}  // namespace xamg
