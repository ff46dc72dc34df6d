// cycle.hpp -- V-cycle, CG driver and SpMM entry as templates over the
// number of columns M; instantiated once per M (inst_m*.hip) so the
// kernels of each column count compile in their own translation unit.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "solver.hpp"

namespace xamg {

using namespace dev;

// ---------------------------------------------------------------------------
// finalize functors (one block; tot[] holds the dot totals)
// ---------------------------------------------------------------------------
struct FinInit {   // tot: (b,b)[M], (r,r)[M]
    ColState* st;
    double tol;
    int M;
    int max_iters;
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
            st->rst[j] = 1;
            st->pz[j] = 0;
            st->cp[j] = 0;
            st->brk[j] = 0;
            st->skip[j] = 0;
            st->half[j] = 0;
            st->failed[j] = 0;
            st->nrst[j] = 0;
            st->alpha[j] = st->beta[j] = 0.0;
            st->xpend[j] = 0.0;
            st->omega[j] = 1.0;
            st->rz[j] = 1.0;
        }
        if (j == 0) {
            st->ppar = 0;
            st->tol = tol;
            st->max_iters = max_iters;
            int bad = 0;
            for (int q = 0; q < M; ++q) bad |= !isfinite(tot[q]);
            st->nrestart = bad ? -1 : 0;
        }
        recount_active(st, M);
    }
};

struct FinAlpha {   // tot: (p, q)[M]
    ColState* st;
    int M;
    int merged = 0;   // merged CG form: alpha also becomes the pending x update;
                      // form 2 swaps the p buffers its SpMM just used
    __device__ void operator()(const double* tot) const
    {
        const int j = threadIdx.x;
        if (j < M) {
            double a = 0.0;
            if (st->active[j]) {
                const double pq = tot[j];
                if (!(pq > 0.0) || !isfinite(pq)) {
                    st->active[j] = 0;
                    st->failed[j] = 1;
                } else {
                    a = st->rz[j] / pq;
                }
            }
            st->alpha[j] = a;
            if (merged) st->xpend[j] = a;
        }
        if (merged == 2 && j == 0) st->ppar ^= 1;
        recount_active(st, M);
    }
};

struct FinRR {   // tot: (r, r)[M]
    ColState* st;
    int M;
    __device__ void operator()(const double* tot) const
    {
        const int j = threadIdx.x;
        if (j < M && st->active[j]) {
            const double rr = tot[j];
            st->rr[j] = rr;
            st->iters[j] += 1;
            const double rel = sqrt(rr) / sqrt(st->bn2[j]);
            st->relres[j] = rel;
            if (rel <= st->tol) {
                st->active[j] = 0;
                st->conv[j] = 1;
            } else if (st->iters[j] >= st->max_iters) {
                st->active[j] = 0;   // iteration cap: not converged
            }
        }
        recount_active(st, M);
    }
};

struct FinMG {   // tot: (b, b)[M], (r, r)[M] of the recomputed residual r = b - A x
    ColState* st;
    int M;
    __device__ void operator()(const double* tot) const
    {
        const int j = threadIdx.x;
        if (j < M && st->active[j]) {
            const double rr = tot[M + j];
            st->rr[j] = rr;
            st->iters[j] += 1;
            const double rel = sqrt(rr) / sqrt(st->bn2[j]);
            st->relres[j] = rel;
            st->true_relres[j] = rel;
            if (rel <= st->tol) {
                st->active[j] = 0;
                st->conv[j] = 1;
            } else if (st->iters[j] >= st->max_iters) {
                st->active[j] = 0;   // iteration cap: not converged
            }
        }
        recount_active(st, M);
    }
};

struct FinBeta {   // tot: (r, z)[M] and, flexible, (z, q)[M]
    ColState* st;
    int M;
    int flexible;
    __device__ void operator()(const double* tot) const
    {
        const int j = threadIdx.x;
        if (j < M && st->active[j]) {
            const double rzn = tot[j];
            double b = 0.0;
            if (st->rst[j]) {
                st->pz[j] = 1;
                st->rst[j] = 0;
            } else {
                st->pz[j] = 0;
                // flexible: (z_new, r_new - r_old) = -alpha (z_new, q)
                b = flexible ? -st->alpha[j] * tot[M + j] / st->rz[j] : rzn / st->rz[j];
            }
            st->beta[j] = b;
            st->rz[j] = rzn;
        }
    }
};

struct FinTrue {   // tot: (b, b)[M], (t, t)[M];  t = b - A x
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
            if (allow_restart && st->conv[j] && bb > 0.0 && !(tr <= st->tol) && !st->failed[j] &&
                st->iters[j] < st->max_iters) {
                st->conv[j] = 0;
                st->active[j] = 1;
                st->rst[j] = 1;
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

// ---------------------------------------------------------------------------
// V-cycle
// ---------------------------------------------------------------------------
struct Cheb {
    double theta, c1, c2, omega_deg1;
};

inline Cheb cheb_consts(const Handle& h, int l)
{
    const double hi = h.opt.cheby_hi_frac * h.lev[l].lmax;
    const double lo = h.opt.cheby_lo_frac * hi;
    Cheb c;
    c.theta = 0.5 * (hi + lo);
    const double delta = 0.5 * (hi - lo);
    const double sigma = c.theta / delta;
    const double rho0 = 1.0 / sigma;
    const double rho1 = 1.0 / (2.0 * sigma - rho0);
    c.c1 = rho1 * rho0;
    c.c2 = (2.0 * rho1) / delta;
    c.omega_deg1 = 1.0 / c.theta;
    return c;
}

template <typename T>
static const DCsr& matA(const LevelDev& L) { if constexpr (sizeof(T) == 8) return L.A64; else return L.A32; }
template <typename T>
static const DCsr& matP(const LevelDev& L) { if constexpr (sizeof(T) == 8) return L.P64; else return L.P32; }
template <typename T>
static const DCsr& matR(const LevelDev& L) { if constexpr (sizeof(T) == 8) return L.R64; else return L.R32; }
template <typename T>
static const T* dinv_of(const LevelDev& L) { if constexpr (sizeof(T) == 8) return L.dinv64; else return L.dinv32; }

template <typename T>
static T* lvbuf(void* p) { return static_cast<T*>(p); }

template <typename T>
static const T* dl1_of(const LevelDev& L) { if constexpr (sizeof(T) == 8) return L.dl1inv64; else return L.dl1inv32; }

// one l1-hybrid Gauss-Seidel sweep over the rows of A (block size from the
// options: 4, 8 or 16 rows; `split` lane groups per block, normally A's
// Gauss-Seidel split, tuned on its own and kept in the pre-smoothing slot,
// since this smoother has no separate pre-smoothing pass)
template <int M, bool BWD, bool ZERO, typename MT, typename XT, typename BT, typename OT>
static void launch_hgs(Handle& h, const DCsr& A, const MT* dl1, const BT* b, const XT* xo, OT* xn,
                       const int* na, int split)
{
    constexpr int CPT = cpt_for<MT, M>();
    constexpr int G = M / CPT;
    const int n = A.nr;
    const MT* av = static_cast<const MT*>(A.v);
    auto go = [&](auto blk, auto sgr) {
        constexpr int BLK = decltype(blk)::value;
        constexpr int S = decltype(sgr)::value;
        constexpr int NG = kGsThreads / (G * S);
        const int nblk = (n + BLK - 1) / BLK;
        const int grid = std::max(1, (nblk + NG - 1) / NG);
        hipLaunchKernelGGL((hgs_kernel<M, CPT, S, BLK, BWD, ZERO, MT, XT, BT, OT>), dim3(grid),
                           dim3(kGsThreads), 0, h.stream, A.rp, A.ci, av, dl1, b, xo, xn, n, na);
    };
    auto with_s = [&](auto blk) {
        const int s = split & (kSweep - 1);
        if constexpr (G * 8 <= kGsThreads) {
            if (s >= 8) return go(blk, std::integral_constant<int, 8>{});
        }
        if constexpr (G * 4 <= kGsThreads) {
            if (s >= 4) return go(blk, std::integral_constant<int, 4>{});
        }
        if constexpr (G * 2 <= kGsThreads) {
            if (s >= 2) return go(blk, std::integral_constant<int, 2>{});
        }
        go(blk, std::integral_constant<int, 1>{});
    };
    if (h.opt.gs_block == 4) with_s(std::integral_constant<int, 4>{});
    else if (h.opt.gs_block == 16) with_s(std::integral_constant<int, 16>{});
    else with_s(std::integral_constant<int, 8>{});
}

// dots (b, x) [and (q, x)] as a pure vector pass (used when the finest
// level is also the coarsest and no smoothing pass exists to fuse them into)
template <int M, int CPT, int D>
struct OpDotsBX {
    using AT = double;
    static constexpr bool kMatrix = false;
    static constexpr int kDots = D;
    const int* rp = nullptr;
    const double* val = nullptr;
    Idx32 idx{nullptr};
    const double *b, *x, *q;
    __device__ __forceinline__ bool active_any() const { return true; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int, int) const { return Pack<AT, CPT>{}; }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&)[CPT], double (&d)[ND][CPT]) const
    {
        const size_t o = size_t(i) * M + j0;
        const auto bi = load_pack<double, CPT>(b + o);
        const auto xi = load_pack<double, CPT>(x + o);
#pragma unroll
        for (int t = 0; t < CPT; ++t) d[0][t] += bi.v[t] * xi.v[t];
        if constexpr (D == 2) {
            const auto qi = load_pack<double, CPT>(q + o);
#pragma unroll
            for (int t = 0; t < CPT; ++t) d[1][t] += qi.v[t] * xi.v[t];
        }
    }
};



// One level of V(1,1) from a zero guess.  b: right-hand side of the level
// (BT), xout: corrected solution (OT).  At the finest level the last pass
// also accumulates the dots (b, xout) [and (q, xout)].  Returns the block
// count of the last launch (the one that wrote partial dots).
// x = A_L^-1 b on the coarsest level (nL rows): the inverse staged in LDS by
// one block up to kCoarseLds rows, else read from global memory by one
// thread per entry of x (the same sums in the same order)
template <int M, typename T>
void launch_coarse(Handle& h, const T* inv, int nL, const T* b, T* x, const int* nactive)
{
    if (nL <= kCoarseLds)
        hipLaunchKernelGGL((coarse_kernel<M, T>), dim3(1), dim3(256), 0, h.stream, inv, nL, b, x,
                           nactive);
    else
        hipLaunchKernelGGL((coarse_global_kernel<M, T>), dim3((nL * M + 255) / 256), dim3(256), 0,
                           h.stream, inv, nL, b, x, nactive);
}

template <int M, typename T, typename BT, typename OT>
static int vlevel(Handle& h, int l, const BT* b, OT* xout, int ndots, const double* q,
                  const double* bd = nullptr)
{
    const LevelDev& L = h.lev[l];
    const int* na = &h.st->nactive;
    const int cap = h.nb_cap;
    auto& W = h.w.lev[l];
    int nb = 1;
    if (l == h.nlev - 1) {
        // coarsest level: the dense inverse applied
        if constexpr (std::is_same<BT, T>::value && std::is_same<OT, T>::value) {
            const T* inv;
            if constexpr (sizeof(T) == 8) inv = h.inv64; else inv = h.inv32;
            launch_coarse<M, T>(h, inv, L.n, b, xout, na);
        } else {
            set_error("internal: coarsest level with mixed boundary types");
            throw DevFail{XAMG_EINVAL};
        }
        return 0;
    }
    const DCsr& A = matA<T>(L);
    const T* dinv = dinv_of<T>(L);
    T* X = lvbuf<T>(W.X);
    T* R = lvbuf<T>(W.R);
    T* Tb = lvbuf<T>(W.T);
    T* Bc = lvbuf<T>(h.w.lev[l + 1].B);
    T* Xc = lvbuf<T>(h.w.lev[l + 1].X2);
    const bool cheb2 = h.opt.smoother == XAMG_CHEBYSHEV && h.opt.cheby_degree == 2;
    const Cheb ch = cheb_consts(h, l);
    const T omega = T(h.opt.smoother == XAMG_CHEBYSHEV ? ch.omega_deg1 : h.opt.omega);
    const int* rp = A.rp;
    const T* av = static_cast<const T*>(A.v);
    const T* avd = static_cast<const T*>(A.vd);
    const int sA = A.template split_of<M>(), sPre = A.template split_pre_of<M>();

    const bool gs = h.opt.smoother == XAMG_GAUSS_SEIDEL;
    if (!gs && !A.vd) {
        set_error("internal: level %d has no column-scaled matrix for pre-smoothing", l);
        throw DevFail{XAMG_EINVAL};
    }
    // r = b - A X (the residual after pre-smoothing)
    auto residual_pass = [&]() {
        launch_op<M, T, T>(h, A, sA, L.n, cap, [&](auto cpt, auto ix) {
            return OpResid<M, decltype(cpt)::value, T, T, BT, decltype(ix), 0>{rp, av, ix, X, b, R,
                                                                               na};
        });
    };
    // pre-smoothing from zero (+ residual)
    if (l == 0) h.timer_begin(XAMG_TIMER_PRESMOOTH);
    if (gs) {
        // symmetric sweep from zero: forward into T, backward into X
        const T* dl1 = dl1_of<T>(L);
        launch_hgs<M, false, true>(h, A, dl1, b, static_cast<const T*>(nullptr), Tb, na, sPre);
        if (l == 0) h.timer_end(XAMG_TIMER_PRESMOOTH);
        launch_hgs<M, true, false>(h, A, dl1, b, static_cast<const T*>(Tb), X, na, sPre);
        residual_pass();
    } else if (!cheb2) {
        launch_op<M, T, T>(h, A, sPre, L.n, cap, [&](auto cpt, auto ix) {
            return OpJacPre<M, decltype(cpt)::value, T, T, BT, decltype(ix)>{rp, avd, ix, dinv,
                                                                             omega, b, X, R, na};
        });
        if (l == 0) h.timer_end(XAMG_TIMER_PRESMOOTH);
    } else {
        launch_op<M, T, T>(h, A, sPre, L.n, cap, [&](auto cpt, auto ix) {
            return OpChebPre<M, decltype(cpt)::value, T, T, BT, decltype(ix)>{
                rp, avd, ix, dinv, T(1.0 / ch.theta), T(ch.c1), T(ch.c2), b, X, na};
        });
        if (l == 0) h.timer_end(XAMG_TIMER_PRESMOOTH);
        residual_pass();
    }
    // restriction b_{l+1} = R_l r_l
    {
        const DCsr& Rm = matR<T>(L);
        launch_op<M, T, T>(h, Rm, Rm.template split_of<M>(), Rm.nr, cap, [&](auto cpt, auto ix) {
            return OpAx<M, decltype(cpt)::value, T, T, decltype(ix), 0>{
                Rm.rp, static_cast<const T*>(Rm.v), ix, R, Bc, na};
        });
    }
    vlevel<M, T, T, T>(h, l + 1, Bc, Xc, 0, nullptr);
    // prolongation x_l += P_l x_{l+1}
    {
        const DCsr& Pm = matP<T>(L);
        launch_op<M, T, T>(h, Pm, Pm.template split_of<M>(), Pm.nr, cap, [&](auto cpt, auto ix) {
            return OpProlongAdd<M, decltype(cpt)::value, T, T, decltype(ix)>{
                Pm.rp, static_cast<const T*>(Pm.v), ix, Xc, X, na};
        });
    }
    // post-smoothing (+ finest-level dots).  The last pass of the finest
    // level of a mixed cycle writes the FP64 z and reads the FP64 b (and q)
    // of its dots: it takes the FP64 lane layout (16 bytes of those rows per
    // lane; measured 3% faster on the mixed solve than the FP32 layout's
    // two loads per lane)
    using LT = std::conditional_t<(sizeof(OT) > sizeof(T)), OT, T>;   // lane layout of that pass
    auto post = [&](auto dots_tag) {
        constexpr int D = decltype(dots_tag)::value;
        if (gs) {
            // symmetric sweep: forward X -> T, backward T -> xout; the
            // finest level's dots in a pass of their own
            const T* dl1 = dl1_of<T>(L);
            launch_hgs<M, false, false>(h, A, dl1, b, static_cast<const T*>(X), Tb, na, sPre);
            launch_hgs<M, true, false>(h, A, dl1, b, static_cast<const T*>(Tb), xout, na, sPre);
            if constexpr (D > 0) {
                if constexpr (std::is_same<BT, double>::value && std::is_same<OT, double>::value) {
                    constexpr int CPD = cpt_for<double, M>();
                    OpDotsBX<M, CPD, D> op;
                    op.b = b;
                    op.x = xout;
                    op.q = q;
                    nb = launch_rows<M, CPD>(h, op, L.n, cap);
                }
            }
        } else if (!cheb2) {
            nb = launch_op<M, LT, T>(h, A, sA, L.n, cap, [&](auto cpt, auto ix) {
                return OpJacPost<M, decltype(cpt)::value, T, T, BT, OT, decltype(ix), D>{
                    rp, av, ix, dinv, omega, X, b, xout, q, na, bd};
            });
        } else {
            launch_op<M, T, T>(h, A, sA, L.n, cap, [&](auto cpt, auto ix) {
                return OpChebPost1<M, decltype(cpt)::value, T, T, BT, decltype(ix)>{
                    rp, av, ix, dinv, X, b, Tb, na};
            });
            nb = launch_op<M, LT, T>(h, A, sA, L.n, cap, [&](auto cpt, auto ix) {
                return OpChebPost2<M, decltype(cpt)::value, T, T, BT, OT, decltype(ix), D>{
                    rp,  av, ix, dinv, T(1.0 / ch.theta), T(ch.c1), T(ch.c2), Tb, X, b, xout, q,
                    na,  bd};
            });
        }
    };
    if (ndots == 2) post(std::integral_constant<int, 2>{});
    else if (ndots == 1) post(std::integral_constant<int, 1>{});
    else post(std::integral_constant<int, 0>{});
    return nb;
}

// z = M^-1 r for the whole hierarchy; returns the block count of the
// launch that produced the finest-level dots (0 if ndots == 0).
template <int M>
int vcycle(Handle& h, const double* r, double* z, int ndots, const double* q,
           const float* r32)
{
    constexpr int CPT = cpt_for<double, M>();
    if (h.nlev == 1) {
        launch_coarse<M, double>(h, h.inv64, h.lev[0].n, r, z, &h.st->nactive);
        if (ndots == 0) return 0;
        if (ndots == 2) {
            OpDotsBX<M, CPT, 2> op{nullptr, nullptr, Idx32{nullptr}, r, z, q};
            return launch_rows<M, CPT>(h, op, h.lev[0].n, h.nb_cap);
        }
        OpDotsBX<M, CPT, 1> op{nullptr, nullptr, Idx32{nullptr}, r, z, q};
        return launch_rows<M, CPT>(h, op, h.lev[0].n, h.nb_cap);
    }
    if (h.opt.precision == XAMG_MIXED) {
        // with an FP32 copy of r the finest level gathers and reads that copy,
        // and only the dots of its last pass read the FP64 r
        if (r32) return vlevel<M, float, float, double>(h, 0, r32, z, ndots, q, r);
        return vlevel<M, float, double, double>(h, 0, r, z, ndots, q);
    }
    return vlevel<M, double, double, double>(h, 0, r, z, ndots, q);
}


// z = M^-1 r for the Krylov drivers: the V-cycle, or z = r when the handle
// runs without a preconditioner (the dots of the finest level then come
// from a vector pass of their own)
template <int M>
int apply_prec(Handle& h, const double* r, double* z, int ndots, const double* q,
               const float* r32 = nullptr)
{
    constexpr int CPT = cpt_for<double, M>();
    if (h.opt.precond) return vcycle<M>(h, r, z, ndots, q, r32);
    hipLaunchKernelGGL((copy_cols_kernel<double, double>), dim3(2048), dim3(256), 0, h.stream,
                       r, M, z, M, h.lev[0].n, M);
    if (ndots == 0) return 0;
    if (ndots == 2) {
        OpDotsBX<M, CPT, 2> op{nullptr, nullptr, Idx32{nullptr}, r, z, q};
        return launch_rows<M, CPT>(h, op, h.lev[0].n, h.nb_cap);
    }
    OpDotsBX<M, CPT, 1> op{nullptr, nullptr, Idx32{nullptr}, r, z, q};
    return launch_rows<M, CPT>(h, op, h.lev[0].n, h.nb_cap);
}

// ---------------------------------------------------------------------------
// preconditioned CG, all m columns at once
// ---------------------------------------------------------------------------
// The CG driver in enqueue-only pieces (no host synchronisation inside),
// so the batched solver can capture iterations into a graph.
template <int M>
int pcg_flex(const Handle& h)
{
    return h.opt.precision == XAMG_MIXED ? 1 : h.opt.flexible;
}

// z = M^-1 r (dots (r, z) [, (z, q)]), beta, p = z + beta p (merged form
// 1: with x += xpend p before p changes; form 2: in the SpMM that follows)
template <int M>
void pcg_precondition(Handle& h, double* X)
{
    constexpr int CPT = cpt_for<double, M>();
    const int flex = pcg_flex<M>(h);
    const int nd = flex ? 2 : 1;
    const int nb = apply_prec<M>(h, h.w.r, h.w.z, nd, h.w.q, h.w.r32);
    launch_fin(h, nb, nd * M, FinBeta{h.st, M, flex});
    if (h.opt.merged == 2) return;
    if (h.opt.merged == 1) {
        OpUpdPX<M, CPT> up{nullptr, nullptr, Idx32{nullptr}, h.st, h.w.p, X, h.w.z};
        launch_rows<M, CPT>(h, up, h.lev[0].n, h.nb_cap);
        return;
    }
    OpUpdP<M, CPT> up{nullptr, nullptr, Idx32{nullptr}, h.st, h.w.p, h.w.z};
    launch_rows<M, CPT>(h, up, h.lev[0].n, h.nb_cap);
}

template <int M>
__global__ void clear_xpend_kernel(ColState* st)
{
    if (int(threadIdx.x) < M) st->xpend[threadIdx.x] = 0.0;
}

// merged CG: apply the pending x += xpend p and clear xpend (before a true
// residual is formed from x)
template <int M>
void pcg_flush(Handle& h, double* X)
{
    constexpr int CPT = cpt_for<double, M>();
    if (h.opt.merged == 0 || h.opt.method != XAMG_CG) return;
    OpFlushX<M, CPT> op{nullptr, nullptr, Idx32{nullptr}, h.st, X, h.w.p, h.w.p2};
    launch_rows<M, CPT>(h, op, h.lev[0].n, h.nb_cap);
    hipLaunchKernelGGL(clear_xpend_kernel<M>, dim3(1), dim3(64), 0, h.stream, h.st);
}

// r32 = float(r), where a pass other than OpUpdXR has rewritten r
template <int M>
void sync_r32(Handle& h)
{
    if (!h.w.r32) return;
    hipLaunchKernelGGL((copy_cols_kernel<double, float>), dim3(2048), dim3(256), 0, h.stream,
                       h.w.r, M, h.w.r32, M, h.lev[0].n, M);
}

// r = b - A x, column state (the first iteration computes z = M^-1 r, p = z)
template <int M>
void pcg_start(Handle& h, const double* B, double* X, double tol)
{
    constexpr int CPT = cpt_for<double, M>();
    const int n = h.lev[0].n;
    const DCsr& A = h.lev[0].A64;
    const double* av = static_cast<const double*>(A.v);
    if (h.opt.x0_mode == XAMG_X0_ZERO)
        hipLaunchKernelGGL((copy_cols_kernel<double, double>), dim3(1024), dim3(256), 0, h.stream,
                           nullptr, M, X, M, n, 0);
    {
        const int nb = launch_op<M, double, double>(
            h, A, A.template split_of<M>(), n, h.nb_cap, [&](auto cpt, auto ix) {
                return OpResid<M, decltype(cpt)::value, double, double, double, decltype(ix), 2>{
                    A.rp, av, ix, X, B, h.w.r, nullptr};
            });
        launch_fin(h, nb, 2 * M, FinInit{h.st, tol, M, h.opt.max_iters});
    }
    if (h.opt.x0_mode == XAMG_X0_GIVEN) {
        OpFixCols<M, CPT> op{nullptr, nullptr, Idx32{nullptr}, h.st, nullptr, nullptr, X};
        launch_rows<M, CPT>(h, op, n, h.nb_cap);
    }
    // q must be finite for the flexible dot of the first cycle
    if (pcg_flex<M>(h))
        hipLaunchKernelGGL((copy_cols_kernel<double, double>), dim3(1024), dim3(256), 0, h.stream,
                           nullptr, M, h.w.q, M, n, 0);
    sync_r32<M>(h);
}

// one iteration: z = M^-1 r, beta, p = z + beta p (beta = 0 on a column's
// first or restarted iteration), q = A p, alpha, x += alpha p,
// r -= alpha q, convergence test.  The test comes last, so no
// preconditioner runs after the last column has converged.
template <int M>
void pcg_iteration(Handle& h, double* X)
{
    constexpr int CPT = cpt_for<double, M>();
    const int n = h.lev[0].n;
    const DCsr& A = h.lev[0].A64;
    const double* av = static_cast<const double*>(A.v);
    ColState* st = h.st;
    const int merged = h.opt.merged;
    pcg_precondition<M>(h, X);
    {
        h.timer_begin(XAMG_TIMER_KRYLOV_SPMM);
        int nb;
        if (merged == 2) {
            nb = launch_op<M, double, double>(
                h, A, A.template split_of<M>(), n, h.nb_cap, [&](auto cpt, auto ix) {
                    return OpAxPX<M, decltype(cpt)::value, decltype(ix)>{
                        A.rp, av, ix, st, h.w.p, h.w.p2, h.w.z, h.w.q, X};
                });
        } else {
            nb = launch_op<M, double, double>(
                h, A, A.template split_of<M>(), n, h.nb_cap, [&](auto cpt, auto ix) {
                    return OpAx<M, decltype(cpt)::value, double, double, decltype(ix), 1>{
                        A.rp, av, ix, h.w.p, h.w.q, &st->nactive};
                });
        }
        h.timer_end(XAMG_TIMER_KRYLOV_SPMM);
        launch_fin(h, nb, M, FinAlpha{st, M, merged});
    }
    {
        // merged: r only (x's update waits in xpend; p is not read)
        OpUpdXR<M, CPT> op{nullptr, nullptr, Idx32{nullptr}, st,      merged ? nullptr : X,
                           h.w.r,   h.w.p,   h.w.q,          h.w.r32};
        const int nb = launch_rows<M, CPT>(h, op, n, h.nb_cap);
        launch_fin(h, nb, M, FinRR{st, M});
    }
}

// true residual of the columns the recurrence froze; columns that fail it
// restart (r = b - A x; their next iteration takes z = M^-1 r, p = z).
// Synchronises; returns the number of restarted columns.
// In two halves, so a batch can check many systems with one wait: enqueue
// the check and the copy of the column state, then (after the stream has
// been synchronised) act on the restarts.
template <int M>
void pcg_true_enqueue(Handle& h, const double* B, double* X, int allow_restart)
{
    const int n = h.lev[0].n;
    const DCsr& A = h.lev[0].A64;
    const double* av = static_cast<const double*>(A.v);
    pcg_flush<M>(h, X);
    const int nb = launch_op<M, double, double>(
        h, A, A.template split_of<M>(), n, h.nb_cap, [&](auto cpt, auto ix) {
            return OpResid<M, decltype(cpt)::value, double, double, double, decltype(ix), 2>{
                A.rp, av, ix, X, B, h.w.t, nullptr};
        });
    launch_fin(h, nb, 2 * M, FinTrue{h.st, M, allow_restart});
    h.check(hipMemcpyAsync(h.st_host, h.st, sizeof(ColState), hipMemcpyDeviceToHost, h.stream),
            "state copy");
}

template <int M>
int pcg_true_finish(Handle& h)
{
    constexpr int CPT = cpt_for<double, M>();
    const int nr = h.st_host->nrestart;
    if (nr > 0) {
        OpFixCols<M, CPT> cp{nullptr, nullptr, Idx32{nullptr}, h.st, h.w.r, h.w.t, nullptr};
        launch_rows<M, CPT>(h, cp, h.lev[0].n, h.nb_cap);
        sync_r32<M>(h);
    }
    return nr;
}

template <int M>
int pcg_true_check(Handle& h, const double* B, double* X, int allow_restart)
{
    pcg_true_enqueue<M>(h, B, X, allow_restart);
    h.check(hipStreamSynchronize(h.stream), "stream sync");
    return pcg_true_finish<M>(h);
}

// Multigrid as a standalone solver (Section 2.1, Table 1): per column
// x <- x + V(b - A x) until ||b - A x|| / ||b|| <= tol; the residual is
// recomputed from x each iteration, so it is the true residual.
template <int M>
int mg_solve(Handle& h, const double* B, double* X, double tol)
{
    constexpr int CPT = cpt_for<double, M>();
    const int n = h.lev[0].n;
    const DCsr& A = h.lev[0].A64;
    const double* av = static_cast<const double*>(A.v);
    pcg_start<M>(h, B, X, tol);   // r = b - A x, column state
    poll_state(h);
    if (h.st_host->nrestart < 0) return XAMG_EINVAL;   // NaN/Inf in B
    PollPlan plan{h.opt.check_every};
    int next = plan.next_after(0, h.st_host->worst, tol);
    for (int it = 0; h.st_host->nactive > 0 && it < h.opt.max_iters;) {
        ++it;
        vcycle<M>(h, h.w.r, h.w.z, 0, nullptr);
        OpAddActive<M, CPT> up{nullptr, nullptr, Idx32{nullptr}, h.st, X, h.w.z};
        launch_rows<M, CPT>(h, up, n, h.nb_cap);
        const int nb = launch_op<M, double, double>(
            h, A, A.template split_of<M>(), n, h.nb_cap, [&](auto cpt, auto ix) {
                return OpResid<M, decltype(cpt)::value, double, double, double, decltype(ix), 2>{
                    A.rp, av, ix, X, B, h.w.r, nullptr};
            });
        launch_fin(h, nb, 2 * M, FinMG{h.st, M});
        if (it >= next || it >= h.opt.max_iters) {
            poll_state(h);
            next = plan.next_after(it, h.st_host->worst, tol);
        }
    }
    sync_state(h);
    return XAMG_OK;
}

template <int M>
int pcg(Handle& h, const double* B, double* X, double tol)
{
    pcg_start<M>(h, B, X, tol);
    poll_state(h);
    if (h.st_host->nrestart < 0) return XAMG_EINVAL;   // NaN/Inf in B
    int it = 0;
    PollPlan plan{h.opt.check_every};
    int next = plan.next_after(0, h.st_host->worst, tol);
    for (;;) {
        if (h.st_host->nactive == 0 || it >= h.opt.max_iters) {
            const int nr = pcg_true_check<M>(h, B, X, it < h.opt.max_iters ? 1 : 0);
            if (nr == 0 || it >= h.opt.max_iters) break;
            plan = PollPlan{h.opt.check_every};
            next = plan.next_after(it, h.st_host->worst, tol);
            continue;
        }
        ++it;
        pcg_iteration<M>(h, X);
        if (it >= next || it >= h.opt.max_iters) {
            poll_state(h);
            next = plan.next_after(it, h.st_host->worst, tol);
        }
    }
    return XAMG_OK;
}

template <int M>
void spmm64(Handle& h, const DCsr& d, const double* X, double* Y)
{
    launch_op<M, double, double>(h, d, d.template split_of<M>(), d.nr, h.nb_cap,
                                 [&](auto cpt, auto ix) {
                                     return OpAx<M, decltype(cpt)::value, double, double,
                                                 decltype(ix), 0>{
                                         d.rp, static_cast<const double*>(d.v), ix, X, Y, nullptr};
                                 });
}


// ---------------------------------------------------------------------------
// autotuner: for every operator of the hierarchy, time the plain SpMM
// y = Op x with a row split (lane groups per row, optionally sweeping) using HIP
// events, and keep the fastest for this column count.  Runs once per M on
// the first solve (or on request); setup cost, not solve cost.
// ---------------------------------------------------------------------------
// kind: 0 = residual pass r = b - A x (the post-smoothing and residual
// passes gather x), 1 = plain product y = Op x (restriction),
// 2 = pre-smoothing pass from zero (gathers b against A D^-1), or with the
// Gauss-Seidel smoother a forward sweep (dinv = its l1 diagonal), 3 =
// prolongation y += Op x (reads and writes the fine vector)
template <int M, typename T>
float time_op(Handle& h, const DCsr& d, int kind, const T* dinv, int split, T* x, T* y, T* z,
              hipEvent_t e0, hipEvent_t e1)
{
    const T* av = static_cast<const T*>(d.v);
    const T* avd = static_cast<const T*>(d.vd);
    auto launch = [&]() {
        if (kind == 2 && h.opt.smoother == XAMG_GAUSS_SEIDEL) {
            launch_hgs<M, false, false>(h, d, dinv, static_cast<const T*>(z),
                                        static_cast<const T*>(x), y, nullptr, split);
        } else if (kind == 0) {
            launch_op<M, T, T>(h, d, split, d.nr, h.nb_cap, [&](auto cpt, auto ix) {
                return OpResid<M, decltype(cpt)::value, T, T, T, decltype(ix), 0>{d.rp, av, ix, x, z,
                                                                                  y, nullptr};
            });
        } else if (kind == 1) {
            launch_op<M, T, T>(h, d, split, d.nr, h.nb_cap, [&](auto cpt, auto ix) {
                return OpAx<M, decltype(cpt)::value, T, T, decltype(ix), 0>{d.rp, av, ix, x, y,
                                                                            nullptr};
            });
        } else if (kind == 3) {
            launch_op<M, T, T>(h, d, split, d.nr, h.nb_cap, [&](auto cpt, auto ix) {
                return OpProlongAdd<M, decltype(cpt)::value, T, T, decltype(ix)>{d.rp, av, ix, x,
                                                                                 y, nullptr};
            });
        } else if (h.opt.smoother == XAMG_CHEBYSHEV && h.opt.cheby_degree == 2) {
            launch_op<M, T, T>(h, d, split, d.nr, h.nb_cap, [&](auto cpt, auto ix) {
                return OpChebPre<M, decltype(cpt)::value, T, T, T, decltype(ix)>{
                    d.rp, avd, ix, dinv, T(1), T(0), T(0), x, y, nullptr};
            });
        } else {
            launch_op<M, T, T>(h, d, split, d.nr, h.nb_cap, [&](auto cpt, auto ix) {
                return OpJacPre<M, decltype(cpt)::value, T, T, T, decltype(ix)>{
                    d.rp, avd, ix, dinv, T(0.5), x, y, z, nullptr};
            });
        }
    };
    // Before each timed run: stream through two other work blocks (Krylov
    // q -> t, n0 x mcap each), so the operator is no longer in L2 or the
    // memory-side cache, then rewrite the run's input blocks (zeros), so
    // they are -- as in the V-cycle, where a pass reads the vectors the
    // previous pass of the level has just written while the matrix streams
    // from HBM.
    auto prepare = [&]() {
        const int mc = h.w.mcap;
        hipLaunchKernelGGL((copy_cols_kernel<double, double>), dim3(4096), dim3(256), 0, h.stream,
                           h.w.q, mc, h.w.t, mc, h.lev[0].n, mc);
        hipLaunchKernelGGL((copy_cols_kernel<T, T>), dim3(2048), dim3(256), 0, h.stream,
                           static_cast<const T*>(nullptr), M, x, M, d.nc, 0);
        if (kind == 0)
            hipLaunchKernelGGL((copy_cols_kernel<T, T>), dim3(2048), dim3(256), 0, h.stream,
                               static_cast<const T*>(nullptr), M, z, M, d.nr, 0);
    };
    float best = 0.0f;
    launch();
    for (int r = 0; r < 5; ++r) {
        float ms = 0.0f;
        prepare();
        h.check(hipEventRecord(e0, h.stream), "tune event");
        launch();
        h.check(hipEventRecord(e1, h.stream), "tune event");
        h.check(hipEventSynchronize(e1), "tune sync");
        h.check(hipEventElapsedTime(&ms, e0, e1), "tune elapsed");
        if (r == 0 || ms < best) best = ms;
    }
    return best;
}

// Tuning cache: the choices of tune_matrix, kept for the process per device
// and keyed by what the timed pass depends on -- the operator's shape and
// storage (rows, columns, nonzeros, stored row length, bandwidth, value
// bytes, 16-bit offsets), the pass, the pre-smoothing variant and M.  A
// later handle with an operator of the same key takes the cached choice
// without timing, so equal problems run on equal launch shapes (and give
// bit-identical results); an explicit re-tune times afresh and replaces it.
struct TuneKey {
    int dev, nr, nc;
    int64_t nnz;
    int rowlen, bw, vbytes, idx16, kind, variant, m;
    bool operator<(const TuneKey& o) const
    {
        return std::tie(dev, nr, nc, nnz, rowlen, bw, vbytes, idx16, kind, variant, m) <
               std::tie(o.dev, o.nr, o.nc, o.nnz, o.rowlen, o.bw, o.vbytes, o.idx16, o.kind,
                        o.variant, o.m);
    }
};

inline std::map<TuneKey, int>& tune_cache()
{
    static std::map<TuneKey, int> cache;
    return cache;
}

inline std::mutex& tune_cache_mutex()
{
    static std::mutex mu;
    return mu;
}

// whether pass `kind` over d is tuned at all (it exists and runs)
inline bool tuned_pass(const Handle& h, const DCsr& d, int kind)
{
    if (!d.rp || d.nr == 0) return false;
    const bool gs_sweep = kind == 2 && h.opt.smoother == XAMG_GAUSS_SEIDEL;
    return !(kind == 2 && !gs_sweep && !d.vd);
}

template <int M, typename T>
TuneKey tune_key(const Handle& h, const DCsr& d, int kind)
{
    const bool gs_sweep = kind == 2 && h.opt.smoother == XAMG_GAUSS_SEIDEL;
    // the pre-smoothing pass runs a different kernel per smoother
    const int variant = kind != 2 ? 0
                        : gs_sweep ? 100 + h.opt.gs_block
                        : (h.opt.smoother == XAMG_CHEBYSHEV && h.opt.cheby_degree == 2) ? 2
                                                                                          : 1;
    return TuneKey{h.device, d.nr, d.nc, d.nnz, d.rowlen, d.bw, int(sizeof(T)),
                   d.off != nullptr ? 1 : 0, kind, variant, M};
}

// the cached choice for pass `kind` over d, if any, applied without timing
template <int M, typename T>
bool cached_choice(const Handle& h, DCsr& d, int kind)
{
    constexpr int k = M == 1 ? 0 : M == 2 ? 1 : M == 4 ? 2 : M == 8 ? 3 : M == 16 ? 4 : 5;
    if (!tuned_pass(h, d, kind)) return true;
    std::lock_guard<std::mutex> lock(tune_cache_mutex());
    const auto it = tune_cache().find(tune_key<M, T>(h, d, kind));
    if (it == tune_cache().end()) return false;
    (kind == 2 ? d.split_pre : d.split)[k] = it->second;
    return true;
}

template <int M, typename T>
void tune_matrix(Handle& h, DCsr& d, int kind, const T* dinv, T* x, T* y, T* z, hipEvent_t e0,
                 hipEvent_t e1)
{
    constexpr int C0 = cpt_for<T, M>();
    constexpr int G = M / C0;
    constexpr int k = M == 1 ? 0 : M == 2 ? 1 : M == 4 ? 2 : M == 8 ? 3 : M == 16 ? 4 : 5;
    if (!tuned_pass(h, d, kind)) return;
    if (!h.tune_fresh && cached_choice<M, T>(h, d, kind)) return;
    const bool gs_sweep = kind == 2 && h.opt.smoother == XAMG_GAUSS_SEIDEL;
    const TuneKey key = tune_key<M, T>(h, d, kind);
    int& slot = (kind == 2 ? d.split_pre : d.split)[k];
    // candidates from the simplest launch up; a later one replaces the
    // current choice only when it is more than 3% faster, so that near-ties
    // (within the timing noise) resolve the same way from run to run.
    // First the lane groups per row and the launch mode ...
    float best = 0.0f;
    int bestS = 1;
    for (int S : {1, 2, 4, 8}) {
        if (G * S > 64) break;
        for (int sw : {0, kSweep}) {
            if (gs_sweep && sw) continue;   // the sweep kernel has one launch shape
            const float t = time_op<M, T>(h, d, kind, dinv, S | sw, x, y, z, e0, e1);
            if ((S == 1 && sw == 0) || t < 0.97f * best) {
                best = t;
                bestS = S | sw;
            }
        }
    }
    // ... then, one at a time on top of the best, the 32-bit indices of a
    // 16-bit-encoded operator, twice the columns per lane, and blocks of
    // twice the threads (the Gauss-Seidel sweep has none of these)
    if (!gs_sweep) {
        std::vector<int> flags;
        if (d.off) flags.push_back(kIdx32);
        if (2 * C0 <= M) flags.push_back(kWide);
        flags.push_back(kBig);
        for (int f : flags) {
            const float t = time_op<M, T>(h, d, kind, dinv, bestS | f, x, y, z, e0, e1);
            if (t < 0.97f * best) {
                best = t;
                bestS |= f;
            }
        }
        // ... and the banded XCD walk with segments of one, a half and a
        // quarter bandwidth (square operators)
        if (d.bw > 0) {
            const int base = bestS;
            for (int f : {kSegBw, kSegHalf, kSegQuarter}) {
                const float t = time_op<M, T>(h, d, kind, dinv, base | f, x, y, z, e0, e1);
                if (t < 0.97f * best) {
                    best = t;
                    bestS = base | f;
                }
            }
        }
    }
    slot = bestS;
    std::lock_guard<std::mutex> lock(tune_cache_mutex());
    tune_cache()[key] = bestS;
}

// the passes the autotuner times, in order: f(T{}, d, kind, dinv) for the
// FP64 (T = double) or FP32 (T = float) copy of each operator the V-cycle
// and the Krylov method run
template <int M, class F>
void for_each_tuned_pass(Handle& h, F&& f)
{
    const bool mixed = h.opt.precision == XAMG_MIXED;
    const bool gs = h.opt.smoother == XAMG_GAUSS_SEIDEL;
    for (int l = 0; l < h.nlev; ++l) {
        auto& L = h.lev[l];
        const bool last = l + 1 == h.nlev;
        if (l == 0 || !mixed) {
            f(double{}, L.A64, 0, L.dinv64);
            if (!last && !mixed) f(double{}, L.A64, 2, gs ? L.dl1inv64 : L.dinv64);
        }
        if (!last) {
            if (!mixed) {
                f(double{}, L.P64, 3, L.dinv64);
                f(double{}, L.R64, 1, L.dinv64);
            } else {
                f(float{}, L.A32, 0, L.dinv32);
                f(float{}, L.A32, 2, gs ? L.dl1inv32 : L.dinv32);
                f(float{}, L.P32, 3, L.dinv32);
                f(float{}, L.R32, 1, L.dinv32);
            }
        }
    }
}

template <int M>
void autotune(Handle& h)
{
    constexpr int k = M == 1 ? 0 : M == 2 ? 1 : M == 4 ? 2 : M == 8 ? 3 : M == 16 ? 4 : 5;
    if (h.tuned_mask & (1u << k)) return;
    const int n0 = h.lev[0].n;
    // scratch: the Krylov r and z blocks (n0 x mcap doubles), zero-filled
    hipLaunchKernelGGL((copy_cols_kernel<double, double>), dim3(1024), dim3(256), 0, h.stream,
                       nullptr, M, h.w.r, M, n0, 0);
    // the timing events, released however the tuning ends (a device error
    // throws out of it)
    struct Events {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Events()
        {
            for (hipEvent_t ev : e)
                if (ev) hipEventDestroy(ev);
        }
    } ev;
    h.check(hipEventCreate(&ev.e[0]), "hipEventCreate");
    h.check(hipEventCreate(&ev.e[1]), "hipEventCreate");
    double* z = h.w.p;   // right-hand side of the residual pass (finite: zeroed)
    hipLaunchKernelGGL((copy_cols_kernel<double, double>), dim3(1024), dim3(256), 0, h.stream,
                       nullptr, M, z, M, n0, 0);
    for_each_tuned_pass<M>(h, [&](auto tag, DCsr& d, int kind, const auto* dinv) {
        using T = decltype(tag);
        tune_matrix<M, T>(h, d, kind, dinv, reinterpret_cast<T*>(h.w.r),
                          reinterpret_cast<T*>(h.w.z), reinterpret_cast<T*>(z), ev.e[0], ev.e[1]);
    });
    h.tuned_mask |= 1u << k;
    h.tune_epoch += 1;
}

// For a handle not yet tuned for M: the choices the tuning cache holds for
// its passes, applied without timing, launching or touching work memory
// (passes without a cached choice keep their current shape).  The
// allocation-free solve calls it.
template <int M>
void apply_cached_tuning(Handle& h)
{
    constexpr int k = M == 1 ? 0 : M == 2 ? 1 : M == 4 ? 2 : M == 8 ? 3 : M == 16 ? 4 : 5;
    if (!h.autotune || (h.tuned_mask & (1u << k))) return;
    bool changed = false;
    for_each_tuned_pass<M>(h, [&](auto tag, DCsr& d, int kind, const auto*) {
        using T = decltype(tag);
        changed |= tuned_pass(h, d, kind) && cached_choice<M, T>(h, d, kind);
    });
    if (changed) h.tune_epoch += 1;
}

}  // namespace xamg
