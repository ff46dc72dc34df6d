// ops.hpp -- operations plugged into rows_kernel (see kernels.hpp).
//
// Naming: T = vector type of the level (double, or float for a reduced-
// precision preconditioner), MT = matrix value type, BT = type of the
// right-hand side read by a smoother (double at the finest level of a
// mixed-precision cycle, where the cycle's input is the FP64 Krylov
// residual), OT = output type of the last smoothing pass (double at the
// finest level: the FP64 preconditioned residual z).
//
// Smoothers (on D^-1 A):
//   Jacobi     x <- x + w D^-1 (b - A x)
//   Chebyshev  degree 2 on [lo, hi]: with theta = (hi+lo)/2,
//              delta = (hi-lo)/2, sigma = theta/delta, rho0 = 1/sigma,
//              rho1 = 1/(2 sigma - rho0), c1 = rho1 rho0, c2 = 2 rho1/delta:
//                r0 = D^-1 (b - A x), d0 = r0/theta, x1 = x + d0,
//                r1 = r0 - D^-1 A d0, d1 = c1 d0 + c2 r1, x2 = x1 + d1
//              (Saad, Iterative Methods for Sparse Linear Systems,
//              Algorithm 12.1, two steps).
// From a zero guess the first pass needs no product with x: the
// pre-smoother gathers b itself against the column-scaled matrix A D^-1
// (stored once at setup), scales the row sum by w (Jacobi) or 1/theta
// (Chebyshev), and fuses the residual (Jacobi) or the second Chebyshev step
// into the same pass over A.
#pragma once

#include "kernels.hpp"

namespace xamg {
namespace dev {

// Per-column Krylov state, resident on the device (one solve at a time).
struct ColState {
    // polled by the host (the first 16 bytes): columns still iterating, the
    // restart count of the last true-residual check (-1: B not finite), and
    // the largest recurrence relative residual among the active columns
    int nactive;
    int nrestart;
    double worst;
    double bn2[32];       // ||b_j||^2
    double rz[32];        // CG: (r, z); BiCGStab: rho
    double alpha[32], beta[32], omega[32];
    double xpend[32];     // merged CG: alpha of the x += alpha p not yet applied
    double rhs[32], rhz[32];   // pipelined BiCGStab: (rh, s) and (rh, z) of the iteration
    double rr[32];        // ||r_j||^2 (recurrence)
    double relres[32];
    double true_relres[32];
    double tol;
    int active[32];       // column still iterating
    int conv[32];         // recurrence residual passed the test
    int iters[32];
    int rst[32];          // restart requested
    int pz[32];           // next p update is p = z (CG) / p = r (BiCGStab)
    int cp[32];           // copy t -> r for this column (restart)
    int brk[32];          // breakdowns in a row (BiCGStab)
    int skip[32];         // rest of this iteration skipped (BiCGStab)
    int half[32];         // converged at the half step (BiCGStab)
    int failed[32];       // stopped by a persistent breakdown
    int nrst[32];         // restarts so far (true-residual and breakdown)
    int max_iters;        // per-column iteration cap
    int ppar;             // merged CG form 2: the current p is in the second buffer
};

// ------------------------------------------------------------------------
// Y = A X  (optionally dot (X_i, Y_i) per column: the Krylov (p, A p))
// ------------------------------------------------------------------------
template <int M, int CPT, typename MT, typename T, class IdxT, int DOT>
struct OpAx {
    using AT = MT;
    static constexpr bool kMatrix = true;
    static constexpr int kDots = DOT;
    const int* rp;
    const MT* val;
    IdxT idx;
    const T* x;
    T* y;
    const int* nactive;   // may be null: always active
    __device__ __forceinline__ bool active_any() const { return !nactive || *nactive > 0; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int c, int j0) const
    {
        const auto v = load_pack<T, CPT>(x + size_t(c) * M + j0);
        Pack<AT, CPT> r;
#pragma unroll
        for (int t = 0; t < CPT; ++t) r.v[t] = AT(v.v[t]);
        return r;
    }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&acc)[CPT],
                                        double (&d)[ND][CPT]) const
    {
        Pack<T, CPT> o;
#pragma unroll
        for (int t = 0; t < CPT; ++t) o.v[t] = T(acc[t]);
        store_pack<T, CPT>(y + size_t(i) * M + j0, o);
        if constexpr (DOT > 0) {
            const auto xl = load_pack<T, CPT>(x + size_t(i) * M + j0);
#pragma unroll
            for (int t = 0; t < CPT; ++t) d[0][t] += double(AT(xl.v[t])) * double(o.v[t]);
        }
    }
    // > 0: every row holds exactly rowlen entries, row i at i * rowlen (no row
    // pointers are read); 0: CSR row pointers
    int rowlen = 0;
};

// ------------------------------------------------------------------------
// x_fine += P x_coarse
// ------------------------------------------------------------------------
template <int M, int CPT, typename MT, typename T, class IdxT>
struct OpProlongAdd {
    using AT = MT;
    static constexpr bool kMatrix = true;
    static constexpr int kDots = 0;
    const int* rp;
    const MT* val;
    IdxT idx;
    const T* xc;
    T* xf;
    const int* nactive;
    __device__ __forceinline__ bool active_any() const { return !nactive || *nactive > 0; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int c, int j0) const
    {
        const auto v = load_pack<T, CPT>(xc + size_t(c) * M + j0);
        Pack<AT, CPT> r;
#pragma unroll
        for (int t = 0; t < CPT; ++t) r.v[t] = AT(v.v[t]);
        return r;
    }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&acc)[CPT],
                                        double (&)[ND][CPT]) const
    {
        auto o = load_pack<T, CPT>(xf + size_t(i) * M + j0);
#pragma unroll
        for (int t = 0; t < CPT; ++t) o.v[t] = T(AT(o.v[t]) + acc[t]);
        store_pack<T, CPT>(xf + size_t(i) * M + j0, o);
    }
    // > 0: every row holds exactly rowlen entries, row i at i * rowlen (no row
    // pointers are read); 0: CSR row pointers
    int rowlen = 0;
};

// ------------------------------------------------------------------------
// r = b - A x, dots (b, b) and (r, r)  (FP64 Krylov level only)
// ------------------------------------------------------------------------
template <int M, int CPT, typename MT, typename T, typename BT, class IdxT, int ND_>
struct OpResid {
    using AT = MT;
    static constexpr bool kMatrix = true;
    static constexpr int kDots = ND_;
    const int* rp;
    const MT* val;
    IdxT idx;
    const T* x;
    const BT* b;
    T* r;
    const int* nactive;
    __device__ __forceinline__ bool active_any() const { return !nactive || *nactive > 0; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int c, int j0) const
    {
        const auto v = load_pack<T, CPT>(x + size_t(c) * M + j0);
        Pack<AT, CPT> r;
#pragma unroll
        for (int t = 0; t < CPT; ++t) r.v[t] = AT(v.v[t]);
        return r;
    }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&acc)[CPT],
                                        double (&d)[ND][CPT]) const
    {
        const auto bi = load_pack<BT, CPT>(b + size_t(i) * M + j0);
        Pack<T, CPT> o;
#pragma unroll
        for (int t = 0; t < CPT; ++t) o.v[t] = T(AT(bi.v[t]) - acc[t]);
        store_pack<T, CPT>(r + size_t(i) * M + j0, o);
        if constexpr (ND_ == 2) {
#pragma unroll
            for (int t = 0; t < CPT; ++t) {
                d[0][t] += double(bi.v[t]) * double(bi.v[t]);
                d[1][t] += double(o.v[t]) * double(o.v[t]);
            }
        }
    }
    // > 0: every row holds exactly rowlen entries, row i at i * rowlen (no row
    // pointers are read); 0: CSR row pointers
    int rowlen = 0;
};

// ------------------------------------------------------------------------
// Jacobi pre-smoothing from x = 0, fused with the residual:
//   x_i = (w d_i) b_i,  r_i = b_i - sum_k a_ik (w d_k) b_k
// ------------------------------------------------------------------------
template <int M, int CPT, typename MT, typename T, typename BT, class IdxT>
struct OpJacPre {
    using AT = MT;
    static constexpr bool kMatrix = true;
    static constexpr int kDots = 0;
    const int* rp;
    const MT* val;       // column-scaled values a_ij d_j (A D^-1)
    IdxT idx;
    const MT* dinv;
    MT omega;
    const BT* b;
    T* x;
    T* r;
    const int* nactive;
    __device__ __forceinline__ bool active_any() const { return !nactive || *nactive > 0; }
    // gathers b_c; the row sum is (A D^-1 b)_i, and x = w D^-1 b gives
    // (A x)_i = w (A D^-1 b)_i
    __device__ __forceinline__ Pack<AT, CPT> fetch(int c, int j0) const
    {
        const auto v = load_pack<BT, CPT>(b + size_t(c) * M + j0);
        Pack<AT, CPT> r;
#pragma unroll
        for (int t = 0; t < CPT; ++t) r.v[t] = AT(v.v[t]);
        return r;
    }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&acc)[CPT],
                                        double (&)[ND][CPT]) const
    {
        const auto bi = load_pack<BT, CPT>(b + size_t(i) * M + j0);
        const AT wd = omega * dinv[i];
        Pack<T, CPT> xo, ro;
#pragma unroll
        for (int t = 0; t < CPT; ++t) {
            xo.v[t] = T(wd * AT(bi.v[t]));
            ro.v[t] = T(AT(bi.v[t]) - omega * acc[t]);
        }
        store_pack<T, CPT>(x + size_t(i) * M + j0, xo);
        store_pack<T, CPT>(r + size_t(i) * M + j0, ro);
    }
    // > 0: every row holds exactly rowlen entries, row i at i * rowlen (no row
    // pointers are read); 0: CSR row pointers
    int rowlen = 0;
};

// ------------------------------------------------------------------------
// Jacobi post-smoothing: xo_i = x_i + (w d_i)(b_i - (A x)_i)
// DOT >= 1: (b_i, xo_i); DOT == 2: also (q_i, xo_i)  [finest level only]
// ------------------------------------------------------------------------
template <int M, int CPT, typename MT, typename T, typename BT, typename OT, class IdxT,
          int DOT>
struct OpJacPost {
    using AT = MT;
    static constexpr bool kMatrix = true;
    static constexpr int kDots = DOT;
    const int* rp;
    const MT* val;
    IdxT idx;
    const MT* dinv;
    MT omega;
    const T* x;
    const BT* b;
    OT* xo;
    const double* q;
    const int* nactive;
    // FP64 right-hand side for the dot (b, xo) when b itself is an FP32 copy
    const double* bd = nullptr;
    __device__ __forceinline__ bool active_any() const { return !nactive || *nactive > 0; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int c, int j0) const
    {
        const auto v = load_pack<T, CPT>(x + size_t(c) * M + j0);
        Pack<AT, CPT> r;
#pragma unroll
        for (int t = 0; t < CPT; ++t) r.v[t] = AT(v.v[t]);
        return r;
    }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&acc)[CPT],
                                        double (&d)[ND][CPT]) const
    {
        const auto bi = load_pack<BT, CPT>(b + size_t(i) * M + j0);
        const auto xl = load_pack<T, CPT>(x + size_t(i) * M + j0);
        Pack<AT, CPT> xi;
#pragma unroll
        for (int t = 0; t < CPT; ++t) xi.v[t] = AT(xl.v[t]);
        const AT wd = omega * dinv[i];
        Pack<OT, CPT> o;
#pragma unroll
        for (int t = 0; t < CPT; ++t)
            o.v[t] = OT(xi.v[t] + wd * (AT(bi.v[t]) - acc[t]));
        store_pack<OT, CPT>(xo + size_t(i) * M + j0, o);
        if constexpr (DOT >= 1) {
            if (bd) {
                const auto bv = load_pack<double, CPT>(bd + size_t(i) * M + j0);
#pragma unroll
                for (int t = 0; t < CPT; ++t) d[0][t] += bv.v[t] * double(o.v[t]);
            } else {
#pragma unroll
                for (int t = 0; t < CPT; ++t) d[0][t] += double(bi.v[t]) * double(o.v[t]);
            }
        }
        if constexpr (DOT >= 2) {
            const auto qi = load_pack<double, CPT>(q + size_t(i) * M + j0);
#pragma unroll
            for (int t = 0; t < CPT; ++t) d[1][t] += qi.v[t] * double(o.v[t]);
        }
    }
    // > 0: every row holds exactly rowlen entries, row i at i * rowlen (no row
    // pointers are read); 0: CSR row pointers
    int rowlen = 0;
};

// ------------------------------------------------------------------------
// Chebyshev (degree 2) pre-smoothing from x = 0 in one pass:
//   d0_k = (d_k b_k) / theta (times a precomputed 1 / theta) gathered on the fly,
//   x_i = d0_i + (c1 d0_i + c2 (d_i b_i - d_i (A d0)_i))
// ------------------------------------------------------------------------
template <int M, int CPT, typename MT, typename T, typename BT, class IdxT>
struct OpChebPre {
    using AT = MT;
    static constexpr bool kMatrix = true;
    static constexpr int kDots = 0;
    const int* rp;
    const MT* val;       // column-scaled values a_ij d_j (A D^-1)
    IdxT idx;
    const MT* dinv;
    MT inv_theta, c1, c2;   // 1 / theta, precomputed on the host
    const BT* b;
    T* x;
    const int* nactive;
    __device__ __forceinline__ bool active_any() const { return !nactive || *nactive > 0; }
    // gathers b_c; the row sum is (A D^-1 b)_i = theta (A d0)_i with
    // d0 = D^-1 b / theta
    __device__ __forceinline__ Pack<AT, CPT> fetch(int c, int j0) const
    {
        const auto v = load_pack<BT, CPT>(b + size_t(c) * M + j0);
        Pack<AT, CPT> r;
#pragma unroll
        for (int t = 0; t < CPT; ++t) r.v[t] = AT(v.v[t]);
        return r;
    }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&acc)[CPT],
                                        double (&)[ND][CPT]) const
    {
        const auto bi = load_pack<BT, CPT>(b + size_t(i) * M + j0);
        const AT di = dinv[i];
        Pack<T, CPT> o;
#pragma unroll
        for (int t = 0; t < CPT; ++t) {
            const AT r0 = AT(bi.v[t]) * di;
            const AT d0 = r0 * inv_theta;
            const AT r1 = r0 - di * (acc[t] * inv_theta);
            const AT d1 = c1 * d0 + c2 * r1;
            o.v[t] = T(d0 + d1);
        }
        store_pack<T, CPT>(x + size_t(i) * M + j0, o);
    }
    // > 0: every row holds exactly rowlen entries, row i at i * rowlen (no row
    // pointers are read); 0: CSR row pointers
    int rowlen = 0;
};

// ------------------------------------------------------------------------
// Chebyshev post-smoothing, pass 1:  r0_i = d_i (b_i - (A x)_i)
// ------------------------------------------------------------------------
template <int M, int CPT, typename MT, typename T, typename BT, class IdxT>
struct OpChebPost1 {
    using AT = MT;
    static constexpr bool kMatrix = true;
    static constexpr int kDots = 0;
    const int* rp;
    const MT* val;
    IdxT idx;
    const MT* dinv;
    const T* x;
    const BT* b;
    T* r0;
    const int* nactive;
    __device__ __forceinline__ bool active_any() const { return !nactive || *nactive > 0; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int c, int j0) const
    {
        const auto v = load_pack<T, CPT>(x + size_t(c) * M + j0);
        Pack<AT, CPT> r;
#pragma unroll
        for (int t = 0; t < CPT; ++t) r.v[t] = AT(v.v[t]);
        return r;
    }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&acc)[CPT],
                                        double (&)[ND][CPT]) const
    {
        const auto bi = load_pack<BT, CPT>(b + size_t(i) * M + j0);
        const AT di = dinv[i];
        Pack<T, CPT> o;
#pragma unroll
        for (int t = 0; t < CPT; ++t) o.v[t] = T((AT(bi.v[t]) - acc[t]) * di);
        store_pack<T, CPT>(r0 + size_t(i) * M + j0, o);
    }
    // > 0: every row holds exactly rowlen entries, row i at i * rowlen (no row
    // pointers are read); 0: CSR row pointers
    int rowlen = 0;
};

// ------------------------------------------------------------------------
// Chebyshev post-smoothing, pass 2 (gathers d0 = r0/theta on the fly):
//   r1 = r0_i - d_i (A d0)_i, d1 = c1 d0_i + c2 r1, xo_i = (x_i + d0_i) + d1
// DOT as in OpJacPost.
// ------------------------------------------------------------------------
template <int M, int CPT, typename MT, typename T, typename BT, typename OT, class IdxT,
          int DOT>
struct OpChebPost2 {
    using AT = MT;
    static constexpr bool kMatrix = true;
    static constexpr int kDots = DOT;
    const int* rp;
    const MT* val;
    IdxT idx;
    const MT* dinv;
    MT inv_theta, c1, c2;   // 1 / theta, precomputed on the host
    const T* r0;
    const T* x;
    const BT* b;
    OT* xo;
    const double* q;
    const int* nactive;
    // FP64 right-hand side for the dot (b, xo) when b itself is an FP32 copy
    const double* bd = nullptr;
    __device__ __forceinline__ Pack<double, CPT> dot_b(int i, int j0) const
    {
        Pack<double, CPT> v;
        if (bd) {
            v = load_pack<double, CPT>(bd + size_t(i) * M + j0);
        } else {
            const auto bl = load_pack<BT, CPT>(b + size_t(i) * M + j0);
#pragma unroll
            for (int t = 0; t < CPT; ++t) v.v[t] = double(bl.v[t]);
        }
        return v;
    }
    __device__ __forceinline__ bool active_any() const { return !nactive || *nactive > 0; }
    // gathers r0 itself; the 1/theta of d0 = r0/theta is applied to the sum
    __device__ __forceinline__ Pack<AT, CPT> fetch(int c, int j0) const
    {
        const auto v = load_pack<T, CPT>(r0 + size_t(c) * M + j0);
        Pack<AT, CPT> r;
#pragma unroll
        for (int t = 0; t < CPT; ++t) r.v[t] = AT(v.v[t]);
        return r;
    }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&acc)[CPT],
                                        double (&d)[ND][CPT]) const
    {
        const auto rl = load_pack<T, CPT>(r0 + size_t(i) * M + j0);
        Pack<AT, CPT> ri;
#pragma unroll
        for (int t = 0; t < CPT; ++t) ri.v[t] = AT(rl.v[t]);
        const auto xi = load_pack<T, CPT>(x + size_t(i) * M + j0);
        const AT di = dinv[i];
        Pack<OT, CPT> o;
#pragma unroll
        for (int t = 0; t < CPT; ++t) {
            const AT d0 = ri.v[t] * inv_theta;
            const AT r1 = ri.v[t] - di * (acc[t] * inv_theta);
            const AT d1 = c1 * d0 + c2 * r1;
            o.v[t] = OT((AT(xi.v[t]) + d0) + d1);
        }
        store_pack<OT, CPT>(xo + size_t(i) * M + j0, o);
        if constexpr (DOT >= 1) {
            const auto bi = dot_b(i, j0);
#pragma unroll
            for (int t = 0; t < CPT; ++t) d[0][t] += bi.v[t] * double(o.v[t]);
        }
        if constexpr (DOT >= 2) {
            const auto qi = load_pack<double, CPT>(q + size_t(i) * M + j0);
#pragma unroll
            for (int t = 0; t < CPT; ++t) d[1][t] += qi.v[t] * double(o.v[t]);
        }
    }
    // > 0: every row holds exactly rowlen entries, row i at i * rowlen (no row
    // pointers are read); 0: CSR row pointers
    int rowlen = 0;
};

// ------------------------------------------------------------------------
// Krylov vector updates (no matrix)
// ------------------------------------------------------------------------
// CG: x += alpha p, r -= alpha q on active columns; dot (r, r).  x null
// (merged form): r only, x's update is applied later (OpUpdPX, OpAxPX)
template <int M, int CPT>
struct OpUpdXR {
    using AT = double;
    static constexpr bool kMatrix = false;
    static constexpr int kDots = 1;
    const int* rp = nullptr;
    const double* val = nullptr;
    Idx32 idx{nullptr};
    const ColState* st;
    double *x, *r;
    const double *p, *q;
    float* r32 = nullptr;   // optional FP32 copy of r (input of a mixed V-cycle)
    __device__ __forceinline__ bool active_any() const { return st->nactive > 0; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int, int) const { return Pack<AT, CPT>{}; }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&)[CPT],
                                        double (&d)[ND][CPT]) const
    {
        const size_t o = size_t(i) * M + j0;
        auto ri = load_pack<double, CPT>(r + o);
        const auto qi = load_pack<double, CPT>(q + o);
        if (x) {
            auto xi = load_pack<double, CPT>(x + o);
            const auto pi = load_pack<double, CPT>(p + o);
#pragma unroll
            for (int t = 0; t < CPT; ++t)
                if (ac_[t]) xi.v[t] = fma(al_[t], pi.v[t], xi.v[t]);
            store_pack<double, CPT>(x + o, xi);
        }
#pragma unroll
        for (int t = 0; t < CPT; ++t) {
            if (ac_[t]) ri.v[t] -= al_[t] * qi.v[t];
            d[0][t] += ri.v[t] * ri.v[t];
        }
        store_pack<double, CPT>(r + o, ri);
        if (r32) {
            Pack<float, CPT> rf;
#pragma unroll
            for (int t = 0; t < CPT; ++t) rf.v[t] = float(ri.v[t]);
            store_pack<float, CPT>(r32 + o, rf);
        }
    }
    // the lane's columns' alpha and active flag, loaded once per thread
    static constexpr bool kBegin = true;
    double al_[CPT] = {};
    int ac_[CPT] = {};
    __device__ __forceinline__ void begin(int j0)
    {
#pragma unroll
        for (int t = 0; t < CPT; ++t) {
            ac_[t] = st->active[j0 + t];
            al_[t] = st->alpha[j0 + t];
        }
    }
};

// CG: p = z + beta p (p = z when pz is set) on active columns
template <int M, int CPT>
struct OpUpdP {
    using AT = double;
    static constexpr bool kMatrix = false;
    static constexpr int kDots = 0;
    const int* rp = nullptr;
    const double* val = nullptr;
    Idx32 idx{nullptr};
    const ColState* st;
    double* p;
    const double* z;
    __device__ __forceinline__ bool active_any() const { return st->nactive > 0; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int, int) const { return Pack<AT, CPT>{}; }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&)[CPT],
                                        double (&)[ND][CPT]) const
    {
        const size_t o = size_t(i) * M + j0;
        auto pi = load_pack<double, CPT>(p + o);
        const auto zi = load_pack<double, CPT>(z + o);
#pragma unroll
        for (int t = 0; t < CPT; ++t)
            if (ac_[t]) pi.v[t] = pz_[t] ? zi.v[t] : fma(be_[t], pi.v[t], zi.v[t]);
        store_pack<double, CPT>(p + o, pi);
    }
    static constexpr bool kBegin = true;
    double be_[CPT] = {};
    int ac_[CPT] = {}, pz_[CPT] = {};
    __device__ __forceinline__ void begin(int j0)
    {
#pragma unroll
        for (int t = 0; t < CPT; ++t) {
            ac_[t] = st->active[j0 + t];
            pz_[t] = st->pz[j0 + t];
            be_[t] = st->beta[j0 + t];
        }
    }
};

// Merged CG (Section 2.1's merged formulations: vector updates regrouped
// so fewer passes read and write the vectors).  x's update of an iteration
// is postponed into the pass of the next iteration that reads the old p
// anyway; its alpha waits in ColState::xpend (FinAlpha stores it, OpFlushX
// applies what is left before a true residual).  The pass always runs, also
// with no active column, so xpend is applied exactly once; x only changes
// where xpend != 0 (p of an inactive column need not be finite).
//
// the per-column coefficients both merged passes load once per thread
template <int CPT>
struct MergedCoef {
    double be[CPT] = {}, xp[CPT] = {};
    int ac[CPT] = {}, pz[CPT] = {};
    __device__ __forceinline__ void load(const ColState* st, int j0)
    {
#pragma unroll
        for (int t = 0; t < CPT; ++t) {
            ac[t] = st->active[j0 + t];
            pz[t] = st->pz[j0 + t];
            be[t] = st->beta[j0 + t];
            xp[t] = st->xpend[j0 + t];
        }
    }
    // the new p of one row (as OpUpdP forms it)
    __device__ __forceinline__ Pack<double, CPT> pnew(const Pack<double, CPT>& z,
                                                      const Pack<double, CPT>& p) const
    {
        Pack<double, CPT> o;
#pragma unroll
        for (int t = 0; t < CPT; ++t)
            o.v[t] = ac[t] ? (pz[t] ? z.v[t] : fma(be[t], p.v[t], z.v[t])) : p.v[t];
        return o;
    }
    __device__ __forceinline__ void addx(double* x, const Pack<double, CPT>& p) const
    {
        auto xi = load_pack<double, CPT>(x);
#pragma unroll
        for (int t = 0; t < CPT; ++t)
            if (xp[t] != 0.0) xi.v[t] = fma(xp[t], p.v[t], xi.v[t]);
        store_pack<double, CPT>(x, xi);
    }
};

// merged CG, standalone pass: x += xpend p, then p = z + beta p
template <int M, int CPT>
struct OpUpdPX {
    using AT = double;
    static constexpr bool kMatrix = false;
    static constexpr int kDots = 0;
    const int* rp = nullptr;
    const double* val = nullptr;
    Idx32 idx{nullptr};
    const ColState* st;
    double *p, *x;
    const double* z;
    __device__ __forceinline__ bool active_any() const { return true; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int, int) const { return Pack<AT, CPT>{}; }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&)[CPT],
                                        double (&)[ND][CPT]) const
    {
        const size_t o = size_t(i) * M + j0;
        const auto pi = load_pack<double, CPT>(p + o);
        const auto zi = load_pack<double, CPT>(z + o);
        cf_.addx(x + o, pi);
        store_pack<double, CPT>(p + o, cf_.pnew(zi, pi));
    }
    static constexpr bool kBegin = true;
    MergedCoef<CPT> cf_;
    __device__ __forceinline__ void begin(int j0) { cf_.load(st, j0); }
};

// merged CG, in the SpMM: q = A pn with pn = z + beta p formed where A
// gathers it (from z and the old p), pn written to the other p buffer
// (other rows still gather the old one; ColState::ppar says which buffer
// holds the current p and FinAlpha flips it, so a captured graph of any
// number of iterations stays valid), x += xpend p_old; dot (pn, q)
template <int M, int CPT, class IdxT>
struct OpAxPX {
    using AT = double;
    static constexpr bool kMatrix = true;
    static constexpr int kDots = 1;
    const int* rp;
    const double* val;
    IdxT idx;
    const ColState* st;
    double *pa, *pb;   // the two p buffers
    const double* z;
    double *q, *x;
    __device__ __forceinline__ bool active_any() const { return true; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int c, int j0) const
    {
        const size_t o = size_t(c) * M + j0;
        return cf_.pnew(load_pack<double, CPT>(z + o), load_pack<double, CPT>(pin_ + o));
    }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&acc)[CPT],
                                        double (&d)[ND][CPT]) const
    {
        const size_t o = size_t(i) * M + j0;
        const auto pi = load_pack<double, CPT>(pin_ + o);
        const auto pn = cf_.pnew(load_pack<double, CPT>(z + o), pi);
        cf_.addx(x + o, pi);
        store_pack<double, CPT>(pout_ + o, pn);
        Pack<double, CPT> qo;
#pragma unroll
        for (int t = 0; t < CPT; ++t) {
            qo.v[t] = acc[t];
            d[0][t] += pn.v[t] * qo.v[t];
        }
        store_pack<double, CPT>(q + o, qo);
    }
    static constexpr bool kBegin = true;
    MergedCoef<CPT> cf_;
    const double* pin_ = nullptr;
    double* pout_ = nullptr;
    __device__ __forceinline__ void begin(int j0)
    {
        cf_.load(st, j0);
        const bool second = st->ppar != 0;
        pin_ = second ? pb : pa;
        pout_ = second ? pa : pb;
    }
    int rowlen = 0;
};

// The two Krylov SpMM kernels of CG, q = A p with the dot (p, q) and merged
// form 2's OpAxPX, are launched on one grid size, so their dots add the
// same per-block partial sums in the same order and the forms' iterates
// agree bitwise: a sweeping launch of either is capped by the occupancy of
// both (grid_twin names the other kernel's op).
template <class Op>
struct grid_twin {
    using type = void;
};
template <int M, int CPT, class IdxT>
struct grid_twin<OpAx<M, CPT, double, double, IdxT, 1>> {
    using type = OpAxPX<M, CPT, IdxT>;
};
template <int M, int CPT, class IdxT>
struct grid_twin<OpAxPX<M, CPT, IdxT>> {
    using type = OpAx<M, CPT, double, double, IdxT, 1>;
};

// merged CG: the update still pending, x += xpend p (all columns; p from
// the buffer ColState::ppar names, pb null when there is one buffer)
template <int M, int CPT>
struct OpFlushX {
    using AT = double;
    static constexpr bool kMatrix = false;
    static constexpr int kDots = 0;
    const int* rp = nullptr;
    const double* val = nullptr;
    Idx32 idx{nullptr};
    const ColState* st;
    double* x;
    const double *pa, *pb;
    __device__ __forceinline__ bool active_any() const { return true; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int, int) const { return Pack<AT, CPT>{}; }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&)[CPT],
                                        double (&)[ND][CPT]) const
    {
        const size_t o = size_t(i) * M + j0;
        cf_.addx(x + o, load_pack<double, CPT>(p_ + o));
    }
    static constexpr bool kBegin = true;
    MergedCoef<CPT> cf_;
    const double* p_ = nullptr;
    __device__ __forceinline__ void begin(int j0)
    {
        cf_.load(st, j0);
        p_ = (pb && st->ppar) ? pb : pa;
    }
};

// multigrid iteration: x += z on the active columns
template <int M, int CPT>
struct OpAddActive {
    using AT = double;
    static constexpr bool kMatrix = false;
    static constexpr int kDots = 0;
    const int* rp = nullptr;
    const double* val = nullptr;
    Idx32 idx{nullptr};
    const ColState* st;
    double* x;
    const double* z;
    __device__ __forceinline__ bool active_any() const { return st->nactive > 0; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int, int) const { return Pack<AT, CPT>{}; }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&)[CPT],
                                        double (&)[ND][CPT]) const
    {
        const size_t o = size_t(i) * M + j0;
        auto xi = load_pack<double, CPT>(x + o);
        const auto zi = load_pack<double, CPT>(z + o);
#pragma unroll
        for (int t = 0; t < CPT; ++t)
            if (ac_[t]) xi.v[t] += zi.v[t];
        store_pack<double, CPT>(x + o, xi);
    }
    static constexpr bool kBegin = true;
    int ac_[CPT] = {};
    __device__ __forceinline__ void begin(int j0)
    {
#pragma unroll
        for (int t = 0; t < CPT; ++t) ac_[t] = st->active[j0 + t];
    }
};

// columns flagged in st->cp: dst = src;  columns with b_j = 0: x = 0
template <int M, int CPT>
struct OpFixCols {
    using AT = double;
    static constexpr bool kMatrix = false;
    static constexpr int kDots = 0;
    const int* rp = nullptr;
    const double* val = nullptr;
    Idx32 idx{nullptr};
    const ColState* st;
    double* dst;        // r (restart copy)
    const double* src;  // t
    double* x;          // zeroed where b_j = 0 (may be null)
    __device__ __forceinline__ bool active_any() const { return true; }
    __device__ __forceinline__ Pack<AT, CPT> fetch(int, int) const { return Pack<AT, CPT>{}; }
    template <int ND>
    __device__ __forceinline__ void out(int i, int j0, const AT (&)[CPT],
                                        double (&)[ND][CPT]) const
    {
        const size_t o = size_t(i) * M + j0;
        if (dst) {
            auto di = load_pack<double, CPT>(dst + o);
            const auto si = load_pack<double, CPT>(src + o);
#pragma unroll
            for (int t = 0; t < CPT; ++t)
                if (st->cp[j0 + t]) di.v[t] = si.v[t];
            store_pack<double, CPT>(dst + o, di);
        }
        if (x) {
            auto xi = load_pack<double, CPT>(x + o);
#pragma unroll
            for (int t = 0; t < CPT; ++t)
                if (st->bn2[j0 + t] == 0.0) xi.v[t] = 0.0;
            store_pack<double, CPT>(x + o, xi);
        }
    }
};

// element-wise fill / cast copy between interleaved blocks with column padding
template <typename TS, typename TD>
__global__ void copy_cols_kernel(const TS* __restrict__ src, int ms, TD* __restrict__ dst,
                                 int md, int n, int mcopy)
{
    const size_t total = size_t(n) * md;
    for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += size_t(gridDim.x) * blockDim.x) {
        const size_t i = e / md;
        const int j = int(e % md);
        dst[e] = (src && j < mcopy) ? TD(src[i * ms + j]) : TD(0);
    }
}

// ------------------------------------------------------------------------
// l1-hybrid Gauss-Seidel sweep (Baker, Falgout, Kolev, Yang 2011): rows in
// blocks of BLK consecutive rows; inside a block Gauss-Seidel in row order
// (backward: reverse order), across blocks the previous iterate xo (Jacobi),
// with the l1 diagonal d_i = a_ii + sum_{j outside the block} |a_ij|:
//   xn_i = xo_i + (b_i - sum_j a_ij v_j) / d_i,
//   v_j = xn_j for the block's rows already updated in this sweep, xo_j else.
// ZERO: xo = 0 (the pre-smoothing sweep from a zero guess; no gathers).
// S lane groups (M / CPT lanes each) per block share out each row's
// nonzeros (batches of U per group, as in rows_kernel) and combine their sums
// with a fixed xor butterfly; the block's rows are processed one after the
// other.  The rows already updated are kept in LDS: every group computes the
// new values of its columns, so each lane reads back slots it has written
// itself (with the same values the other groups wrote; no barrier needed).
// xo and xn must not overlap.  Launch: kGsThreads threads per workgroup.
// ------------------------------------------------------------------------
constexpr int kGsThreads = 64;

template <int M, int CPT, int S, int BLK, bool BWD, bool ZERO, typename MT, typename XT,
          typename BT, typename OT>
__global__ __launch_bounds__(kGsThreads) void hgs_kernel(
    const int* __restrict__ rp, const int* __restrict__ ci, const MT* __restrict__ val,
    const MT* __restrict__ dl1inv, const BT* __restrict__ b, const XT* __restrict__ xo,
    OT* __restrict__ xn, int nrows, const int* nactive)
{
    constexpr int G = M / CPT;
    static_assert(G * S <= kGsThreads, "a block's lanes must fit in the workgroup");
    constexpr int NG = kGsThreads / (G * S);   // blocks of rows per workgroup
    constexpr int U = S == 1 ? 8 : (S == 2 ? 4 : 2);
    using AT = MT;
    __shared__ AT fresh[NG][BLK][M];
    if (nactive && *nactive == 0) return;
    const int g = threadIdx.x % G;
    const int sg = (threadIdx.x / G) % S;
    const int q = threadIdx.x / (G * S);
    const int j0 = g * CPT;
    const int lo = (blockIdx.x * NG + q) * BLK;
    if (lo >= nrows) return;
    const int hi = min(nrows, lo + BLK);
    for (int s = 0; s < hi - lo; ++s) {
        const int r = BWD ? hi - lo - 1 - s : s;
        const int i = lo + r;
        AT acc[CPT];
#pragma unroll
        for (int t = 0; t < CPT; ++t) acc[t] = AT(0);
        const int kb = rp[i], ke = rp[i + 1];
        for (int k0 = kb + sg * U; k0 < ke; k0 += S * U) {
            int cc[U];
            AT aa[U];
            if constexpr (G > 1) {
                // the G lanes of a group load every G-th entry and exchange them
                constexpr int PL = (U + G - 1) / G;
                int cown[PL];
                AT aown[PL];
#pragma unroll
                for (int p = 0; p < PL; ++p) {
                    const int u = g + G * p;
                    const int k = k0 + u;
                    const bool ok = u < U && k < ke;
                    cown[p] = ok ? ci[k] : -1;
                    aown[p] = ok ? AT(val[k]) : AT(0);
                }
                grp_share<G, U, PL, int>(cown, cc);
                grp_share<G, U, PL, AT>(aown, aa);
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int k = k0 + u;
                    cc[u] = k < ke ? ci[k] : -1;
                    aa[u] = k < ke ? AT(val[k]) : AT(0);
                }
            }
            Pack<AT, CPT> vv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = cc[u];
                const int rc = c - lo;
                const bool upd = c >= 0 && rc >= 0 && rc < hi - lo && (BWD ? rc > r : rc < r);
                if (upd) {
#pragma unroll
                    for (int t = 0; t < CPT; ++t) vv[u].v[t] = fresh[q][rc][j0 + t];
                } else if (!ZERO && c >= 0) {
                    const auto x = load_pack<XT, CPT>(xo + size_t(c) * M + j0);
#pragma unroll
                    for (int t = 0; t < CPT; ++t) vv[u].v[t] = AT(x.v[t]);
                } else {
#pragma unroll
                    for (int t = 0; t < CPT; ++t) vv[u].v[t] = AT(0);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int t = 0; t < CPT; ++t) acc[t] += aa[u] * vv[u].v[t];
        }
        if constexpr (S > 1) {
#pragma unroll
            for (int off = G; off < G * S; off <<= 1)
#pragma unroll
                for (int t = 0; t < CPT; ++t) acc[t] += __shfl_xor(acc[t], off, 64);
        }
        const auto bi = load_pack<BT, CPT>(b + size_t(i) * M + j0);
        const AT di = dl1inv[i];
        Pack<OT, CPT> o;
        if constexpr (ZERO) {
#pragma unroll
            for (int t = 0; t < CPT; ++t) {
                const AT v = di * (AT(bi.v[t]) - acc[t]);
                fresh[q][r][j0 + t] = v;
                o.v[t] = OT(v);
            }
        } else {
            const auto xi = load_pack<XT, CPT>(xo + size_t(i) * M + j0);
#pragma unroll
            for (int t = 0; t < CPT; ++t) {
                const AT v = AT(xi.v[t]) + di * (AT(bi.v[t]) - acc[t]);
                fresh[q][r][j0 + t] = v;
                o.v[t] = OT(v);
            }
        }
        if (sg == 0) store_pack<OT, CPT>(xn + size_t(i) * M + j0, o);
    }
}

// ------------------------------------------------------------------------
// coarsest level: x = A_L^-1 b, the inverse staged in LDS (n_L <= 64)
// ------------------------------------------------------------------------
template <int M, typename T>
__global__ __launch_bounds__(256) void coarse_kernel(const T* __restrict__ inv, int nL,
                                                     const T* __restrict__ b, T* __restrict__ x,
                                                     const int* nactive)
{
    __shared__ T sa[64 * 64];
    __shared__ T sb[64 * M];
    if (nactive && *nactive == 0) return;
    for (int e = threadIdx.x; e < nL * nL; e += blockDim.x) sa[e] = inv[e];
    for (int e = threadIdx.x; e < nL * M; e += blockDim.x) sb[e] = b[e];
    __syncthreads();
    for (int e = threadIdx.x; e < nL * M; e += blockDim.x) {
        const int i = e / M, j = e % M;
        T s = T(0);
        for (int k = 0; k < nL; ++k) s += sa[i * nL + k] * sb[k * M + j];
        x[e] = s;
    }
}

// the same product for a coarsest level too large for LDS: the inverse is
// read from global memory (it stays in L2 across cycles), one thread per
// entry of x, the sum over k in the same increasing order
template <int M, typename T>
__global__ __launch_bounds__(256) void coarse_global_kernel(const T* __restrict__ inv, int nL,
                                                            const T* __restrict__ b,
                                                            T* __restrict__ x, const int* nactive)
{
    if (nactive && *nactive == 0) return;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nL * M) return;
    const int i = e / M, j = e % M;
    const T* row = inv + size_t(i) * nL;
    T s = T(0);
    for (int k = 0; k < nL; ++k) s += row[k] * b[size_t(k) * M + j];
    x[e] = s;
}

}  // namespace dev
}  // namespace xamg
