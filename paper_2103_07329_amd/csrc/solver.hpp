// solver.hpp -- device-side handle and launch helpers shared by the solver
// translation units of libxamg (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "internal.h"
#include "kernels.hpp"
#include "ops.hpp"

struct xamg_handle {};   // opaque ABI tag; the real object is xamg::Handle

namespace xamg {

struct DevFail {
    int code;
};

// device CSR (values FP64 or FP32; optional 16-bit index encoding)
struct DCsr {
    int nr = 0, nc = 0;
    int64_t nnz = 0;
    int bw = 0;   // bandwidth max |j - i| of a square operator (0: rectangular)
    // > 0: stored with exactly rowlen entries per row (shorter rows padded
    // with explicit zeros at unused columns), so row i starts at i * rowlen
    int rowlen = 0;
    int* rp = nullptr;
    int* ci = nullptr;
    void* v = nullptr;
    // values scaled by the inverse diagonal of their column (a_ij / a_jj,
    // i.e. A D^-1) for the Jacobi / Chebyshev pre-smoothing pass from zero;
    // same type as v; null where no such pass runs
    void* vd = nullptr;
    bool fp32 = false;
    uint16_t* off = nullptr;
    int4* base = nullptr;
    // lane groups per row (1, 2, 4 or 8, plus kSweep for a sweeping launch)
    // for each column count M = 2^k, k = 0..5: a mean-row-length guess at
    // upload, replaced by the autotuner's measured choice
    int split[6] = {1, 1, 1, 1, 1, 1};
    // the same for the pre-smoothing pass of a square operator, which
    // gathers b and D^-1 instead of x and is tuned on its own
    int split_pre[6] = {1, 1, 1, 1, 1, 1};
    template <int M>
    int split_of() const
    {
        return split[M == 1 ? 0 : M == 2 ? 1 : M == 4 ? 2 : M == 8 ? 3 : M == 16 ? 4 : 5];
    }
    template <int M>
    int split_pre_of() const
    {
        return split_pre[M == 1 ? 0 : M == 2 ? 1 : M == 4 ? 2 : M == 8 ? 3 : M == 16 ? 4 : 5];
    }
};

// a square CSR operator padded to one row length (host copy for the upload)
struct UniformCsr {
    int rowlen = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> v;
    xamg_csr_t view{};
};
bool pad_uniform(const xamg_csr_t& c, UniformCsr& u);

struct LevelDev {
    int n = 0;
    double lmax = 0.0;
    DCsr A64, P64, R64;      // FP64 operators (the Krylov level uses A64 of level 0)
    DCsr A32, P32, R32;      // FP32 copies for a mixed-precision preconditioner
    double* dinv64 = nullptr;
    float* dinv32 = nullptr;
    double* dl1inv64 = nullptr;   // 1 / l1 diagonal of the Gauss-Seidel blocks
    float* dl1inv32 = nullptr;
    double frac16[3] = {0, 0, 0};   // fraction of A/P/R nonzeros in 16-bit form
};

struct LevelWork {
    void* B = nullptr;   // right-hand side of the level (l >= 1)
    void* X = nullptr;   // pre-smoothed + corrected iterate
    void* X2 = nullptr;  // post-smoothed output (l >= 1)
    void* R = nullptr;   // residual
    void* T = nullptr;   // Chebyshev temporary
};

struct Work {
    int mcap = 0;
    std::vector<LevelWork> lev;
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *t = nullptr;
    double* p2 = nullptr;   // merged CG form 2: the second p buffer (ColState::ppar)
    // pipelined BiCGStab: rt = M r, w = K r, wh = M w, y = K q, zh = M z, qh = M q
    double *rt = nullptr, *pw = nullptr, *wh = nullptr, *y = nullptr, *zh = nullptr,
           *qh = nullptr;
    double *rh = nullptr, *v = nullptr, *s = nullptr, *ph = nullptr, *sh = nullptr;
    double *bpad = nullptr, *xpad = nullptr;
    // FP32 copies of the finest-level inputs of a mixed V-cycle (Jacobi or
    // Chebyshev smoother): r for CG, kept equal to float(r) wherever r
    // changes; p and s for BiCGStab, written by the passes that form them
    float* r32 = nullptr;
    float *p32 = nullptr, *s32 = nullptr;
};

struct Handle : xamg_handle {
    int nlev = 0;
    std::vector<LevelDev> lev;
    double* inv64 = nullptr;
    float* inv32 = nullptr;
    xamg_options_t opt{};
    hipStream_t stream = nullptr;
    Work w;
    Work w_na;   // work of xamg_solve_noalloc: slices of the scratch array (lev sized at setup)
    dev::ColState* st = nullptr;
    dev::ColState* st_host = nullptr;
    double* part = nullptr;
    int nb_cap = 1024;
    int num_cu = 256;            // compute units of the device (sizes sweeping launches)
    int device = 0;              // the device the handle was set up on
    std::vector<void*> allocs;
    int autotune = 1;            // tune row splits on the first solve per M
    unsigned tuned_mask = 0;     // bit k: M = 2^k tuned
    bool tune_fresh = false;     // time every choice again (not from the tuning cache)
    int tune_epoch = 0;          // bumped whenever launch shapes may change
    // kernel timer (measurement only)
    int timer_kind = 0;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    double timer_ms = 0.0;
    int64_t timer_count = 0;
    void timer_begin(int kind);
    void timer_end(int kind);
    void timer_collect();

    ~Handle();
    void check(hipError_t e, const char* what);
    void* alloc_bytes(size_t bytes);
    template <typename T>
    T* alloc(size_t n) { return static_cast<T*>(alloc_bytes(n * sizeof(T))); }
    void release(void* p);
};

// ---- launch helpers -------------------------------------------------------
template <typename T, int M>
constexpr int cpt_for()
{
    // 16 bytes of the row's columns per lane (one dwordx4 load per gathered
    // nonzero): the lanes of a row then read each 64-byte piece of it with
    // a single load instruction, which measured faster than 32 bytes per
    // lane in two loads (fewer cache lines per instruction)
    if constexpr (sizeof(T) == 8) return M >= 2 ? 2 : M;
    else return M >= 4 ? 4 : M;
}

// groups of lanes that split one row's nonzeros, from the mean row length
inline int split_for(int64_t nnz, int nrows)
{
    const double avg = nrows > 0 ? double(nnz) / nrows : 0.0;
    return avg > 48.0 ? 8 : (avg > 24.0 ? 4 : 1);
}

// A launch shape ("row split" value): S (1, 2, 4 or 8 lane groups per row)
// plus the flags below, chosen per operator and pass by the autotuner.
//   kSweep: at most `cap` blocks (no more than the device holds at once)
//           sweep the tiles instead of one block per tile;
//   kBig:   blocks of kMaxBlock threads (tiles of twice the rows);
//   kIdx32: an operator that also has 16-bit column offsets is read through
//           its 32-bit indices;
//   kWide:  each lane takes twice the default columns (32 instead of 16
//           bytes of the row's columns per gathered nonzero).
//   kSeg*:  (two bits) the banded XCD walk of rows_kernel with segments of
//           the operator's bandwidth (kSegBw), half (kSegHalf) or a quarter
//           (kSegQuarter) of it.
constexpr int kSweep = 16;
constexpr int kBig = 32;
constexpr int kIdx32 = 64;
constexpr int kWide = 128;
constexpr int kSegShift = 8;
constexpr int kSegMask = 3 << kSegShift;
constexpr int kSegBw = 1 << kSegShift, kSegHalf = 2 << kSegShift, kSegQuarter = 3 << kSegShift;
constexpr int kShapeFlags = kSweep | kBig | kIdx32 | kWide | kSegMask;
constexpr int kSweepPerCu = 5;
// coarsest level sizes: up to kCoarseLds rows its dense inverse is applied
// from LDS, up to kMaxCoarse rows from global memory
constexpr int kCoarseLds = 64;
constexpr int kMaxCoarse = 1024;

// blocks of rows_kernel<M, CPT, S, Op> of `block` threads that the device
// holds at once (its occupancy, from the kernel's registers and LDS, times
// the CU count)
template <int M, int CPT, int S, class Op>
int resident_blocks(const Handle& h, int block)
{
    static int per_cu[2] = {0, 0};
    int& b = per_cu[block == dev::kMaxBlock ? 1 : 0];
    if (b == 0) {
        int v = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, dev::rows_kernel<M, CPT, S, Op>,
                                                         block, 0) != hipSuccess)
            v = 1;
        b = std::max(1, v);
    }
    return b * h.num_cu;
}

template <int M, int CPT, int S, class Op>
int launch_rows_s(Handle& h, const Op& op, int nrows, int cap, bool sweep = false,
                  int block = dev::kBlock, int seg_rows = 0)
{
    constexpr int G = M / CPT;
    const int RPB = block / (G * S);
    const int ntiles = (nrows + RPB - 1) / RPB;
    // banded XCD walk: segments of seg_rows rows, in tiles, rounded up to a
    // multiple of the XCD count; off for operators of fewer than 4 segments
    int seg = 0;
    if (seg_rows > 0) {
        seg = (seg_rows + RPB - 1) / RPB;
        seg = (seg + dev::kNumXcd - 1) / dev::kNumXcd * dev::kNumXcd;
        if (ntiles < 4 * seg) seg = 0;
    }
    // one tile per block, unless the kernel has dot products (at most `cap`
    // blocks so their partial sums stay few) or the operator sweeps; a
    // sweeping grid is no larger than what the device holds at once, so
    // every block starts in the first round and none waits for a free slot,
    // and a matrix pass has at most kSweepPerCu blocks per CU (the window of
    // rows the sweep works on at a time; measured best on 7- and 19-point
    // rows whatever the occupancy; streaming vector ops use every slot)
    const bool capped = Op::kDots > 0 || sweep;
    // one block per visit (a banded walk pads each segment to whole chunks)
    int nb = seg > 0 ? (ntiles + seg - 1) / seg * seg : ntiles;
    if (capped) {
        int res = resident_blocks<M, CPT, S, Op>(h, block);
        using Twin = typename dev::grid_twin<Op>::type;
        if constexpr (!std::is_void_v<Twin>)
            res = std::min(res, resident_blocks<M, CPT, S, Twin>(h, block));
        nb = std::min({ntiles, cap, res,
                       Op::kMatrix ? kSweepPerCu * h.num_cu * dev::kBlock / block : ntiles});
    }
    nb = std::max(1, nb);
    if (capped && nb >= dev::kNumXcd) nb -= nb % dev::kNumXcd;   // even over the 8 XCDs
    if (seg > 0 && nb < dev::kNumXcd) seg = 0;                   // the walk needs every XCD
    hipLaunchKernelGGL((dev::rows_kernel<M, CPT, S, Op>), dim3(nb), dim3(block), 0, h.stream, op,
                       nrows, h.part, seg);
    return nb;
}

// row-wise vector operation (no matrix)
template <int M, int CPT, class Op>
int launch_rows(Handle& h, const Op& op, int nrows, int cap)
{
    return launch_rows_s<M, CPT, 1>(h, op, nrows, cap);
}

// operation over the rows of matrix d, with d's launch shape (see kSweep)
// (bw: the operator's bandwidth max |j - i|, for the banded XCD walk)
template <int M, int CPT, class Op>
int launch_mat(Handle& h, const Op& op, int split, int nrows, int cap, int bw = 0)
{
    constexpr int G = M / CPT;
    const bool sweep = (split & kSweep) != 0;
    const int block = (split & kBig) ? dev::kMaxBlock : dev::kBlock;
    const int sm = (split & kSegMask) >> kSegShift;
    const int seg_rows = (sm == 0 || bw <= 0) ? 0 : bw >> (sm - 1);
    const int s = split & (kSweep - 1);
    if constexpr (G * 8 <= 64) {
        if (s >= 8) return launch_rows_s<M, CPT, 8>(h, op, nrows, cap, sweep, block, seg_rows);
    }
    if constexpr (G * 4 <= 64) {
        if (s >= 4) return launch_rows_s<M, CPT, 4>(h, op, nrows, cap, sweep, block, seg_rows);
    }
    if constexpr (G * 2 <= 64) {
        if (s >= 2) return launch_rows_s<M, CPT, 2>(h, op, nrows, cap, sweep, block, seg_rows);
    }
    return launch_rows_s<M, CPT, 1>(h, op, nrows, cap, sweep, block, seg_rows);
}

// The op that make(cpt, ix) builds, launched with the shape `split` over
// the rows of matrix d: cpt (std::integral_constant) is the columns per
// lane -- cpt_for<T, M>(), or twice that with kWide where the row's columns
// allow it -- and ix the column-index decoder of d (its 16-bit offsets when
// it has them, unless kIdx32).
// (Only FP32 copies carry 16-bit offsets: MT is d's value type.)
template <int M, typename T, typename MT, class Make>
int launch_op(Handle& h, const DCsr& d, int split, int nrows, int cap, Make&& make)
{
    constexpr int C0 = cpt_for<T, M>();
    auto go = [&](auto cpt) {
        constexpr int CPT = decltype(cpt)::value;
        if constexpr (sizeof(MT) == 4) {
            if (d.off && !(split & kIdx32)) {
                dev::Idx16 ix;
                ix.off = d.off;
                ix.ci = d.ci;
                ix.base = d.base;
                auto op = make(cpt, ix);
                op.rowlen = d.rowlen;
                return launch_mat<M, CPT>(h, op, split, nrows, cap, d.bw);
            }
        }
        auto op = make(cpt, dev::Idx32{d.ci});
        op.rowlen = d.rowlen;
        return launch_mat<M, CPT>(h, op, split, nrows, cap, d.bw);
    };
    if constexpr (2 * C0 <= M) {
        if (split & kWide) return go(std::integral_constant<int, 2 * C0>{});
    }
    return go(std::integral_constant<int, C0>{});
}

template <class Fin>
void launch_fin(Handle& h, int nb, int npair, const Fin& f)
{
    hipLaunchKernelGGL((dev::finalize_kernel<Fin>), dim3(1), dim3(dev::kFinThreads), 0, h.stream,
                       h.part, nb, npair, f);
}

__device__ __forceinline__ void recount_active(dev::ColState* st, int M)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        int c = 0;
        double w = 0.0;
        for (int j = 0; j < M; ++j) {
            c += st->active[j];
            if (st->active[j]) w = fmax(w, st->relres[j]);
        }
        st->nactive = c;
        st->worst = w;
    }
}

// When the host next reads the solve's progress (16 bytes: active columns
// and the largest active relative residual).  every > 0: a fixed period.
// every == 0: predicted from the observed decay of the largest residual,
// assumed geometric, so that the read falls on the iteration where it
// should pass tol; never more than 16 iterations ahead.
struct PollPlan {
    int every = 0;
    int last_it = 0;
    double last_worst = 0.0;
    int next_after(int it, double worst, double tol)
    {
        if (every > 0) return it + every;
        int step = 1;
        if (last_it > 0 && last_worst > 0.0 && worst > 0.0 && worst < last_worst && tol > 0.0 &&
            worst > tol) {
            const double rate = std::log(worst / last_worst) / double(it - last_it);
            const double need = std::log(tol / worst) / rate;
            if (need > 1.0) step = int(std::min(16.0, std::ceil(need)));
        }
        last_it = it;
        last_worst = worst;
        return it + step;
    }
};

// ---- solver entry points (explicitly instantiated for M = 1..32) ----------
template <int M>
int vcycle(Handle& h, const double* r, double* z, int ndots, const double* q,
           const float* r32 = nullptr);
template <int M>
int pcg(Handle& h, const double* B, double* X, double tol);
template <int M>
int bicgstab(Handle& h, const double* B, double* X, double tol);
template <int M>
int pbicgstab(Handle& h, const double* B, double* X, double tol);
template <int M>
int mg_solve(Handle& h, const double* B, double* X, double tol);
template <int M>
void spmm64(Handle& h, const DCsr& d, const double* X, double* Y);
// the CG driver in enqueue-only pieces (no host synchronisation inside), for
// the batched solver's graph capture
template <int M>
void pcg_start(Handle& h, const double* B, double* X, double tol);
template <int M>
void pcg_iteration(Handle& h, double* X);
template <int M>
void pcg_true_enqueue(Handle& h, const double* B, double* X, int allow_restart);
template <int M>
int pcg_true_finish(Handle& h);
// time each operator's SpMM over the row splits and keep the fastest
template <int M>
void autotune(Handle& h);
// the tuning cache's choices for a handle not yet tuned for M, no timing
template <int M>
void apply_cached_tuning(Handle& h);

void ensure_work(Handle& h, int mp, bool bicg);
// the BiCGStab work vectors (r-hat, v, s, p-hat, s-hat) are needed
inline bool bicg_like(const xamg_options_t& o)
{
    return o.method == XAMG_BICGSTAB || o.method == XAMG_PBICGSTAB;
}
// Lay the work buffers of mp columns (plus the padding copies of B and X
// when pad) out in the region base[0, cap): fills w (whose lev must hold
// nlev entries) when the region is large enough; returns the bytes needed.
size_t carve_work(const Handle& h, int mp, bool bicg, bool pad, Work& w, char* base,
                  size_t cap);
void sync_state(Handle& h);
// copy the 16 polled bytes of the column state to the host and wait
void poll_state(Handle& h);
int padded_m(int m);
int solve_impl(Handle& h, const double* B, double* X, int m, double tol, xamg_stats_t* stats);
int solve_run(Handle& h, const double* B, double* X, int m, double tol, xamg_stats_t* stats);

}  // namespace xamg
