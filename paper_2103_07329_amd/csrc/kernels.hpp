// kernels.hpp -- gfx950 kernels of the multi-RHS AMG-Krylov solve phase.
//
// Every hot operation of the solve is a pass over the rows of one CSR
// operator with the m right-hand sides interleaved (x[i*M + j]), so that a
// matrix entry is loaded once and applied to all M columns (the "blas2"
// multi-RHS SpMV of the paper, Sections 2.2-2.3).  One generic kernel,
// rows_kernel<M, CPT, Op>, covers them all:
//
//   * G = M / CPT lanes of a 64-wide wavefront share a row; each lane owns
//     CPT consecutive columns and gathers them with one vector load per
//     nonzero, so a row's M columns are one contiguous, coalesced segment;
//   * the op supplies the gathered input (x itself, or a value computed on
//     the fly from b and D^-1 so smoothers from a zero guess need no extra
//     pass), and the epilogue that turns the row sums into outputs (residual,
//     Jacobi / Chebyshev updates, prolongation add, ...);
//   * per-column dot products of the epilogue are reduced in the block in a
//     fixed tree order and written as one partial per block; a one-block
//     finalize kernel adds the partials in block order (deterministic) and
//     updates the Krylov scalars on the device.
//
// Tiles of rows are taken in block order, so the device works on one
// contiguous window of rows at a time and the x rows that neighbouring rows
// share are reused from L2 or the memory-side cache.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace xamg {
namespace dev {

constexpr int kBlock = 256;      // threads per block of the row kernels (default)
constexpr int kMaxBlock = 512;   // the larger block a launch may take instead
constexpr int kMaxDots = 5;      // dots per kernel
constexpr int kNumXcd = 8;
constexpr int kUnroll = 8;      // nonzeros per batch in the row loop

// ---------------------------------------------------------------------------
// vector loads/stores of CPT consecutive elements
// ---------------------------------------------------------------------------
// (aligned to its size up to 16 bytes: a 32-byte pack is two 16-byte loads,
// and the ABI promises callers' blocks 16-byte alignment only)
template <typename T, int N>
struct alignas(sizeof(T) * N > 16 ? 16 : sizeof(T) * N) Pack {
    T v[N];
};

template <typename T, int N>
__device__ __forceinline__ Pack<T, N> load_pack(const T* p)
{
    return *reinterpret_cast<const Pack<T, N>*>(p);
}

template <typename T, int N>
__device__ __forceinline__ void store_pack(T* p, const Pack<T, N>& x)
{
    *reinterpret_cast<Pack<T, N>*>(p) = x;
}

// ---------------------------------------------------------------------------
// column index decoders
// ---------------------------------------------------------------------------
// plain 32-bit CSR columns
struct Idx32 {
    const int* ci;
    __device__ __forceinline__ void row_begin(int) {}
    __device__ __forceinline__ int col(int k) const { return ci[k]; }
};

// 16-bit compressed columns: rows are grouped in blocks of kIdxRows; each
// block stores up to 4 int32 bases (int4: x, y, z, w; w < 0 marks a block
// kept in 32 bits).  A compressed entry is (window << 14) | offset with
// column = base[window] + offset, offset < 2^14.
constexpr int kIdxRows = 64;
struct Idx16 {
    const uint16_t* off;
    const int* ci;          // 32-bit fallback (full array)
    const int4* base;
    int b0, b1, b2, b3;
    bool wide;
    __device__ __forceinline__ void row_begin(int i)
    {
        const int4 b = base[i / kIdxRows];
        b0 = b.x; b1 = b.y; b2 = b.z; b3 = b.w;
        wide = b3 < 0;
    }
    __device__ __forceinline__ int col(int k) const
    {
        if (wide) return ci[k];
        const unsigned e = off[k];
        const unsigned w = e >> 14;
        const int o = int(e & 0x3fffu);
        const int b = (w == 0) ? b0 : (w == 1) ? b1 : (w == 2) ? b2 : b3;
        return b + o;
    }
};

// ---------------------------------------------------------------------------
// value of lane K of the caller's group of G consecutive lanes (groups
// aligned to G): DPP quad permutes for G = 2, 4 (vector ALU moves), a
// bit-mode swizzle for G = 8, 16 (the source lane (l & ~(G-1)) | K within
// each 32-lane half is encoded in the instruction, so no address register
// is held per broadcast), a shuffle for G = 32, 64
// ---------------------------------------------------------------------------
template <int G, int K>
__device__ __forceinline__ int grp_bcast(int v)
{
    if constexpr (G == 4)
        return __builtin_amdgcn_mov_dpp(v, K | (K << 2) | (K << 4) | (K << 6), 0xF, 0xF, false);
    else if constexpr (G == 2)
        return __builtin_amdgcn_mov_dpp(v, K | (K << 2) | ((K + 2) << 4) | ((K + 2) << 6), 0xF,
                                        0xF, false);
    else if constexpr (G == 8 || G == 16)
        return __builtin_amdgcn_ds_swizzle(v, (0x1f & ~(G - 1)) | (K << 5));
    else
        return __shfl(v, ((threadIdx.x & 63) & ~(G - 1)) + K, 64);
}

template <int G, int K>
__device__ __forceinline__ float grp_bcast(float v)
{
    return __int_as_float(grp_bcast<G, K>(__float_as_int(v)));
}

template <int G, int K>
__device__ __forceinline__ double grp_bcast(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = grp_bcast<G, K>(int(b & 0xffffffffLL));
    const int hi = grp_bcast<G, K>(int(b >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                static_cast<long long>(static_cast<unsigned>(lo)));
}

// out[u] = entry u of a batch, from the entries each lane of the group
// loaded (lane g holds entries g, g + G, ...)
template <int G, int U, int PL, typename V, int u = 0>
__device__ __forceinline__ void grp_share(const V (&own)[PL], V (&out)[U])
{
    if constexpr (u < U) {
        out[u] = grp_bcast<G, u % G>(own[u / G]);
        grp_share<G, U, PL, V, u + 1>(own, out);
    }
}

// ---------------------------------------------------------------------------
// block-level deterministic reduction of per-column dots
// ---------------------------------------------------------------------------
template <int M, int CPT, int ND>
__device__ __forceinline__ void reduce_dots(double (&d)[ND > 0 ? ND : 1][CPT],
                                            double* __restrict__ part, int blk)
{
    if constexpr (ND > 0) {
        constexpr int G = M / CPT;
        const int RPB = int(blockDim.x) / G;
        __shared__ double sh[ND * (kMaxBlock / G) * M];
        const int g = threadIdx.x % G, rl = threadIdx.x / G;
#pragma unroll
        for (int q = 0; q < ND; ++q)
#pragma unroll
            for (int c = 0; c < CPT; ++c) sh[(q * RPB + rl) * M + g * CPT + c] = d[q][c];
        __syncthreads();
#pragma unroll
        for (int s = RPB / 2; s >= 1; s >>= 1) {
            if (rl < s) {
#pragma unroll
                for (int q = 0; q < ND; ++q)
#pragma unroll
                    for (int c = 0; c < CPT; ++c)
                        sh[(q * RPB + rl) * M + g * CPT + c] +=
                            sh[(q * RPB + rl + s) * M + g * CPT + c];
            }
            __syncthreads();
        }
        if (threadIdx.x < ND * M) {
            const int q = threadIdx.x / M, j = threadIdx.x % M;
            part[size_t(blk) * (ND * M) + threadIdx.x] = sh[(q * RPB) * M + j];
        }
    }
}

// ---------------------------------------------------------------------------
// the generic row kernel
// ---------------------------------------------------------------------------
// Op interface:
//   using MT (matrix value type), AT (accumulator type), Idx (decoder)
//   static constexpr bool kMatrix  -- false: pure row-wise vector op
//   static constexpr int kDots     -- per-column dots produced (0..2)
//   const int* rp; const MT* val; Idx idx;
//   Pack<AT, CPT> fetch(int c, int j0)   the gathered input in(c, j0..j0+CPT)
//   void out(int i, int j0, const AT (&acc)[CPT], double (&d)[ND][CPT])
//   bool active_any()   -- false: whole op is a no-op (every column frozen)
// ops that read per-column coefficients (Krylov alpha, beta, flags) load
// them once per thread in begin(j0) instead of once per row
template <class T, class = void>
struct op_has_begin : std::false_type {};
template <class T>
struct op_has_begin<T, std::void_t<decltype(T::kBegin)>> : std::bool_constant<T::kBegin> {};

// seg > 0 (matrix passes): the banded XCD walk.  The tiles are cut into
// segments of seg tiles (a multiple of the XCD count), each segment into
// kNumXcd equal chunks; the blocks of XCD k (blocks are dealt to the XCDs
// round-robin) take chunk k of every segment, segment after segment.  With
// a segment about one bandwidth of the matrix long, a row's couplings lie
// in the same chunk of the neighbouring segments, so the vector rows they
// share are reused from the XCD's own L2.
template <int M, int CPT, int S, class Op>
__global__ __launch_bounds__(kMaxBlock) void rows_kernel(Op op_in, int nrows, double* part,
                                                         int seg)
{
    Op op = op_in;
    // G lanes share the columns of a row; S such groups split the row's
    // nonzeros (long rows of coarse levels) and combine their sums with a
    // fixed butterfly over the wavefront; U nonzeros per batch and group.
    // A block of kBlock or kMaxBlock threads holds RPB rows (a tile).
    constexpr int G = M / CPT;
    const int RPB = int(blockDim.x) / (G * S);
    constexpr int U = S == 1 ? kUnroll : (S == 2 ? kUnroll / 2 : 2);
    constexpr int ND = Op::kDots;
    static_assert(G * S <= 64, "a row must stay inside one wavefront");
    using AT = typename Op::AT;
    const int g = threadIdx.x % G;
    const int sg = (threadIdx.x / G) % S;
    const int rl = threadIdx.x / (G * S);
    const int j0 = g * CPT;
    const int blk = blockIdx.x;
    if constexpr (op_has_begin<Op>::value) op.begin(j0);
    double dsum[ND > 0 ? ND : 1][CPT];
#pragma unroll
    for (int q = 0; q < (ND > 0 ? ND : 1); ++q)
#pragma unroll
        for (int c = 0; c < CPT; ++c) dsum[q][c] = 0.0;

    if (op.active_any()) {
        // Matrix passes take tiles in block order: a launch with one block
        // per tile, or a sweep by as many blocks as the device holds at
        // once, each taking every gridDim-th tile, so the chip works on one
        // contiguous window of rows at a time and the x rows they share stay
        // in L2 or the memory-side cache between their uses (measured faster
        // than per-XCD slabs).  A sweeping row-wise vector op (pure
        // streaming) gives each XCD (blocks are dealt to the 8 XCDs
        // round-robin) a contiguous slab of tiles instead, which streams
        // faster.
        const int ntiles = (nrows + RPB - 1) / RPB;
        int tb = 0, te = ntiles, t0 = blockIdx.x, tstep = gridDim.x;
        const int xcd = blockIdx.x % kNumXcd;
        const int ct = seg / kNumXcd;   // tiles per chunk of a segment
        if (seg > 0) {
            // this XCD's visits: chunk `xcd` of every segment, in order
            te = ((ntiles + seg - 1) / seg) * ct;
            t0 = blockIdx.x / kNumXcd;
            tstep = gridDim.x / kNumXcd;
        } else if (!Op::kMatrix && gridDim.x % kNumXcd == 0 && int(gridDim.x) < ntiles) {
            const int per = (ntiles + kNumXcd - 1) / kNumXcd;
            tb = xcd * per;
            te = min(ntiles, tb + per);
            t0 = tb + blockIdx.x / kNumXcd;
            tstep = gridDim.x / kNumXcd;
        }
        for (int v = t0; v < te; v += tstep) {
            int t = v;
            if (seg > 0) {
                const int sgm = v / ct;
                t = sgm * seg + xcd * ct + (v - sgm * ct);
            }
            const int i = t * RPB + rl;
            const bool live = i < nrows;
            AT acc[CPT];
#pragma unroll
            for (int c = 0; c < CPT; ++c) acc[c] = AT(0);
            if constexpr (Op::kMatrix) {
                // nonzeros in batches of U: all column indices and values
                // first, then every gather, then the multiply-adds in
                // nonzero order (more loads in flight per lane)
                if (live) {
                    auto idx = op.idx;
                    idx.row_begin(i);
                    const int kb = op.rowlen ? i * op.rowlen : op.rp[i];
                    const int ke = op.rowlen ? kb + op.rowlen : op.rp[i + 1];
                    for (int k0 = kb + sg * U; k0 < ke; k0 += S * U) {
                        int cc[U];
                        AT aa[U];
                        if constexpr (G > 1) {
                            // the G lanes of the row load every G-th entry of
                            // the batch and exchange them (fewer load
                            // instructions through the address units)
                            constexpr int PL = (U + G - 1) / G;
                            int cown[PL];
                            AT aown[PL];
#pragma unroll
                            for (int q = 0; q < PL; ++q) {
                                const int u = g + G * q;
                                const int k = k0 + u;
                                const bool ok = u < U && k < ke;
                                cown[q] = ok ? idx.col(k) : -1;
                                aown[q] = ok ? AT(op.val[k]) : AT(0);
                            }
                            grp_share<G, U, PL, int>(cown, cc);
                            grp_share<G, U, PL, AT>(aown, aa);
                        } else {
#pragma unroll
                            for (int u = 0; u < U; ++u) {
                                const int k = k0 + u;
                                cc[u] = k < ke ? idx.col(k) : -1;
                                aa[u] = k < ke ? AT(op.val[k]) : AT(0);
                            }
                        }
                        // padding entries (past the row's end) keep a zero
                        // gathered value and a zero coefficient, so the
                        // multiply-adds below need no per-entry condition
                        // (a conditional update costs selects and registers)
                        Pack<AT, CPT> vv[U];
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            vv[u] = Pack<AT, CPT>{};
                            if (cc[u] >= 0) vv[u] = op.fetch(cc[u], j0);
                        }
#pragma unroll
                        for (int u = 0; u < U; ++u)
#pragma unroll
                            for (int c = 0; c < CPT; ++c) acc[c] += aa[u] * vv[u].v[c];
                    }
                }
                if constexpr (S > 1) {
#pragma unroll
                    for (int off = G; off < G * S; off <<= 1)
#pragma unroll
                        for (int c = 0; c < CPT; ++c) acc[c] += __shfl_xor(acc[c], off, 64);
                }
            }
            if (live && sg == 0) op.out(i, j0, acc, dsum);
        }
    }
    reduce_dots<M, CPT, ND>(dsum, part, blk);
}

// ---------------------------------------------------------------------------
// finalize: sum block partials in block order, then a per-column functor
// ---------------------------------------------------------------------------
constexpr int kFinThreads = 1024;

// npair <= kMaxDots * 32 partial sums per block; thread t takes pair t % P and slice
// t / P (P = npair rounded up to a power of two), sums the blocks of its
// slice in increasing order (8 loads in flight), then the slices are
// combined by a fixed tree in LDS.
template <class Fin>
__global__ __launch_bounds__(kFinThreads) void finalize_kernel(const double* __restrict__ part,
                                                               int nb, int npair, Fin fin)
{
    __shared__ double red[kFinThreads];
    __shared__ double tot[kMaxDots * 32];
    int P = 1;
    while (P < npair) P <<= 1;
    const int nsl = kFinThreads / P;
    const int p = threadIdx.x % P, s = threadIdx.x / P;
    double acc = 0.0;
    if (p < npair) {
        for (int b0 = s; b0 < nb; b0 += 8 * nsl) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int b = b0 + u * nsl;
                v[u] = b < nb ? part[size_t(b) * npair + p] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += v[u];
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = nsl / 2; h >= 1; h >>= 1) {
        if (s < h) red[threadIdx.x] += red[threadIdx.x + h * P];
        __syncthreads();
    }
    if (threadIdx.x < kMaxDots * 32) tot[threadIdx.x] = threadIdx.x < npair ? red[threadIdx.x] : 0.0;
    __syncthreads();
    fin(tot);
}

}  // namespace dev
}  // namespace xamg
