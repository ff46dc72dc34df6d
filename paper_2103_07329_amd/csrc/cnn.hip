// cnn.hip -- learned warm start: a small bias-free 3D CNN maps a right-hand
// side b to an initial guess x0 for the solve (an extension of the
// multi-RHS solver; Section 2.4 lists an initial guess as an optional input).
//
// Network: four 3x3x3 convolutions (channels 1 -> 16 -> 16 -> 16 -> 1),
// zero padding, ReLU after the first three, no bias, so f(c b) = c f(b) for
// c > 0.  A column is normalised by s = ||b|| / sqrt(n) before the network
// and the output is multiplied by s.  Weights and activations are BF16
// (round to nearest even), accumulation FP32, master weights FP32 (Adam).
//
// Layout: volumes of N^3 voxels (r = x + N y + N^2 z), channels last:
// a[r*C + c].  Tap t = (dz+1)*9 + (dy+1)*3 + (dx+1); a layer computes
// out[r, co] = sum_t sum_ci W[co][ci][t] in[r + off(t), ci] (zero outside).
//
// Kernels: the two 16 -> 16 layers (about 94% of the flops) run on the
// v_mfma_f32_16x16x32_bf16 matrix instruction from an LDS-staged tile of the
// input: a wavefront computes rows of 16 consecutive voxels x 16 output
// channels and takes two taps (32 = 2 x 16 input channels) per instruction;
// the input gradient of these layers is the same kernel with the weights
// mirrored and transposed, plus the ReLU mask.  The 1 -> 16 and 16 -> 1
// layers are VALU kernels (BF16 dot products).  The weight gradients of the
// 16 -> 16 and 16 -> 1 layers run on the same MFMA with voxels as the
// contracted dimension, that of the 1 -> 16 layer as an LDS-staged VALU
// reduction; per-block (or per-wave) partials are summed in a fixed order
// (deterministic).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "solver.hpp"

struct xamg_cnn {};   // opaque ABI tag; the real object is xamg::cnn::Net

namespace xamg {
namespace cnn {

constexpr int kTaps = 27;
constexpr int kC = 16;                 // hidden channels
constexpr int kPairs = 14;             // tap pairs of the 1 -> 16 layer (27 -> 28)
// B fragments of a 16 -> 16 MFMA layer: for each dy, the 9 (dz, dx) taps in
// 5 pairs (the last padded with zeros), so an A fragment of input row hy
// serves every output row r with hy - r = dy + 1
constexpr int kDyPairs = 5;
constexpr int kMPairs = 3 * kDyPairs;  // 15
constexpr int kParams1 = kC * 1 * kTaps;
constexpr int kParams2 = kC * kC * kTaps;
constexpr int kParams4 = 1 * kC * kTaps;
constexpr int kParams = kParams1 + 2 * kParams2 + kParams4;   // 14688
constexpr int kColBlocks = 4096;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__host__ __device__ inline uint16_t f2bf(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

__host__ __device__ inline float bf2f(uint16_t h)
{
    const uint32_t u = uint32_t(h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

__device__ inline bool neighbour(int N, int x, int y, int z, int t, long r, long& u)
{
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    const int xx = x + dx, yy = y + dy, zz = z + dz;
    if (xx < 0 || xx >= N || yy < 0 || yy >= N || zz < 0 || zz >= N) return false;
    u = r + dx + long(N) * dy + long(N) * N * dz;
    return true;
}

// BF16 pairs packed in 32-bit words: element 2k in the low half
__device__ inline float bf_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf_hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
__device__ inline uint32_t bf_pack(float lo, float hi)
{
    return uint32_t(f2bf(lo)) | (uint32_t(f2bf(hi)) << 16);
}

// the 16 channels of one voxel as floats
__device__ inline void load16(const uint16_t* p, float* v)
{
    const uint4* q = reinterpret_cast<const uint4*>(p);
    const uint4 a = q[0], b = q[1];
    const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[2 * k] = bf_lo(w[k]);
        v[2 * k + 1] = bf_hi(w[k]);
    }
}

// store 16 floats as BF16 channels of one voxel
__device__ inline void store16(uint16_t* p, const float* v)
{
    uint4* q = reinterpret_cast<uint4*>(p);
    q[0] = make_uint4(bf_pack(v[0], v[1]), bf_pack(v[2], v[3]), bf_pack(v[4], v[5]),
                      bf_pack(v[6], v[7]));
    q[1] = make_uint4(bf_pack(v[8], v[9]), bf_pack(v[10], v[11]), bf_pack(v[12], v[13]),
                      bf_pack(v[14], v[15]));
}

// ---------------------------------------------------------------------------
// 16 -> 16 layer on MFMA (forward, or input gradient with mirrored weights)
// ---------------------------------------------------------------------------
// wpk[p*64 + lane]: the 8 BF16 values lane `lane` feeds as the B operand for
// tap pair p: rows k = 8*(lane/16) + j of the 32 x 16 block, i.e. tap
// 2p + (lane/16)/2, input channel ((lane/16)&1)*8 + j, output channel
// lane % 16.  out = relu?(acc) * (mask > 0 if mask) in BF16.
//
// The volume is cut into tiles of 16 (x) x 4 (y) x 4 (z) output voxels
// (N is a multiple of 16, so tiles are whole).  For a tile, the 18 x 6 x 6
// input voxels around it (one-voxel halo, zero outside the volume; 16 BF16
// channels = 32 bytes each, 20.7 KB) are staged in LDS, so an input voxel is
// read from memory about 2.5 times per layer instead of once per tap.  The
// staged channels 0-7 and 8-15 lie in two planes, so the 16 lanes that feed
// one A fragment read 16 consecutive 16-byte words.
constexpr int kTX = 16, kTY = 4, kTZ = 4;            // output tile
constexpr int kHX = kTX + 2, kHY = kTY + 2, kHZ = kTZ + 2;
constexpr int kHalo = kHX * kHY * kHZ;               // 648 staged voxels
constexpr int kOutPitch = 20;                        // floats per voxel in the output staging
constexpr int kStageRegs = (kHalo * 2 + 255) / 256;  // 16-byte words a thread stages

// tile t of the volume -> its first output voxel (x0, y0, z0)
__device__ inline void tile_origin(int t, int N, int& x0, int& y0, int& z0)
{
    const int ntx = N / kTX, nty = N / kTY;
    x0 = (t % ntx) * kTX;
    y0 = ((t / ntx) % nty) * kTY;
    z0 = (t / (ntx * nty)) * kTZ;
}

// the input words of the halo around the tile at (x0, y0, z0): word e (voxel
// e / 2, channels (e & 1) * 8 ...) for e = threadIdx.x + 256 q
__device__ inline void load_halo(const uint16_t* __restrict__ in, int x0, int y0, int z0, int N,
                                 uint4 (&v)[kStageRegs])
{
#pragma unroll
    for (int q = 0; q < kStageRegs; ++q) {
        const int e = threadIdx.x + 256 * q;
        v[q] = make_uint4(0, 0, 0, 0);
        if (e < kHalo * 2) {
            const int h = e >> 1;
            const int hx = h % kHX, hy = (h / kHX) % kHY, hz = h / (kHX * kHY);
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            if (gx >= 0 && gx < N && gy >= 0 && gy < N && gz >= 0 && gz < N)
                v[q] = *reinterpret_cast<const uint4*>(in + ((long(gz) * N + gy) * N + gx) * kC +
                                                       (e & 1) * 8);
        }
    }
}

// voxel h: tile[h] channels 0-7, tile[kHalo + h] channels 8-15
__device__ inline void store_halo(uint4* tile, const uint4 (&v)[kStageRegs])
{
#pragma unroll
    for (int q = 0; q < kStageRegs; ++q) {
        const int e = threadIdx.x + 256 * q;
        if (e < kHalo * 2) tile[(e & 1) * kHalo + (e >> 1)] = v[q];
    }
}

// Stage the halo of the tile at (x0, y0, z0) in LDS.  No barrier.
__device__ inline void stage_tile16(const uint16_t* __restrict__ in, uint4* tile, int x0, int y0,
                                    int z0, int N)
{
    uint4 v[kStageRegs];
    load_halo(in, x0, y0, z0, N, v);
    store_halo(tile, v);
}

// halo index of output voxel (lx, ly, lz) of a tile shifted by tap t
__device__ inline int halo_of(int lx, int ly, int lz, int t)
{
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    return ((lz + 1 + dz) * kHY + (ly + 1 + dy)) * kHX + (lx + 1 + dx);
}

// 16 -> 16 layer: each block walks the tiles blockIdx.x, + gridDim.x, ...;
// the next tile's halo is loaded into registers while the current one is
// computed.  Wave w takes z-slice w of a tile: for each tap pair p it reads
// the A fragments of its 4 rows (16 voxels each) from LDS and issues 4
// independent MFMAs, with the 14 packed B fragments held in registers.  The
// results go back through LDS (a lane holds one channel of 4 voxels), so
// that each thread writes the 16 channels of one voxel as two 16-byte stores.
__global__ __launch_bounds__(256, 3) void conv16_lds(const uint16_t* __restrict__ in,
                                                  const uint4* __restrict__ wpk,
                                                  uint16_t* __restrict__ out,
                                                  const uint16_t* __restrict__ mask, int relu,
                                                  int N)
{
    __shared__ uint4 tile[kHalo * 2];
    // output staging, apart from the input tile: a tile needs two barriers,
    // one after its halo is stored and one after its results are staged
    __shared__ __align__(16) float stage[kTX * kTY * kTZ * kOutPitch];
    const int ntiles = (N / kTX) * (N / kTY) * (N / kTZ);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, kq = lane >> 4;
    const int half = kq & 1, tsel = kq >> 1;
    uint4 b[kMPairs];
#pragma unroll
    for (int p = 0; p < kMPairs; ++p) b[p] = wpk[p * 64 + lane];
    uint4 pre[kStageRegs];
    int t = blockIdx.x;
    if (t >= ntiles) return;
    int x0, y0, z0;
    tile_origin(t, N, x0, y0, z0);
    load_halo(in, x0, y0, z0, N, pre);
    for (; t < ntiles; t += gridDim.x) {
        // every wave has passed the previous tile's second barrier, so its
        // reads of the halo are done
        store_halo(tile, pre);
        __syncthreads();
        const int cx = x0, cy = y0, cz = z0;
        if (t + int(gridDim.x) < ntiles) {
            tile_origin(t + gridDim.x, N, x0, y0, z0);
            load_halo(in, x0, y0, z0, N, pre);
        }
        f32x4 acc[kTY];
#pragma unroll
        for (int r = 0; r < kTY; ++r) acc[r] = f32x4{0.f, 0.f, 0.f, 0.f};
        const uint4* plane = tile + half * kHalo;
        // input row hy of the halo, (dz, dx) pair k: one A fragment for the
        // output rows r = hy - 2 .. hy (dy = hy - r - 1)
#pragma unroll
        for (int hy = 0; hy < kHY; ++hy) {
#pragma unroll
            for (int k = 0; k < kDyPairs; ++k) {
                const int c = 2 * k + tsel;   // (dz, dx) index of this lane's tap
                const int dz = c / 3 - 1, dx = c % 3 - 1;
                uint4 a = make_uint4(0, 0, 0, 0);
                if (c < 9) a = plane[((wave + 1 + dz) * kHY + hy) * kHX + (m + 1 + dx)];
#pragma unroll
                for (int r = 0; r < kTY; ++r) {
                    const int dyi = hy - r;
                    if (dyi < 0 || dyi > 2) continue;
                    acc[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        __builtin_bit_cast(bf16x8, a),
                        __builtin_bit_cast(bf16x8, b[dyi * kDyPairs + k]), acc[r], 0, 0, 0);
                }
            }
        }
        // lane holds rows (voxels) 4*kq + j of each 16-voxel row, column (channel) m;
        // every wave has passed this tile's first barrier, so the previous
        // tile's staged results have been read
#pragma unroll
        for (int r = 0; r < kTY; ++r)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int lv = (wave * kTY + r) * kTX + 4 * kq + j;
                stage[lv * kOutPitch + m] = relu ? fmaxf(acc[r][j], 0.0f) : acc[r][j];
            }
        __syncthreads();
        const int lv = threadIdx.x;   // 256 threads, 256 voxels
        const int lx = lv % kTX, ly = (lv / kTX) % kTY, lz = lv / (kTX * kTY);
        const long vv = (long(cz + lz) * N + (cy + ly)) * N + cx + lx;
        float o[kC];
        const float4* s4 = reinterpret_cast<const float4*>(stage + lv * kOutPitch);
#pragma unroll
        for (int q = 0; q < kC / 4; ++q) {
            const float4 w = s4[q];
            o[4 * q] = w.x;
            o[4 * q + 1] = w.y;
            o[4 * q + 2] = w.z;
            o[4 * q + 3] = w.w;
        }
        if (mask) {
            float mv[kC];
            load16(mask + vv * kC, mv);
#pragma unroll
            for (int c = 0; c < kC; ++c)
                if (!(mv[c] > 0.0f)) o[c] = 0.0f;
        }
        store16(out + vv * kC, o);
    }
}


typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// a.lo * b.lo + a.hi * b.hi + c (BF16 pairs, FP32 sum)
__device__ inline float dot2(uint32_t a, uint32_t b, float c)
{
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a),
                                           __builtin_bit_cast(bf16x2, b), c, false);
}

// ---------------------------------------------------------------------------
// 1 -> 16 layer (VALU), ReLU, BF16 out.  w1p: [co][tap pair] BF16 pairs.
// One block per 16 x 4 x 4 output tile (grid conv_tile_grid); the input's
// 18 x 6 x 6 halo (zero outside the volume) is staged in LDS, and each
// thread forms the 16 channels of one voxel from 14 tap pairs, each a
// two-term BF16 dot product accumulated in FP32, pairs in tap order.
// (Walking several tiles per block with the next halo prefetched measured
// no faster: the layer is bound by its dot products and LDS reads.)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void conv_in1(const uint16_t* __restrict__ in,
                                               const uint32_t* __restrict__ w1p,
                                               uint16_t* __restrict__ out, int N)
{
    __shared__ uint32_t sw[kC * kPairs];
    __shared__ uint16_t t1[kHalo];
    const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY, z0 = blockIdx.z * kTZ;
    for (int e = threadIdx.x; e < kC * kPairs; e += blockDim.x) sw[e] = w1p[e];
    for (int h = threadIdx.x; h < kHalo; h += blockDim.x) {
        const int hx = h % kHX, hy = (h / kHX) % kHY, hz = h / (kHX * kHY);
        const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
        uint16_t v = 0;
        if (gx >= 0 && gx < N && gy >= 0 && gy < N && gz >= 0 && gz < N)
            v = in[(long(gz) * N + gy) * N + gx];
        t1[h] = v;
    }
    __syncthreads();
    const int lv = threadIdx.x;
    const int lx = lv % kTX, ly = (lv / kTX) % kTY, lz = lv / (kTX * kTY);
    uint32_t nb[kPairs];
#pragma unroll
    for (int q = 0; q < kPairs; ++q) {
        const uint32_t lo = t1[halo_of(lx, ly, lz, 2 * q)];
        const uint32_t hi = 2 * q + 1 < kTaps ? uint32_t(t1[halo_of(lx, ly, lz, 2 * q + 1)]) : 0u;
        nb[q] = lo | (hi << 16);
    }
    float o[kC];
#pragma unroll
    for (int co = 0; co < kC; ++co) {
        float acc = 0.0f;
#pragma unroll
        for (int q = 0; q < kPairs; ++q) acc = dot2(nb[q], sw[co * kPairs + q], acc);
        o[co] = fmaxf(acc, 0.0f);
    }
    const long r = (long(z0 + lz) * N + (y0 + ly)) * N + x0 + lx;
    store16(out + r * kC, o);
}

// ---------------------------------------------------------------------------
// 16 -> 1 layer (VALU), FP32 out.  w4p: [t][channel pair] BF16 pairs.
// One block per output tile (grid conv_tile_grid) over the LDS-staged input
// halo of the 16 -> 16 layers; each thread sums one voxel, taps in order and
// channel pairs in order within a tap, each pair a two-term BF16 dot product
// accumulated in FP32 (taps outside the volume add exact zeros).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void conv_out1(const uint16_t* __restrict__ in,
                                                const uint32_t* __restrict__ w4p,
                                                float* __restrict__ out, int N)
{
    __shared__ uint4 sw[kTaps * 2];
    __shared__ uint4 tile[kHalo * 2];
    const int x0 = blockIdx.x * kTX, y0 = blockIdx.y * kTY, z0 = blockIdx.z * kTZ;
    for (int e = threadIdx.x; e < kTaps * 2; e += blockDim.x)
        sw[e] = reinterpret_cast<const uint4*>(w4p)[e];
    stage_tile16(in, tile, x0, y0, z0, N);
    __syncthreads();
    const int lv = threadIdx.x;
    const int lx = lv % kTX, ly = (lv / kTX) % kTY, lz = lv / (kTX * kTY);
    float acc = 0.0f;
#pragma unroll
    for (int t = 0; t < kTaps; ++t) {
        const int h = halo_of(lx, ly, lz, t);
        const uint4 lo = tile[h], hi = tile[kHalo + h];
        const uint4 wl = sw[2 * t], wh = sw[2 * t + 1];
        acc = dot2(lo.x, wl.x, acc);
        acc = dot2(lo.y, wl.y, acc);
        acc = dot2(lo.z, wl.z, acc);
        acc = dot2(lo.w, wl.w, acc);
        acc = dot2(hi.x, wh.x, acc);
        acc = dot2(hi.y, wh.y, acc);
        acc = dot2(hi.z, wh.z, acc);
        acc = dot2(hi.w, wh.w, acc);
    }
    out[(long(z0 + lz) * N + (y0 + ly)) * N + x0 + lx] = acc;
}

// one block per output tile (the VALU layers; N is a multiple of 16)
inline dim3 conv_tile_grid(int N) { return dim3(N / kTX, N / kTY, N / kTZ); }

// input gradient of the 16 -> 1 layer: g[r, ci] = sum_t w[ci][t] dy[r - off(t)],
// times (act[r, ci] > 0), BF16 out
__global__ __launch_bounds__(256) void dgrad_out1(const float* __restrict__ dy,
                                                 const float* __restrict__ w,
                                                 const uint16_t* __restrict__ act,
                                                 uint16_t* __restrict__ g, int N)
{
    __shared__ float sw[kC * kTaps];
    for (int e = threadIdx.x; e < kC * kTaps; e += blockDim.x) sw[e] = w[e];
    __syncthreads();
    const long n = long(N) * N * N;
    const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int x = int(r % N), y = int((r / N) % N), z = int(r / (long(N) * N));
    float d[kTaps];
#pragma unroll
    for (int t = 0; t < kTaps; ++t) {
        long u;
        d[t] = neighbour(N, x, y, z, 26 - t, r, u) ? dy[u] : 0.0f;   // r - off(t)
    }
    float av[kC], o[kC];
    load16(act + r * kC, av);
#pragma unroll
    for (int ci = 0; ci < kC; ++ci) {
        float s = 0.0f;
#pragma unroll
        for (int t = 0; t < kTaps; ++t) s += sw[ci * kTaps + t] * d[t];
        o[ci] = av[ci] > 0.0f ? s : 0.0f;
    }
    store16(g + r * kC, o);
}

// ---------------------------------------------------------------------------
// 16 -> 16 weight gradient on MFMA: dW[co][ci][t] = sum_r g[r, co] in[r + off(t), ci]
// as D_t = G^T A_t over voxels, v_mfma_f32_16x16x32_bf16 with K = 32 voxels
// (two 16-voxel rows of a tile).  Each block walks the 16 x 4 x 4 tiles
// blockIdx.x, + gridDim.x, ...; per tile, g (256 voxels) and the input halo
// (18 x 6 x 6, zero outside the volume) are staged in LDS channel-major, the
// halo as three copies shifted by dx = -1, 0, 1 so that the 8 voxels a lane
// feeds are one aligned 16-byte word.  Wave w takes the K chunks 2w and
// 2w + 1 of every tile (z-slice w) and accumulates all 27 taps in registers;
// each wave writes its sums as one partial, part[(block * 4 + wave) *
// kParams2 + (co * 16 + ci) * 27 + t].
// DY32: the 16 -> 1 layer's gradient, dW4[ci][t] = sum_r dy[r] in[r + off(t), ci]
// with dy in FP32: dy = hi + mid + lo exactly (three BF16 parts, each the
// rounded remainder of the previous) in rows 0, 1, 2 of G^T (the other rows
// zero), and dW4 = (D[0] + D[1]) + D[2]; partials of kParams4 values.
// ---------------------------------------------------------------------------
constexpr int kWgWaves = 4;
template <bool DY32>
__global__ __launch_bounds__(256, 2) void wgrad16_mfma(const uint16_t* __restrict__ g,
                                                       const float* __restrict__ dy,
                                                       const uint16_t* __restrict__ in, int N,
                                                       float* __restrict__ part)
{
    // aT[((d * 16 + ci) * 36 + hz * 6 + hy) * 16 + lx] = in at halo (lx + d, hy, hz)
    __shared__ __align__(16) uint16_t aT[3 * kC * kHY * kHZ * kTX];
    // gT[co * 256 + lv] = g at tile voxel lv = (lz * 4 + ly) * 16 + lx
    __shared__ __align__(16) uint16_t gT[kC * kTX * kTY * kTZ];
    const int ntiles = (N / kTX) * (N / kTY) * (N / kTZ);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int mn = lane & 15, kq = lane >> 4;
    f32x4 acc[kTaps];
#pragma unroll
    for (int t = 0; t < kTaps; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (DY32) {
        // rows 3..15 of G^T stay zero
        for (int e = threadIdx.x; e < (kC - 3) * kTX * kTY * kTZ; e += blockDim.x)
            gT[3 * kTX * kTY * kTZ + e] = 0;
    }
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        int x0, y0, z0;
        tile_origin(tile, N, x0, y0, z0);
        __syncthreads();   // the previous tile's operands have been read
        for (int e = threadIdx.x; e < kHalo * 2; e += blockDim.x) {
            const int h = e >> 1, half = e & 1;
            const int hx = h % kHX, hy = (h / kHX) % kHY, hz = h / (kHX * kHY);
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (gx >= 0 && gx < N && gy >= 0 && gy < N && gz >= 0 && gz < N)
                v = *reinterpret_cast<const uint4*>(in + ((long(gz) * N + gy) * N + gx) * kC +
                                                    half * 8);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int lx = hx - d;
                if (lx < 0 || lx >= kTX) continue;
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int ci = half * 8 + c;
                    aT[((d * kC + ci) * (kHY * kHZ) + hz * kHY + hy) * kTX + lx] =
                        uint16_t(w[c >> 1] >> ((c & 1) * 16));
                }
            }
        }
        if constexpr (DY32) {
            for (int lv = threadIdx.x; lv < kTX * kTY * kTZ; lv += blockDim.x) {
                const int lx = lv % kTX, ly = (lv / kTX) % kTY, lz = lv / (kTX * kTY);
                const float v = dy[(long(z0 + lz) * N + (y0 + ly)) * N + x0 + lx];
                const uint16_t hi = f2bf(v);
                const float r1 = v - bf2f(hi);
                const uint16_t mid = f2bf(r1);
                const uint16_t lo = f2bf(r1 - bf2f(mid));
                gT[lv] = hi;
                gT[kTX * kTY * kTZ + lv] = mid;
                gT[2 * kTX * kTY * kTZ + lv] = lo;
            }
        } else {
            for (int e = threadIdx.x; e < kTX * kTY * kTZ * 2; e += blockDim.x) {
                const int lv = e >> 1, half = e & 1;
                const int lx = lv % kTX, ly = (lv / kTX) % kTY, lz = lv / (kTX * kTY);
                const uint4 v = *reinterpret_cast<const uint4*>(
                    g + ((long(z0 + lz) * N + (y0 + ly)) * N + x0 + lx) * kC + half * 8);
                const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int c = 0; c < 8; ++c)
                    gT[(half * 8 + c) * (kTX * kTY * kTZ) + lv] =
                        uint16_t(w[c >> 1] >> ((c & 1) * 16));
            }
        }
        __syncthreads();
        // K chunk c = 2 * wave + q: z-slice lz = wave, rows 2q and 2q + 1;
        // K index 8 kq + j -> row 2q + (kq >> 1), x = 8 (kq & 1) + j
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int lz = wave, ly = 2 * q + (kq >> 1), lx0 = 8 * (kq & 1);
            const uint4 a = *reinterpret_cast<const uint4*>(
                &gT[mn * (kTX * kTY * kTZ) + (lz * kTY + ly) * kTX + lx0]);
#pragma unroll
            for (int t = 0; t < kTaps; ++t) {
                const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
                const uint4 b = *reinterpret_cast<const uint4*>(
                    &aT[(((dx + 1) * kC + mn) * (kHY * kHZ) + (lz + 1 + dz) * kHY + (ly + 1 + dy)) *
                            kTX + lx0]);
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                                __builtin_bit_cast(bf16x8, b),
                                                                acc[t], 0, 0, 0);
            }
        }
    }
    // lane holds D[co = 4 kq + j][ci = mn]
    if constexpr (DY32) {
        float* dst = part + (size_t(blockIdx.x) * kWgWaves + wave) * kParams4;
        if (kq == 0) {
#pragma unroll
            for (int t = 0; t < kTaps; ++t) dst[mn * kTaps + t] = (acc[t][0] + acc[t][1]) + acc[t][2];
        }
    } else {
        float* dst = part + (size_t(blockIdx.x) * kWgWaves + wave) * kParams2;
#pragma unroll
        for (int t = 0; t < kTaps; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) dst[((4 * kq + j) * kC + mn) * kTaps + t] = acc[t][j];
    }
}

// ---------------------------------------------------------------------------
// 1 -> 16 weight gradient on MFMA: dW1[co][t] = sum_r g[r, co] in[r + off(t)]
// (one input channel) as D = G^T S over voxels with the taps as the 16
// columns of S (two MFMAs per 32 voxels: taps 0-15 and 16-26, the rest
// zero), S[k][t] = in at voxel k shifted by tap t.  Tiles, g staging and the
// per-wave partials (kParams1 values each) as in wgrad16_mfma; the input
// halo is staged as three x-shifted copies of its one channel.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void wgrad1_mfma(const uint16_t* __restrict__ g,
                                                  const uint16_t* __restrict__ in, int N,
                                                  float* __restrict__ part)
{
    // aT[(d * 36 + hz * 6 + hy) * 16 + lx] = in at halo (lx + d, hy, hz)
    __shared__ __align__(16) uint16_t aT[3 * kHY * kHZ * kTX];
    __shared__ __align__(16) uint16_t gT[kC * kTX * kTY * kTZ];
    const int ntiles = (N / kTX) * (N / kTY) * (N / kTZ);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int mn = lane & 15, kq = lane >> 4;
    f32x4 acc[2] = {f32x4{0.f, 0.f, 0.f, 0.f}, f32x4{0.f, 0.f, 0.f, 0.f}};
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        int x0, y0, z0;
        tile_origin(tile, N, x0, y0, z0);
        __syncthreads();   // the previous tile's operands have been read
        for (int h = threadIdx.x; h < kHalo; h += blockDim.x) {
            const int hx = h % kHX, hy = (h / kHX) % kHY, hz = h / (kHX * kHY);
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            uint16_t v = 0;
            if (gx >= 0 && gx < N && gy >= 0 && gy < N && gz >= 0 && gz < N)
                v = in[(long(gz) * N + gy) * N + gx];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int lx = hx - d;
                if (lx >= 0 && lx < kTX) aT[(d * (kHY * kHZ) + hz * kHY + hy) * kTX + lx] = v;
            }
        }
        for (int e = threadIdx.x; e < kTX * kTY * kTZ * 2; e += blockDim.x) {
            const int lv = e >> 1, half = e & 1;
            const int lx = lv % kTX, ly = (lv / kTX) % kTY, lz = lv / (kTX * kTY);
            const uint4 v = *reinterpret_cast<const uint4*>(
                g + ((long(z0 + lz) * N + (y0 + ly)) * N + x0 + lx) * kC + half * 8);
            const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int c = 0; c < 8; ++c)
                gT[(half * 8 + c) * (kTX * kTY * kTZ) + lv] = uint16_t(w[c >> 1] >> ((c & 1) * 16));
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int lz = wave, ly = 2 * q + (kq >> 1), lx0 = 8 * (kq & 1);
            const uint4 a = *reinterpret_cast<const uint4*>(
                &gT[mn * (kTX * kTY * kTZ) + (lz * kTY + ly) * kTX + lx0]);
#pragma unroll
            for (int sidx = 0; sidx < 2; ++sidx) {
                const int t = mn + 16 * sidx;   // this lane's column of S
                uint4 b = make_uint4(0, 0, 0, 0);
                if (t < kTaps) {
                    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
                    b = *reinterpret_cast<const uint4*>(
                        &aT[((dx + 1) * (kHY * kHZ) + (lz + 1 + dz) * kHY + (ly + 1 + dy)) * kTX + lx0]);
                }
                acc[sidx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                                   __builtin_bit_cast(bf16x8, b),
                                                                   acc[sidx], 0, 0, 0);
            }
        }
    }
    // lane holds D[co = 4 kq + j][t = mn + 16 s]
    float* dst = part + (size_t(blockIdx.x) * kWgWaves + wave) * kParams1;
#pragma unroll
    for (int sidx = 0; sidx < 2; ++sidx) {
        const int t = mn + 16 * sidx;
        if (t < kTaps) {
#pragma unroll
            for (int j = 0; j < 4; ++j) dst[(4 * kq + j) * kTaps + t] = acc[sidx][j];
        }
    }
}

// dst[e] += sum over b of part[b len + e], in two fixed-order stages: the
// kRedSegs segments of consecutive partials (blockIdx.y = segment) into
// seg[s len + e], then the segments in order
constexpr int kRedSegs = 32;
__global__ void reduce_parts(const float* __restrict__ part, int nb, int len,
                             float* __restrict__ seg)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= len) return;
    const int sgi = blockIdx.y;
    const int b0 = int(long(nb) * sgi / kRedSegs), b1 = int(long(nb) * (sgi + 1) / kRedSegs);
    float s = 0.0f;
    for (int b = b0; b < b1; ++b) s += part[size_t(b) * len + e];
    seg[size_t(sgi) * len + e] = s;
}

__global__ void reduce_segs(const float* __restrict__ seg, int len, float* __restrict__ dst)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= len) return;
    float s = 0.0f;
    for (int k = 0; k < kRedSegs; ++k) s += seg[size_t(k) * len + e];
    dst[e] += s;
}

// ---------------------------------------------------------------------------
// loss: per sample e2 = sum (y - t)^2, tt = sum t^2 (block partials)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void loss_parts(const float* __restrict__ y,
                                                 const float* __restrict__ t, long n,
                                                 double* __restrict__ part)
{
    __shared__ double s1[256], s2[256];
    double a = 0.0, b = 0.0;
    for (long r = long(blockIdx.x) * blockDim.x + threadIdx.x; r < n;
         r += long(gridDim.x) * blockDim.x) {
        const double e = double(y[r]) - double(t[r]);
        a += e * e;
        b += double(t[r]) * double(t[r]);
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if (threadIdx.x < h) {
            s1[threadIdx.x] += s1[threadIdx.x + h];
            s2[threadIdx.x] += s2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1[0];
        part[2 * blockIdx.x + 1] = s2[0];
    }
}

// out[0] += e2 / tt / S (the sample's loss); out[1] = 2 / (tt S) (gradient scale)
// one block of 256 threads: thread t adds partials t, t + 256, ... in order,
// then a fixed halving tree (the same order every run)
__global__ __launch_bounds__(256) void loss_finish(const double* __restrict__ part, int nb, int S,
                                                   double* out)
{
    __shared__ double sa[256], sb[256];
    const int t = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int k = t; k < nb; k += 256) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    sa[t] = a;
    sb[t] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            sa[t] += sa[t + w];
            sb[t] += sb[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] += sa[0] / sb[0] / S;
        out[1] = 2.0 / (sb[0] * S);
    }
}

__global__ void loss_grad(const float* __restrict__ y, const float* __restrict__ t, long n,
                          const double* __restrict__ sc, float* __restrict__ dy)
{
    const float s = float(sc[1]);
    for (long r = long(blockIdx.x) * blockDim.x + threadIdx.x; r < n;
         r += long(gridDim.x) * blockDim.x)
        dy[r] = s * (y[r] - t[r]);
}

// Residual loss (the guess judged as a solver's initial guess): r = x - A y
// with A's CSR rows (FP64 products and sums, r kept FP32), and per block
// the partial sums of r^2 and x^2, in the loss_parts layout.
__global__ __launch_bounds__(256) void res_parts(const float* __restrict__ x,
                                                const float* __restrict__ y,
                                                const int* __restrict__ rp,
                                                const int* __restrict__ ci,
                                                const double* __restrict__ av, long n,
                                                float* __restrict__ r, double* __restrict__ part)
{
    __shared__ double s1[256], s2[256];
    double a = 0.0, b = 0.0;
    for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += long(gridDim.x) * blockDim.x) {
        double ax = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) ax += av[k] * double(y[ci[k]]);
        const double e = double(x[i]) - ax;
        r[i] = float(e);
        a += e * e;
        b += double(x[i]) * double(x[i]);
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if (threadIdx.x < h) {
            s1[threadIdx.x] += s1[threadIdx.x + h];
            s2[threadIdx.x] += s2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1[0];
        part[2 * blockIdx.x + 1] = s2[0];
    }
}

// dL/dy = -(2 / (||x||^2 S)) A^T r, with A^T = A (the symmetric operator of
// CG); sc[1] = 2 / (||x||^2 S) from loss_finish
__global__ void res_grad(const float* __restrict__ r, const int* __restrict__ rp,
                         const int* __restrict__ ci, const double* __restrict__ av, long n,
                         const double* __restrict__ sc, float* __restrict__ dy)
{
    const double s = sc[1];
    for (long i = long(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += long(gridDim.x) * blockDim.x) {
        double ar = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; ++k) ar += av[k] * double(r[ci[k]]);
        dy[i] = float(-s * ar);
    }
}

// ---------------------------------------------------------------------------
// weights: Adam on FP32 masters, then BF16 copies in each kernel's layout
// ---------------------------------------------------------------------------
__global__ void adam_step(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v, int len, float lr, float b1, float b2, float eps,
                          float c1, float c2)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= len) return;
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.0f - b1) * gg;
    const float vv = b2 * v[e] + (1.0f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    const float mh = mm / c1, vh = vv / c2;
    w[e] -= lr * mh / (sqrtf(vh) + eps);
}

// Layer offsets in the flat master array: W1 [16][1][27], W2, W3 [16][16][27],
// W4 [1][16][27].
// w1p[co * kPairs + q]: BF16 W1[co][2q] (low half) and W1[co][2q + 1] (high
// half, zero for q = 13); w4p[t * 8 + k]: BF16 W4[2k][t] and W4[2k + 1][t]
__global__ void pack_weights(const float* __restrict__ w, float* __restrict__ w4b,
                             uint16_t* __restrict__ pk,
                             uint32_t* __restrict__ w1p, uint32_t* __restrict__ w4p)
{
    // pk: 4 packs of kMPairs*64*8 BF16: [W2 fwd, W2 dgrad, W3 fwd, W3 dgrad]
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < kParams4) {
        // W4 [0][ci][t] -> [ci][t]
        w4b[e] = bf2f(f2bf(w[kParams1 + 2 * kParams2 + e]));
    }
    if (e < kC * kPairs) {
        const int co = e / kPairs, q = e % kPairs;
        const uint32_t lo = f2bf(w[co * kTaps + 2 * q]);
        const uint32_t hi = 2 * q + 1 < kTaps ? f2bf(w[co * kTaps + 2 * q + 1]) : 0u;
        w1p[e] = lo | (hi << 16);
    }
    if (e < kTaps * 8) {
        const int t = e / 8, k = e % 8;
        const float* W4 = w + kParams1 + 2 * kParams2;   // [ci][t]
        w4p[e] = uint32_t(f2bf(W4[(2 * k) * kTaps + t])) |
                 (uint32_t(f2bf(W4[(2 * k + 1) * kTaps + t])) << 16);
    }
    constexpr int per = kMPairs * 64 * 8;
    if (e >= 4 * per) return;
    const int which = e / per, rem = e % per;
    const int p = rem / (64 * 8), lane = (rem / 8) % 64, j = rem % 8;
    const int kq = lane >> 4, col = lane & 15;
    // fragment p = dyi * kDyPairs + k: taps (dz, dy = dyi - 1, dx) with
    // (dz + 1) * 3 + (dx + 1) = 2k + kq / 2 (none for 9)
    const int dyi = p / kDyPairs, c = 2 * (p % kDyPairs) + (kq >> 1);
    const int t = c < 9 ? (c / 3) * 9 + dyi * 3 + c % 3 : kTaps;
    const int row = (kq & 1) * 8 + j;   // input channel of this pass
    const float* W = w + kParams1 + (which / 2) * kParams2;   // [co][ci][t]
    float val = 0.0f;
    if (t < kTaps) {
        if ((which & 1) == 0)
            val = W[(col * kC + row) * kTaps + t];            // fwd: B[ci][co]
        else
            val = W[(row * kC + col) * kTaps + (26 - t)];     // dgrad: B[co][ci], mirrored
    }
    pk[e] = f2bf(val);
}

// ---------------------------------------------------------------------------
// data preparation / warm start
// ---------------------------------------------------------------------------
// All m columns at once through an LDS tile of kTRows rows x m columns, so
// that both the interleaved block and the volumes are accessed contiguously.
constexpr int kTRows = 64;

// vol[j n + r] = BF16(B[r m + j] / s_j) (zero for a zero column)
__global__ __launch_bounds__(256) void cols_to_bf16(const double* __restrict__ B, int m, long n,
                                                    const double* __restrict__ s,
                                                    uint16_t* __restrict__ vol)
{
    __shared__ float inv[XAMG_MAX_M];
    __shared__ uint16_t tb[kTRows * (XAMG_MAX_M + 1)];
    if (int(threadIdx.x) < m)
        inv[threadIdx.x] = s[threadIdx.x] > 0.0 ? float(1.0 / s[threadIdx.x]) : 0.0f;
    __syncthreads();
    for (long r0 = long(blockIdx.x) * kTRows; r0 < n; r0 += long(gridDim.x) * kTRows) {
        const int rows = int(n - r0 < kTRows ? n - r0 : kTRows);
        for (int f = threadIdx.x; f < rows * m; f += blockDim.x) {
            const int i = f / m, j = f % m;
            tb[i * (m + 1) + j] = f2bf(float(B[r0 * m + f]) * inv[j]);
        }
        __syncthreads();
        for (int f = threadIdx.x; f < rows * m; f += blockDim.x) {
            const int j = f / rows, i = f % rows;
            vol[size_t(j) * n + r0 + i] = tb[i * (m + 1) + j];
        }
        __syncthreads();
    }
}

// X0[r m + j] = s_j y_j[r] (zero for a zero column)
__global__ __launch_bounds__(256) void vols_to_cols(const float* __restrict__ y, int m, long n,
                                                    const double* __restrict__ s,
                                                    double* __restrict__ X0)
{
    __shared__ double sc[XAMG_MAX_M];
    __shared__ float tb[kTRows * (XAMG_MAX_M + 1)];
    if (int(threadIdx.x) < m) sc[threadIdx.x] = s[threadIdx.x];
    __syncthreads();
    for (long r0 = long(blockIdx.x) * kTRows; r0 < n; r0 += long(gridDim.x) * kTRows) {
        const int rows = int(n - r0 < kTRows ? n - r0 : kTRows);
        for (int f = threadIdx.x; f < rows * m; f += blockDim.x) {
            const int j = f / rows, i = f % rows;
            tb[i * (m + 1) + j] = y[size_t(j) * n + r0 + i];
        }
        __syncthreads();
        for (int f = threadIdx.x; f < rows * m; f += blockDim.x) {
            const int i = f / m, j = f % m;
            X0[r0 * m + f] = sc[j] > 0.0 ? sc[j] * double(tb[i * (m + 1) + j]) : 0.0;
        }
        __syncthreads();
    }
}

__global__ void f32_to_bf16(const float* __restrict__ x, long n, uint16_t* __restrict__ out)
{
    for (long r = long(blockIdx.x) * blockDim.x + threadIdx.x; r < n;
         r += long(gridDim.x) * blockDim.x)
        out[r] = f2bf(x[r]);
}

// Per-column sums of squares over a contiguous row range per block:
// part[(block * m + j) * 2] = sum b_rj^2 and, with a matrix, part[... + 1] =
// sum (b - A x)_rj^2.  With CW adjacent columns a thread (mg = m / CW column
// groups), thread t < g mg (g = 256 / mg) takes column group t % mg and rows
// q, q + g, ... of the range (q = t / mg), so loads stay contiguous; the
// threads' sums of a column are added in q order.
// With rows stored at one length (rowlen > 0: row r's entries at r rowlen,
// padded with exact zeros) four rows are taken at a time with their loads
// interleaved; every sum keeps the same terms in the same order.
template <int CW>
__global__ __launch_bounds__(256) void col_sq(const double* __restrict__ B,
                                             const double* __restrict__ X,
                                             const int* __restrict__ rp, const int* __restrict__ ci,
                                             const double* __restrict__ v, int m, long n,
                                             double* __restrict__ part, int rowlen)
{
    typedef double vec __attribute__((ext_vector_type(CW)));
    __shared__ double s0[256 * CW], s1[256 * CW];
    const int mg = m / CW;   // column groups of CW adjacent columns
    const int t = threadIdx.x, g = 256 / mg;
    const int jg = t % mg, q = t / mg;
    const long per = (n + gridDim.x - 1) / gridDim.x;
    const long r0 = long(blockIdx.x) * per, r1 = std::min(n, r0 + per);
    vec bb = vec(0.0), rr = vec(0.0);
    auto ld = [&](const double* p, long row) {
        return *reinterpret_cast<const vec*>(p + row * m + jg * CW);
    };
    if (q < g && rp && rowlen > 0) {
        for (long r = r0 + q; r < r1; r += 4L * g) {
            vec bv[4], sv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const long ru = r + long(u) * g;
                bv[u] = ru < r1 ? ld(B, ru) : vec(0.0);
                sv[u] = bv[u];
            }
            for (int k = 0; k < rowlen; ++k) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const long ru = r + long(u) * g;
                    if (ru < r1) {
                        const long e = ru * rowlen + k;
                        sv[u] -= v[e] * ld(X, ci[e]);
                    }
                }
            }
            // rows past the range add exact zeros
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                bb += bv[u] * bv[u];
                rr += sv[u] * sv[u];
            }
        }
    } else if (q < g) {
        for (long r = r0 + q; r < r1; r += g) {
            const vec b = ld(B, r);
            bb += b * b;
            if (rp) {
                vec sv = b;
                for (int k = rp[r]; k < rp[r + 1]; ++k) sv -= v[k] * ld(X, ci[k]);
                rr += sv * sv;
            }
        }
    }
#pragma unroll
    for (int c = 0; c < CW; ++c) {
        s0[t * CW + c] = bb[c];
        s1[t * CW + c] = rr[c];
    }
    __syncthreads();
    if (t < m) {
        double a = 0.0, c = 0.0;
        for (int k = 0; k < g; ++k) {
            a += s0[k * m + t];
            c += s1[k * m + t];
        }
        part[(size_t(blockIdx.x) * m + t) * 2] = a;
        part[(size_t(blockIdx.x) * m + t) * 2 + 1] = c;
    }
}

// col_sq with two adjacent columns a thread (16-byte loads) when m is even
inline void launch_col_sq(int nb, hipStream_t st, const double* B, const double* X, const int* rp,
                          const int* ci, const double* v, int m, long n, double* part, int rowlen)
{
    if (m % 2 == 0)
        hipLaunchKernelGGL(col_sq<2>, dim3(nb), dim3(256), 0, st, B, X, rp, ci, v, m, n, part, rowlen);
    else
        hipLaunchKernelGGL(col_sq<1>, dim3(nb), dim3(256), 0, st, B, X, rp, ci, v, m, n, part, rowlen);
}

// sums[2j + k] = the sum over blocks of part[(b m + j) 2 + k], one block per
// column: thread t adds blocks t, t + 256, ... in order, then a fixed halving
// tree over the 256 threads (the same order every run); with scales,
// s_j = sqrt(sums[2j] / n)
__global__ __launch_bounds__(256) void col_sq_finish(const double* __restrict__ part, int nb, int m,
                                                     long n, double* __restrict__ sums,
                                                     double* __restrict__ scales)
{
    __shared__ double s0[256], s1[256];
    const int j = blockIdx.x, t = threadIdx.x;
    double a = 0.0, c = 0.0;
    for (int b = t; b < nb; b += 256) {
        a += part[(size_t(b) * m + j) * 2];
        c += part[(size_t(b) * m + j) * 2 + 1];
    }
    s0[t] = a;
    s1[t] = c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            s0[t] += s0[t + w];
            s1[t] += s1[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        sums[2 * j] = s0[0];
        sums[2 * j + 1] = s1[0];
        if (scales) scales[j] = sqrt(s0[0] / double(n));
    }
}

__global__ void zero_col(double* __restrict__ X0, int m, int j, long n)
{
    for (long r = long(blockIdx.x) * blockDim.x + threadIdx.x; r < n;
         r += long(gridDim.x) * blockDim.x)
        X0[r * m + j] = 0.0;
}

// ---------------------------------------------------------------------------
// host object
// ---------------------------------------------------------------------------
struct Net : xamg_cnn {
    int N = 0;
    long n = 0;
    hipStream_t stream = nullptr;
    std::vector<void*> allocs;
    float *w = nullptr, *g = nullptr, *mo = nullptr, *ve = nullptr;   // masters, grads, Adam
    float* w4b = nullptr;
    uint32_t *w1p = nullptr, *w4p = nullptr;   // BF16 pairs for the dot2 layers
    uint16_t* pk = nullptr;
    uint16_t *a0 = nullptr, *a1 = nullptr, *a2 = nullptr, *a3 = nullptr;
    uint16_t *g1 = nullptr, *g2 = nullptr, *g3 = nullptr;
    float *y = nullptr, *dy = nullptr, *wpart = nullptr, *wseg = nullptr;
    float* rres = nullptr;   // residual of the residual loss
    double *lpart = nullptr, *lacc = nullptr, *scales = nullptr, *sums = nullptr;
    double* cpart = nullptr;   // col_sq partials
    int64_t adam_t = 0;
    int conv_blocks = 1;   // resident blocks of conv16_lds (at most one per tile)
    int wg_blocks = 1;     // resident blocks of wgrad16_mfma (at most one per tile)
    int wg4_blocks = 1;    // the same for its 16 -> 1 form
    int wg1_blocks = 1;    // resident blocks of wgrad1_mfma (at most one per tile)
    // kernel timer (measurement only): event pairs around the selected launches
    int timer_kind = 0;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    double timer_ms = 0.0;
    int64_t timer_count = 0;

    ~Net()
    {
        for (hipEvent_t e : ev_pool) hipEventDestroy(e);
        for (void* p : allocs) hipFree(p);
    }
    void tbegin(int kind)
    {
        if (timer_kind != kind) return;
        if (ev_used + 2 > ev_pool.size()) {
            for (int k = 0; k < 64; ++k) {
                hipEvent_t e;
                chk(hipEventCreate(&e), "hipEventCreate");
                ev_pool.push_back(e);
            }
        }
        chk(hipEventRecord(ev_pool[ev_used], stream), "hipEventRecord");
    }
    void tend(int kind)
    {
        if (timer_kind != kind) return;
        chk(hipEventRecord(ev_pool[ev_used + 1], stream), "hipEventRecord");
        ev_used += 2;
    }
    // after a stream synchronisation
    void tcollect()
    {
        for (size_t k = 0; k + 1 < ev_used; k += 2) {
            float ms = 0.0f;
            chk(hipEventElapsedTime(&ms, ev_pool[k], ev_pool[k + 1]), "hipEventElapsedTime");
            timer_ms += ms;
            timer_count += 1;
        }
        ev_used = 0;
    }
    void chk(hipError_t e, const char* what)
    {
        if (e != hipSuccess) {
            set_error("HIP error %d (%s) in %s", int(e), hipGetErrorString(e), what);
            throw DevFail{e == hipErrorOutOfMemory ? XAMG_ENOMEM : XAMG_EHIP};
        }
    }
    template <typename T>
    T* alloc(size_t count)
    {
        void* p = nullptr;
        chk(hipMalloc(&p, std::max<size_t>(count * sizeof(T), 256)), "hipMalloc");
        allocs.push_back(p);
        return static_cast<T*>(p);
    }
    const uint4* pack(int which) const
    {
        return reinterpret_cast<const uint4*>(pk + size_t(which) * kMPairs * 64 * 8);
    }
    int grid(long count, int per = 256) const { return int((count + per - 1) / per); }
    // dst[0 .. len) += the sum of the nb weight-gradient partials in wpart
    void reduce(int len, int nb, float* dst)
    {
        hipLaunchKernelGGL(reduce_parts, dim3(grid(len), kRedSegs), dim3(256), 0, stream, wpart, nb,
                           len, wseg);
        hipLaunchKernelGGL(reduce_segs, dim3(grid(len)), dim3(256), 0, stream, wseg, len, dst);
    }

    void repack()
    {
        const int total = std::max(4 * kMPairs * 64 * 8, kParams1);
        hipLaunchKernelGGL(pack_weights, dim3(grid(total)), dim3(256), 0, stream, w, w4b, pk,
                           w1p, w4p);
    }

    // forward of one normalised sample: yout = f(ain) (a1..a3 hold the activations)
    void forward(const uint16_t* ain, float* yout)
    {
        hipLaunchKernelGGL(conv_in1, conv_tile_grid(N), dim3(256), 0, stream, ain, w1p, a1, N);
        tbegin(XAMG_CNN_TIMER_CONV16);
        hipLaunchKernelGGL(conv16_lds, dim3(conv_blocks), dim3(256), 0, stream, a1, pack(0), a2,
                           static_cast<const uint16_t*>(nullptr), 1, N);
        tend(XAMG_CNN_TIMER_CONV16);
        tbegin(XAMG_CNN_TIMER_CONV16);
        hipLaunchKernelGGL(conv16_lds, dim3(conv_blocks), dim3(256), 0, stream, a2, pack(2), a3,
                           static_cast<const uint16_t*>(nullptr), 1, N);
        tend(XAMG_CNN_TIMER_CONV16);
        hipLaunchKernelGGL(conv_out1, conv_tile_grid(N), dim3(256), 0, stream, a3, w4p, yout, N);
    }
    void forward() { forward(a0, y); }

    // per-column volumes of the warm start (m BF16 inputs, m FP32 outputs),
    // grown on demand
    uint16_t* cols_in = nullptr;
    float* cols_out = nullptr;
    int cols_cap = 0;
    void release(void* p)
    {
        if (!p) return;
        for (size_t k = 0; k < allocs.size(); ++k)
            if (allocs[k] == p) {
                allocs.erase(allocs.begin() + long(k));
                break;
            }
        (void)hipFree(p);
    }
    void ensure_cols(int m)
    {
        if (m <= cols_cap) return;
        chk(hipStreamSynchronize(stream), "sync");
        release(cols_in);
        release(cols_out);
        cols_in = nullptr;
        cols_out = nullptr;
        cols_cap = 0;
        cols_in = alloc<uint16_t>(size_t(m) * n);
        cols_out = alloc<float>(size_t(m) * n);
        cols_cap = m;
    }

    // backward of one sample (dy set); weight gradients accumulate into g
    void backward()
    {
        // layer 4: dW4 and g3 = W4^T dy masked by a3 > 0
        hipLaunchKernelGGL(wgrad16_mfma<true>, dim3(wg4_blocks), dim3(256), 0, stream,
                           static_cast<const uint16_t*>(nullptr), dy, a3, N, wpart);
        reduce(kParams4, kWgWaves * wg4_blocks, g + kParams1 + 2 * kParams2);
        hipLaunchKernelGGL(dgrad_out1, dim3(grid(n)), dim3(256), 0, stream, dy, w4b, a3, g3, N);
        // layer 3: dW3 from (g3, a2); g2 = dgrad masked by a2 > 0
        tbegin(XAMG_CNN_TIMER_WGRAD16);
        hipLaunchKernelGGL(wgrad16_mfma<false>, dim3(wg_blocks), dim3(256), 0, stream, g3,
                           static_cast<const float*>(nullptr), a2, N, wpart);
        tend(XAMG_CNN_TIMER_WGRAD16);
        reduce(kParams2, kWgWaves * wg_blocks, g + kParams1 + kParams2);
        hipLaunchKernelGGL(conv16_lds, dim3(conv_blocks), dim3(256), 0, stream, g3, pack(3), g2, a2, 0, N);
        // layer 2: dW2 from (g2, a1); g1 = dgrad masked by a1 > 0
        tbegin(XAMG_CNN_TIMER_WGRAD16);
        hipLaunchKernelGGL(wgrad16_mfma<false>, dim3(wg_blocks), dim3(256), 0, stream, g2,
                           static_cast<const float*>(nullptr), a1, N, wpart);
        tend(XAMG_CNN_TIMER_WGRAD16);
        reduce(kParams2, kWgWaves * wg_blocks, g + kParams1);
        hipLaunchKernelGGL(conv16_lds, dim3(conv_blocks), dim3(256), 0, stream, g2, pack(1), g1, a1, 0, N);
        // layer 1: dW1 from (g1, a0)
        hipLaunchKernelGGL(wgrad1_mfma, dim3(wg1_blocks), dim3(256), 0, stream, g1, a0, N, wpart);
        reduce(kParams1, kWgWaves * wg1_blocks, g);
    }
};

}  // namespace cnn
}  // namespace xamg

using xamg::cnn::Net;

extern "C" {

int xamg_cnn_create(int32_t N, const float* w_init, void* stream, xamg_cnn_t** out)
{
    xamg::clear_error();
    if (!w_init || !out) return xamg::fail(XAMG_EINVAL, "null argument");
    if (N < 16 || N % 16 != 0 || N > 1024) return xamg::fail(XAMG_EINVAL, "N must be a multiple of 16");
    *out = nullptr;
    Net* net = new (std::nothrow) Net;
    if (!net) return xamg::fail(XAMG_ENOMEM, "host allocation");
    using namespace xamg::cnn;
    try {
        net->N = N;
        net->n = long(N) * N * N;
        net->stream = static_cast<hipStream_t>(stream);
        const long n = net->n;
        net->w = net->alloc<float>(kParams);
        net->g = net->alloc<float>(kParams);
        net->mo = net->alloc<float>(kParams);
        net->ve = net->alloc<float>(kParams);
        net->w4b = net->alloc<float>(kParams4);
        net->w1p = net->alloc<uint32_t>(kC * kPairs);
        net->w4p = net->alloc<uint32_t>(kTaps * 8);
        net->pk = net->alloc<uint16_t>(4 * kMPairs * 64 * 8);
        net->a0 = net->alloc<uint16_t>(n);
        net->a1 = net->alloc<uint16_t>(n * kC);
        net->a2 = net->alloc<uint16_t>(n * kC);
        net->a3 = net->alloc<uint16_t>(n * kC);
        net->g1 = net->alloc<uint16_t>(n * kC);
        net->g2 = net->alloc<uint16_t>(n * kC);
        net->g3 = net->alloc<uint16_t>(n * kC);
        net->y = net->alloc<float>(n);
        net->dy = net->alloc<float>(n);
        net->rres = net->alloc<float>(n);
        net->wseg = net->alloc<float>(size_t(kRedSegs) * kParams2);
        net->lpart = net->alloc<double>(2 * 1024);
        net->lacc = net->alloc<double>(2);
        net->scales = net->alloc<double>(64);
        net->sums = net->alloc<double>(2 * 64);
        net->cpart = net->alloc<double>(size_t(kColBlocks) * 2 * 64);
        {
            int dev = 0, cus = 0, per_cu = 0;
            net->chk(hipGetDevice(&dev), "hipGetDevice");
            net->chk(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev), "CUs");
            const long ntiles = n / (kTX * kTY * kTZ);
            auto resident = [&](const void* fn) {
                net->chk(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0),
                         "occupancy");
                return int(std::min<long>(ntiles, long(std::max(1, per_cu)) * std::max(1, cus)));
            };
            net->conv_blocks = resident(reinterpret_cast<const void*>(conv16_lds));
            net->wg_blocks = resident(reinterpret_cast<const void*>(wgrad16_mfma<false>));
            net->wg4_blocks = resident(reinterpret_cast<const void*>(wgrad16_mfma<true>));
            net->wg1_blocks = resident(reinterpret_cast<const void*>(wgrad1_mfma));
        }
        // weight-gradient partials: one per wave of the weight-gradient kernels
        net->wpart = net->alloc<float>(
            size_t(kWgWaves) * std::max({net->wg_blocks, net->wg4_blocks, net->wg1_blocks}) *
            kParams2);
        net->chk(hipMemcpy(net->w, w_init, kParams * sizeof(float), hipMemcpyHostToDevice), "weights");
        std::vector<float> zero(kParams, 0.0f);
        net->chk(hipMemcpy(net->mo, zero.data(), kParams * sizeof(float), hipMemcpyHostToDevice), "adam");
        net->chk(hipMemcpy(net->ve, zero.data(), kParams * sizeof(float), hipMemcpyHostToDevice), "adam");
        net->repack();
        net->chk(hipStreamSynchronize(net->stream), "create sync");
    } catch (const xamg::DevFail& f) {
        delete net;
        return f.code;
    }
    *out = static_cast<xamg_cnn_t*>(net);
    return XAMG_OK;
}

int xamg_cnn_get_weights(xamg_cnn_t* h, float* w_host)
{
    Net* net = static_cast<Net*>(h);
    if (!net || !w_host) return xamg::fail(XAMG_EINVAL, "null argument");
    try {
        net->chk(hipStreamSynchronize(net->stream), "sync");
        net->chk(hipMemcpy(w_host, net->w, xamg::cnn::kParams * sizeof(float), hipMemcpyDeviceToHost),
                 "weights");
    } catch (const xamg::DevFail& f) {
        return f.code;
    }
    return XAMG_OK;
}

int xamg_cnn_set_weights(xamg_cnn_t* h, const float* w_host)
{
    Net* net = static_cast<Net*>(h);
    if (!net || !w_host) return xamg::fail(XAMG_EINVAL, "null argument");
    try {
        net->chk(hipMemcpy(net->w, w_host, xamg::cnn::kParams * sizeof(float), hipMemcpyHostToDevice),
                 "weights");
        net->repack();
        net->chk(hipStreamSynchronize(net->stream), "sync");
    } catch (const xamg::DevFail& f) {
        return f.code;
    }
    return XAMG_OK;
}

// One forward (and, with targets, backward) pass over S normalised samples.
// x: S x n FP32 inputs, t: S x n FP32 targets or NULL, y_out: S x n FP32
// (device) or NULL.  With targets the weight gradients are summed over the
// samples into the gradient buffer and *loss = mean relative squared error.
int xamg_cnn_pass(xamg_cnn_t* h, const float* x, const float* t, int32_t S, float* y_out,
                  double* loss)
{
    using namespace xamg::cnn;
    Net* net = static_cast<Net*>(h);
    if (!net || !x || S < 1) return xamg::fail(XAMG_EINVAL, "bad arguments");
    try {
        const long n = net->n;
        if (t) {
            net->chk(hipMemsetAsync(net->g, 0, kParams * sizeof(float), net->stream), "grad zero");
            net->chk(hipMemsetAsync(net->lacc, 0, 2 * sizeof(double), net->stream), "loss zero");
        }
        for (int s = 0; s < S; ++s) {
            hipLaunchKernelGGL(f32_to_bf16, dim3(1024), dim3(256), 0, net->stream, x + size_t(s) * n,
                               n, net->a0);
            net->forward();
            if (y_out)
                net->chk(hipMemcpyAsync(y_out + size_t(s) * n, net->y, n * sizeof(float),
                                        hipMemcpyDeviceToDevice, net->stream), "y copy");
            if (t) {
                const float* ts = t + size_t(s) * n;
                hipLaunchKernelGGL(loss_parts, dim3(1024), dim3(256), 0, net->stream, net->y, ts, n,
                                   net->lpart);
                hipLaunchKernelGGL(loss_finish, dim3(1), dim3(256), 0, net->stream, net->lpart, 1024, S,
                                   net->lacc);
                hipLaunchKernelGGL(loss_grad, dim3(1024), dim3(256), 0, net->stream, net->y, ts, n,
                                   net->lacc, net->dy);
                net->backward();
            }
        }
        if (t && loss) {
            double l[2];
            net->chk(hipMemcpyAsync(l, net->lacc, 2 * sizeof(double), hipMemcpyDeviceToHost,
                                    net->stream), "loss copy");
            net->chk(hipStreamSynchronize(net->stream), "sync");
            *loss = l[0];
        }
        net->chk(hipGetLastError(), "cnn pass");
        if (net->ev_used) {
            net->chk(hipStreamSynchronize(net->stream), "sync");
            net->tcollect();
        }
    } catch (const xamg::DevFail& f) {
        return f.code;
    }
    return XAMG_OK;
}

// Forward and backward with the residual loss over S samples: the operator
// is level 0 of a solver handle on the same grid (FP64 CSR).
int xamg_cnn_pass_residual(xamg_cnn_t* h, xamg_handle_t* solver, const float* x, int32_t S,
                           double* loss)
{
    using namespace xamg::cnn;
    xamg::clear_error();
    Net* net = static_cast<Net*>(h);
    if (!net || !solver || !x || S < 1) return xamg::fail(XAMG_EINVAL, "bad arguments");
    const xamg::Handle* sh = static_cast<const xamg::Handle*>(solver);
    if (sh->lev[0].n != net->n) return xamg::fail(XAMG_EINVAL, "solver size differs from the network grid");
    try {
        const long n = net->n;
        const xamg::DCsr& A = sh->lev[0].A64;
        const double* av = static_cast<const double*>(A.v);
        net->chk(hipMemsetAsync(net->g, 0, kParams * sizeof(float), net->stream), "grad zero");
        net->chk(hipMemsetAsync(net->lacc, 0, 2 * sizeof(double), net->stream), "loss zero");
        for (int s = 0; s < S; ++s) {
            const float* xs = x + size_t(s) * n;
            hipLaunchKernelGGL(f32_to_bf16, dim3(1024), dim3(256), 0, net->stream, xs, n, net->a0);
            net->forward();
            hipLaunchKernelGGL(res_parts, dim3(1024), dim3(256), 0, net->stream, xs, net->y, A.rp,
                               A.ci, av, n, net->rres, net->lpart);
            hipLaunchKernelGGL(loss_finish, dim3(1), dim3(256), 0, net->stream, net->lpart, 1024, S,
                               net->lacc);
            hipLaunchKernelGGL(res_grad, dim3(1024), dim3(256), 0, net->stream, net->rres, A.rp, A.ci,
                               av, n, net->lacc, net->dy);
            net->backward();
        }
        if (loss) {
            double l[2];
            net->chk(hipMemcpyAsync(l, net->lacc, 2 * sizeof(double), hipMemcpyDeviceToHost,
                                    net->stream), "loss copy");
            net->chk(hipStreamSynchronize(net->stream), "sync");
            *loss = l[0];
        }
        net->chk(hipGetLastError(), "cnn residual pass");
        if (net->ev_used) {
            net->chk(hipStreamSynchronize(net->stream), "sync");
            net->tcollect();
        }
    } catch (const xamg::DevFail& f) {
        return f.code;
    }
    return XAMG_OK;
}

// Copy the summed weight gradients of the last pass (host, 14688 floats).
int xamg_cnn_get_grads(xamg_cnn_t* h, float* g_host)
{
    Net* net = static_cast<Net*>(h);
    if (!net || !g_host) return xamg::fail(XAMG_EINVAL, "null argument");
    try {
        net->chk(hipStreamSynchronize(net->stream), "sync");
        net->chk(hipMemcpy(g_host, net->g, xamg::cnn::kParams * sizeof(float), hipMemcpyDeviceToHost),
                 "grads");
    } catch (const xamg::DevFail& f) {
        return f.code;
    }
    return XAMG_OK;
}

// Adam step with the gradients of the last pass.
int xamg_cnn_adam(xamg_cnn_t* h, float lr, float beta1, float beta2, float eps)
{
    using namespace xamg::cnn;
    Net* net = static_cast<Net*>(h);
    if (!net || !(lr > 0.0f)) return xamg::fail(XAMG_EINVAL, "bad arguments");
    try {
        net->adam_t += 1;
        const float c1 = 1.0f - std::pow(beta1, float(net->adam_t));
        const float c2 = 1.0f - std::pow(beta2, float(net->adam_t));
        hipLaunchKernelGGL(adam_step, dim3(net->grid(kParams)), dim3(256), 0, net->stream, net->w,
                           net->g, net->mo, net->ve, kParams, lr, beta1, beta2, eps, c1, c2);
        net->repack();
        net->chk(hipGetLastError(), "adam");
    } catch (const xamg::DevFail& f) {
        return f.code;
    }
    return XAMG_OK;
}

// Single-layer kernels for tests (device pointers, BF16 as uint16).
// layer 1..4; in: n x cin, out: n x cout (layer 4: FP32 out).  mode 0 =
// forward, mode 1 = input gradient (layers 2..4; `mask` = activation whose
// sign gates the result), mode 2 = weight gradient (out = FP32 [cout][cin][27]
// added to the net's gradient buffer, read with xamg_cnn_get_grads).
int xamg_cnn_layer(xamg_cnn_t* h, int32_t layer, int32_t mode, const void* in, const void* mask,
                   void* out)
{
    using namespace xamg::cnn;
    Net* net = static_cast<Net*>(h);
    if (!net || !in || !out || layer < 1 || layer > 4 || mode < 0 || mode > 2)
        return xamg::fail(XAMG_EINVAL, "bad arguments");
    if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(mask) |
         reinterpret_cast<uintptr_t>(out)) & 15)
        return xamg::fail(XAMG_EINVAL, "in, mask and out must be 16-byte aligned");
    try {
        const long n = net->n;
        const int N = net->N;
        const uint16_t* i16 = static_cast<const uint16_t*>(in);
        const uint16_t* m16 = static_cast<const uint16_t*>(mask);
        if (mode == 0) {
            if (layer == 1)
                hipLaunchKernelGGL(conv_in1, conv_tile_grid(N), dim3(256), 0, net->stream, i16, net->w1p,
                                   static_cast<uint16_t*>(out), N);
            else if (layer == 4)
                hipLaunchKernelGGL(conv_out1, conv_tile_grid(N), dim3(256), 0, net->stream, i16, net->w4p,
                                   static_cast<float*>(out), N);
            else
                hipLaunchKernelGGL(conv16_lds, dim3(net->conv_blocks), dim3(256), 0, net->stream, i16,
                                   net->pack(layer == 2 ? 0 : 2), static_cast<uint16_t*>(out),
                                   static_cast<const uint16_t*>(nullptr), 1, N);
        } else if (mode == 1) {
            if (layer == 1) return xamg::fail(XAMG_EINVAL, "no input gradient for layer 1");
            if (!mask) return xamg::fail(XAMG_EINVAL, "mask required");
            if (layer == 4)
                hipLaunchKernelGGL(dgrad_out1, dim3(net->grid(n)), dim3(256), 0, net->stream,
                                   static_cast<const float*>(in), net->w4b, m16,
                                   static_cast<uint16_t*>(out), N);
            else
                hipLaunchKernelGGL(conv16_lds, dim3(net->conv_blocks), dim3(256), 0, net->stream, i16,
                                   net->pack(layer == 2 ? 1 : 3), static_cast<uint16_t*>(out), m16,
                                   0, N);
        } else {
            // in = gradient at the layer's output, mask = the layer's input
            if (!mask) return xamg::fail(XAMG_EINVAL, "layer input required");
            net->chk(hipMemsetAsync(net->g, 0, kParams * sizeof(float), net->stream), "grad zero");
            if (layer == 1) {
                hipLaunchKernelGGL(wgrad1_mfma, dim3(net->wg1_blocks), dim3(256), 0, net->stream, i16,
                                   m16, N, net->wpart);
                net->reduce(kParams1, kWgWaves * net->wg1_blocks, net->g);
            } else if (layer == 4) {
                hipLaunchKernelGGL(wgrad16_mfma<true>, dim3(net->wg4_blocks), dim3(256), 0,
                                   net->stream, static_cast<const uint16_t*>(nullptr),
                                   static_cast<const float*>(in), m16, N, net->wpart);
                net->reduce(kParams4, kWgWaves * net->wg4_blocks,
                            net->g + kParams1 + 2 * kParams2);
            } else {
                hipLaunchKernelGGL(wgrad16_mfma<false>, dim3(net->wg_blocks), dim3(256), 0,
                                   net->stream, i16, static_cast<const float*>(nullptr), m16, N,
                                   net->wpart);
                net->reduce(kParams2, kWgWaves * net->wg_blocks,
                            net->g + kParams1 + (layer - 2) * kParams2);
            }
        }
        net->chk(hipGetLastError(), "layer");
        net->chk(hipStreamSynchronize(net->stream), "layer sync");
    } catch (const xamg::DevFail& f) {
        return f.code;
    }
    return XAMG_OK;
}

// Warm start: X0[:, j] = s_j f(B[:, j] / s_j), s_j = ||b_j|| / sqrt(n); then,
// with a solver handle, every column whose initial residual is not smaller
// than ||b_j|| is reset to zero (fallback[j] = 1, host, may be NULL).
int xamg_warmstart(xamg_cnn_t* h, xamg_handle_t* solver, const double* B, double* X0, int32_t m,
                   int32_t* fallback)
{
    using namespace xamg::cnn;
    xamg::clear_error();
    Net* net = static_cast<Net*>(h);
    if (!net || !B || !X0 || m < 1 || m > XAMG_MAX_M) return xamg::fail(XAMG_EINVAL, "bad arguments");
    if (solver && static_cast<xamg::Handle*>(solver)->lev[0].n != net->n)
        return xamg::fail(XAMG_EINVAL, "solver size differs from the network grid");
    try {
        const long n = net->n;
        const int nbc = int(std::min<long>(kColBlocks, std::max<long>(1, n / 64)));
        launch_col_sq(nbc, net->stream, B, nullptr, nullptr, nullptr, nullptr, m, n, net->cpart, 0);
        hipLaunchKernelGGL(col_sq_finish, dim3(m), dim3(256), 0, net->stream, net->cpart, nbc, m, n,
                           net->sums, net->scales);
        net->ensure_cols(m);
        const int nbr = int(std::min<long>(4096, (n + kTRows - 1) / kTRows));
        hipLaunchKernelGGL(cols_to_bf16, dim3(nbr), dim3(256), 0, net->stream, B, m, n,
                           net->scales, net->cols_in);
        for (int j = 0; j < m; ++j)
            net->forward(net->cols_in + size_t(j) * n, net->cols_out + size_t(j) * n);
        hipLaunchKernelGGL(vols_to_cols, dim3(nbr), dim3(256), 0, net->stream, net->cols_out, m, n,
                           net->scales, X0);
        net->chk(hipGetLastError(), "warm start");
        if (solver) {
            // fallback: ||b_j - A x0_j|| >= ||b_j||  =>  x0_j = 0
            const xamg::DCsr& A = static_cast<xamg::Handle*>(solver)->lev[0].A64;
            launch_col_sq(nbc, net->stream, B, X0, A.rp, A.ci, static_cast<const double*>(A.v), m, n,
                          net->cpart, A.rowlen);
            hipLaunchKernelGGL(col_sq_finish, dim3(m), dim3(256), 0, net->stream, net->cpart, nbc, m,
                               n, net->sums, static_cast<double*>(nullptr));
            double sums[2 * 64];
            net->chk(hipMemcpyAsync(sums, net->sums, 2 * m * sizeof(double), hipMemcpyDeviceToHost,
                                    net->stream), "norm copy");
            net->chk(hipStreamSynchronize(net->stream), "sync");
            for (int j = 0; j < m; ++j) {
                const bool fb = !(sums[2 * j + 1] < sums[2 * j]);
                if (fb)
                    hipLaunchKernelGGL(zero_col, dim3(1024), dim3(256), 0, net->stream, X0, m, j, n);
                if (fallback) fallback[j] = fb ? 1 : 0;
            }
            net->chk(hipGetLastError(), "fallback");
        } else if (fallback) {
            for (int j = 0; j < m; ++j) fallback[j] = 0;
        }
        net->chk(hipStreamSynchronize(net->stream), "sync");
        net->tcollect();
    } catch (const xamg::DevFail& f) {
        return f.code;
    }
    return XAMG_OK;
}

int xamg_cnn_timer_enable(xamg_cnn_t* h, int32_t kind)
{
    Net* net = static_cast<Net*>(h);
    if (!net) return xamg::fail(XAMG_EINVAL, "null argument");
    if (kind < XAMG_CNN_TIMER_OFF || kind > XAMG_CNN_TIMER_WGRAD16)
        return xamg::fail(XAMG_EINVAL, "timer kind");
    try {
        net->chk(hipStreamSynchronize(net->stream), "sync");
        net->tcollect();
    } catch (const xamg::DevFail& f) {
        return f.code;
    }
    net->timer_kind = kind;
    net->timer_ms = 0.0;
    net->timer_count = 0;
    return XAMG_OK;
}

int xamg_cnn_timer_read(xamg_cnn_t* h, double* ms, int64_t* count)
{
    Net* net = static_cast<Net*>(h);
    if (!net || !ms || !count) return xamg::fail(XAMG_EINVAL, "null argument");
    try {
        net->chk(hipStreamSynchronize(net->stream), "sync");
        net->tcollect();
    } catch (const xamg::DevFail& f) {
        return f.code;
    }
    *ms = net->timer_ms;
    *count = net->timer_count;
    return XAMG_OK;
}

int xamg_cnn_destroy(xamg_cnn_t* h)
{
    Net* net = static_cast<Net*>(h);
    if (!net) return XAMG_OK;
    hipStreamSynchronize(net->stream);
    delete net;
    return XAMG_OK;
}

}  // extern "C"
