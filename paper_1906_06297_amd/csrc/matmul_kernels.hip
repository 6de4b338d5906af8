// gfx950 kernels of the matrix-multiply formulation of the checkerboard sweep
// (Sec. 3.2, the tensor-core implementation), kept as a measured negative
// control beside the bit-packed kernels.
//
// Storage: one fp16 per spin (+1 = 0x3C00, -1 = 0xBC00), the lattice cut into
// 256 x 256 sub-lattices, each stored as four 128 x 128 row-major blocks
// sigma_ab holding the sites (2r + a, 2q + b) (block index 2a + b).  Colour
// c = (a + b) & 1: black blocks 00, 11, white blocks 01, 10.
//
// Neighbour sums of a target block (a, b): its horizontal neighbours live in
// block P = (a, 1 - b), its vertical ones in Q = (1 - a, b), and the paper's
// four block equations are one form,
//     nn = P M1 + M2 Q,   M1 = (b ? K^T : K),   M2 = (a ? K : K^T),
// with K the 128 x 128 matrix of ones on the diagonal and the first
// superdiagonal.  The two products run as dense fp16 MFMA
// (v_mfma_f32_16x16x32_f16, fp32 sums -- exact for these small integers);
// K's fragments are formed in registers from the indices, once per tile and
// only where they are nonzero (the products stay dense).  The products miss
// one neighbour on one edge row and one edge column of the block, which
// comes from the adjacent sub-lattice (the boundary step).  The spin update
// then decides each run of 64 same-colour spins of a row -- one word of the
// bit-packed layout -- with the same Philox counters, planes and exact
// compare as the bit-packed kernels, so every variant yields the same
// lattice bit for bit.
//
// Two structures: the paper's (products writing fp16 sums to HBM, a boundary
// kernel, an update kernel), and one fused kernel that keeps the sums in LDS.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"
#include "ising_rows.hpp"
#include "matmul.hpp"

namespace ising {
namespace mm {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kB = 128;         // block edge
constexpr int kLd = kB + 8;     // LDS row stride in halves (272 B, 16-byte aligned rows)
constexpr int kThreads = 256;   // 4 wavefronts per block tile
constexpr uint16_t kPlus = 0x3C00, kMinus = 0xBC00;

// element offset of block (a, b) of sub-lattice (I, J); S sub-lattices per side
__device__ __forceinline__ size_t block_off(uint32_t S, uint32_t I, uint32_t J, uint32_t a,
                                            uint32_t b)
{
    return (((size_t)I * S + J) * 4 + (2 * a + b)) * (size_t)(kB * kB);
}

// The tile a workgroup owns: sub-lattice (I, J) and the target block (a, b)
// of colour c; both targets of a sub-lattice and neighbouring sub-lattices
// stay on one XCD (shared L2 for the edge reads).
struct Tile {
    uint32_t I, J, a, b, u;
};

__device__ __forceinline__ Tile tile_of(uint32_t S, int c)
{
    const uint32_t g = rows::xcd_block(blockIdx.x, gridDim.x);
    const uint32_t sl = g >> 1, u = g & 1u;
    Tile t;
    t.I = sl / S;
    t.J = sl - t.I * S;
    t.u = u;
    t.a = u;
    t.b = (u + (uint32_t)c) & 1u;
    return t;
}

// 128 x 128 fp16 block from global into LDS, row-major
__device__ __forceinline__ void load_block(_Float16 (*dst)[kLd], const uint16_t *src)
{
#pragma unroll
    for (int it = 0; it < kB * kB / 8 / kThreads; ++it) {
        const int v = it * kThreads + (int)threadIdx.x;
        const int row = v >> 4, col = (v & 15) * 8;
        *reinterpret_cast<uint4 *>(&dst[row][col]) =
            *reinterpret_cast<const uint4 *>(src + row * kB + col);
    }
}

// ... and transposed (dst[col][row]): the B operand of M2 Q reads columns of Q
__device__ __forceinline__ void load_block_t(_Float16 (*dst)[kLd], const uint16_t *src)
{
#pragma unroll
    for (int it = 0; it < kB * kB / 8 / kThreads; ++it) {
        const int v = it * kThreads + (int)threadIdx.x;
        const int row = v >> 4, col = (v & 15) * 8;
        const uint4 x = *reinterpret_cast<const uint4 *>(src + row * kB + col);
        const uint32_t w[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const uint16_t h = (uint16_t)(w[e >> 1] >> (16 * (e & 1)));
            dst[col + e][row] = __builtin_bit_cast(_Float16, h);
        }
    }
}

__device__ __forceinline__ void store_block(uint16_t *dst, _Float16 (*src)[kLd])
{
#pragma unroll
    for (int it = 0; it < kB * kB / 8 / kThreads; ++it) {
        const int v = it * kThreads + (int)threadIdx.x;
        const int row = v >> 4, col = (v & 15) * 8;
        *reinterpret_cast<uint4 *>(dst + row * kB + col) =
            *reinterpret_cast<const uint4 *>(&src[row][col]);
    }
}

// K (ones at [x][x] and [x][x + 1]) or its transpose, as 8 consecutive
// k-entries of one row (A operand) or one column (B operand).
__device__ __forceinline__ half8 k_row(uint32_t row, uint32_t k0, bool transposed)
{
    half8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const uint32_t k = k0 + e;
        // K[row][k]: k == row or k == row + 1; K^T[row][k]: row == k or row == k + 1
        const bool one = (k == row) || (transposed ? (row == k + 1) : (k == row + 1));
        v[e] = one ? (_Float16)1.0f : (_Float16)0.0f;
    }
    return v;
}

__device__ __forceinline__ half8 k_col(uint32_t col, uint32_t k0, bool transposed)
{
    // column col of M = row col of M^T
    return k_row(col, k0, !transposed);
}

// nn = P M1 + M2 Q for the whole block: wavefront w owns rows 32w .. 32w + 31
// (two 16-row MFMA tiles) by all 128 columns (eight 16-column tiles), four
// 32-deep k steps, two products each.  Leaves the sums in `out` (fp16,
// row-major), which may alias P's buffer: every wavefront has finished its
// products when the first sum is written.
__device__ __forceinline__ void block_products(_Float16 (*sP)[kLd], _Float16 (*sQt)[kLd], bool a,
                                               bool b, _Float16 (*out)[kLd])
{
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    const uint32_t r16 = lane & 15u, kq = lane >> 4;
    f32x4 acc[2][8];
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int n = 0; n < 8; ++n)
            acc[mi][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    // M1's fragment of column tile n at k step ks depends only on n - 2 ks
    // and is zero unless that is -1 .. 2: the four nonzero ones, formed once
    // (indices shifted by 32, as only differences of row and column matter)
    half8 m1f[4];
#pragma unroll
    for (int d = 0; d < 4; ++d)
        m1f[d] = k_col((uint32_t)(16 * d + 16) + r16, 32 + kq * 8, b); // n - 2 ks = d - 1
    const half8 zero8 = {};
#pragma unroll
    for (uint32_t k0 = 0; k0 < (uint32_t)kB; k0 += 32) {
        const uint32_t kk = k0 + kq * 8;
        half8 pa[2], ma[2];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
            const uint32_t row = (2 * w + mi) * 16 + r16;
            pa[mi] = *reinterpret_cast<const half8 *>(&sP[row][kk]);
            // M2 = K for a = 1, K^T for a = 0; zero unless the row tile is within
            // one of this k step's diagonal block (a wave-uniform test)
            const int d = (int)(2 * w + mi) - (int)(k0 / 16);
            ma[mi] = (d >= -1 && d <= 2) ? k_row(row, kk, !a) : zero8;
        }
#pragma unroll
        for (int n = 0; n < 8; ++n) {
            const uint32_t col = n * 16 + r16;
            const int d = n - (int)(k0 / 16); // n - 2 ks
            const half8 mb = (d >= -1 && d <= 2) ? m1f[d + 1] : zero8; // M1 = K^T (b) or K
            const half8 qb = *reinterpret_cast<const half8 *>(&sQt[col][kk]);
#pragma unroll
            for (int mi = 0; mi < 2; ++mi) {
                acc[mi][n] = __builtin_amdgcn_mfma_f32_16x16x32_f16(pa[mi], mb, acc[mi][n], 0, 0, 0);
                acc[mi][n] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ma[mi], qb, acc[mi][n], 0, 0, 0);
            }
        }
    }
    __syncthreads(); // products done before `out` (P's buffer) is overwritten
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int n = 0; n < 8; ++n)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                out[(2 * w + mi) * 16 + kq * 4 + e][n * 16 + r16] = (_Float16)acc[mi][n][e];
}

// The neighbour of each edge site that lies in the adjacent sub-lattice:
// thread t < 128 adds the horizontal one of row t (column edge), thread
// 128 + q the vertical one of column q (row edge); the corner takes both from
// the row thread.  `sum(row, col)` returns a reference to the sum.
template <typename SumRef>
__device__ __forceinline__ void add_edges(const uint16_t *spins, uint32_t S, const Tile &tl,
                                          SumRef sum)
{
    const uint32_t t = threadIdx.x;
    const uint32_t qe = tl.b ? kB - 1 : 0, re = tl.a ? kB - 1 : 0;
    const uint32_t Jn = tl.b ? (tl.J + 1 == S ? 0 : tl.J + 1) : (tl.J == 0 ? S - 1 : tl.J - 1);
    const uint32_t In = tl.a ? (tl.I + 1 == S ? 0 : tl.I + 1) : (tl.I == 0 ? S - 1 : tl.I - 1);
    // horizontal: block (a, 1 - b) of (I, Jn), its column 0 (b = 1) or 127 (b = 0)
    const uint16_t *ph = spins + block_off(S, tl.I, Jn, tl.a, 1 - tl.b);
    // vertical: block (1 - a, b) of (In, J), its row 0 (a = 1) or 127 (a = 0)
    const uint16_t *pv = spins + block_off(S, In, tl.J, 1 - tl.a, tl.b);
    const uint32_t hcol = tl.b ? 0 : kB - 1, vrow = tl.a ? 0 : kB - 1;
    auto val = [](uint16_t h) { return (float)__builtin_bit_cast(_Float16, h); };
    if (t < (uint32_t)kB) {
        float add = val(ph[t * kB + hcol]);
        if (t == re)
            add += val(pv[vrow * kB + qe]);
        auto &x = sum(t, qe);
        x = (_Float16)((float)x + add);
    } else {
        const uint32_t q = t - kB;
        if (q != qe) {
            auto &x = sum(re, q);
            x = (_Float16)((float)x + val(pv[vrow * kB + q]));
        }
    }
}

// Each thread decides one run of 64 same-colour spins (row r = t / 2, half
// h = t % 2 of the block row), which is word i * (L / 128) + 2 J + h of the
// bit-packed colour array, with that word's Philox blocks; spins and sums
// are read from LDS and the new spins written back in place.
template <bool Anti, bool Plain>
__device__ __forceinline__ void update_words(_Float16 (*sT)[kLd], _Float16 (*sN)[kLd],
                                             uint32_t S, const Tile &tl, const SweepArgs2 &a)
{
    const uint32_t t = threadIdx.x, r = t >> 1, h = t & 1u;
    const uint32_t i = 256 * tl.I + 2 * r + tl.a;
    const uint32_t chunk = i * (2 * S) + 2 * tl.J + h;
    const rows::ClassMasks cm = rows::class_masks(a.m);
    rows::State s;
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        uint32_t tb = 0, ge2 = 0, one = 0, zero = 0;
#pragma unroll
        for (int v8 = 0; v8 < 4; ++v8) {
            const uint32_t col = 64 * h + 32 * hh + 8 * v8;
            const half8 sp = *reinterpret_cast<const half8 *>(&sT[r][col]);
            const half8 nn = *reinterpret_cast<const half8 *>(&sN[r][col]);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const bool up = (float)sp[e] > 0.f;
                const int n = (int)(float)nn[e];
                const int aligned = (4 + (up ? n : -n)) / 2;
                // J > 0: classes by the number of unlike neighbours; J < 0: by
                // the number of like ones
                const int cnt = Anti ? aligned : 4 - aligned;
                const uint32_t bit = 1u << (8 * v8 + e);
                tb |= up ? bit : 0u;
                ge2 |= cnt >= 2 ? bit : 0u;
                one |= cnt == 1 ? bit : 0u;
                zero |= cnt == 0 ? bit : 0u;
            }
        }
        rows::start_half<Plain>(s, hh, tb, rows::Split{ge2, one, zero}, cm);
    }
    for (uint32_t q = 0; q < 16 && (s.p[0] | s.p[1]) != 0; ++q)
        rows::block_uniform(s, q, chunk, a);
#pragma unroll
    for (int hh = 0; hh < 2; ++hh)
#pragma unroll
        for (int x = 0; x < 32; ++x)
            sT[r][64 * h + 32 * hh + x] =
                __builtin_bit_cast(_Float16, ((s.tf[hh] >> x) & 1u) ? kPlus : kMinus);
}

// ----------------------------------------------------------- fused half-sweep
template <bool Anti, bool Plain>
__global__ __launch_bounds__(kThreads) void k_mm_fused(uint16_t *__restrict__ spins, uint32_t S,
                                                       int c, SweepArgs2 a)
{
    __shared__ _Float16 sP[kB][kLd], sQt[kB][kLd];
    const Tile tl = tile_of(S, c);
    load_block(sP, spins + block_off(S, tl.I, tl.J, tl.a, 1 - tl.b));
    load_block_t(sQt, spins + block_off(S, tl.I, tl.J, 1 - tl.a, tl.b));
    __syncthreads();
    block_products(sP, sQt, tl.a, tl.b, sP); // sums replace P
    __syncthreads();
    uint16_t *tgt = spins + block_off(S, tl.I, tl.J, tl.a, tl.b);
    load_block(sQt, tgt); // target spins replace Q^T
    add_edges(spins, S, tl, [&](uint32_t r, uint32_t q) -> _Float16 & { return sP[r][q]; });
    __syncthreads();
    update_words<Anti, Plain>(sQt, sP, S, tl, a);
    __syncthreads();
    store_block(tgt, sQt);
}

// --------------------------------------------- the paper's three-step form
// (1) products: fp16 sums of every target block to HBM, tile (sub-lattice,
// u) at (sl * 2 + u) * 128 * 128.
__global__ __launch_bounds__(kThreads) void k_mm_products(const uint16_t *__restrict__ spins,
                                                          uint16_t *__restrict__ sums, uint32_t S,
                                                          int c)
{
    __shared__ _Float16 sP[kB][kLd], sQt[kB][kLd];
    const Tile tl = tile_of(S, c);
    load_block(sP, spins + block_off(S, tl.I, tl.J, tl.a, 1 - tl.b));
    load_block_t(sQt, spins + block_off(S, tl.I, tl.J, 1 - tl.a, tl.b));
    __syncthreads();
    block_products(sP, sQt, tl.a, tl.b, sP);
    __syncthreads();
    store_block(sums + ((size_t)(tl.I * S + tl.J) * 2 + tl.u) * (kB * kB), sP);
}

// (2) boundary: the edge neighbours added to the sums in HBM (the column
// edge is strided in memory).
__global__ __launch_bounds__(kThreads) void k_mm_boundary(const uint16_t *__restrict__ spins,
                                                          uint16_t *__restrict__ sums, uint32_t S,
                                                          int c)
{
    const Tile tl = tile_of(S, c);
    uint16_t *tile = sums + ((size_t)(tl.I * S + tl.J) * 2 + tl.u) * (kB * kB);
    add_edges(spins, S, tl, [&](uint32_t r, uint32_t q) -> _Float16 & {
        return *reinterpret_cast<_Float16 *>(tile + r * kB + q);
    });
}

// (3) update: sums and target spins from HBM, new spins to HBM.
template <bool Anti, bool Plain>
__global__ __launch_bounds__(kThreads) void k_mm_update(uint16_t *__restrict__ spins,
                                                        const uint16_t *__restrict__ sums,
                                                        uint32_t S, int c, SweepArgs2 a)
{
    __shared__ _Float16 sN[kB][kLd], sT[kB][kLd];
    const Tile tl = tile_of(S, c);
    uint16_t *tgt = spins + block_off(S, tl.I, tl.J, tl.a, tl.b);
    load_block(sN, sums + ((size_t)(tl.I * S + tl.J) * 2 + tl.u) * (kB * kB));
    load_block(sT, tgt);
    __syncthreads();
    update_words<Anti, Plain>(sT, sN, S, tl, a);
    __syncthreads();
    store_block(tgt, sT);
}

// ----------------------------------------------------- layout conversions
// One thread per bit-packed word (both colours, grid-stride): word k of
// colour c is row i = k / (L / 128), column word w; its 64 spins are the run
// of block (i & 1, (i + c) & 1) of sub-lattice (i / 256, w / 2), block row
// (i % 256) / 2, columns 64 (w & 1) .. + 63.
__global__ __launch_bounds__(256) void k_mm_from_words(const uint64_t *__restrict__ words,
                                                       uint16_t *__restrict__ spins, uint32_t S,
                                                       int64_t W)
{
    const uint32_t Wr = 2 * S;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < 2 * W; g += stride) {
        const int c = g >= W;
        const int64_t k = g - (c ? W : 0);
        const uint32_t i = (uint32_t)(k / Wr), w = (uint32_t)(k - (int64_t)i * Wr);
        const uint32_t a = i & 1u, b = (i + (uint32_t)c) & 1u, r = (i & 255u) >> 1;
        uint16_t *dst = spins + block_off(S, i >> 8, w >> 1, a, b) + r * kB + 64 * (w & 1u);
        const uint64_t x = words[g];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            uint32_t p[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int bit = 8 * v + 2 * e;
                p[e] = (uint32_t)(((x >> bit) & 1u) ? kPlus : kMinus) |
                       ((uint32_t)(((x >> (bit + 1)) & 1u) ? kPlus : kMinus) << 16);
            }
            *reinterpret_cast<uint4 *>(dst + 8 * v) = uint4{p[0], p[1], p[2], p[3]};
        }
    }
}

__global__ __launch_bounds__(256) void k_mm_to_words(const uint16_t *__restrict__ spins,
                                                     uint64_t *__restrict__ words, uint32_t S,
                                                     int64_t W)
{
    const uint32_t Wr = 2 * S;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < 2 * W; g += stride) {
        const int c = g >= W;
        const int64_t k = g - (c ? W : 0);
        const uint32_t i = (uint32_t)(k / Wr), w = (uint32_t)(k - (int64_t)i * Wr);
        const uint32_t a = i & 1u, b = (i + (uint32_t)c) & 1u, r = (i & 255u) >> 1;
        const uint16_t *src = spins + block_off(S, i >> 8, w >> 1, a, b) + r * kB + 64 * (w & 1u);
        uint64_t x = 0;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            const uint4 q = *reinterpret_cast<const uint4 *>(src + 8 * v);
            const uint32_t p[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const uint16_t hv = (uint16_t)(p[e >> 1] >> (16 * (e & 1)));
                x |= (uint64_t)((hv & 0x8000u) == 0) << (8 * v + e); // sign bit clear: +1
            }
        }
        words[g] = x;
    }
}

// ------------------------------------------------------------------ launches
namespace {
constexpr uint32_t kMaxStrideBlocks = 1u << 20;

uint32_t stride_blocks(int64_t n)
{
    const int64_t nb = (n + 255) / 256;
    return (uint32_t)(nb < (int64_t)kMaxStrideBlocks ? nb : kMaxStrideBlocks);
}
} // namespace

hipError_t launch_from_words(const uint64_t *words, uint16_t *spins, int64_t L, hipStream_t s)
{
    const int64_t W = L * L / 128;
    hipLaunchKernelGGL(k_mm_from_words, dim3(stride_blocks(2 * W)), dim3(256), 0, s, words, spins,
                       (uint32_t)(L / 256), W);
    return hipGetLastError();
}

hipError_t launch_to_words(const uint16_t *spins, uint64_t *words, int64_t L, hipStream_t s)
{
    const int64_t W = L * L / 128;
    hipLaunchKernelGGL(k_mm_to_words, dim3(stride_blocks(2 * W)), dim3(256), 0, s, spins, words,
                       (uint32_t)(L / 256), W);
    return hipGetLastError();
}

hipError_t launch_half_sweep(uint16_t *spins, uint16_t *sums, int64_t L, int c, const Metro2 &m,
                             uint64_t t, uint64_t seed, uint32_t stream_id, bool fused,
                             hipStream_t s)
{
    const uint32_t S = (uint32_t)(L / 256);
    const dim3 grid(2 * S * S), block(kThreads);
    const SweepArgs2 a{m, (uint32_t)t, (uint32_t)(t >> 32), stream_id, (uint32_t)seed,
                       (uint32_t)(seed >> 32)};
    const bool plain = m.randA && m.randB && !m.alwaysA && !m.alwaysB;
    const int sel = (m.anti ? 2 : 0) + (plain ? 1 : 0);
    if (fused) {
        using Kernel = void (*)(uint16_t *, uint32_t, int, SweepArgs2);
        static const Kernel kernels[4] = {k_mm_fused<false, false>, k_mm_fused<false, true>,
                                          k_mm_fused<true, false>, k_mm_fused<true, true>};
        hipLaunchKernelGGL(kernels[sel], grid, block, 0, s, spins, S, c, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_mm_products, grid, block, 0, s, spins, sums, S, c);
    hipLaunchKernelGGL(k_mm_boundary, grid, block, 0, s, spins, sums, S, c);
    using Kernel = void (*)(uint16_t *, const uint16_t *, uint32_t, int, SweepArgs2);
    static const Kernel kernels[4] = {k_mm_update<false, false>, k_mm_update<false, true>,
                                      k_mm_update<true, false>, k_mm_update<true, true>};
    hipLaunchKernelGGL(kernels[sel], grid, block, 0, s, spins, sums, S, c, a);
    return hipGetLastError();
}

} // namespace mm
} // namespace ising
