// gfx950 kernels of the +-J spin glass (the extension the paper's conclusions
// name): bond-sign arrays, the half-sweep and the observables.
//
// Couplings J_ij = J * (1 - 2 b_ij), b_ij one bit per bond.  Four bit arrays
// in the colour-compact layout of the spins (W words each, padding bits 0),
// interleaved word by word (word 4 k + x is word k of array x): x = 0, 1: the
// bond to the right of each colour-x site; x = 2, 3: the bond below each
// colour-(x - 2) site.  Every bond is stored once, and the four words that a
// spin word k needs sit in one 32-byte chunk.  For a target word of colour c
// the four bond vectors, aligned bit for bit with the target spins, are: up =
// down bonds of colour 1 - c one row above, down = down bonds of colour c,
// right = right bonds of colour c, left = right bonds of colour 1 - c at the
// left neighbour (the same word, or the side shift of Sec. 3.3 when the left
// neighbour is the side neighbour).  XORing a bond bit into the neighbour bit
// turns s * b * n into s * n', so the aligned-count classes, thresholds and
// compare of the ferromagnetic kernels apply unchanged.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "glass.hpp"
#include "ising_device.hpp"
#include "ising_rows.hpp"
#include "launch.hpp"

namespace ising {

enum : uint32_t { kDomainCouplings = 4 };

// Random bond signs (probability 1/2): array x word k (stored at 4 k + x) is
// x0 | x1 << 32 of Philox block (stream << 8 | 4 << 4 | x, 0, 0, k), padding
// bits cleared.
__global__ __launch_bounds__(256) void k_glass_bonds_init(uint64_t *__restrict__ bonds, int64_t M,
                                                          int64_t W, uint32_t key0, uint32_t key1,
                                                          uint32_t stream_id)
{
    // grid-stride: 4 W can exceed the 2^32 work-items of one dispatch
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < 4 * W; g += stride) {
        const uint32_t x = (uint32_t)(g & 3);
        const int64_t k = g >> 2;
        const Block b = philox4x32_10(ctr_word0(stream_id, kDomainCouplings, x), 0u, 0u,
                                      (uint32_t)k, key0, key1);
        bonds[g] = ((uint64_t)b.x0 | ((uint64_t)b.x1 << 32)) & valid_mask(k, M);
    }
}

// Bond vectors of target word (row i, column word w) of colour c; `left`:
// the side neighbour is the left one.
struct BondVectors {
    uint64_t up, dn, ce, sd;
};

__device__ __forceinline__ BondVectors bond_vectors(const uint64_t *__restrict__ bonds, int64_t Wr,
                                                    int64_t L, int c, int64_t i, int64_t w,
                                                    int64_t wl, bool left)
{
    // word (row, column word) of array x
    const auto at = [&](int64_t row, int64_t col, int x) { return bonds[4 * (row * Wr + col) + x]; };
    const int64_t iu = (i == 0) ? L - 1 : i - 1;
    BondVectors v;
    v.up = at(iu, w, 3 - c);
    v.dn = at(i, w, 2 + c);
    const uint64_t right = at(i, w, c);
    const uint64_t left_aligned = at(i, w, 1 - c);
    if (left) { // centre = right neighbour, side = left neighbour (jc - 1)
        v.ce = right;
        v.sd = side_vector(left_aligned, at(i, wl, 1 - c), true);
    } else { // centre = left neighbour, side = right neighbour
        v.ce = left_aligned;
        v.sd = right;
    }
    return v;
}

// Half-sweep of colour c, row-aligned lattices: one thread per word column
// of a band of kGlassRows rows (three spin rows in registers), each word
// decided on its own (blocks until all its spins are decided).
constexpr int kGlassRows = 16;

template <bool Anti, bool Plain>
__global__ __launch_bounds__(256) void k_glass_rows(uint64_t *__restrict__ tgt,
                                                    const uint64_t *__restrict__ src,
                                                    const uint64_t *__restrict__ bonds, int64_t L,
                                                    int64_t Wr, int64_t blocks_per_band, int c,
                                                    SweepArgs2 a)
{
    const int64_t band = blockIdx.x / blocks_per_band;
    const int64_t w = (blockIdx.x - band * blocks_per_band) * (int64_t)blockDim.x + threadIdx.x;
    if (w >= Wr)
        return;
    const int64_t i0 = band * kGlassRows;
    const int64_t wl = (w == 0) ? Wr - 1 : w - 1;
    const int64_t wr = (w == Wr - 1) ? 0 : w + 1;
    const rows::ClassMasks cm = rows::class_masks(a.m);
    uint64_t prev = src[((i0 == 0) ? L - 1 : i0 - 1) * Wr + w];
    uint64_t cur = src[i0 * Wr + w];
    for (int r = 0; r < kGlassRows; ++r) {
        const int64_t i = i0 + r;
        if (i >= L)
            break;
        const uint64_t next = src[((i + 1 == L) ? 0 : i + 1) * Wr + w];
        const int64_t idx = i * Wr + w;
        const bool left = ((i + c) & 1) == 0;
        const uint64_t t = tgt[idx];
        const uint64_t sd = side_vector(cur, src[i * Wr + (left ? wl : wr)], left);
        const BondVectors b = bond_vectors(bonds, Wr, L, c, i, w, wl, left);
        const uint64_t nu = prev ^ b.up, nd = next ^ b.dn, nc = cur ^ b.ce, ns = sd ^ b.sd;
        rows::State s;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const auto half = [h](uint64_t v) { return h ? rows::hi32(v) : rows::lo32(v); };
            rows::start_half<Plain>(
                s, h, half(t),
                rows::split_classes<Anti>(half(t), half(nu), half(nd), half(nc), half(ns)), cm);
        }
        for (uint32_t q = 0; q < 16 && (s.p[0] | s.p[1]) != 0; ++q)
            rows::block_uniform(s, q, (uint32_t)idx, a);
        tgt[idx] = rows::join(s.tf[0], s.tf[1]);
        prev = cur;
        cur = next;
    }
}

// Bond sum sum over bonds of (J_ij / J) s_i s_j and magnetisation: over black
// words, the aligned count of the bond-corrected neighbours gives each black
// site's four bonds once.
__global__ __launch_bounds__(256) void k_glass_observables(const uint64_t *__restrict__ black,
                                                           const uint64_t *__restrict__ white,
                                                           const uint64_t *__restrict__ bonds,
                                                           int64_t L, int64_t Wr,
                                                           int64_t *bond_out, int64_t *mag_out)
{
    int64_t bond = 0, mag = 0;
    const int64_t W = L * Wr, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < W; k += stride) {
        const int64_t i = k / Wr, w = k - i * Wr;
        const uint64_t t = black[k], ce = white[k];
        const uint64_t up = white[((i == 0) ? L - 1 : i - 1) * Wr + w];
        const uint64_t dn = white[((i + 1 == L) ? 0 : i + 1) * Wr + w];
        const bool left = (i & 1) == 0; // colour 0: side neighbour on the left on even rows
        const int64_t wl = (w == 0) ? Wr - 1 : w - 1, wr = (w + 1 == Wr) ? 0 : w + 1;
        const uint64_t sd = side_vector(ce, white[i * Wr + (left ? wl : wr)], left);
        const BondVectors b = bond_vectors(bonds, Wr, L, 0, i, w, wl, left);
        const int64_t aligned =
            (int64_t)__popcll(~(t ^ up ^ b.up)) + (int64_t)__popcll(~(t ^ dn ^ b.dn)) +
            (int64_t)__popcll(~(t ^ ce ^ b.ce)) + (int64_t)__popcll(~(t ^ sd ^ b.sd));
        bond += 2 * aligned - 4 * 64;
        mag += 2 * ((int64_t)__popcll(t) + (int64_t)__popcll(ce)) - 2 * 64;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        bond += __shfl_xor(bond, off, 64);
        mag += __shfl_xor(mag, off, 64);
    }
    __shared__ int64_t part[2][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        part[0][wv] = bond;
        part[1][wv] = mag;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t bs = 0, ms = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
            bs += part[0][q];
            ms += part[1][q];
        }
        atomicAdd((unsigned long long *)bond_out, (unsigned long long)bs);
        atomicAdd((unsigned long long *)mag_out, (unsigned long long)ms);
    }
}

__global__ void k_glass_zero2(int64_t *a, int64_t *b)
{
    if (threadIdx.x == 0) {
        *a = 0;
        *b = 0;
    }
}

// ------------------------------------------------------------------ launches
hipError_t launch_glass_bonds_init(uint64_t *bonds, int64_t L, uint64_t seed, uint32_t stream_id,
                                   hipStream_t s)
{
    const int64_t M = L * L / 2, W = (M + 63) / 64;
    const int64_t nb = (4 * W + 255) / 256;
    hipLaunchKernelGGL(k_glass_bonds_init, dim3((uint32_t)(nb < (1 << 20) ? nb : (1 << 20))),
                       dim3(256), 0, s, bonds, M, W, (uint32_t)seed, (uint32_t)(seed >> 32),
                       stream_id);
    return hipGetLastError();
}

hipError_t launch_glass_half_sweep(uint64_t *words, const uint64_t *bonds, int64_t L, int c,
                                   const Metro2 &m, uint64_t t, uint64_t seed, uint32_t stream_id,
                                   hipStream_t s, int variant)
{
    const int64_t Wr = L / 128, W = L * Wr;
    uint64_t *tgt = words + (int64_t)c * W;
    const uint64_t *src = words + (int64_t)(1 - c) * W;
    const SweepArgs2 a{m, (uint32_t)t, (uint32_t)(t >> 32), stream_id, (uint32_t)seed,
                       (uint32_t)(seed >> 32)};
    if (variant != kVariantGeneral && variant != kVariantRowsPlain)
        return launch_rows_queue(tgt, src, bonds, L, c, m, a, s,
                                 variant == kVariantQueue16 ? 16
                                                            : (variant == kVariantQueue8 ? 8 : 32));
    const int threads = Wr >= 256 ? 256 : (Wr >= 64 ? 64 * (int)((Wr + 63) / 64) : 64);
    const int64_t bpb = (Wr + threads - 1) / threads;
    const int64_t bands = (L + kGlassRows - 1) / kGlassRows;
    const bool plain = m.randA && m.randB && !m.alwaysA && !m.alwaysB;
    using Kernel = void (*)(uint64_t *, const uint64_t *, const uint64_t *, int64_t, int64_t,
                            int64_t, int, SweepArgs2);
    static const Kernel kernels[4] = {k_glass_rows<false, false>, k_glass_rows<false, true>,
                                      k_glass_rows<true, false>, k_glass_rows<true, true>};
    hipLaunchKernelGGL(kernels[(m.anti ? 2 : 0) + (plain ? 1 : 0)], dim3((uint32_t)(bands * bpb)),
                       dim3(threads), 0, s, tgt, src, bonds, L, Wr, bpb, c, a);
    return hipGetLastError();
}

hipError_t launch_glass_observables(const uint64_t *words, const uint64_t *bonds, int64_t L,
                                    int64_t *bond, int64_t *mag, hipStream_t s)
{
    const int64_t Wr = L / 128, W = L * Wr;
    hipLaunchKernelGGL(k_glass_zero2, dim3(1), dim3(64), 0, s, bond, mag);
    const uint32_t nb = (uint32_t)((W + 255) / 256 < 4096 ? (W + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_glass_observables, dim3(nb), dim3(256), 0, s, words, words + W, bonds, L,
                       Wr, bond, mag);
    return hipGetLastError();
}

} // namespace ising
