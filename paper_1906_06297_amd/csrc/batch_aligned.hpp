// Neighbour vectors for the batch kernel when a colour row is a whole number
// of words (H = L/2 a multiple of 64, i.e. L % 128 == 0): no word straddles
// two rows, so the vertical neighbours are whole words Wr = H/64 away and the
// side neighbour is the centre word shifted by one spin, with the edge spin
// taken from the adjacent word of the same row, or from the other end of the
// row at a row's first and last word (periodic rows; Sec. 3.3, Fig. 3).
// Gives what neighbours_ext_rm gives for these sizes, without its row-mask
// loop, division and funnel shifts.  Plain bit logic, compiled for the host
// in the tests too.
#pragma once

#include <stdint.h>

#include "ising_device.hpp"

namespace ising {

// Row of word k for Wr <= 5 words per row and k < 4096 words per colour:
// floor(k / Wr) as a multiply by ceil(2^16 / Wr); the rounding error
// k / 2^16 < 1/16 stays below the 1/Wr gap to the next integer.
__host__ __device__ __forceinline__ uint32_t aligned_row(uint32_t k, uint32_t inv_wr)
{
    return (k * inv_wr) >> 16;
}

__host__ __device__ __forceinline__ uint32_t aligned_inv(uint32_t Wr)
{
    return (65536u + Wr - 1) / Wr;
}

// Word k of colour c (0 = black) from the other colour's W words in E;
// Wr words per row, inv_wr = aligned_inv(Wr).
template <typename Ptr>
__host__ __device__ __forceinline__ Neighbours neighbours_aligned(Ptr E, uint32_t W, uint32_t Wr,
                                                                  uint32_t inv_wr, uint32_t k,
                                                                  int c)
{
    const uint32_t row = aligned_row(k, inv_wr), col = k - row * Wr;
    Neighbours nb;
    nb.ce = E[k];
    nb.up = E[k >= Wr ? k - Wr : k + W - Wr];
    nb.dn = E[k + Wr < W ? k + Wr : k + Wr - W];
    // the spin before the word's first and after its last, within the row
    const uint64_t before = E[col == 0 ? k + Wr - 1 : k - 1];
    const uint64_t after = E[col == Wr - 1 ? k + 1 - Wr : k + 1];
    const uint64_t left = (nb.ce << 1) | (before >> 63);
    const uint64_t right = (nb.ce >> 1) | (after << 63);
    // rows whose side neighbour is on the left: (row + c) even
    nb.sd = ((row + (uint32_t)c) & 1u) == 0 ? left : right;
    return nb;
}

// Colour rows of a whole number of 32-bit halves (H = L/2 a multiple of 32,
// i.e. L % 64 == 0; used where H is not a multiple of 64, as for L = 64 and
// 192): every half lies in one row, so the vertical neighbours of half h are
// the halves Hr = H/32 away (periodic over the colour's 2W halves) and its
// side neighbour is half h shifted by one spin with the edge spin taken from
// the adjacent half of its row, or from the row's other end.  E is the other
// colour as 32-bit halves (half h = bits 32(h&1).. of word h>>1).

// Row of half h for h < 8192 and Hr <= 11: floor(h / Hr) as a multiply by
// ceil(2^18 / Hr); the error h / 2^18 < 1/32 stays below the 1/Hr gap.
__host__ __device__ __forceinline__ uint32_t half_row(uint32_t h, uint32_t inv_hr)
{
    return (h * inv_hr) >> 18;
}

__host__ __device__ __forceinline__ uint32_t half_inv(uint32_t Hr)
{
    return ((1u << 18) + Hr - 1) / Hr;
}

template <typename Ptr32>
__host__ __device__ __forceinline__ Neighbours neighbours_half_aligned(Ptr32 E, uint32_t W,
                                                                       uint32_t Hr,
                                                                       uint32_t inv_hr, uint32_t k,
                                                                       int c)
{
    const uint32_t NH = 2 * W, h0 = 2 * k;
    const uint32_t r0 = half_row(h0, inv_hr), o0 = h0 - r0 * Hr;
    uint32_t up[2], dn[2], ce[2], sd[2];
#pragma unroll
    for (uint32_t hh = 0; hh < 2; ++hh) {
        const uint32_t h = h0 + hh;
        const bool next_row = hh == 1 && o0 + 1 == Hr;
        const uint32_t r = r0 + (next_row ? 1u : 0u), o = next_row ? 0u : o0 + hh;
        ce[hh] = E[h];
        up[hh] = E[h >= Hr ? h - Hr : h + NH - Hr];
        dn[hh] = E[h + Hr < NH ? h + Hr : h + Hr - NH];
        const uint32_t before = E[o == 0 ? h + Hr - 1 : h - 1];
        const uint32_t after = E[o == Hr - 1 ? h + 1 - Hr : h + 1];
        const uint32_t left = (ce[hh] << 1) | (before >> 31);
        const uint32_t right = (ce[hh] >> 1) | (after << 31);
        // rows whose side neighbour is on the left: (row + c) even
        sd[hh] = ((r + (uint32_t)c) & 1u) == 0 ? left : right;
    }
    Neighbours nb;
    nb.ce = (uint64_t)ce[0] | ((uint64_t)ce[1] << 32);
    nb.up = (uint64_t)up[0] | ((uint64_t)up[1] << 32);
    nb.dn = (uint64_t)dn[0] | ((uint64_t)dn[1] << 32);
    nb.sd = (uint64_t)sd[0] | ((uint64_t)sd[1] << 32);
    return nb;
}

// The general extraction (any geometry, extended colour array) on 32-bit
// halves: a 64-spin window at spin x is two funnel shifts of three
// consecutive halves, and the wrapped positions are 32-bit (every spin index
// of a batch lattice is below 2^18).  Same vectors as neighbours_ext_rm.
__host__ __device__ __forceinline__ uint32_t funnel32(uint32_t hi, uint32_t lo, uint32_t sh)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_alignbit(hi, lo, sh);
#else
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> sh);
#endif
}

template <typename Ptr32>
__host__ __device__ __forceinline__ uint64_t ext_bits32(Ptr32 E, uint32_t x)
{
    const uint32_t w = x >> 5, sh = x & 31;
    const uint32_t d0 = E[w], d1 = E[w + 1], d2 = E[w + 2];
    return (uint64_t)funnel32(d1, d0, sh) | ((uint64_t)funnel32(d2, d1, sh) << 32);
}

__host__ __device__ __forceinline__ uint32_t wrap32(int32_t x, uint32_t M)
{
    return (uint32_t)(x < 0 ? x + (int32_t)M : (x >= (int32_t)M ? x - (int32_t)M : x));
}

template <typename Ptr32>
__host__ __device__ __forceinline__ Neighbours neighbours_ext32(Ptr32 E, uint32_t H, uint32_t M,
                                                                uint32_t k, const RowMasks &rm)
{
    const int32_t n0 = (int32_t)(k << 6), h = (int32_t)H;
    Neighbours nb;
    nb.ce = ext_bits32(E, (uint32_t)n0);
    nb.up = ext_bits32(E, wrap32(n0 - h, M));
    nb.dn = ext_bits32(E, wrap32(n0 + h, M));
    const uint64_t left = (ext_bits32(E, wrap32(n0 - 1, M)) & ~rm.row_start) |
                          (ext_bits32(E, wrap32(n0 + h - 1, M)) & rm.row_start);
    const uint64_t right = (ext_bits32(E, wrap32(n0 + 1, M)) & ~rm.row_end) |
                           (ext_bits32(E, wrap32(n0 - h + 1, M)) & rm.row_end);
    nb.sd = (left & rm.left_rows) | (right & ~rm.left_rows);
    return nb;
}

} // namespace ising
