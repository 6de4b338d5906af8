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

} // namespace ising
