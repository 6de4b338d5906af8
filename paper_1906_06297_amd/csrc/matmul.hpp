// Host-side launchers of the matrix-multiply formulation (internal to libising).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"

namespace ising {
namespace mm {

// Bit-packed colour arrays (2 * L * L / 128 words) <-> fp16 block layout
// (L * L halves); L % 256 == 0.
hipError_t launch_from_words(const uint64_t *words, uint16_t *spins, int64_t L, hipStream_t s);
hipError_t launch_to_words(const uint16_t *spins, uint64_t *words, int64_t L, hipStream_t s);
// Half-sweep of colour c: fused (sums in LDS; `sums` unused) or the
// three-kernel form (sums of the colour, L * L / 2 halves, through HBM).
hipError_t launch_half_sweep(uint16_t *spins, uint16_t *sums, int64_t L, int c, const Metro2 &m,
                             uint64_t t, uint64_t seed, uint32_t stream_id, bool fused,
                             hipStream_t s);

} // namespace mm
} // namespace ising
