// Host-side launchers of the +-J spin-glass kernels (internal to libising).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"

namespace ising {

// Random bond signs into the four bond arrays (4 * ceil(L*L/128) words).
hipError_t launch_glass_bonds_init(uint64_t *bonds, int64_t L, uint64_t seed, uint32_t stream_id,
                                   hipStream_t s);
// Half-sweep of colour c of a row-aligned lattice (L % 128 == 0): the queued
// row kernel (kVariantDefault: 32-row bands, kVariantQueue16, kVariantQueue8),
// or the per-word row kernel (kVariantGeneral, kVariantRowsPlain).
hipError_t launch_glass_half_sweep(uint64_t *words, const uint64_t *bonds, int64_t L, int c,
                                   const Metro2 &m, uint64_t t, uint64_t seed, uint32_t stream_id,
                                   hipStream_t s, int variant);
hipError_t launch_glass_observables(const uint64_t *words, const uint64_t *bonds, int64_t L,
                                    int64_t *bond, int64_t *mag, hipStream_t s);

} // namespace ising
