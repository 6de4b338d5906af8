// Host-side launchers of the sweep kernels (C++ linkage, internal to libising).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"

namespace ising {

hipError_t launch_init(uint64_t *words, int64_t L, uint64_t seed, uint32_t stream_id,
                       hipStream_t s);
hipError_t launch_half_sweep(uint64_t *words, int64_t L, int c, const Accept &ap, uint64_t t,
                             uint64_t seed, uint32_t stream_id, hipStream_t s);
hipError_t launch_observables(const uint64_t *words, int64_t L, int64_t *bond, int64_t *mag,
                              hipStream_t s);

} // namespace ising
