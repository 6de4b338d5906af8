// Host-side launchers of the sweep kernels (C++ linkage, internal to libising).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"
#include "ising_rows.hpp"

namespace ising {

hipError_t launch_init(uint64_t *words, int64_t L, uint64_t seed, uint32_t stream_id,
                       hipStream_t s);
// Half-sweep kernel choice: the default is the queued row kernel with 32-row
// bands for row-aligned sizes (L % 128 == 0) and the general kernel
// otherwise; the queued kernel with 16- or 8-row bands on request.
enum {
    kVariantDefault = 0,
    kVariantGeneral = 1,
    kVariantRowsPlain = 2,
    kVariantQueue16 = 4,
    kVariantQueue8 = 5
};

hipError_t launch_half_sweep(uint64_t *words, int64_t L, int c, const Metro2 &m, uint64_t t,
                             uint64_t seed, uint32_t stream_id, hipStream_t s,
                             int variant = kVariantDefault);
// The queued row kernel on the target / source colour arrays of a
// row-aligned lattice; `bonds` (the interleaved bond words) for a +-J glass,
// or nullptr for the ferromagnet.
hipError_t launch_rows_queue(uint64_t *tgt, const uint64_t *src, const uint64_t *bonds,
                             int64_t L, int c, const Metro2 &m, const SweepArgs2 &a, hipStream_t s,
                             int band);
// Half-sweep under any 5-entry acceptance table (heat bath); the variants
// choose kernels as for launch_half_sweep.
hipError_t launch_half_sweep5(uint64_t *words, int64_t L, int c, const rows::Table5 &tab,
                              uint64_t t, uint64_t seed, uint32_t stream_id, hipStream_t s,
                              int variant);
hipError_t launch_philox_rate(uint64_t nwords, uint32_t nq, uint64_t seed, uint32_t stream_id,
                              uint64_t t, uint32_t *sink, uint32_t sink_words, hipStream_t s);
hipError_t launch_observables(const uint64_t *words, int64_t L, int64_t *bond, int64_t *mag,
                              hipStream_t s);

} // namespace ising
