// Batched simulation of many independent lattices: device descriptors shared
// by the batch kernels and the host planner (internal to libising).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"

namespace ising {

// One lattice of a batch.  Its 2*W words (colour 0 then colour 1, the layout
// of a single lattice) start at word_off of the batch buffer.
struct BatchLattice {
    uint64_t word_off;
    uint32_t L, H, M, W; // size, spins per colour row, spins per colour, words per colour
    Metro2 m;            // acceptance at this lattice's beta
    uint32_t key0, key1, stream_id, pad;
};

// A work item of the persistent kernel: `count` lattices of one size, swept
// together by one workgroup.  Thread t serves lattice slot t / tpl; within
// the slot, lanes form groups of lpw adjacent lanes, and group g serves
// words g + j * (tpl / lpw), j < wpt.
struct BatchBundle {
    uint32_t first; // index of the first slot in the member list
    uint32_t count; // lattices in the bundle
    uint32_t wpt;   // words per lane group (per colour)
    uint32_t tpl;   // threads per lattice: ceil(W / wpt) * lpw
    uint32_t lpw;   // lanes per word: 1, or 2 (the pair computes alternate Philox blocks)
    uint32_t pad;
};

constexpr int kBatchThreads = 1024;

// LDS words a lattice occupies in the persistent kernel: two extended colour arrays.
__host__ __device__ inline uint32_t batch_lds_words(uint32_t W) { return 2 * (W + 2); }

hipError_t launch_batch_init(const BatchLattice *lats, uint32_t n, uint64_t *words,
                             hipStream_t s);
hipError_t launch_batch_sweep(const BatchLattice *lats, const uint32_t *members,
                              const BatchBundle *bundles, uint32_t nbundles, uint32_t grid,
                              size_t lds_bytes, uint32_t *next_bundle, uint64_t *words,
                              uint64_t *rng_counter, int64_t nsweeps, hipStream_t s);
// Workgroups of the persistent sweep kernel one compute unit holds at once
// with lds_bytes of dynamic LDS each (registers, wavefront slots and LDS).
hipError_t batch_sweep_blocks_per_cu(size_t lds_bytes, int *blocks);
hipError_t launch_batch_to_spins(const BatchLattice *lats, uint32_t n, const uint64_t *words,
                                 const int64_t *spin_off, int8_t *spins, hipStream_t s);
hipError_t launch_batch_from_spins(const BatchLattice *lats, uint32_t n, uint64_t *words,
                                   const int64_t *spin_off, const int8_t *spins, hipStream_t s);
hipError_t launch_batch_observables(const BatchLattice *lats, uint32_t n, const uint64_t *words,
                                    int64_t *bond, int64_t *mag, hipStream_t s);

} // namespace ising
