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

// One lattice of a work item and the threads that serve it: threads
// thread0 .. thread0 + tpl - 1 of the workgroup, in groups of lpw adjacent
// lanes; group g serves words g + j * (tpl / lpw), j < wpt.  Its two extended
// colour arrays start at LDS word lds_off.
struct BatchSlot {
    uint32_t lat;     // lattice index
    uint32_t thread0; // first thread (even where lpw = 2)
    uint32_t tpl;     // threads: ceil(W / wpt) * lpw
    uint32_t tile;    // wpt | lpw << 16 (lpw 1, or 2: the pair computes alternate Philox blocks)
    uint32_t lds_off; // first LDS word of the lattice
};

__host__ __device__ inline uint32_t slot_tile(uint32_t wpt, uint32_t lpw) { return wpt | (lpw << 16); }

// A work item of the persistent kernel: `count` slots -- lattices of one size
// or of several, each with its own tile -- swept together by one workgroup.
// Slots are in increasing thread0 and their thread ranges are disjoint.
struct BatchBundle {
    uint32_t first;   // index of the first slot in the slot list
    uint32_t count;   // slots
    uint32_t refresh; // 1 if some lattice's colour is not a whole number of words, or one word
    uint32_t pad;
};

constexpr int kBatchThreads = 1024;

// LDS words a lattice occupies in the persistent kernel: two extended colour arrays.
__host__ __device__ inline uint32_t batch_lds_words(uint32_t W) { return 2 * (W + 2); }

hipError_t launch_batch_init(const BatchLattice *lats, uint32_t n, uint64_t *words,
                             hipStream_t s);
// bundle_clock (optional, 2 x nbundles): each bundle's start and end on the
// device's constant-rate wall clock.
hipError_t launch_batch_sweep(const BatchLattice *lats, const BatchSlot *slots,
                              const BatchBundle *bundles, uint32_t nbundles, uint32_t grid,
                              size_t lds_bytes, uint32_t *next_bundle, uint64_t *words,
                              uint64_t *rng_counter, int64_t nsweeps, hipStream_t s,
                              uint64_t *bundle_clock = nullptr);
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
