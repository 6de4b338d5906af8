// gfx950 kernels for batches of independent lattices that fit in LDS: the
// persistent sweep kernel, initial states and per-lattice observables.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "batch.hpp"
#include "ising_rows.hpp"
#include "pair_decision.hpp"
#include "batch_aligned.hpp"

namespace ising {

// Initial state of every lattice; one workgroup per lattice.
__global__ __launch_bounds__(256) void k_batch_init(const BatchLattice *__restrict__ lats,
                                                    uint64_t *__restrict__ words)
{
    const BatchLattice lt = lats[blockIdx.x];
    for (uint32_t k = threadIdx.x; k < 2 * lt.W; k += blockDim.x) {
        const uint32_t c = k >= lt.W;
        words[lt.word_off + k] =
            init_word(k - c * lt.W, c, lt.M, lt.stream_id, lt.key0, lt.key1);
    }
}

// Writes the cyclic continuation of one extended colour array.
__device__ __forceinline__ void ext_refresh(uint64_t *E, uint32_t M, uint32_t W)
{
    uint64_t tail[3];
    ext_tail_fast(E, M, W, tail);
    E[W - 1] = tail[0];
    E[W] = tail[1];
    E[W + 1] = tail[2];
}

__device__ __forceinline__ rows::BlockDecision shuffle_xor1(const rows::BlockDecision &x)
{
    return rows::BlockDecision{{(uint32_t)__shfl_xor((int)x.d[0], 1, 64),
                                (uint32_t)__shfl_xor((int)x.d[1], 1, 64)},
                               {(uint32_t)__shfl_xor((int)x.f[0], 1, 64),
                                (uint32_t)__shfl_xor((int)x.f[1], 1, 64)}};
}

// Decision of one word by a pair of adjacent lanes: each lane computes every
// other Philox block (lane parity p takes q = 2j + p) and what that block
// decides on its own, the pair swaps those and both apply them in block
// order, so the pair reaches the sequential result in half the dependent
// steps.  Both lanes hold the same state.
__device__ __forceinline__ uint64_t decide_word_pair(uint64_t t, const Neighbours &nb,
                                                     uint64_t valid, uint32_t chunk,
                                                     const SweepArgs2 &a, uint32_t parity)
{
    rows::State s = rows::start_word_any(t, nb, valid, a.m);
    for (uint32_t q0 = 0; q0 < 16 && (s.p[0] | s.p[1]) != 0; q0 += 2) {
        const Block mine =
            rows::philox_fast<rows::kCtrKeyLane>(ctr_word0(a.stream_id, kDomainSweep, q0 + parity),
                                                 a.t_lo, a.t_hi, chunk, a.key0, a.key1);
        const rows::BlockDecision dm = rows::block_decision_lane(s, mine, q0 + parity, a.m);
        const rows::BlockDecision other = shuffle_xor1(dm);
        rows::apply_decision(s, parity ? other : dm);
        rows::apply_decision(s, parity ? dm : other);
    }
    return t ^ rows::join(s.tf[0], s.tf[1]);
}

// Persistent sweep kernel.  Workgroups take bundles from an atomic counter
// (the host orders them by decreasing work), copy the bundle's lattices into
// LDS, run every sweep there -- all spins of one colour from the other
// colour, a barrier, then the other colour (Sec. 2) -- and copy them back.
// Sweep s of the call uses half-sweep index t = 2*(rng_counter + s) + colour.
// A bundle may mix lattice sizes and tiles: every thread finds its slot and
// takes that lattice's geometry, neighbour extraction and tile as its own.
__global__ __launch_bounds__(kBatchThreads) void k_batch_sweep(
    const BatchLattice *__restrict__ lats, const BatchSlot *__restrict__ slots,
    const BatchBundle *__restrict__ bundles, uint32_t nbundles, uint32_t *__restrict__ next_bundle,
    uint64_t *__restrict__ words, const uint64_t *__restrict__ rng_counter, int64_t nsweeps,
    uint64_t *__restrict__ bundle_clock)
{
    extern __shared__ uint64_t lds[];
    __shared__ uint32_t item;
    const uint64_t ctr = *rng_counter;
    const uint32_t tid = threadIdx.x;
    for (;;) {
        __syncthreads(); // the previous bundle is written back and `item` consumed
        if (tid == 0)
            item = atomicAdd(next_bundle, 1u);
        __syncthreads();
        const uint32_t b = item;
        if (b >= nbundles)
            return;
        const BatchBundle bd = bundles[b];
        if (bundle_clock && tid == 0) // (optional) start and end of each bundle
            bundle_clock[2 * b] = (uint64_t)wall_clock64();
        // this thread's slot: the last one starting at or before it
        uint32_t lo = 0, hi = bd.count;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (slots[bd.first + mid].thread0 <= tid)
                lo = mid;
            else
                hi = mid;
        }
        const BatchSlot sl = slots[bd.first + lo];
        const uint32_t li = tid - sl.thread0;
        const bool on = tid >= sl.thread0 && li < sl.tpl;
        const uint32_t wpt = sl.tile & 0xFFFFu, lpw = sl.tile >> 16;
        const uint32_t group = lpw == 2 ? li >> 1 : li, parity = lpw == 2 ? li & 1u : 0u;
        const uint32_t groups = lpw == 2 ? sl.tpl >> 1 : sl.tpl;
        BatchLattice lt{};
        if (on)
            lt = lats[sl.lat];
        // When a colour is a whole number of words (M % 64 == 0, W >= 2) its
        // continuation is a copy of words 0 and 1: the lanes that write those
        // write the copies too, and the refresh drops out of every
        // half-sweep (with its barrier, where no lattice of the bundle needs it).
        const bool copy_ext = (lt.M & 63) == 0 && lt.W >= 2;
        // whole-word colour rows: the row-aligned neighbour vectors (their
        // row arithmetic holds for W < 4096, which L <= 722 keeps)
        const bool aligned = (lt.H & 63) == 0 && lt.W < 4096;
        const uint32_t Wr = lt.H >> 6, inv_wr = aligned ? aligned_inv(Wr) : 0;
        // colour rows of whole 32-bit halves (L % 64 == 0, e.g. 64 and 192)
        const bool half_aligned = !aligned && (lt.H & 31) == 0 && lt.W < 4096;
        const uint32_t Hr = lt.H >> 5, inv_hr = half_aligned ? half_inv(Hr) : 0;
        // general geometry: the row masks of the lane group's first word,
        // the same every half-sweep, taken once per bundle
        RowMasks rm0{};
        if (on && !aligned && !half_aligned && group < lt.W)
            rm0 = row_masks32(group, lt.H, lt.M, 0);
        uint64_t *E0 = lds + sl.lds_off;
        uint64_t *E1 = E0 + lt.W + 2;
        if (on)
            for (uint32_t k = li; k < 2 * lt.W; k += sl.tpl) {
                const uint32_t c = k >= lt.W;
                (c ? E1 : E0)[k - c * lt.W] = words[lt.word_off + k];
            }
        __syncthreads();
        if (on && li == 0) {
            ext_refresh(E0, lt.M, lt.W);
            ext_refresh(E1, lt.M, lt.W);
        }
        __syncthreads();
        for (int64_t sw = 0; sw < nsweeps; ++sw) {
            for (int c = 0; c < 2; ++c) {
                const uint64_t t = 2 * (ctr + (uint64_t)sw) + (uint64_t)c;
                uint64_t *tgt = c ? E1 : E0;
                const uint64_t *src = c ? E0 : E1;
                if (on) {
                    const SweepArgs2 a{lt.m,      (uint32_t)t, (uint32_t)(t >> 32), lt.stream_id,
                                       lt.key0, lt.key1};
                    for (uint32_t j = 0; j < wpt; ++j) {
                        const uint32_t k = group + j * groups;
                        if (k >= lt.W)
                            break;
                        Neighbours nb;
                        if (aligned) {
                            nb = neighbours_aligned(src, lt.W, Wr, inv_wr, k, c);
                        } else if (half_aligned) {
                            nb = neighbours_half_aligned((const uint32_t *)src, lt.W, Hr, inv_hr,
                                                         k, c);
                        } else {
                            RowMasks rm = j == 0 ? rm0 : row_masks32(k, lt.H, lt.M, 0);
                            if (c)
                                rm.left_rows = ~rm.left_rows; // rows of the other parity
                            nb = neighbours_ext32((const uint32_t *)src, lt.H, lt.M, k, rm);
                        }
                        const uint64_t tw = tgt[k];
                        const uint64_t valid = valid_mask(k, lt.M);
                        const uint64_t flips = (lpw == 2)
                                                   ? decide_word_pair(tw, nb, valid, k, a, parity)
                                                   : rows::decide_word_any(tw, nb, valid, k, a);
                        if (parity == 0) {
                            tgt[k] = tw ^ flips;
                            if (copy_ext && k < 2)
                                tgt[lt.W + k] = tw ^ flips;
                        }
                    }
                }
                __syncthreads();
                if (bd.refresh) {
                    if (on && li == 0 && !copy_ext)
                        ext_refresh(tgt, lt.M, lt.W);
                    __syncthreads();
                }
            }
        }
        if (on)
            for (uint32_t k = li; k < 2 * lt.W; k += sl.tpl) {
                const uint32_t c = k >= lt.W;
                const uint32_t kk = k - c * lt.W;
                words[lt.word_off + k] = (c ? E1 : E0)[kk] & valid_mask(kk, lt.M);
            }
        if (bundle_clock) {
            __syncthreads();
            if (tid == 0)
                bundle_clock[2 * b + 1] = (uint64_t)wall_clock64();
        }
    }
}

__global__ void k_batch_prepare(uint32_t *next_bundle)
{
    if (threadIdx.x == 0)
        *next_bundle = 0;
}

__global__ void k_batch_advance(uint64_t *rng_counter, int64_t nsweeps)
{
    if (threadIdx.x == 0)
        *rng_counter += (uint64_t)nsweeps;
}

hipError_t batch_sweep_blocks_per_cu(size_t lds_bytes, int *blocks)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch_sweep, kBatchThreads,
                                                        lds_bytes);
}

// Per-lattice bond sum and magnetisation; one workgroup per lattice.
__global__ __launch_bounds__(256) void k_batch_observables(const BatchLattice *__restrict__ lats,
                                                           const uint64_t *__restrict__ words,
                                                           int64_t *bond_out, int64_t *mag_out)
{
    const BatchLattice lt = lats[blockIdx.x];
    const uint64_t *black = words + lt.word_off, *white = black + lt.W;
    int64_t bond = 0, mag = 0;
    for (uint32_t k = threadIdx.x; k < lt.W; k += blockDim.x) {
        const uint64_t valid = valid_mask(k, lt.M);
        const uint64_t t = black[k];
        const Neighbours nb = neighbours_general(white, lt.H, lt.M, lt.W, k, 0);
        const int64_t aligned =
            (int64_t)__popcll(~(t ^ nb.up) & valid) + (int64_t)__popcll(~(t ^ nb.dn) & valid) +
            (int64_t)__popcll(~(t ^ nb.ce) & valid) + (int64_t)__popcll(~(t ^ nb.sd) & valid);
        const int64_t nvalid = (int64_t)__popcll(valid);
        bond += 2 * aligned - 4 * nvalid;
        mag += 2 * ((int64_t)__popcll(t & valid) + (int64_t)__popcll(white[k] & valid)) -
               2 * nvalid;
    }
    __shared__ int64_t sb[256], sm[256];
    sb[threadIdx.x] = bond;
    sm[threadIdx.x] = mag;
    __syncthreads();
    for (uint32_t h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            sb[threadIdx.x] += sb[threadIdx.x + h];
            sm[threadIdx.x] += sm[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bond_out[blockIdx.x] = sb[0];
        mag_out[blockIdx.x] = sm[0];
    }
}

// Bit-packed lattices <-> int8 rasters (one workgroup per lattice).
__global__ __launch_bounds__(256) void k_batch_to_spins(const BatchLattice *__restrict__ lats,
                                                        const uint64_t *__restrict__ words,
                                                        const int64_t *__restrict__ spin_off,
                                                        int8_t *__restrict__ spins)
{
    const BatchLattice lt = lats[blockIdx.x];
    int8_t *out = spins + spin_off[blockIdx.x];
    for (uint32_t p = threadIdx.x; p < lt.L * lt.L; p += blockDim.x) {
        const uint32_t i = p / lt.L, j = p % lt.L, c = (i + j) & 1, n = i * lt.H + (j >> 1);
        const uint64_t w = words[lt.word_off + (uint64_t)c * lt.W + (n >> 6)];
        out[p] = ((w >> (n & 63)) & 1u) ? 1 : -1;
    }
}

__global__ __launch_bounds__(256) void k_batch_from_spins(const BatchLattice *__restrict__ lats,
                                                          uint64_t *__restrict__ words,
                                                          const int64_t *__restrict__ spin_off,
                                                          const int8_t *__restrict__ spins)
{
    const BatchLattice lt = lats[blockIdx.x];
    const int8_t *in = spins + spin_off[blockIdx.x];
    for (uint32_t k = threadIdx.x; k < 2 * lt.W; k += blockDim.x) {
        const uint32_t c = k >= lt.W, kk = k - c * lt.W;
        uint64_t w = 0;
        for (uint32_t b = 0; b < 64; ++b) {
            const uint32_t n = kk * 64 + b;
            if (n >= lt.M)
                break;
            const uint32_t i = n / lt.H, jc = n % lt.H, j = 2 * jc + ((i + c) & 1);
            if (in[i * lt.L + j] > 0)
                w |= 1ull << b;
        }
        words[lt.word_off + k] = w;
    }
}

hipError_t launch_batch_to_spins(const BatchLattice *lats, uint32_t n, const uint64_t *words,
                                 const int64_t *spin_off, int8_t *spins, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_to_spins, dim3(n), dim3(256), 0, s, lats, words, spin_off, spins);
    return hipGetLastError();
}

hipError_t launch_batch_from_spins(const BatchLattice *lats, uint32_t n, uint64_t *words,
                                   const int64_t *spin_off, const int8_t *spins, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_from_spins, dim3(n), dim3(256), 0, s, lats, words, spin_off, spins);
    return hipGetLastError();
}

hipError_t launch_batch_init(const BatchLattice *lats, uint32_t n, uint64_t *words,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_init, dim3(n), dim3(256), 0, s, lats, words);
    return hipGetLastError();
}

hipError_t launch_batch_sweep(const BatchLattice *lats, const BatchSlot *slots,
                              const BatchBundle *bundles, uint32_t nbundles, uint32_t grid,
                              size_t lds_bytes, uint32_t *next_bundle, uint64_t *words,
                              uint64_t *rng_counter, int64_t nsweeps, hipStream_t s,
                              uint64_t *bundle_clock)
{
    hipLaunchKernelGGL(k_batch_prepare, dim3(1), dim3(64), 0, s, next_bundle);
    hipLaunchKernelGGL(k_batch_sweep, dim3(grid), dim3(kBatchThreads), lds_bytes, s, lats,
                       slots, bundles, nbundles, next_bundle, words,
                       (const uint64_t *)rng_counter, nsweeps, bundle_clock);
    hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, s, rng_counter, nsweeps);
    return hipGetLastError();
}

hipError_t launch_batch_observables(const BatchLattice *lats, uint32_t n, const uint64_t *words,
                                    int64_t *bond, int64_t *mag, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_observables, dim3(n), dim3(256), 0, s, lats, words, bond, mag);
    return hipGetLastError();
}

} // namespace ising
