// gfx950 kernels of the checkerboard Metropolis sweep: initial state,
// half-sweep (general geometry and row-aligned streaming), observables.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"
#include "launch.hpp"

namespace ising {

// ------------------------------------------------------------ initial state
__global__ __launch_bounds__(256) void k_init(uint64_t *__restrict__ words, int64_t M, int64_t W,
                                              uint32_t key0, uint32_t key1, uint32_t stream_id)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * W)
        return;
    const uint32_t c = (uint32_t)(idx / W);
    const int64_t chunk = idx - (int64_t)c * W;
    words[idx] = init_word(chunk, c, M, stream_id, key0, key1);
}

// ------------------------------------------------- half-sweep, any geometry
// One thread per target word; neighbour vectors by cyclic extraction from the
// other colour (row-straddling words, partial last word, tiny lattices).
__global__ __launch_bounds__(256) void k_sweep_general(uint64_t *__restrict__ tgt,
                                                       const uint64_t *__restrict__ src, int64_t H,
                                                       int64_t M, int64_t W, int c, SweepArgs2 a)
{
    const int64_t chunk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (chunk >= W)
        return;
    tgt[chunk] = update_word_general(tgt[chunk], src, H, M, W, chunk, c, a);
}

// ------------------------------------------- half-sweep, row-aligned lattices
// L % 128 == 0: each colour row is Wr = L/128 whole words, so the up, down and
// centre neighbours of word (i, w) are words (i-1, w), (i+1, w), (i, w) of the
// other colour and the side neighbour is the centre word shifted by one spin
// with the adjacent word's edge bit shifted in (Sec. 3.3, Fig. 3).  A thread
// owns one word column of a band of kRows rows and marches down it keeping
// three source rows in registers, so each source word is read from memory
// (kRows + 2) / kRows times.
constexpr int kRows = 16;

__global__ __launch_bounds__(256) void k_sweep_rows(uint64_t *__restrict__ tgt,
                                                    const uint64_t *__restrict__ src, int64_t L,
                                                    int64_t Wr, int64_t blocks_per_band, int c,
                                                    SweepArgs2 a)
{
    const int64_t band = blockIdx.x / blocks_per_band;
    const int64_t w = (blockIdx.x - band * blocks_per_band) * (int64_t)blockDim.x + threadIdx.x;
    if (w >= Wr)
        return;
    const int64_t i0 = band * kRows;
    const int64_t wl = (w == 0) ? Wr - 1 : w - 1;
    const int64_t wr = (w == Wr - 1) ? 0 : w + 1;
    uint64_t prev = src[((i0 == 0) ? L - 1 : i0 - 1) * Wr + w];
    uint64_t cur = src[i0 * Wr + w];
    for (int r = 0; r < kRows; ++r) {
        const int64_t i = i0 + r;
        if (i >= L)
            break;
        const int64_t inext = (i + 1 == L) ? 0 : i + 1;
        const uint64_t next = src[inext * Wr + w];
        const int64_t idx = i * Wr + w;
        const bool left = ((i + c) & 1) == 0;
        const uint64_t adj = src[i * Wr + (left ? wl : wr)];
        tgt[idx] = update_word_rows(tgt[idx], prev, next, cur, adj, left, (uint32_t)idx, a);
        prev = cur;
        cur = next;
    }
}

// ------------------------------- half-sweep, row-aligned, with a work queue
// The lazy compare needs a different number of Philox blocks per word (about
// 3.8 on average near T_c, up to 16); a wavefront that waits for its slowest
// word spends about 6.8.  Here every word first gets kStreamBlocks blocks in
// lock step; words still undecided then go to a per-wavefront FIFO queue in
// LDS, which is drained 64 entries at a time so that every lane works on some
// undecided word.  Each word still receives its blocks q = 0, 1, 2, ... in
// order, so the result is the same as deciding each word on its own.  The
// FIFO order finishes words soon after their row, so partly written cache
// lines are completed before they leave L2.
constexpr int kBandRows = 32;
constexpr uint32_t kStreamBlocks = 3;
constexpr uint32_t kQueueCap = 128; // < 64 entries left after a drain + 64 pushed per row
constexpr int kWaves = 4;

struct WaveQueue {
    uint64_t t[kQueueCap];       // target word before the half-sweep
    uint64_t flips[kQueueCap];   // flips decided so far
    uint64_t pending[kQueueCap]; // spins still undecided
    uint64_t classA[kQueueCap];  // undecided spins of class A
    uint32_t chunk[kQueueCap];   // word index in its colour
    uint32_t q[kQueueCap];       // next Philox block
};

__device__ __forceinline__ uint32_t lanes_below(uint64_t ballot)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(ballot >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0u));
}

__device__ __forceinline__ void queue_put(WaveQueue &wq, uint32_t e, uint64_t t,
                                          const WordState &s, uint32_t chunk, uint32_t q)
{
    wq.t[e] = t;
    wq.flips[e] = s.flips;
    wq.pending[e] = s.pending;
    wq.classA[e] = s.classA;
    wq.chunk[e] = chunk;
    wq.q[e] = q;
}

// One pass over the oldest n (<= 64) queue entries: one Philox block each;
// finished words are stored, the rest appended again at the tail.
__device__ __forceinline__ void drain_once(WaveQueue &wq, uint32_t &head, uint32_t &len,
                                           uint32_t n, uint64_t *__restrict__ tgt,
                                           const SweepArgs2 &a, int lane)
{
    const bool mine = (uint32_t)lane < n;
    WordState s{0, 0, 0};
    uint64_t t = 0;
    uint32_t chunk = 0, q = 0;
    if (mine) {
        const uint32_t e = (head + (uint32_t)lane) & (kQueueCap - 1);
        t = wq.t[e];
        s.flips = wq.flips[e];
        s.pending = wq.pending[e];
        s.classA = wq.classA[e];
        chunk = wq.chunk[e];
        q = wq.q[e];
        advance_block(s, q, chunk, a.m, a.t_lo, a.t_hi, a.stream_id, a.key0, a.key1);
        ++q;
    }
    __builtin_amdgcn_wave_barrier();
    head = (head + n) & (kQueueCap - 1);
    len -= n;
    const bool keep = mine && s.pending != 0;
    if (mine && !keep)
        tgt[chunk] = t ^ s.flips;
    const uint64_t bal = __ballot(keep);
    if (keep)
        queue_put(wq, (head + len + lanes_below(bal)) & (kQueueCap - 1), t, s, chunk, q);
    __builtin_amdgcn_wave_barrier();
    len += (uint32_t)__popcll(bal);
}

// L % 128 == 0.  A wavefront owns 64 consecutive word columns of a band of
// kBandRows colour rows and marches down it, holding the three source rows it
// needs in registers; the side neighbour comes from the adjacent word of the
// same source row (Sec. 3.3, Fig. 3).  Word indices fit in 32 bits.
__global__ __launch_bounds__(256) void k_sweep_rows_q(uint64_t *__restrict__ tgt,
                                                      const uint64_t *__restrict__ src,
                                                      uint32_t L, uint32_t Wr,
                                                      uint32_t waves_per_band, uint32_t nbands,
                                                      int c, SweepArgs2 a)
{
    __shared__ WaveQueue queues[kWaves];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    WaveQueue &wq = queues[wv];
    const uint32_t gwave = blockIdx.x * kWaves + wv;
    const uint32_t band = gwave / waves_per_band;
    if (band >= nbands)
        return; // whole wavefront
    const uint32_t w = (gwave - band * waves_per_band) * 64 + lane;
    const bool active = w < Wr;
    const uint32_t wl = (w == 0) ? Wr - 1 : w - 1;
    const uint32_t wr = (w + 1 >= Wr) ? 0 : w + 1;
    const uint32_t i0 = band * kBandRows;
    uint64_t prev = 0, cur = 0;
    if (active) {
        prev = src[((i0 == 0) ? L - 1 : i0 - 1) * Wr + w];
        cur = src[i0 * Wr + w];
    }
    uint32_t head = 0, len = 0;
    for (int r = 0; r < kBandRows; ++r) {
        const uint32_t i = i0 + r;
        if (i >= L)
            break;
        const uint32_t inext = (i + 1 == L) ? 0 : i + 1;
        const uint32_t idx = i * Wr + w;
        const bool left = ((i + c) & 1) == 0;
        uint64_t next = 0, t = 0;
        WordState s{0, 0, 0};
        if (active) {
            next = src[inext * Wr + w];
            t = tgt[idx];
            const uint64_t adj = src[i * Wr + (left ? wl : wr)];
            const Classes k = classify(t, prev, next, cur, side_vector(cur, adj, left));
            s = start_word(k, ~0ull, a.m);
        }
#pragma unroll
        for (uint32_t q = 0; q < kStreamBlocks; ++q) {
            if (__ballot(s.pending != 0) == 0)
                break;
            if (s.pending != 0)
                advance_block_uniform(s, q, idx, a.m, a.t_lo, a.t_hi, a.stream_id, a.key0,
                                      a.key1);
        }
        const bool push = active && s.pending != 0;
        if (active && !push)
            tgt[idx] = t ^ s.flips;
        const uint64_t bal = __ballot(push);
        if (push)
            queue_put(wq, (head + len + lanes_below(bal)) & (kQueueCap - 1), t, s, idx,
                      kStreamBlocks);
        __builtin_amdgcn_wave_barrier();
        len += (uint32_t)__popcll(bal);
        while (len >= 64)
            drain_once(wq, head, len, 64, tgt, a, lane);
        prev = cur;
        cur = next;
    }
    while (len > 0)
        drain_once(wq, head, len, len < 64 ? len : 64, tgt, a, lane);
}

// --------------------------------------------------------------- observables
__global__ __launch_bounds__(256) void k_fill_i64(int64_t *__restrict__ p, int64_t n, int64_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

__device__ __forceinline__ int64_t wave_sum(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

// Bond sum and magnetisation.  Each bond joins a black and a white site, so
// summing (2a - 4) over black sites (a = aligned neighbours) counts every
// bond once.  M = sum over both colours of (2*popcount - spins).
__global__ __launch_bounds__(256) void k_observables(const uint64_t *__restrict__ black,
                                                     const uint64_t *__restrict__ white, int64_t H,
                                                     int64_t M, int64_t W, int64_t *bond_out,
                                                     int64_t *mag_out)
{
    int64_t bond = 0, mag = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t chunk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; chunk < W;
         chunk += stride) {
        const uint64_t valid = valid_mask(chunk, M);
        const uint64_t t = black[chunk];
        const Neighbours nb = neighbours_general(white, H, M, W, chunk, 0);
        // popcounts are unsigned: widen to signed 64-bit before subtracting
        const int64_t aligned =
            (int64_t)__popcll(~(t ^ nb.up) & valid) + (int64_t)__popcll(~(t ^ nb.dn) & valid) +
            (int64_t)__popcll(~(t ^ nb.ce) & valid) + (int64_t)__popcll(~(t ^ nb.sd) & valid);
        const int64_t nvalid = (int64_t)__popcll(valid);
        const int64_t up_spins =
            (int64_t)__popcll(t & valid) + (int64_t)__popcll(white[chunk] & valid);
        bond += 2 * aligned - 4 * nvalid;
        mag += 2 * up_spins - 2 * nvalid;
    }
    bond = wave_sum(bond);
    mag = wave_sum(mag);
    __shared__ int64_t part[2][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        part[0][wv] = bond;
        part[1][wv] = mag;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t b = 0, m = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
            b += part[0][q];
            m += part[1][q];
        }
        atomicAdd((unsigned long long *)bond_out, (unsigned long long)b);
        atomicAdd((unsigned long long *)mag_out, (unsigned long long)m);
    }
}

// Row-aligned lattices (L % 128 == 0): the same sums with the neighbour words
// addressed directly, as in the row sweep.
__global__ __launch_bounds__(256) void k_observables_rows(const uint64_t *__restrict__ black,
                                                          const uint64_t *__restrict__ white,
                                                          int64_t L, int64_t Wr, int64_t *bond_out,
                                                          int64_t *mag_out)
{
    int64_t bond = 0, mag = 0;
    const int64_t W = L * Wr, stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < W; k += stride) {
        const int64_t i = k / Wr, w = k - i * Wr;
        const uint64_t t = black[k], ce = white[k];
        const uint64_t up = white[((i == 0) ? L - 1 : i - 1) * Wr + w];
        const uint64_t dn = white[((i + 1 == L) ? 0 : i + 1) * Wr + w];
        const bool left = (i & 1) == 0; // colour 0: side neighbour on the left on even rows
        const int64_t wa = left ? (w == 0 ? Wr - 1 : w - 1) : (w + 1 == Wr ? 0 : w + 1);
        const uint64_t sd = side_vector(ce, white[i * Wr + wa], left);
        const int64_t aligned = (int64_t)__popcll(~(t ^ up)) + (int64_t)__popcll(~(t ^ dn)) +
                                (int64_t)__popcll(~(t ^ ce)) + (int64_t)__popcll(~(t ^ sd));
        bond += 2 * aligned - 4 * 64;
        mag += 2 * ((int64_t)__popcll(t) + (int64_t)__popcll(ce)) - 2 * 64;
    }
    bond = wave_sum(bond);
    mag = wave_sum(mag);
    __shared__ int64_t part[2][4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        part[0][wv] = bond;
        part[1][wv] = mag;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t b = 0, m = 0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
            b += part[0][q];
            m += part[1][q];
        }
        atomicAdd((unsigned long long *)bond_out, (unsigned long long)b);
        atomicAdd((unsigned long long *)mag_out, (unsigned long long)m);
    }
}

// ------------------------------------------------------------------ launches
static inline uint32_t blocks_for(int64_t n, int threads)
{
    return (uint32_t)((n + threads - 1) / threads);
}

hipError_t launch_init(uint64_t *words, int64_t L, uint64_t seed, uint32_t stream_id,
                       hipStream_t s)
{
    const int64_t M = L * L / 2, W = (M + 63) / 64;
    hipLaunchKernelGGL(k_init, dim3(blocks_for(2 * W, 256)), dim3(256), 0, s, words, M, W,
                       (uint32_t)seed, (uint32_t)(seed >> 32), stream_id);
    return hipGetLastError();
}

hipError_t launch_half_sweep(uint64_t *words, int64_t L, int c, const Metro2 &m, uint64_t t,
                             uint64_t seed, uint32_t stream_id, hipStream_t s, int variant)
{
    const int64_t H = L / 2, M = L * L / 2, W = (M + 63) / 64;
    uint64_t *tgt = words + (int64_t)c * W;
    const uint64_t *src = words + (int64_t)(1 - c) * W;
    const SweepArgs2 a{m, (uint32_t)t, (uint32_t)(t >> 32), stream_id, (uint32_t)seed,
                       (uint32_t)(seed >> 32)};
    if (L % 128 == 0 && variant != kVariantGeneral) {
        const int64_t Wr = L / 128;
        if (variant == kVariantRowsPlain) {
            const int threads = Wr >= 256 ? 256 : (Wr >= 64 ? 64 * (int)((Wr + 63) / 64) : 64);
            const int64_t bpb = (Wr + threads - 1) / threads;
            const int64_t bands = (L + kRows - 1) / kRows;
            hipLaunchKernelGGL(k_sweep_rows, dim3((uint32_t)(bands * bpb)), dim3(threads), 0, s,
                               tgt, src, L, Wr, bpb, c, a);
        } else {
            const int64_t wpb = (Wr + 63) / 64;
            const int64_t nbands = (L + kBandRows - 1) / kBandRows;
            const int64_t waves = wpb * nbands;
            hipLaunchKernelGGL(k_sweep_rows_q, dim3((uint32_t)((waves + kWaves - 1) / kWaves)),
                               dim3(64 * kWaves), 0, s, tgt, src, (uint32_t)L, (uint32_t)Wr,
                               (uint32_t)wpb, (uint32_t)nbands, c, a);
        }
    } else {
        hipLaunchKernelGGL(k_sweep_general, dim3(blocks_for(W, 256)), dim3(256), 0, s, tgt, src,
                           H, M, W, c, a);
    }
    return hipGetLastError();
}

hipError_t launch_observables(const uint64_t *words, int64_t L, int64_t *bond, int64_t *mag,
                              hipStream_t s)
{
    const int64_t H = L / 2, M = L * L / 2, W = (M + 63) / 64;
    hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, s, bond, (int64_t)1, (int64_t)0);
    hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, s, mag, (int64_t)1, (int64_t)0);
    const uint32_t nb = (uint32_t)((W + 255) / 256 < 4096 ? (W + 255) / 256 : 4096);
    if (L % 128 == 0)
        hipLaunchKernelGGL(k_observables_rows, dim3(nb), dim3(256), 0, s, words, words + W, L,
                           L / 128, bond, mag);
    else
        hipLaunchKernelGGL(k_observables, dim3(nb), dim3(256), 0, s, words, words + W, H, M, W,
                           bond, mag);
    return hipGetLastError();
}

} // namespace ising
