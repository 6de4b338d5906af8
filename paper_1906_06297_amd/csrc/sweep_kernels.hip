// gfx950 kernels of the checkerboard Metropolis sweep: initial state,
// half-sweep (general geometry and row-aligned streaming), observables.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"
#include "ising_rows.hpp"
#include "launch.hpp"

namespace ising {

// ------------------------------------------------------------ initial state
// A dispatch counts its grid in 32-bit work-items, so kernels over up to 2^33
// words loop over a capped grid.
constexpr uint32_t kMaxStrideBlocks = 1u << 20; // x 256 threads < 2^32

__global__ __launch_bounds__(256) void k_init(uint64_t *__restrict__ words, int64_t M, int64_t W,
                                              uint32_t key0, uint32_t key1, uint32_t stream_id)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < 2 * W;
         idx += stride) {
        const uint32_t c = (uint32_t)(idx / W);
        const int64_t chunk = idx - (int64_t)c * W;
        words[idx] = init_word(chunk, c, M, stream_id, key0, key1);
    }
}

// ------------------------------------------------- half-sweep, any geometry
// One thread per target word; neighbour vectors by cyclic extraction from the
// other colour (row-straddling words, partial last word, tiny lattices).  The
// size limit (fewer than 2^32 - 2^16 words per colour) keeps the grid below
// 2^32 work-items.
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
// per-word steps run on 32-bit halves with gfx950's three-input logic
// instruction (ising_rows.hpp).
//
// New words are collected in a ring of R rows in LDS (R = 4 under Metropolis,
// 2 under the heat bath, whose larger queue entries leave less LDS: the
// smaller ring keeps a fifth wavefront per SIMD, ~4 % faster), and row r goes
// to memory as one coalesced 512-byte store when row r + R needs its slot,
// so that HBM sees whole lines instead of the scattered 8-byte stores of
// words finished in the queue.  A word still undecided then (a few per
// thousand) is stored on its own when it is final.
// two 64-bit words in one 16-byte load
typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));
constexpr uint32_t kStreamBlocks = 3;
constexpr uint32_t kQueueCap = 128; // < 64 entries left after a drain + 64 pushed per row
constexpr int kWaves = 4;

// The decision rule of the queued kernel: its per-word state, the words a
// queue entry holds, and the start and block steps (ising_rows.hpp).
// Metropolis: two drawing classes; state = flips so far, pending spins,
// class-A spins.
struct RuleMetro {
    using State = rows::State;
    using Args = SweepArgs2;
    static constexpr int kWords = 3;
    static constexpr uint32_t kRing = 4; // LDS row-ring depth
    struct Setup {
        rows::ClassMasks cm;
    };
    __device__ static Setup setup(const Args &a) { return Setup{rows::class_masks(a.m)}; }
    // The lock-step planes branch on threshold bits that are the same for
    // the whole launch.  Taken as they are, the compiler hoists every
    // plane's test out of the row loop and keeps each as a 64-bit lane mask,
    // a dozen scalar-register pairs that then spill; passing the two words
    // through an empty asm statement per row leaves them opaque, so each
    // test is a scalar bit test where it is used.
    __device__ static Args per_row(Args a)
    {
        asm volatile("" : "+s"(a.m.thrA), "+s"(a.m.thrB));
        return a;
    }
    template <bool Anti, bool Plain>
    __device__ static State start(uint64_t t, uint64_t up, uint64_t dn, uint64_t ce, uint32_t sl,
                                  uint32_t sh, const Setup &su, const Args &)
    {
        return rows::start_from_halves<Anti, Plain>(t, up, dn, ce, sl, sh, su.cm);
    }
    __device__ static void block(State &s, uint32_t q, uint32_t chunk, const Args &a)
    {
        rows::block_uniform(s, q, chunk, a);
    }
    // Per-lane blocks take their threshold masks from a table of the 16
    // blocks in LDS, one 16-byte read instead of four bit extracts and the
    // bit-index arithmetic.
    struct LaneTable {
        rows::BlockMasks m[16];
    };
    __device__ static void fill_table(LaneTable &tab, const Args &a, uint32_t tid)
    {
        if (tid < 16)
            tab.m[tid] = rows::block_masks(tid, a.m);
    }
    __device__ static void block_lane(State &s, uint32_t q, uint32_t chunk, const Args &a,
                                      const LaneTable &tab)
    {
        rows::apply_block_masks(s,
                                rows::philox_fast<rows::kCtrLane>(
                                    ctr_word0(a.stream_id, kDomainSweep, q), a.t_lo, a.t_hi,
                                    chunk, a.key0, a.key1),
                                tab.m[q]);
    }
    __device__ static uint64_t word(const State &s, int k)
    {
        return k == 0 ? rows::join(s.tf[0], s.tf[1])
                      : (k == 1 ? rows::join(s.p[0], s.p[1]) : rows::join(s.a[0], s.a[1]));
    }
    __device__ static void set_word(State &s, int k, uint64_t v)
    {
        uint32_t *h = k == 0 ? s.tf : (k == 1 ? s.p : s.a);
        h[0] = rows::lo32(v);
        h[1] = rows::hi32(v);
    }
};

// Any 5-entry table (heat bath): every class may draw; state = flips so far,
// pending spins, the aligned count as three bit slices.
struct Rule5 {
    using State = rows::State5;
    using Args = rows::SweepArgs5;
    static constexpr int kWords = 5;
    static constexpr uint32_t kRing = 2;
    struct Setup {};
    __device__ static Setup setup(const Args &) { return Setup{}; }
    __device__ static Args per_row(const Args &a) { return a; }
    template <bool Anti, bool Plain>
    __device__ static State start(uint64_t t, uint64_t up, uint64_t dn, uint64_t ce, uint32_t sl,
                                  uint32_t sh, const Setup &, const Args &a)
    {
        return rows::start5_from_halves(t, up, dn, ce, sl, sh, a.tab);
    }
    __device__ static void block(State &s, uint32_t q, uint32_t chunk, const Args &a)
    {
        rows::block5<false>(s, q, chunk, a);
    }
    struct LaneTable {};
    __device__ static void fill_table(LaneTable &, const Args &, uint32_t) {}
    __device__ static void block_lane(State &s, uint32_t q, uint32_t chunk, const Args &a,
                                      const LaneTable &)
    {
        rows::block5<true>(s, q, chunk, a);
    }
    template <class S>
    __device__ static auto half_pair(S &s, int k) -> decltype(&s.tf[0])
    {
        return k == 0 ? s.tf : (k == 1 ? s.p : (k == 2 ? s.b0 : (k == 3 ? s.b1 : s.b2)));
    }
    __device__ static uint64_t word(const State &s, int k)
    {
        const uint32_t *h = half_pair(s, k);
        return rows::join(h[0], h[1]);
    }
    __device__ static void set_word(State &s, int k, uint64_t v)
    {
        uint32_t *h = half_pair(s, k);
        h[0] = rows::lo32(v);
        h[1] = rows::hi32(v);
    }
};

template <int N>
struct WaveQueue {
    uint64_t w[N][kQueueCap]; // the rule's state words (first: flips so far, second: pending)
    uint64_t cm[kQueueCap];   // word index in its colour | queue_meta() << 32
};

// Queue entry metadata: next Philox block (4 bits) | the word's ring cell
// (slot * 64 + lane, 8 bits) << 4 | band row << 12.
__device__ __forceinline__ uint32_t queue_meta(uint32_t q, uint32_t cell, uint32_t r)
{
    return q | (cell << 4) | (r << 12);
}

template <uint32_t R> // rows, a power of two
struct WaveRing {
    uint64_t word[R][64]; // new words of the last R rows
    uint8_t done[R][64];  // 1 where the word is final
};

__device__ __forceinline__ uint32_t lanes_below(uint64_t ballot)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(ballot >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)ballot, 0u));
}

template <class Rule>
__device__ __forceinline__ void queue_put(WaveQueue<Rule::kWords> &wq, uint32_t e,
                                          const typename Rule::State &s, uint32_t chunk,
                                          uint32_t meta)
{
#pragma unroll
    for (int k = 0; k < Rule::kWords; ++k)
        wq.w[k][e] = Rule::word(s, k);
    wq.cm[e] = rows::join(chunk, meta);
}

template <class State>
__device__ __forceinline__ bool undecided(const State &s) { return (s.p[0] | s.p[1]) != 0; }

// Writes ring slot `sl` to row pointer `rowp`: every word, or (`only_done`)
// the final ones.
template <uint32_t R>
__device__ __forceinline__ void ring_store(const WaveRing<R> &rg, uint32_t sl,
                                           uint64_t *__restrict__ rowp, uint32_t wc, bool active,
                                           int lane, bool only_done)
{
    __builtin_amdgcn_wave_barrier();
    const bool st = active && (!only_done || rg.done[sl][lane] != 0);
    if (st)
        __builtin_nontemporal_store(rg.word[sl][lane], &rowp[wc]);
}

// One pass over the oldest n (<= 64) queue entries: one Philox block each;
// finished words go to their ring slot (or, for a row already written, to
// memory), the rest are appended again at the tail.  A word still undecided
// after block 15 (all 32 planes) has r == T: rejected, and final as it is.
// Rows up to r_cur - Rule::kRing have left the ring.  `Head` >= 0: the
// queue's head is known to be Head (n = 64 passes from an empty queue leave
// it at 0 or 64), so the entries' LDS addresses are fixed offsets.
template <class Rule, int Head = -1>
__device__ __forceinline__ void drain_once(WaveQueue<Rule::kWords> &wq,
                                           WaveRing<Rule::kRing> &rg,
                                           uint32_t &head, uint32_t &len, uint32_t n,
                                           uint32_t r_cur, uint64_t *__restrict__ tgt,
                                           const typename Rule::Args &a,
                                           const typename Rule::LaneTable &tab, int lane)
{
    const bool mine = (uint32_t)lane < n;
    typename Rule::State s{};
    uint32_t chunk = 0, meta = 0, q = 0;
    if (mine) {
        const uint32_t e = Head >= 0 ? (uint32_t)Head + (uint32_t)lane
                                     : (head + (uint32_t)lane) & (kQueueCap - 1);
#pragma unroll
        for (int k = 0; k < Rule::kWords; ++k)
            Rule::set_word(s, k, wq.w[k][e]);
        const uint64_t cm = wq.cm[e];
        chunk = rows::lo32(cm);
        meta = rows::hi32(cm);
        q = meta & 15u;
        Rule::block_lane(s, q, chunk, a, tab);
    }
    __builtin_amdgcn_wave_barrier();
    head = (head + n) & (kQueueCap - 1);
    len -= n;
    const bool keep = mine && q < 15u && undecided(s);
    const bool fin = mine && !keep;
    // the word's row is still in the ring iff row >= r_cur + 1 - kRing
    const uint32_t own_min = r_cur + 1 >= Rule::kRing ? (r_cur + 1 - Rule::kRing) << 12 : 0u;
    const bool owned = meta >= own_min;
    if (fin) {
        const uint64_t v = rows::join(s.tf[0], s.tf[1]);
        if (owned) {
            const uint32_t cell = (meta >> 4) & 255u;
            (&rg.word[0][0])[cell] = v;
            (&rg.done[0][0])[cell] = 1;
        } else {
            tgt[chunk] = v;
        }
    }
    const uint64_t bal = __builtin_amdgcn_ballot_w64(keep);
    if (keep)
        queue_put<Rule>(wq, (head + len + lanes_below(bal)) & (kQueueCap - 1), s, chunk, meta + 1);
    __builtin_amdgcn_wave_barrier();
    len += (uint32_t)__popcll(bal);
}

// A load from a wave-uniform row of nwords 64-bit words through a buffer
// resource that the scalar unit builds from the row pointer: the per-lane
// byte offset voff is a loop-invariant register and a wave-uniform byte
// offset soff goes in the scalar offset, so the load takes no vector address
// arithmetic (and it stays a vector-memory load, in flight like the others,
// where a wave-uniform address would otherwise become a scalar load that is
// waited for at once).  The hardware range-checks voff + soff + 8 against
// the row's bytes; every offset used here lies inside the row.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int kRsrcWord3 = 0x00020000; // resource word 3 on gfx9: 32-bit data format
constexpr int kLoadNT = 2;              // cache-policy operand: non-temporal

template <int Policy>
__device__ __forceinline__ uint64_t row_load(const uint64_t *rowp, uint32_t nwords, uint32_t voff,
                                             uint32_t soff)
{
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)rowp, (short)0, (int)(nwords * 8u), kRsrcWord3);
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, Policy);
    return (uint64_t)v.x | ((uint64_t)v.y << 32);
}

// Edge half of the side vector of a wavefront that owns whole 64-word row
// segments: every lane takes its neighbour lane's centre word by a wavefront
// shift (DPP wave_shr:1 / wave_shl:1); the shift leaves lane 0 (left
// neighbours) or lane 63 (right neighbours) with `edge`, the half of the word
// past the segment, which the caller holds in every lane.
__device__ __forceinline__ uint32_t side_half_dpp(uint32_t cur_lo, uint32_t cur_hi, uint32_t edge,
                                                  bool left)
{
    return left ? (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)cur_hi, 0x138, 0xF, 0xF,
                                                        false)
                : (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)cur_lo, 0x130, 0xF, 0xF,
                                                        false);
}

// L % 128 == 0.  A wavefront owns 64 consecutive word columns of a band of
// Band rows (32; 16 or 8 where a lattice has too few bands to fill the chip)
// and marches down it, keeping the three source rows it needs
// in registers and loading the next row's words one step ahead; the side
// neighbour comes from the adjacent word of the same source row (Sec. 3.3,
// Fig. 3).  `Dpp` (Wr % 64 == 0): the adjacent words are the neighbour lanes'
// centre words, except at the segment edge.  Otherwise lanes past the row's
// last word (Wr < 64) read the last word and store nothing, and every lane
// loads its adjacent word.  The source row that streams in is read
// non-temporally, so that L2 keeps the target lines, whose words are stored
// at different times, until they are complete.  Word indices fit in 32 bits.
//
// `Glass`: +-J couplings from the interleaved bond words (4 per spin word:
// right bonds of colour 0, 1, down bonds of colour 0, 1; bit 1 = -J), XORed
// into the neighbour words before the class split (glass_kernels.hip has the
// layout).  A lane's four bond words are one 32-byte load per row, streamed
// like the spin rows; the left bond of a target spin whose left neighbour is
// the side one takes the same one-spin shift.
//
// `Rule`: Metropolis (RuleMetro) or any 5-entry table (Rule5, heat bath).
template <class Rule, int Band, bool Anti, bool Plain, bool Dpp, bool Glass>
__global__ __launch_bounds__(256) void k_sweep_rows_q(uint64_t *__restrict__ tgt,
                                                      const uint64_t *__restrict__ src,
                                                      const uint64_t *__restrict__ bonds,
                                                      uint32_t L, uint32_t Wr,
                                                      uint32_t waves_per_band, uint32_t nbands,
                                                      int c, typename Rule::Args a)
{
    using Queue = WaveQueue<Rule::kWords>;
    __shared__ Queue queues[kWaves];
    constexpr uint32_t kRing = Rule::kRing;
    static_assert(kRing * 64 <= 256 && Band <= 1 << 19, "queue_meta fields");
    static_assert(kQueueCap == 128, "64-entry passes alternate the head between 0 and 64");
    __shared__ WaveRing<kRing> rings[kWaves];
    __shared__ __align__(16) typename Rule::LaneTable lane_tab;
    Rule::fill_table(lane_tab, a, threadIdx.x);
    __syncthreads(); // before any wavefront can leave
    const int lane = threadIdx.x & 63;
    // wave-uniform: the row arithmetic stays on the scalar unit
    const uint32_t wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    Queue &wq = queues[wv];
    WaveRing<kRing> &rg = rings[wv];
    const uint32_t gwave = rows::xcd_block(blockIdx.x, gridDim.x) * kWaves + wv;
    const uint32_t band = gwave / waves_per_band;
    if (band >= nbands)
        return; // whole wavefront
    const uint32_t w0 = (gwave - band * waves_per_band) * 64;
    const uint32_t w = w0 + lane;
    const bool active = w < Wr;
    const uint32_t wc = active ? w : Wr - 1;
    const uint32_t wl = (wc == 0) ? Wr - 1 : wc - 1;
    const uint32_t wr = (wc + 1 >= Wr) ? 0 : wc + 1;
    // Dpp (glass bonds): the one word the left edge lane reads
    const bool edge_l = lane == 0;
    const uint32_t i0 = band * Band;
    const typename Rule::Setup su = Rule::setup(a);
    auto row = [&](uint32_t i) { return src + (size_t)i * Wr; }; // wave-uniform pointer
    auto side_word = [&](uint32_t i, bool left) -> uint64_t { return row(i)[left ? wl : wr]; };
    // Dpp: the segment's edge words are the same for every lane of the
    // wavefront (left of lane 0, right of lane 63), so each is one
    // wave-uniform load
    const uint32_t wl_edge = w0 == 0 ? Wr - 1 : w0 - 1;
    const uint32_t wr_edge = w0 + 64 >= Wr ? 0 : w0 + 64;
    // (the whole word is kept until the row is decided, so that the load
    // stays in flight meanwhile)
    auto edge_word = [&](uint32_t i, bool left) -> uint64_t {
        return row_load<0>(row(i), Wr, 0u, (left ? wl_edge : wr_edge) * 8u);
    };
    const uint32_t lane_off = wc * 8u; // byte offset of the lane's word in a row
    uint64_t prev = row((i0 == 0) ? L - 1 : i0 - 1)[wc];
    uint64_t cur = row(i0)[wc];
    // Glass: bond words of the target colour (right, down) and of the other
    // colour (right ro, down dO) at word 4 k + x
    const uint32_t xro = 1u - (uint32_t)c, xdo = 3u - (uint32_t)c;
    auto bword = [&](uint32_t i, uint32_t w_) { return bonds + 4 * ((size_t)i * Wr + w_); };
    struct RowBonds {
        uint64_t dn, rt, ro, dnext; // down, right, other colour's right (aligned), dO of this row
        uint64_t radj;              // other colour's right bond at the left word (no Dpp)
        uint32_t redge;             // its high half at the segment edge (Dpp)
    };
    auto row_bonds = [&](uint32_t i, bool lft) {
        RowBonds rb{};
        if (Glass) {
            const u64x2 *p = reinterpret_cast<const u64x2 *>(bword(i, wc));
            const u64x2 r01 = __builtin_nontemporal_load(p), d01 = __builtin_nontemporal_load(p + 1);
            rb.rt = c ? r01.y : r01.x;
            rb.ro = c ? r01.x : r01.y;
            rb.dn = c ? d01.y : d01.x;
            rb.dnext = c ? d01.x : d01.y;
            if (lft) {
                if (Dpp) {
                    if (edge_l)
                        rb.redge = rows::hi32(bword(i, wl)[xro]);
                } else {
                    rb.radj = bword(i, wl)[xro];
                }
            }
        }
        return rb;
    };
    uint64_t bup = Glass ? bword((i0 == 0) ? L - 1 : i0 - 1, wc)[xdo] : 0;
    // row i0 operands
    bool left = ((i0 + c) & 1) == 0;
    uint64_t next = __builtin_nontemporal_load(&row((i0 + 1 == L) ? 0 : i0 + 1)[wc]);
    uint64_t t = tgt[(size_t)i0 * Wr + wc];
    uint64_t adj = 0;
    uint64_t edge = 0;
    if (Dpp)
        edge = edge_word(i0, left);
    else
        adj = side_word(i0, left);
    RowBonds rb = row_bonds(i0, left);
    auto trow = [&](uint32_t i) { return tgt + (size_t)i * Wr; }; // wave-uniform pointer
    uint32_t head = 0, len = 0;
    // L % 128 == 0 and Band divides 128, so every band has Band rows; the
    // loop is unrolled by four (a multiple of the ring depth), so ring slots
    // are constants and the row registers rotate without copies
#pragma unroll 4
    for (uint32_t r = 0; r < (uint32_t)Band; ++r) {
        const uint32_t i = i0 + r;
        const uint32_t idx = i * Wr + wc;
        const uint32_t sl = r & (kRing - 1);
        if (r >= kRing) // row r - kRing leaves the ring
            ring_store(rg, sl, trow(i - kRing), wc, active, lane, true);
        // loads of row i + 1, in flight while row i is decided.  They are
        // issued on every row, so that every path through the loop has the
        // same loads outstanding and the wait for this row's operands leaves
        // the new ones in flight; on the band's last row they re-read row i
        // (lines just read, so no new HBM traffic) and the results are unused.
        const bool more = r + 1 < (uint32_t)Band;
        const uint32_t i1 = !more ? i : ((i + 1 == L) ? 0 : i + 1);
        const uint32_t i2 = !more ? i : ((i1 + 1 == L) ? 0 : i1 + 1);
        const bool left1 = !left;
        uint64_t adj1 = 0, edge1 = 0;
        const uint64_t next1 = row_load<kLoadNT>(row(i2), Wr, lane_off, 0u);
        const uint64_t t1 = row_load<0>(trow(i1), Wr, lane_off, 0u);
        if (Dpp)
            edge1 = edge_word(i1, left1);
        else
            adj1 = side_word(i1, left1);
        // (the glass's bond words are read non-temporally and are gone from
        // L2 by then: the last row skips them rather than fetch them again)
        const RowBonds rb1 = (Glass && !more) ? RowBonds{} : row_bonds(i1, left1);
        const uint32_t adj_half =
            Dpp ? side_half_dpp(rows::lo32(cur), rows::hi32(cur),
                                left ? rows::hi32(edge) : rows::lo32(edge), left)
                : (left ? rows::hi32(adj) : rows::lo32(adj));
        uint32_t shl, shh;
        rows::side_halves(cur, adj_half, left, shl, shh);
        uint64_t nu = prev, nd = next, nc = cur;
        if (Glass) {
            nu ^= bup;
            nd ^= rb.dn;
            if (left) { // centre = right neighbour; side = left neighbour, shifted bonds
                nc ^= rb.rt;
                const uint32_t radj_half = Dpp ? side_half_dpp(rows::lo32(rb.ro), rows::hi32(rb.ro),
                                                               rb.redge, true)
                                               : rows::hi32(rb.radj);
                uint32_t bl, bh;
                rows::side_halves(rb.ro, radj_half, true, bl, bh);
                shl ^= bl;
                shh ^= bh;
            } else { // centre = left neighbour; side = right neighbour
                nc ^= rb.ro;
                shl ^= rows::lo32(rb.rt);
                shh ^= rows::hi32(rb.rt);
            }
        }
        typename Rule::State s = Rule::template start<Anti, Plain>(t, nu, nd, nc, shl, shh, su, a);
        // (a block applied to a decided word changes nothing; with both
        // classes random a whole wavefront is practically never decided
        // early, so only the other cases test for it)
        // (the threshold words are re-read per row, see Rule::per_row)
        const typename Rule::Args ar = Rule::per_row(a);
#pragma unroll
        for (uint32_t q = 0; q < kStreamBlocks; ++q) {
            if (!Plain && __ballot(active && undecided(s)) == 0)
                break;
            Rule::block(s, q, idx, ar);
        }
        const bool push = active && undecided(s);
        rg.word[sl][lane] = rows::join(s.tf[0], s.tf[1]);
        rg.done[sl][lane] = push ? 0 : 1;
        const uint64_t bal = __builtin_amdgcn_ballot_w64(push);
        if (push)
            queue_put<Rule>(wq, (head + len + lanes_below(bal)) & (kQueueCap - 1), s, idx,
                            queue_meta(kStreamBlocks, sl * 64 + (uint32_t)lane, r));
        __builtin_amdgcn_wave_barrier();
        len += (uint32_t)__popcll(bal);
        while (len >= 64) {
            if (head == 0)
                drain_once<Rule, 0>(wq, rg, head, len, 64, r, tgt, a, lane_tab, lane);
            else
                drain_once<Rule, 64>(wq, rg, head, len, 64, r, tgt, a, lane_tab, lane);
        }
        prev = cur;
        cur = next;
        next = next1;
        t = t1;
        adj = adj1;
        edge = edge1;
        left = left1;
        if (Glass) {
            bup = rb.dnext;
            rb = rb1;
        }
    }
    while (len > 0)
        drain_once<Rule>(wq, rg, head, len, len < 64 ? len : 64, Band - 1, tgt, a, lane_tab,
                         lane);
    // the last rows, all words final
    static_assert(Band >= (int)kRing && Band % 4 == 0 && 128 % Band == 0,
                  "whole bands of at least kRing rows");
#pragma unroll
    for (uint32_t r = Band - kRing; r < (uint32_t)Band; ++r)
        ring_store(rg, r & (kRing - 1), trow(i0 + r), wc, active, lane, false);
}


// ------------------------------------------- any 5-entry table (heat bath)
// The other local rule of Sec. 2: every class may draw, so the decision is
// decide_word5(); the geometry is handled as in the Metropolis kernels.
__global__ __launch_bounds__(256) void k_sweep_general5(uint64_t *__restrict__ tgt,
                                                        const uint64_t *__restrict__ src, int64_t H,
                                                        int64_t M, int64_t W, int c,
                                                        rows::SweepArgs5 a)
{
    const int64_t chunk = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (chunk >= W)
        return;
    const Neighbours nb = neighbours_general(src, H, M, W, chunk, c);
    tgt[chunk] = rows::decide_word5(tgt[chunk], nb, valid_mask(chunk, M), (uint32_t)chunk, a);
}

// Row-aligned lattices: one thread per word column of a band of kRows rows,
// three source rows in registers (as k_sweep_rows).
__global__ __launch_bounds__(256) void k_sweep_rows5(uint64_t *__restrict__ tgt,
                                                     const uint64_t *__restrict__ src, int64_t L,
                                                     int64_t Wr, int64_t blocks_per_band, int c,
                                                     rows::SweepArgs5 a)
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
        const uint64_t next = src[((i + 1 == L) ? 0 : i + 1) * Wr + w];
        const int64_t idx = i * Wr + w;
        const bool left = ((i + c) & 1) == 0;
        const Neighbours nb{prev, next, cur, side_vector(cur, src[i * Wr + (left ? wl : wr)], left)};
        tgt[idx] = rows::decide_word5(tgt[idx], nb, ~0ull, (uint32_t)idx, a);
        prev = cur;
        cur = next;
    }
}

hipError_t launch_half_sweep5(uint64_t *words, int64_t L, int c, const rows::Table5 &tab,
                              uint64_t t, uint64_t seed, uint32_t stream_id, hipStream_t s,
                              int variant)
{
    const int64_t H = L / 2, M = L * L / 2, W = (M + 63) / 64;
    uint64_t *tgt = words + (int64_t)c * W;
    const uint64_t *src = words + (int64_t)(1 - c) * W;
    const rows::SweepArgs5 a{tab, (uint32_t)t, (uint32_t)(t >> 32), stream_id, (uint32_t)seed,
                             (uint32_t)(seed >> 32)};
    if (L % 128 == 0 && variant != kVariantGeneral && variant != kVariantRowsPlain) {
        // the queued row kernel under the table
        const int band = variant == kVariantQueue16 ? 16 : (variant == kVariantQueue8 ? 8 : 32);
        const int64_t Wr = L / 128, wpb = (Wr + 63) / 64, nbands = (L + band - 1) / band;
        const int64_t waves = wpb * nbands;
        using Kernel = void (*)(uint64_t *, const uint64_t *, const uint64_t *, uint32_t, uint32_t,
                                uint32_t, uint32_t, int, rows::SweepArgs5);
        static const Kernel kernels[3][2] = {
            {k_sweep_rows_q<Rule5, 32, false, false, false, false>,
             k_sweep_rows_q<Rule5, 32, false, false, true, false>},
            {k_sweep_rows_q<Rule5, 16, false, false, false, false>,
             k_sweep_rows_q<Rule5, 16, false, false, true, false>},
            {k_sweep_rows_q<Rule5, 8, false, false, false, false>,
             k_sweep_rows_q<Rule5, 8, false, false, true, false>}};
        const Kernel k = kernels[band == 32 ? 0 : (band == 16 ? 1 : 2)][Wr % 64 == 0 ? 1 : 0];
        hipLaunchKernelGGL(k, dim3((uint32_t)((waves + kWaves - 1) / kWaves)), dim3(64 * kWaves),
                           0, s, tgt, src, nullptr, (uint32_t)L, (uint32_t)Wr, (uint32_t)wpb,
                           (uint32_t)nbands, c, a);
    } else if (L % 128 == 0 && variant == kVariantRowsPlain) {
        const int64_t Wr = L / 128;
        const int threads = Wr >= 256 ? 256 : (Wr >= 64 ? 64 * (int)((Wr + 63) / 64) : 64);
        const int64_t bpb = (Wr + threads - 1) / threads;
        const int64_t bands = (L + kRows - 1) / kRows;
        hipLaunchKernelGGL(k_sweep_rows5, dim3((uint32_t)(bands * bpb)), dim3(threads), 0, s, tgt,
                           src, L, Wr, bpb, c, a);
    } else {
        hipLaunchKernelGGL(k_sweep_general5, dim3((uint32_t)((W + 255) / 256)), dim3(256), 0, s,
                           tgt, src, H, M, W, c, a);
    }
    return hipGetLastError();
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
    const uint32_t nb = blocks_for(2 * W, 256);
    hipLaunchKernelGGL(k_init, dim3(nb < kMaxStrideBlocks ? nb : kMaxStrideBlocks), dim3(256), 0, s,
                       words, M, W,
                       (uint32_t)seed, (uint32_t)(seed >> 32), stream_id);
    return hipGetLastError();
}

// The queued row kernel for a row-aligned lattice (L % 128 == 0), with the
// bond arrays of a +-J glass or without (bonds == nullptr); band = 32, 16 or
// 8 rows.
hipError_t launch_rows_queue(uint64_t *tgt, const uint64_t *src, const uint64_t *bonds,
                             int64_t L, int c, const Metro2 &m, const SweepArgs2 &a, hipStream_t s,
                             int band)
{
    if (L % 128 != 0 || (band != 8 && band != 16 && band != 32))
        return hipErrorInvalidValue; // the kernel assumes whole bands of whole 64-word rows
    const int64_t Wr = L / 128;
    const int64_t wpb = (Wr + 63) / 64;
    const int64_t nbands = L / band;
    const int64_t waves = wpb * nbands;
    const dim3 grid((uint32_t)((waves + kWaves - 1) / kWaves)), block(64 * kWaves);
    const bool plain = m.randA && m.randB && !m.alwaysA && !m.alwaysB;
    const bool dpp = Wr % 64 == 0;
    using Kernel = void (*)(uint64_t *, const uint64_t *, const uint64_t *, uint32_t, uint32_t,
                            uint32_t, uint32_t, int, SweepArgs2);
#define ISING_ROWS_Q8(B, G)                                                                       \
    k_sweep_rows_q<RuleMetro, B, false, false, false, G>,                                         \
        k_sweep_rows_q<RuleMetro, B, false, false, true, G>,                                      \
        k_sweep_rows_q<RuleMetro, B, false, true, false, G>,                                      \
        k_sweep_rows_q<RuleMetro, B, false, true, true, G>,                                       \
        k_sweep_rows_q<RuleMetro, B, true, false, false, G>,                                      \
        k_sweep_rows_q<RuleMetro, B, true, false, true, G>,                                       \
        k_sweep_rows_q<RuleMetro, B, true, true, false, G>,                                       \
        k_sweep_rows_q<RuleMetro, B, true, true, true, G>
    static const Kernel kernels[6][8] = {
        {ISING_ROWS_Q8(32, false)}, {ISING_ROWS_Q8(16, false)}, {ISING_ROWS_Q8(8, false)},
        {ISING_ROWS_Q8(32, true)},  {ISING_ROWS_Q8(16, true)},  {ISING_ROWS_Q8(8, true)}};
#undef ISING_ROWS_Q8
    const int set = (bonds ? 3 : 0) + (band == 32 ? 0 : (band == 16 ? 1 : 2));
    const Kernel k = kernels[set][(m.anti ? 4 : 0) + (plain ? 2 : 0) + (dpp ? 1 : 0)];
    hipLaunchKernelGGL(k, grid, block, 0, s, tgt, src, bonds, (uint32_t)L, (uint32_t)Wr,
                       (uint32_t)wpb, (uint32_t)nbands, c, a);
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
            const int band = variant == kVariantQueue16 ? 16 : (variant == kVariantQueue8 ? 8 : 32);
            return launch_rows_queue(tgt, src, nullptr, L, c, m, a, s, band);
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
