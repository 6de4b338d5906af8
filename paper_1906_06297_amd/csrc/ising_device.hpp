// Device building blocks of the checkerboard Metropolis sweep on gfx950.
//
// One 64-bit word holds 64 spins of one colour (bit = 1 <=> +1).  For a word
// of target spins the kernels build four 64-bit neighbour vectors (up, down,
// centre, side) from the other colour, count per spin the neighbours that are
// aligned with it with a bit-sliced adder (the multi-spin coding idea of
// Sec. 3.3, here at one bit per spin), and take the Metropolis decision
// (Sec. 2) exactly in integers against the threshold table, comparing the
// spin's 32-bit uniform most significant bit first, one Philox block (two
// bit-planes) at a time, and stopping as soon as every spin of the word is
// decided.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32->64 products; the key advances by the two Weyl constants between
// rounds.
struct Block {
    uint32_t x0, x1, x2, x3;
};

__host__ __device__ __forceinline__ Block philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                               uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t pa = (uint64_t)0xD2511F53u * c0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        const uint32_t n1 = (uint32_t)pb;
        const uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        const uint32_t n3 = (uint32_t)pa;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    return Block{c0, c1, c2, c3};
}

enum : uint32_t { kDomainSweep = 0, kDomainInit = 1 };

// Counter word 0 of a Philox block.
__host__ __device__ __forceinline__ uint32_t ctr_word0(uint32_t stream_id, uint32_t domain, uint32_t q)
{
    return (stream_id << 8) | (domain << 4) | q;
}

// ----------------------------------------------------- aligned-count classes
// One-hot masks e[a], a = 0..4: bit set where exactly a of the four
// neighbours equal the target spin.
struct Classes {
    uint64_t e[5];
};

__host__ __device__ __forceinline__ Classes classify(uint64_t t, uint64_t up, uint64_t dn, uint64_t ce,
                                            uint64_t sd)
{
    const uint64_t x1 = ~(t ^ up), x2 = ~(t ^ dn), x3 = ~(t ^ ce), x4 = ~(t ^ sd);
    const uint64_t s1 = x1 ^ x2, c1 = x1 & x2;
    const uint64_t s2 = x3 ^ x4, c2 = x3 & x4;
    const uint64_t a0 = s1 ^ s2, c3 = s1 & s2;
    // c3 = 1 forces x1 != x2 and x3 != x4, so at most c1 and c2 are both set
    const uint64_t a1 = c1 ^ c2 ^ c3, a2 = c1 & c2;
    Classes k;
    k.e[4] = a2;
    k.e[3] = a1 & a0;
    k.e[2] = a1 & ~a0;
    k.e[1] = a0 & ~a1;
    k.e[0] = ~(a0 | a1 | a2);
    return k;
}

// --------------------------------------------- Metropolis, two random classes
// Under the Metropolis rule (Sec. 2) at most two classes have dE > 0: for
// J > 0 the spins with a = 3 and a = 4 aligned neighbours (dE = 4J, 8J), for
// J < 0 those with a = 1 and a = 0.  Call them A (|dE| = 4|J|) and B
// (|dE| = 8|J|); every other class has dE <= 0 and always flips.
struct Metro2 {
    uint32_t thrA, thrB;       // thresholds of A and B when they need a random number
    uint32_t randA, randB;     // 1: 0 < T < 2^32, compare against thr
    uint32_t alwaysA, alwaysB; // 1: T = 2^32 (dE rounds to a certain flip)
    uint32_t anti;             // 1: J < 0 (A = 1 aligned, B = 0 aligned)
};

// Decision state of one word: flips decided so far, spins still undecided,
// and which undecided spins belong to class A (the rest are class B).
struct WordState {
    uint64_t flips, pending, classA;
};

__host__ __device__ __forceinline__ WordState start_word(const Classes &k, uint64_t valid,
                                                         const Metro2 &m)
{
    const uint64_t eA = m.anti ? k.e[1] : k.e[3];
    const uint64_t eB = m.anti ? k.e[0] : k.e[4];
    const uint64_t base = m.anti ? (k.e[2] | k.e[3] | k.e[4]) : (k.e[0] | k.e[1] | k.e[2]);
    WordState s;
    s.flips = (base | (m.alwaysA ? eA : 0) | (m.alwaysB ? eB : 0)) & valid;
    s.classA = m.randA ? (eA & valid) : 0;
    s.pending = s.classA | (m.randB ? (eB & valid) : 0);
    return s;
}

// All ones where bit `bit` of thr is set, else zero (32 bits).
__host__ __device__ __forceinline__ uint32_t bit_mask(uint32_t thr, int bit)
{
    // move the bit to the sign position and sign-extend: one shift pair
    return (uint32_t)((int32_t)(thr << (31 - bit)) >> 31);
}

// Per 32-bit half: bits of m1 where sel is set, bits of m0 elsewhere.
__host__ __device__ __forceinline__ uint32_t select_bits(uint32_t sel, uint32_t m1, uint32_t m0)
{
    return (sel & m1) | (~sel & m0);
}

// One bit-plane of the exact compare r < T: spins whose r bit differs from
// their threshold bit are decided (accepted where the threshold bit is 1).
// mA, mB: the plane's threshold bit of classes A and B as all-ones/zero.
__host__ __device__ __forceinline__ void compare_plane(WordState &s, uint64_t plane, uint32_t mA,
                                                       uint32_t mB)
{
    const uint64_t tb = (uint64_t)select_bits((uint32_t)s.classA, mA, mB) |
                        ((uint64_t)select_bits((uint32_t)(s.classA >> 32), mA, mB) << 32);
    const uint64_t differ = s.pending & (plane ^ tb);
    s.flips |= differ & tb;
    s.pending ^= differ;
}

// Applies the two bit-planes of Philox block q of a word.  After the last
// block a spin still undecided has r == T, which is not < T: rejected.
__host__ __device__ __forceinline__ void apply_block(WordState &s, const Block &x, uint32_t q,
                                                     const Metro2 &m)
{
    const int bit = 31 - 2 * (int)q;
    compare_plane(s, (uint64_t)x.x0 | ((uint64_t)x.x1 << 32), bit_mask(m.thrA, bit),
                  bit_mask(m.thrB, bit));
    compare_plane(s, (uint64_t)x.x2 | ((uint64_t)x.x3 << 32), bit_mask(m.thrA, bit - 1),
                  bit_mask(m.thrB, bit - 1));
    if (q == 15)
        s.pending = 0;
}

// Philox block q of word `chunk`: bit-planes 2q and 2q+1.
__host__ __device__ __forceinline__ void advance_block(WordState &s, uint32_t q, uint32_t chunk,
                                                       const Metro2 &m, uint32_t t_lo,
                                                       uint32_t t_hi, uint32_t stream_id,
                                                       uint32_t key0, uint32_t key1)
{
    apply_block(s,
                philox4x32_10(ctr_word0(stream_id, kDomainSweep, q), t_lo, t_hi, chunk, key0, key1),
                q, m);
}

// Sweep parameters shared by every word of one half-sweep launch.
struct SweepArgs2 {
    Metro2 m;
    uint32_t t_lo, t_hi, stream_id, key0, key1;
};

// Complete decision for one word (all its blocks in order).
__host__ __device__ __forceinline__ uint64_t decide_word(const Classes &k, uint64_t valid,
                                                         uint32_t chunk, const SweepArgs2 &a)
{
    WordState s = start_word(k, valid, a.m);
    for (uint32_t q = 0; q < 16 && s.pending != 0; ++q)
        advance_block(s, q, chunk, a.m, a.t_lo, a.t_hi, a.stream_id, a.key0, a.key1);
    return s.flips;
}

// ------------------------------------------- general colour-linear geometry
// 64 consecutive spins of a colour-linear bit string of M spins starting at
// spin x, cyclically (x taken mod M).  Bits past M in the last word are zero.
template <typename Ptr>
__host__ __device__ __forceinline__ uint64_t cyclic_bits(Ptr src, int64_t M, int64_t W, int64_t x)
{
    x %= M;
    if (x < 0)
        x += M;
    if (M >= 64) {
        const int64_t w = x >> 6;
        const int sh = (int)(x & 63);
        uint64_t lo = src[w] >> sh;
        if (sh != 0 && w + 1 < W)
            lo |= src[w + 1] << (64 - sh);
        const int64_t avail = M - x;
        if (avail >= 64)
            return lo;
        return (lo & ((1ull << avail) - 1)) | (src[0] << avail);
    }
    // fewer than 64 spins: the whole colour sits in word 0; repeat it
    const uint64_t full = (1ull << M) - 1;
    const uint64_t p = src[0] & full;
    const uint64_t rot = x ? (((p >> x) | (p << (M - x))) & full) : p;
    uint64_t r = 0;
    for (int64_t f = 0; f < 64; f += M)
        r |= rot << f;
    return r;
}

// Row structure of word `chunk` of colour c: which bits start or end a
// colour row, and which bits sit on rows whose side neighbour is on the left
// ((i + c) even: column j/2 - 1 of the other colour, Fig. 2 and Fig. 3).
struct RowMasks {
    uint64_t left_rows, row_start, row_end;
};

__host__ __device__ __forceinline__ RowMasks row_masks(int64_t chunk, int64_t H, int64_t M, int c)
{
    const int64_t n0 = chunk << 6;
    const int64_t end = (n0 + 64 < M) ? n0 + 64 : M;
    int64_t i = n0 / H;
    RowMasks r{0, 0, 0};
    for (int64_t rs = i * H; rs < end; ++i, rs += H) {
        const int64_t a = (rs > n0 ? rs : n0) - n0;
        const int64_t b = ((rs + H < end) ? rs + H : end) - n0;
        const uint64_t seg = (b - a >= 64) ? ~0ull : (((1ull << (b - a)) - 1) << a);
        if (((i + c) & 1) == 0)
            r.left_rows |= seg;
        if (rs >= n0)
            r.row_start |= 1ull << (rs - n0);
        if (rs + H - 1 < end)
            r.row_end |= 1ull << (rs + H - 1 - n0);
    }
    return r;
}

struct Neighbours {
    uint64_t up, dn, ce, sd;
};

// The four neighbour vectors of target word `chunk` of colour c, read from
// the other colour's bit string `src` (any lattice size).
template <typename Ptr>
__host__ __device__ __forceinline__ Neighbours neighbours_general(Ptr src, int64_t H, int64_t M, int64_t W,
                                                         int64_t chunk, int c)
{
    const int64_t n0 = chunk << 6;
    const RowMasks rm = row_masks(chunk, H, M, c);
    Neighbours nb;
    nb.ce = cyclic_bits(src, M, W, n0);
    nb.up = cyclic_bits(src, M, W, n0 - H);
    nb.dn = cyclic_bits(src, M, W, n0 + H);
    const uint64_t left = (cyclic_bits(src, M, W, n0 - 1) & ~rm.row_start) |
                          (cyclic_bits(src, M, W, n0 + H - 1) & rm.row_start);
    const uint64_t right = (cyclic_bits(src, M, W, n0 + 1) & ~rm.row_end) |
                           (cyclic_bits(src, M, W, n0 - H + 1) & rm.row_end);
    nb.sd = (left & rm.left_rows) | (right & ~rm.left_rows);
    return nb;
}

__host__ __device__ __forceinline__ uint64_t valid_mask(int64_t chunk, int64_t M)
{
    const int64_t n0 = chunk << 6;
    return (n0 + 64 <= M) ? ~0ull : ((1ull << (M - n0)) - 1);
}

// -------------------------------- extended colour arrays (lattices in LDS)
// An extended colour array E holds the W words of one colour, then two more
// words; the padding bits of word W-1 and the two extra words continue the
// bit string cyclically (spin M follows spin M-1 with spin 0).  64 spins
// starting at any x in [0, M) are then one funnel shift of E[x/64], E[x/64+1].
template <typename Ptr>
__host__ __device__ __forceinline__ uint64_t ext_bits(Ptr E, uint32_t x)
{
    const uint32_t w = x >> 6, sh = x & 63;
    const uint64_t lo = E[w], hi = E[w + 1];
    return sh ? (lo >> sh) | (hi << (64 - sh)) : lo;
}

// New contents of E[W-1], E[W], E[W+1] after the W words of the colour changed.
template <typename Ptr>
__host__ __device__ __forceinline__ void ext_tail(Ptr E, uint32_t M, uint32_t W, uint64_t out[3])
{
    const uint32_t r = M & 63;
    const uint64_t head = cyclic_bits(E, M, W, 0);
    out[0] = r ? ((E[W - 1] & ((1ull << r) - 1)) | (head << r)) : E[W - 1];
    out[1] = cyclic_bits(E, M, W, (int64_t)64 * W - M);
    out[2] = cyclic_bits(E, M, W, (int64_t)64 * W + 64 - M);
}

__host__ __device__ __forceinline__ uint32_t wrap_spin(int64_t x, uint32_t M)
{
    return (uint32_t)(x < 0 ? x + M : (x >= (int64_t)M ? x - M : x));
}

// Neighbour vectors of target word k of colour c from an extended source array.
template <typename Ptr>
__host__ __device__ __forceinline__ Neighbours neighbours_ext(Ptr E, uint32_t H, uint32_t M,
                                                              uint32_t k, int c)
{
    const int64_t n0 = (int64_t)k << 6;
    const RowMasks rm = row_masks(k, H, M, c);
    Neighbours nb;
    nb.ce = ext_bits(E, (uint32_t)n0);
    nb.up = ext_bits(E, wrap_spin(n0 - H, M));
    nb.dn = ext_bits(E, wrap_spin(n0 + H, M));
    const uint64_t left = (ext_bits(E, wrap_spin(n0 - 1, M)) & ~rm.row_start) |
                          (ext_bits(E, wrap_spin(n0 + H - 1, M)) & rm.row_start);
    const uint64_t right = (ext_bits(E, wrap_spin(n0 + 1, M)) & ~rm.row_end) |
                           (ext_bits(E, wrap_spin(n0 - H + 1, M)) & rm.row_end);
    nb.sd = (left & rm.left_rows) | (right & ~rm.left_rows);
    return nb;
}

// Row masks of word k for lattices whose spin counts fit 32 bits.
__host__ __device__ __forceinline__ RowMasks row_masks32(uint32_t k, uint32_t H, uint32_t M, int c)
{
    const uint32_t n0 = k << 6;
    const uint32_t end = (n0 + 64 < M) ? n0 + 64 : M;
    uint32_t i = n0 / H;
    RowMasks r{0, 0, 0};
    for (uint32_t rs = i * H; rs < end; ++i, rs += H) {
        const uint32_t a = (rs > n0 ? rs : n0) - n0;
        const uint32_t b = ((rs + H < end) ? rs + H : end) - n0;
        const uint64_t seg = (b - a >= 64) ? ~0ull : (((1ull << (b - a)) - 1) << a);
        if (((i + c) & 1) == 0)
            r.left_rows |= seg;
        if (rs >= n0)
            r.row_start |= 1ull << (rs - n0);
        if (rs + H - 1 < end)
            r.row_end |= 1ull << (rs + H - 1 - n0);
    }
    return r;
}

// As neighbours_ext with precomputed row masks.
template <typename Ptr>
__host__ __device__ __forceinline__ Neighbours neighbours_ext_rm(Ptr E, uint32_t H, uint32_t M,
                                                                 uint32_t k, const RowMasks &rm)
{
    const int64_t n0 = (int64_t)k << 6;
    Neighbours nb;
    nb.ce = ext_bits(E, (uint32_t)n0);
    nb.up = ext_bits(E, wrap_spin(n0 - H, M));
    nb.dn = ext_bits(E, wrap_spin(n0 + H, M));
    const uint64_t left = (ext_bits(E, wrap_spin(n0 - 1, M)) & ~rm.row_start) |
                          (ext_bits(E, wrap_spin(n0 + H - 1, M)) & rm.row_start);
    const uint64_t right = (ext_bits(E, wrap_spin(n0 + 1, M)) & ~rm.row_end) |
                           (ext_bits(E, wrap_spin(n0 - H + 1, M)) & rm.row_end);
    nb.sd = (left & rm.left_rows) | (right & ~rm.left_rows);
    return nb;
}

// Tail of an extended colour array, cheap when M is a multiple of 64 and the
// colour has at least two words (then the tail repeats words 0 and 1).
template <typename Ptr>
__host__ __device__ __forceinline__ void ext_tail_fast(Ptr E, uint32_t M, uint32_t W,
                                                       uint64_t out[3])
{
    if ((M & 63) == 0 && W >= 2) {
        out[0] = E[W - 1];
        out[1] = E[0];
        out[2] = E[1];
    } else {
        ext_tail(E, M, W, out);
    }
}

// New value of target word `chunk` of colour c, any geometry.
template <typename Ptr>
__host__ __device__ __forceinline__ uint64_t update_word_general(uint64_t t, Ptr src, int64_t H,
                                                                 int64_t M, int64_t W,
                                                                 int64_t chunk, int c,
                                                                 const SweepArgs2 &a)
{
    const Neighbours nb = neighbours_general(src, H, M, W, chunk, c);
    const Classes k = classify(t, nb.up, nb.dn, nb.ce, nb.sd);
    return t ^ decide_word(k, valid_mask(chunk, M), (uint32_t)chunk, a);
}

// Row-aligned geometry (each colour row is a whole number of words): the side
// vector of a target word from the centre source word and the adjacent source
// word of the same row, left (j/2 - 1) or right (j/2 + 1) neighbours.
__host__ __device__ __forceinline__ uint64_t side_vector(uint64_t centre, uint64_t adjacent,
                                                         bool left)
{
    return left ? (centre << 1) | (adjacent >> 63) : (centre >> 1) | (adjacent << 63);
}

// New value of row-aligned target word `chunk` from its four source words.
__host__ __device__ __forceinline__ uint64_t update_word_rows(uint64_t t, uint64_t up, uint64_t dn,
                                                              uint64_t centre, uint64_t adjacent,
                                                              bool left, uint32_t chunk,
                                                              const SweepArgs2 &a)
{
    const Classes k = classify(t, up, dn, centre, side_vector(centre, adjacent, left));
    return t ^ decide_word(k, ~0ull, chunk, a);
}

// Initial value of word `chunk` of colour c.
__host__ __device__ __forceinline__ uint64_t init_word(int64_t chunk, uint32_t c, int64_t M,
                                                       uint32_t stream_id, uint32_t key0,
                                                       uint32_t key1)
{
    const Block x = philox4x32_10(ctr_word0(stream_id, kDomainInit, 0), c, 0u, (uint32_t)chunk,
                                  key0, key1);
    return ((uint64_t)x.x0 | ((uint64_t)x.x1 << 32)) & valid_mask(chunk, M);
}

} // namespace ising
