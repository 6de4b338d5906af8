// Streaming half-sweep of row-aligned lattices (L % 128 == 0) on gfx950: the
// per-word steps written on 32-bit halves with the three-input logic
// instruction of gfx950, so that the Philox rounds, the neighbour count and
// the bit-plane compare take as few vector instructions as the hardware
// allows.  Every helper here computes exactly what the 64-bit helpers of
// ising_device.hpp compute (same Philox counters, same planes, same
// thresholds); only the instruction count differs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"

namespace ising {
namespace rows {

// ------------------------------------------------------ three-input logic
// v_bitop3_b32 d, a, b, c, TT: bit (4a + 2b + c) of the 8-bit immediate TT is
// the result for input bits a, b, c.  kA, kB, kC are the tables of the three
// inputs themselves, so the table of a logic expression is that expression
// evaluated on them.
constexpr uint32_t kA = 0xF0, kB = 0xCC, kC = 0xAA;
constexpr uint32_t tt(uint32_t v) { return v & 0xFFu; }

template <uint32_t TT>
__host__ __device__ __forceinline__ uint32_t lop3(uint32_t a, uint32_t b, uint32_t c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_bitop3_b32(a, b, c, TT);
#else
    // the instruction's definition, for the host build of these helpers
    uint32_t r = 0;
    for (uint32_t i = 0; i < 8; ++i)
        if ((TT >> i) & 1u)
            r |= ((i & 4u) ? a : ~a) & ((i & 2u) ? b : ~b) & ((i & 1u) ? c : ~c);
    return r;
#endif
}

constexpr uint32_t kXor3 = tt(kA ^ kB ^ kC);

__host__ __device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return lop3<kXor3>(a, b, c);
}

// ------------------------------------------------------------------ Philox
// Philox4x32-10 as in ising_device.hpp, with each round's "high product ^
// counter word ^ key" terms as single three-input XORs.  Which terms vary per
// lane is fixed by the counter and the key: counter words 1 and 2 (the
// half-sweep index) are the same in every lane, word 3 (the word index) is
// not; word 0 (stream, domain, block) and the key vary per lane or not
// according to the mode.  The early rounds still have wave-uniform terms,
// which the scalar unit computes; a XOR with at most one lane-varying input
// is one vector XOR once the scalar unit has combined the other two.
enum PhiloxMode {
    kCtrUniform = 0, // word 0 and key wave-uniform (lock-step blocks of a row)
    kCtrLane = 1,    // word 0 per lane (block index per lane), key uniform
    kCtrKeyLane = 2, // word 0 and key per lane (lattices of a batch)
};

template <int Mode>
__host__ __device__ __forceinline__ Block philox_fast(uint32_t c0, uint32_t c1, uint32_t c2,
                                                      uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t pa = (uint64_t)0xD2511F53u * c0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        const bool plain0 = Mode == kCtrUniform ? round <= 3 : (Mode == kCtrLane ? round <= 1 : round == 0);
        const bool plain2 = Mode == kCtrUniform ? round <= 2 : (Mode == kCtrLane ? (round == 1 || round == 2) : false);
        const uint32_t n0 = plain0 ? ((uint32_t)(pb >> 32) ^ c1 ^ k0)
                                   : xor3((uint32_t)(pb >> 32), c1, k0);
        const uint32_t n2 = plain2 ? ((uint32_t)(pa >> 32) ^ c3 ^ k1)
                                   : xor3((uint32_t)(pa >> 32), c3, k1);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
    }
    return Block{c0, c1, c2, c3};
}

// --------------------------------------------------------- neighbour count
// Per 32-bit half, with D_k = 1 where neighbour k is "unfavourable" (differs
// from the spin for J > 0, equals it for J < 0; Sec. 2):
//   zero = no D_k set      -> class B (|dE| = 8|J|),
//   one  = exactly one set -> class A (|dE| = 4|J|),
//   ge2  = two or more set -> dE <= 0, always flipped.
struct Split {
    uint32_t ge2, one, zero;
};

template <bool Anti>
__host__ __device__ __forceinline__ Split split_classes(uint32_t s, uint32_t n0, uint32_t n1,
                                                        uint32_t n2, uint32_t n3)
{
    // D_k = s ^ n_k (J > 0) or ~(s ^ n_k) (J < 0), folded into the tables
    constexpr uint32_t dB = Anti ? (~(kA ^ kB)) : (kA ^ kB);
    constexpr uint32_t dC = Anti ? (~(kA ^ kC)) : (kA ^ kC);
    const uint32_t o01 = lop3<tt(dB | dC)>(s, n0, n1);
    const uint32_t a01 = lop3<tt(dB & dC)>(s, n0, n1);
    const uint32_t o23 = lop3<tt(dB | dC)>(s, n2, n3);
    const uint32_t a23 = lop3<tt(dB & dC)>(s, n2, n3);
    Split r;
    r.ge2 = lop3<tt(kA | kB | kC)>(lop3<tt(kA | (kB & kC))>(a01, o01, o23), a23, 0u);
    r.one = lop3<tt((kA | kB) & ~kC)>(o01, o23, r.ge2);
    r.zero = ~(o01 | o23);
    return r;
}

// ---------------------------------------------------------- decision state
// Per 32-bit half h: tf = target word with the flips decided so far applied,
// p = spins still undecided, a = class-A spins (class B elsewhere).
struct State {
    uint32_t tf[2], p[2], a[2];
};

// Uniform per-launch masks (all ones or zero) of the Metropolis classes.
struct ClassMasks {
    uint32_t alwaysA, alwaysB, randA, randB;
};

__host__ __device__ __forceinline__ ClassMasks class_masks(const Metro2 &m)
{
    return ClassMasks{m.alwaysA ? ~0u : 0u, m.alwaysB ? ~0u : 0u, m.randA ? ~0u : 0u,
                      m.randB ? ~0u : 0u};
}

// Start state of half h.  `Plain`: both classes need a random number and
// neither always flips (every J != 0, 0 < beta < infinity with non-degenerate
// thresholds), the common case.
template <bool Plain>
__host__ __device__ __forceinline__ void start_half(State &s, int h, uint32_t t, const Split &k,
                                                    const ClassMasks &cm)
{
    if (Plain) {
        s.tf[h] = t ^ k.ge2;
        s.a[h] = k.one;
        s.p[h] = ~k.ge2;
    } else {
        const uint32_t f = lop3<tt(kA | (kB & kC))>(k.ge2, k.one, cm.alwaysA) | (k.zero & cm.alwaysB);
        s.tf[h] = t ^ f;
        s.a[h] = k.one & cm.randA;
        s.p[h] = lop3<tt(kA | (kB & kC))>(s.a[h], k.zero, cm.randB);
    }
}

// One bit-plane (both 32-bit halves, Plo and Phi) against threshold bits bA,
// bB that every lane shares: where the r bit differs from the spin's
// threshold bit the spin is decided, accepted (flipped) if the threshold bit
// is 1.
__host__ __device__ __forceinline__ void plane_uniform(State &s, uint32_t Plo, uint32_t Phi,
                                                       bool bA, bool bB)
{
    const uint32_t P[2] = {Plo, Phi};
    if (!bA && !bB) { // r bit 1 rejects
#pragma unroll
        for (int h = 0; h < 2; ++h)
            s.p[h] = lop3<tt(kA & ~kB)>(s.p[h], P[h], 0u);
    } else if (bA && bB) { // r bit 0 accepts
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            s.tf[h] = lop3<tt(kA ^ (kB & ~kC))>(s.tf[h], s.p[h], P[h]);
            s.p[h] &= P[h];
        }
    } else if (bA) { // class A: r bit 0 accepts; class B: r bit 1 rejects
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            s.tf[h] = lop3<tt(kA ^ (kB & kC))>(s.tf[h], lop3<tt(kA & ~kB)>(s.p[h], P[h], 0u), s.a[h]);
            s.p[h] = lop3<tt(kA & ~(kB ^ kC))>(s.p[h], P[h], s.a[h]);
        }
    } else { // class B: r bit 0 accepts; class A: r bit 1 rejects
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            s.tf[h] = lop3<tt(kA ^ (kB & ~kC))>(s.tf[h], lop3<tt(kA & ~kB)>(s.p[h], P[h], 0u), s.a[h]);
            s.p[h] = lop3<tt(kA & (kB ^ kC))>(s.p[h], P[h], s.a[h]);
        }
    }
}

// The same with per-lane threshold masks mA, mB (all ones where the plane's
// bit of T_A, T_B is 1): threshold bit tb = a ? mA : mB.
__host__ __device__ __forceinline__ void plane_lane(State &s, int h, uint32_t P, uint32_t mA,
                                                    uint32_t mB)
{
    uint32_t &tf = s.tf[h], &p = s.p[h];
    const uint32_t tb = lop3<tt((kA & kB) | (~kA & kC))>(s.a[h], mA, mB);
    const uint32_t differ = lop3<tt(kA & (kB ^ kC))>(p, P, tb);
    tf = lop3<tt(kA ^ (kB & kC))>(tf, differ, tb);
    p ^= differ;
}

// All ones where bit `bit` of thr is set (per lane).
__host__ __device__ __forceinline__ uint32_t thr_mask(uint32_t thr, uint32_t bit)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return (uint32_t)__builtin_amdgcn_sbfe((int32_t)thr, bit, 1);
#else
    return ((thr >> bit) & 1u) ? ~0u : 0u;
#endif
}

// Block q (planes 2q, 2q+1) with lane-shared threshold bits.
__host__ __device__ __forceinline__ void block_uniform(State &s, uint32_t q, uint32_t chunk,
                                                       const SweepArgs2 &a)
{
    const Block x = philox_fast<kCtrUniform>(ctr_word0(a.stream_id, kDomainSweep, q), a.t_lo,
                                             a.t_hi, chunk, a.key0, a.key1);
    const uint32_t b0 = 31 - 2 * q, b1 = 30 - 2 * q;
    const bool a0 = (a.m.thrA >> b0) & 1u, B0 = (a.m.thrB >> b0) & 1u;
    const bool a1 = (a.m.thrA >> b1) & 1u, B1 = (a.m.thrB >> b1) & 1u;
    plane_uniform(s, x.x0, x.x1, a0, B0);
    plane_uniform(s, x.x2, x.x3, a1, B1);
}

// Threshold masks of block q (planes 2q, 2q+1): all ones where the plane's
// bit of T_A, T_B is set.
struct BlockMasks {
    uint32_t mA0, mB0, mA1, mB1;
};

__host__ __device__ __forceinline__ BlockMasks block_masks(uint32_t q, const Metro2 &m)
{
    const uint32_t b0 = 31 - 2 * q, b1 = 30 - 2 * q;
    return BlockMasks{thr_mask(m.thrA, b0), thr_mask(m.thrB, b0), thr_mask(m.thrA, b1),
                      thr_mask(m.thrB, b1)};
}

// Philox block x applied with the threshold masks of its block.
__host__ __device__ __forceinline__ void apply_block_masks(State &s, const Block &x,
                                                           const BlockMasks &bm)
{
    plane_lane(s, 0, x.x0, bm.mA0, bm.mB0);
    plane_lane(s, 1, x.x1, bm.mA0, bm.mB0);
    plane_lane(s, 0, x.x2, bm.mA1, bm.mB1);
    plane_lane(s, 1, x.x3, bm.mA1, bm.mB1);
}

// Philox block x applied as block q (planes 2q, 2q+1) with per-lane
// threshold masks.
__host__ __device__ __forceinline__ void apply_block_lane(State &s, const Block &x, uint32_t q,
                                                          const Metro2 &m)
{
    apply_block_masks(s, x, block_masks(q, m));
}

// Block q with per-lane q.  After block 15 (all 32 planes) a spin still
// undecided has r == T, not < T: rejected, which the caller does by dropping
// the word.
__host__ __device__ __forceinline__ void block_lane(State &s, uint32_t q, uint32_t chunk,
                                                    const SweepArgs2 &a)
{
    apply_block_lane(s,
                     philox_fast<kCtrLane>(ctr_word0(a.stream_id, kDomainSweep, q), a.t_lo, a.t_hi,
                                           chunk, a.key0, a.key1),
                     q, a.m);
}

// ----------------------------------------------------------- word helpers
__host__ __device__ __forceinline__ uint32_t lo32(uint64_t v) { return (uint32_t)v; }
__host__ __device__ __forceinline__ uint32_t hi32(uint64_t v) { return (uint32_t)(v >> 32); }
__host__ __device__ __forceinline__ uint64_t join(uint32_t lo, uint32_t hi)
{
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// Funnel shift: low 32 bits of (hi:lo) >> sh, 0 < sh < 32.
__host__ __device__ __forceinline__ uint32_t funnel(uint32_t hi, uint32_t lo, uint32_t sh)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_alignbit(hi, lo, sh);
#else
    return (uint32_t)((((uint64_t)hi << 32) | lo) >> sh);
#endif
}

// Side vector halves: centre shifted by one spin, the adjacent word's edge
// spin shifted in (Sec. 3.3, Fig. 3); `adj_half` = the half of the adjacent
// word that feeds it (high half of the left word when `left`, low half of
// the right word otherwise).
__host__ __device__ __forceinline__ void side_halves(uint64_t ce, uint32_t adj_half, bool left,
                                                     uint32_t &sl, uint32_t &sh)
{
    const uint32_t cl = lo32(ce), ch = hi32(ce);
    sl = left ? funnel(cl, adj_half, 31) : funnel(ch, cl, 1);
    sh = left ? funnel(ch, cl, 31) : funnel(adj_half, ch, 1);
}

// start_half<true>(split_classes<Anti>(...)) with the "two or more" mask
// never formed: 8 three-input ops per half instead of 9.  With x = the
// pairs-level part of ge2, ge2 = x | a23, so tf = t ^ (x | a23),
// p = ~(x | a23), and class A = (o01 | o23) & p.
template <bool Anti>
__host__ __device__ __forceinline__ void start_half_plain(State &s, int h, uint32_t t,
                                                          uint32_t n0, uint32_t n1, uint32_t n2,
                                                          uint32_t n3)
{
    constexpr uint32_t dB = Anti ? (~(kA ^ kB)) : (kA ^ kB);
    constexpr uint32_t dC = Anti ? (~(kA ^ kC)) : (kA ^ kC);
    const uint32_t o01 = lop3<tt(dB | dC)>(t, n0, n1);
    const uint32_t a01 = lop3<tt(dB & dC)>(t, n0, n1);
    const uint32_t o23 = lop3<tt(dB | dC)>(t, n2, n3);
    const uint32_t a23 = lop3<tt(dB & dC)>(t, n2, n3);
    const uint32_t x = lop3<tt(kA | (kB & kC))>(a01, o01, o23);
    s.tf[h] = lop3<tt(kA ^ (kB | kC))>(t, x, a23);
    s.p[h] = lop3<tt(~(kA | kB))>(x, a23, 0u);
    s.a[h] = lop3<tt((kA | kB) & kC)>(o01, o23, s.p[h]);
}

// Start state of a word from its target word and its four neighbour vectors
// (the side one as halves).
template <bool Anti, bool Plain>
__host__ __device__ __forceinline__ State start_from_halves(uint64_t t, uint64_t up, uint64_t dn,
                                                            uint64_t ce, uint32_t sl, uint32_t sh,
                                                            const ClassMasks &cm)
{
    State s;
    if (Plain) {
        start_half_plain<Anti>(s, 0, lo32(t), lo32(up), lo32(dn), lo32(ce), sl);
        start_half_plain<Anti>(s, 1, hi32(t), hi32(up), hi32(dn), hi32(ce), sh);
        return s;
    }
    start_half<Plain>(s, 0, lo32(t),
                      split_classes<Anti>(lo32(t), lo32(up), lo32(dn), lo32(ce), sl), cm);
    start_half<Plain>(s, 1, hi32(t),
                      split_classes<Anti>(hi32(t), hi32(up), hi32(dn), hi32(ce), sh), cm);
    return s;
}

// Start state of a word from its target word and four source words: up, down
// and centre words of the same column and the half of the adjacent source
// word that feeds the side vector.
template <bool Anti, bool Plain>
__host__ __device__ __forceinline__ State start_word_rows(uint64_t t, uint64_t up, uint64_t dn,
                                                          uint64_t ce, uint32_t adj_half,
                                                          bool left, const ClassMasks &cm)
{
    uint32_t sl, sh;
    side_halves(ce, adj_half, left, sl, sh);
    return start_from_halves<Anti, Plain>(t, up, dn, ce, sl, sh, cm);
}

// Start state of a word of any geometry from its four neighbour vectors, with
// the lattice's coupling sign and classes taken per lane; spins past the end
// of the colour (`valid` clear) neither flip nor draw.
__host__ __device__ __forceinline__ State start_word_any(uint64_t t, const Neighbours &nb,
                                                         uint64_t valid, const Metro2 &m)
{
    // J < 0: the unfavourable neighbours are the aligned ones, i.e. those
    // differing from the complemented spin
    const uint32_t f = m.anti ? ~0u : 0u;
    const ClassMasks cm = class_masks(m);
    State s;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t th = h ? hi32(t) : lo32(t), vh = h ? hi32(valid) : lo32(valid);
        const Split k = split_classes<false>(th ^ f, h ? hi32(nb.up) : lo32(nb.up),
                                             h ? hi32(nb.dn) : lo32(nb.dn),
                                             h ? hi32(nb.ce) : lo32(nb.ce),
                                             h ? hi32(nb.sd) : lo32(nb.sd));
        start_half<false>(s, h, th, k, cm);
        s.tf[h] = lop3<tt(kA ^ ((kA ^ kB) & kC))>(th, s.tf[h], vh); // flips on valid spins only
        s.p[h] &= vh;
    }
    return s;
}

// Flip mask of a word of any geometry, each block computed here (per-lane
// lattice parameters).
__host__ __device__ __forceinline__ uint64_t decide_word_any(uint64_t t, const Neighbours &nb,
                                                             uint64_t valid, uint32_t chunk,
                                                             const SweepArgs2 &a)
{
    State s = start_word_any(t, nb, valid, a.m);
    for (uint32_t q = 0; q < 16 && (s.p[0] | s.p[1]) != 0; ++q)
        apply_block_lane(s,
                         philox_fast<kCtrKeyLane>(ctr_word0(a.stream_id, kDomainSweep, q), a.t_lo,
                                                  a.t_hi, chunk, a.key0, a.key1),
                         q, a.m);
    return t ^ join(s.tf[0], s.tf[1]);
}

// ------------------------------------------------------- any 5-entry table
// Rules other than Metropolis give each class a = 0..4 (neighbours aligned
// with the spin) its own threshold: heat bath (Sec. 2) draws for every class.
struct Table5 {
    uint32_t thr[5]; // T[a] of the classes that draw (0 < T < 2^32)
    uint32_t always; // bit a: T[a] = 2^32, always flipped
    uint32_t random; // bit a: 0 < T[a] < 2^32
};

struct SweepArgs5 {
    Table5 tab;
    uint32_t t_lo, t_hi, stream_id, key0, key1;
};

// Number of aligned neighbours (one 32-bit half) as bit slices: count =
// 4 b2 + 2 b1 + b0, a bit-sliced sum of the four "aligned" vectors.
__host__ __device__ __forceinline__ void count_bits(uint32_t s, uint32_t n0, uint32_t n1,
                                                    uint32_t n2, uint32_t n3, uint32_t &b0,
                                                    uint32_t &b1, uint32_t &b2)
{
    constexpr uint32_t kAligned = tt(~(kA ^ kB)); // 1 where the two inputs are equal
    const uint32_t x0 = lop3<kAligned>(s, n0, 0u), x1 = lop3<kAligned>(s, n1, 0u);
    const uint32_t x2 = lop3<kAligned>(s, n2, 0u), x3 = lop3<kAligned>(s, n3, 0u);
    const uint32_t s1 = xor3(x0, x1, x2);
    const uint32_t c1 = lop3<tt((kA & kB) | (kA & kC) | (kB & kC))>(x0, x1, x2); // majority
    const uint32_t cy = s1 & x3;
    b0 = s1 ^ x3;
    b1 = c1 ^ cy;
    b2 = c1 & cy;
}

// The same as one-hot masks e[a], a = 0..4.
__host__ __device__ __forceinline__ void count_classes(uint32_t s, uint32_t n0, uint32_t n1,
                                                       uint32_t n2, uint32_t n3,
                                                       uint32_t (&e)[5])
{
    uint32_t b0, b1, b2;
    count_bits(s, n0, n1, n2, n3, b0, b1, b2);
    e[4] = b2;
    e[3] = b1 & b0;
    e[2] = b1 & ~b0;
    e[1] = b0 & ~b1;
    e[0] = lop3<tt(~(kA | kB | kC))>(b0, b1, b2);
}

// New value of a word of any geometry under table `a.tab`: the same lazy
// most-significant-plane-first compare r < T[a], with the threshold bit of
// each spin taken from its class.  The block index is the loop counter, the
// same in every active lane.
__host__ __device__ __forceinline__ uint64_t decide_word5(uint64_t t, const Neighbours &nb,
                                                          uint64_t valid, uint32_t chunk,
                                                          const SweepArgs5 &a)
{
    uint32_t e[2][5], tf[2], p[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t th = h ? hi32(t) : lo32(t);
        count_classes(th, h ? hi32(nb.up) : lo32(nb.up), h ? hi32(nb.dn) : lo32(nb.dn),
                      h ? hi32(nb.ce) : lo32(nb.ce), h ? hi32(nb.sd) : lo32(nb.sd), e[h]);
        uint32_t f = 0, r = 0;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            f |= ((a.tab.always >> c) & 1u) ? e[h][c] : 0u;
            r |= ((a.tab.random >> c) & 1u) ? e[h][c] : 0u;
        }
        const uint32_t vh = h ? hi32(valid) : lo32(valid);
        tf[h] = th ^ (f & vh);
        p[h] = r & vh;
    }
    for (uint32_t q = 0; q < 16 && (p[0] | p[1]) != 0; ++q) {
        const Block x = philox_fast<kCtrUniform>(ctr_word0(a.stream_id, kDomainSweep, q), a.t_lo,
                                                 a.t_hi, chunk, a.key0, a.key1);
        const uint32_t planes[2][2] = {{x.x0, x.x1}, {x.x2, x.x3}};
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const uint32_t bit = 31 - (2 * q + (uint32_t)k);
            uint32_t m[5];
#pragma unroll
            for (int c = 0; c < 5; ++c)
                m[c] = (((a.tab.random >> c) & (a.tab.thr[c] >> bit)) & 1u) ? ~0u : 0u;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                uint32_t tb = e[h][0] & m[0];
#pragma unroll
                for (int c = 1; c < 5; ++c)
                    tb = lop3<tt(kA | (kB & kC))>(tb, e[h][c], m[c]);
                const uint32_t differ = lop3<tt(kA & (kB ^ kC))>(p[h], planes[k][h], tb);
                tf[h] = lop3<tt(kA ^ (kB & kC))>(tf[h], differ, tb);
                p[h] ^= differ;
            }
        }
    }
    return join(tf[0], tf[1]); // undecided after 32 planes: r == T, rejected
}

// ------------------------------------- 5-entry table, streamed row kernel
// Decision state of a word under a 5-entry table, per 32-bit half: flips
// decided so far, spins still undecided, and each spin's aligned count as
// bit slices (the class that picks its threshold bit on every plane).
struct State5 {
    uint32_t tf[2], p[2], b0[2], b1[2], b2[2];
};

// Start state from the target word and its neighbour halves (as
// start_from_halves): always-flip classes flipped, drawing classes pending.
__host__ __device__ __forceinline__ State5 start5_from_halves(uint64_t t, uint64_t up, uint64_t dn,
                                                              uint64_t ce, uint32_t sl,
                                                              uint32_t sh, const Table5 &tab)
{
    State5 s;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t th = h ? hi32(t) : lo32(t);
        count_bits(th, h ? hi32(up) : lo32(up), h ? hi32(dn) : lo32(dn), h ? hi32(ce) : lo32(ce),
                   h ? sh : sl, s.b0[h], s.b1[h], s.b2[h]);
        const uint32_t e[5] = {lop3<tt(~(kA | kB | kC))>(s.b0[h], s.b1[h], s.b2[h]),
                               s.b0[h] & ~s.b1[h], s.b1[h] & ~s.b0[h], s.b1[h] & s.b0[h],
                               s.b2[h]};
        uint32_t f = 0, r = 0;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            f |= ((tab.always >> c) & 1u) ? e[c] : 0u;
            r |= ((tab.random >> c) & 1u) ? e[c] : 0u;
        }
        s.tf[h] = th ^ f;
        s.p[h] = r;
    }
    return s;
}

// Threshold bit of every spin from its count slices and the five classes'
// bits m[a] (all ones or zero): a multiplexer tree over b0, b1, b2.
__host__ __device__ __forceinline__ uint32_t thr_bits5(uint32_t b0, uint32_t b1, uint32_t b2,
                                                       const uint32_t (&m)[5])
{
    constexpr uint32_t kMux = tt((kA & kB) | (~kA & kC)); // A ? B : C
    const uint32_t lo = lop3<kMux>(b0, m[1], m[0]);     // count 0, 1
    const uint32_t hi = lop3<kMux>(b0, m[3], m[2]);     // count 2, 3
    return lop3<kMux>(b2, m[4], lop3<kMux>(b1, hi, lo));
}

// One plane P of half h: where the r bit differs from the spin's threshold
// bit the spin is decided, flipped if the threshold bit is 1.
__host__ __device__ __forceinline__ void plane5(State5 &s, int h, uint32_t P,
                                                const uint32_t (&m)[5])
{
    const uint32_t tb = thr_bits5(s.b0[h], s.b1[h], s.b2[h], m);
    const uint32_t differ = lop3<tt(kA & (kB ^ kC))>(s.p[h], P, tb);
    s.tf[h] = lop3<tt(kA ^ (kB & kC))>(s.tf[h], differ, tb);
    s.p[h] ^= differ;
}

// Block q (planes 2q, 2q+1) of a word: lock step (`Lane` false: q and the
// class bits shared by the wavefront) or per lane (queued words).
template <bool Lane>
__host__ __device__ __forceinline__ void block5(State5 &s, uint32_t q, uint32_t chunk,
                                                const SweepArgs5 &a)
{
    const Block x = Lane ? philox_fast<kCtrLane>(ctr_word0(a.stream_id, kDomainSweep, q), a.t_lo,
                                                 a.t_hi, chunk, a.key0, a.key1)
                         : philox_fast<kCtrUniform>(ctr_word0(a.stream_id, kDomainSweep, q),
                                                    a.t_lo, a.t_hi, chunk, a.key0, a.key1);
    const uint32_t planes[2][2] = {{x.x0, x.x1}, {x.x2, x.x3}};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const uint32_t bit = 31 - (2 * q + (uint32_t)k);
        uint32_t m[5];
#pragma unroll
        for (int c = 0; c < 5; ++c)
            m[c] = ((a.tab.random >> c) & 1u) ? (Lane ? thr_mask(a.tab.thr[c], bit)
                                                      : (((a.tab.thr[c] >> bit) & 1u) ? ~0u : 0u))
                                              : 0u;
        plane5(s, 0, planes[k][0], m);
        plane5(s, 1, planes[k][1], m);
    }
}

// --------------------------------------------------- XCD-aware block order
// Workgroups are handed to the 8 XCDs of the chip in turn (block b to XCD
// b % 8).  The logical block of hardware block b gives each XCD a contiguous
// range, so neighbouring bands, whose halo rows overlap, share an L2.
__host__ __device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nblocks)
{
    const uint32_t x = b & 7u, j = b >> 3;
    const uint32_t base = nblocks >> 3, extra = nblocks & 7u; // XCDs < extra get base + 1
    return x * base + (x < extra ? x : extra) + j;
}

} // namespace rows
} // namespace ising
