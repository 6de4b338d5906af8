// Host emulation of the sweep kernels: runs the same per-word device helpers
// (ising_device.hpp) over every word on the CPU, with the kernels' indexing,
// so the kernel logic can be checked against the oracle without a GPU.
#include <cstdint>
#include <vector>

#include "../paper_1906_06297_amd/csrc/ising_device.hpp"
#include "../paper_1906_06297_amd/csrc/ising_rows.hpp"
#include "../paper_1906_06297_amd/csrc/pair_decision.hpp"
#include "../paper_1906_06297_amd/csrc/batch_aligned.hpp"

using namespace ising;

// The two dE > 0 classes of the table, as the library's host code maps them.
static Metro2 metro2_from_table(const uint64_t *T, int anti)
{
    Metro2 m{};
    m.anti = (uint32_t)anti;
    const uint64_t tA = anti ? T[1] : T[3], tB = anti ? T[0] : T[4];
    m.alwaysA = tA >= (1ull << 32);
    m.alwaysB = tB >= (1ull << 32);
    m.randA = !m.alwaysA && tA > 0;
    m.randB = !m.alwaysB && tB > 0;
    m.thrA = m.randA ? (uint32_t)tA : 0u;
    m.thrB = m.randB ? (uint32_t)tB : 0u;
    return m;
}

namespace {

// The queued row kernel's sequence for one word: the start state from the
// 32-bit-half class split, three blocks with the lane-shared compare, then
// blocks with the per-lane compare until the word is decided.
template <bool Anti, bool Plain>
static uint64_t queued_word(uint64_t t, uint64_t up, uint64_t dn, uint64_t ce, uint64_t adj,
                            bool left, uint32_t chunk, const SweepArgs2 &a)
{
    const rows::ClassMasks cm = rows::class_masks(a.m);
    rows::State s = rows::start_word_rows<Anti, Plain>(
        t, up, dn, ce, left ? rows::hi32(adj) : rows::lo32(adj), left, cm);
    uint32_t q = 0;
    for (; q < 3; ++q)
        rows::block_uniform(s, q, chunk, a);
    for (; q < 16 && (s.p[0] | s.p[1]) != 0; ++q)
        rows::block_lane(s, q, chunk, a);
    return rows::join(s.tf[0], s.tf[1]);
}

static uint64_t queued_word_any(uint64_t t, uint64_t up, uint64_t dn, uint64_t ce, uint64_t adj,
                                bool left, uint32_t chunk, const SweepArgs2 &a)
{
    const bool plain = a.m.randA && a.m.randB && !a.m.alwaysA && !a.m.alwaysB;
    if (a.m.anti)
        return plain ? queued_word<true, true>(t, up, dn, ce, adj, left, chunk, a)
                     : queued_word<true, false>(t, up, dn, ce, adj, left, chunk, a);
    return plain ? queued_word<false, true>(t, up, dn, ce, adj, left, chunk, a)
                 : queued_word<false, false>(t, up, dn, ce, adj, left, chunk, a);
}

// The queued row kernel's sequence under a 5-entry table: start state from
// the count slices, three lock-step blocks, then per-lane blocks.
static uint64_t queued_word5(uint64_t t, uint64_t up, uint64_t dn, uint64_t ce, uint64_t adj,
                             bool left, uint32_t chunk, const rows::SweepArgs5 &a)
{
    uint32_t sl, sh;
    rows::side_halves(ce, left ? rows::hi32(adj) : rows::lo32(adj), left, sl, sh);
    rows::State5 s = rows::start5_from_halves(t, up, dn, ce, sl, sh, a.tab);
    uint32_t q = 0;
    for (; q < 3; ++q)
        rows::block5<false>(s, q, chunk, a);
    for (; q < 16 && (s.p[0] | s.p[1]) != 0; ++q)
        rows::block5<true>(s, q, chunk, a);
    return rows::join(s.tf[0], s.tf[1]);
}

} // namespace

extern "C" {

// A lane pair's step: blocks q and q + 1 each reduced to what it decides on
// its own and applied in order, against applying their planes one by one,
// over n random states, blocks and thresholds; returns the mismatches.
int emu_block_decision_check(uint64_t seed, int n)
{
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + 1;
    auto next = [&z]() { // splitmix64
        uint64_t x = (z += 0x9E3779B97F4A7C15ull);
        x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
        x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
        return x ^ (x >> 31);
    };
    auto r32 = [&next]() { return (uint32_t)next(); };
    int bad = 0;
    for (int i = 0; i < n; ++i) {
        rows::State s;
        for (int h = 0; h < 2; ++h) {
            s.tf[h] = r32();
            s.p[h] = r32();
            s.a[h] = r32();
        }
        Metro2 m{};
        // thresholds with long runs of equal bits as well as random ones
        m.thrA = (i & 1) ? r32() : (r32() | 0xFFFF0000u);
        m.thrB = (i & 2) ? r32() : (r32() & 0x0000FFFFu);
        const uint32_t q = (uint32_t)(next() % 15);
        const Block x0{r32(), r32(), r32(), r32()}, x1{r32(), r32(), r32(), r32()};
        rows::State ref = s, got = s;
        rows::apply_block_lane(ref, x0, q, m);
        rows::apply_block_lane(ref, x1, q + 1, m);
        rows::apply_decision(got, rows::block_decision_lane(s, x0, q, m));
        rows::apply_decision(got, rows::block_decision_lane(s, x1, q + 1, m));
        for (int h = 0; h < 2; ++h)
            bad += (ref.tf[h] != got.tf[h]) || (ref.p[h] != got.p[h]) || (ref.a[h] != got.a[h]);
    }
    return bad;
}

// The plain start state built straight from the pair-level terms
// (start_from_halves<Anti, true>) against the class split followed by
// start_half<true>, over n random target and neighbour words, both signs of
// J; returns the mismatches.
int emu_start_plain_check(uint64_t seed, int n)
{
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + 7;
    auto next = [&z]() { // splitmix64
        uint64_t x = (z += 0x9E3779B97F4A7C15ull);
        x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
        x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
        return x ^ (x >> 31);
    };
    const rows::ClassMasks cm{0u, 0u, ~0u, ~0u};
    int bad = 0;
    for (int i = 0; i < n; ++i) {
        const uint64_t t = next(), up = next(), dn = next(), ce = next();
        const uint32_t sl = (uint32_t)next(), sh = (uint32_t)next();
        for (int anti = 0; anti < 2; ++anti) {
            const rows::State got = anti ? rows::start_from_halves<true, true>(t, up, dn, ce, sl, sh, cm)
                                         : rows::start_from_halves<false, true>(t, up, dn, ce, sl, sh, cm);
            for (int h = 0; h < 2; ++h) {
                const uint32_t th = h ? rows::hi32(t) : rows::lo32(t);
                const uint32_t n0 = h ? rows::hi32(up) : rows::lo32(up);
                const uint32_t n1 = h ? rows::hi32(dn) : rows::lo32(dn);
                const uint32_t n2 = h ? rows::hi32(ce) : rows::lo32(ce);
                const uint32_t n3 = h ? sh : sl;
                const rows::Split k = anti ? rows::split_classes<true>(th, n0, n1, n2, n3)
                                           : rows::split_classes<false>(th, n0, n1, n2, n3);
                rows::State ref{};
                rows::start_half<true>(ref, h, th, k, cm);
                bad += (ref.tf[h] != got.tf[h]) || (ref.p[h] != got.p[h]) || (ref.a[h] != got.a[h]);
            }
        }
    }
    return bad;
}

// The batch kernel's row-aligned neighbour vectors against the general
// extraction from an extended colour array, for every word of both colours
// of an L x L lattice (L % 128 == 0) filled from `seed`; returns mismatches.
int emu_aligned_neighbours_check(int64_t L, uint64_t seed)
{
    const uint32_t H = (uint32_t)(L / 2), M = (uint32_t)(L * L / 2), W = M / 64, Wr = H / 64;
    std::vector<uint64_t> E(W + 2);
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + 7;
    for (uint32_t k = 0; k < W; ++k) { // splitmix64
        uint64_t x = (z += 0x9E3779B97F4A7C15ull);
        x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
        x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
        E[k] = x ^ (x >> 31);
    }
    E[W] = E[0];
    E[W + 1] = E[1 % W];
    int bad = 0;
    const uint32_t inv = aligned_inv(Wr);
    for (int c = 0; c < 2; ++c)
        for (uint32_t k = 0; k < W; ++k) {
            RowMasks rm = row_masks32(k, H, M, 0);
            if (c)
                rm.left_rows = ~rm.left_rows;
            const Neighbours a = neighbours_ext_rm(E.data(), H, M, k, rm);
            const Neighbours b = neighbours_aligned(E.data(), W, Wr, inv, k, c);
            bad += (a.ce != b.ce) || (a.up != b.up) || (a.dn != b.dn) || (a.sd != b.sd);
        }
    return bad;
}

// The batch kernel's half-aligned neighbour vectors (L % 64 == 0) against the
// general extraction, for every word of both colours; returns mismatches.
int emu_half_aligned_neighbours_check(int64_t L, uint64_t seed)
{
    const uint32_t H = (uint32_t)(L / 2), M = (uint32_t)(L * L / 2), W = M / 64, Hr = H / 32;
    std::vector<uint64_t> E(W + 2);
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + 11;
    for (uint32_t k = 0; k < W; ++k) { // splitmix64
        uint64_t x = (z += 0x9E3779B97F4A7C15ull);
        x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
        x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
        E[k] = x ^ (x >> 31);
    }
    E[W] = E[0];
    E[W + 1] = E[1 % W];
    std::vector<uint32_t> E32(2 * W);
    for (uint32_t k = 0; k < W; ++k) {
        E32[2 * k] = (uint32_t)E[k];
        E32[2 * k + 1] = (uint32_t)(E[k] >> 32);
    }
    int bad = 0;
    const uint32_t inv = half_inv(Hr);
    for (int c = 0; c < 2; ++c)
        for (uint32_t k = 0; k < W; ++k) {
            RowMasks rm = row_masks32(k, H, M, 0);
            if (c)
                rm.left_rows = ~rm.left_rows;
            const Neighbours a = neighbours_ext_rm(E.data(), H, M, k, rm);
            const Neighbours b = neighbours_half_aligned(E32.data(), W, Hr, inv, k, c);
            bad += (a.ce != b.ce) || (a.up != b.up) || (a.dn != b.dn) || (a.sd != b.sd);
        }
    return bad;
}

// The batch kernel's 32-bit general extraction against the 64-bit one, for
// every word of both colours of an L x L lattice (any even L <= 722).
int emu_ext32_neighbours_check(int64_t L, uint64_t seed)
{
    const uint32_t H = (uint32_t)(L / 2), M = (uint32_t)(L * L / 2), W = (M + 63) / 64;
    std::vector<uint64_t> E(W + 2);
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + 5;
    for (uint32_t k = 0; k < W + 2; ++k) { // splitmix64; the continuation is arbitrary here
        uint64_t x = (z += 0x9E3779B97F4A7C15ull);
        x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
        x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
        E[k] = x ^ (x >> 31);
    }
    std::vector<uint32_t> E32(2 * (W + 2));
    for (uint32_t k = 0; k < W + 2; ++k) {
        E32[2 * k] = (uint32_t)E[k];
        E32[2 * k + 1] = (uint32_t)(E[k] >> 32);
    }
    int bad = 0;
    for (int c = 0; c < 2; ++c)
        for (uint32_t k = 0; k < W; ++k) {
            RowMasks rm = row_masks32(k, H, M, 0);
            if (c)
                rm.left_rows = ~rm.left_rows;
            const Neighbours a = neighbours_ext_rm(E.data(), H, M, k, rm);
            const Neighbours b = neighbours_ext32(E32.data(), H, M, k, rm);
            bad += (a.ce != b.ce) || (a.up != b.up) || (a.dn != b.dn) || (a.sd != b.sd);
        }
    return bad;
}

// floor(h / Hr) by the half-aligned multiply, over its whole range.
int emu_half_row_check()
{
    int bad = 0;
    for (uint32_t Hr = 1; Hr <= 11; ++Hr)
        for (uint32_t h = 0; h < 8192; ++h)
            bad += half_row(h, half_inv(Hr)) != h / Hr;
    return bad;
}

// floor(k / Wr) by the batch kernel's multiply, over its whole range.
int emu_aligned_row_check()
{
    int bad = 0;
    for (uint32_t Wr = 1; Wr <= 5; ++Wr)
        for (uint32_t k = 0; k < 4096; ++k)
            bad += aligned_row(k, aligned_inv(Wr)) != k / Wr;
    return bad;
}

// Logical block of hardware block b of a grid of n blocks.
uint32_t emu_xcd_block(uint32_t b, uint32_t n) { return rows::xcd_block(b, n); }

// Philox block with the fused-XOR rounds, in each counter/key mode.
void emu_philox_fast(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                     int mode, uint32_t *out)
{
    const Block x = mode == 0   ? rows::philox_fast<rows::kCtrUniform>(c0, c1, c2, c3, k0, k1)
                    : mode == 1 ? rows::philox_fast<rows::kCtrLane>(c0, c1, c2, c3, k0, k1)
                                : rows::philox_fast<rows::kCtrKeyLane>(c0, c1, c2, c3, k0, k1);
    out[0] = x.x0;
    out[1] = x.x1;
    out[2] = x.x2;
    out[3] = x.x3;
}

void emu_init(uint64_t *words, int64_t L, uint64_t seed, uint32_t stream)
{
    const int64_t M = L * L / 2, W = (M + 63) / 64;
    for (int64_t idx = 0; idx < 2 * W; ++idx)
        words[idx] = init_word(idx % W, (uint32_t)(idx / W), M, stream, (uint32_t)seed,
                               (uint32_t)(seed >> 32));
}

// rows = 1: the row-aligned kernel's formulas (needs L % 128 == 0);
// rows = 2: the same with the queued kernel's compare sequence.
void emu_half_sweep(uint64_t *words, int64_t L, int c, const uint64_t *T, int anti, uint64_t t,
                    uint64_t seed, uint32_t stream, int rows)
{
    const int64_t H = L / 2, M = L * L / 2, W = (M + 63) / 64;
    uint64_t *tgt = words + c * W;
    const uint64_t *src = words + (1 - c) * W;
    const SweepArgs2 a{metro2_from_table(T, anti), (uint32_t)t, (uint32_t)(t >> 32), stream,
                       (uint32_t)seed, (uint32_t)(seed >> 32)};
    if (!rows) {
        for (int64_t k = 0; k < W; ++k)
            tgt[k] = update_word_general(tgt[k], src, H, M, W, k, c, a);
        return;
    }
    const int64_t Wr = L / 128;
    for (int64_t i = 0; i < L; ++i)
        for (int64_t w = 0; w < Wr; ++w) {
            const bool left = ((i + c) & 1) == 0;
            const int64_t adjw = left ? (w == 0 ? Wr - 1 : w - 1) : (w == Wr - 1 ? 0 : w + 1);
            const int64_t idx = i * Wr + w;
            if (rows == 2) {
                tgt[idx] = queued_word_any(tgt[idx], src[((i + L - 1) % L) * Wr + w],
                                           src[((i + 1) % L) * Wr + w], src[idx],
                                           src[i * Wr + adjw], left, (uint32_t)idx, a);
            } else {
                tgt[idx] = update_word_rows(tgt[idx], src[((i + L - 1) % L) * Wr + w],
                                            src[((i + 1) % L) * Wr + w], src[idx],
                                            src[i * Wr + adjw], left, (uint32_t)idx, a);
            }
        }
}

// The heat-bath kernels' word decision (decide_word5) under table T, with
// the general kernel's neighbour extraction (rows = 0) or the row kernel's
// (rows = 1, L % 128 == 0); rows = 2: the queued row kernel's sequence.
void emu_half_sweep5(uint64_t *words, int64_t L, int c, const uint64_t *T, uint64_t t,
                     uint64_t seed, uint32_t stream, int rows5)
{
    const int64_t H = L / 2, M = L * L / 2, W = (M + 63) / 64;
    uint64_t *tgt = words + c * W;
    const uint64_t *src = words + (1 - c) * W;
    rows::Table5 tab{};
    for (int a = 0; a < 5; ++a) {
        if (T[a] >= (1ull << 32))
            tab.always |= 1u << a;
        else if (T[a] > 0) {
            tab.random |= 1u << a;
            tab.thr[a] = (uint32_t)T[a];
        }
    }
    const rows::SweepArgs5 a{tab, (uint32_t)t, (uint32_t)(t >> 32), stream, (uint32_t)seed,
                             (uint32_t)(seed >> 32)};
    if (!rows5) {
        for (int64_t k = 0; k < W; ++k)
            tgt[k] = rows::decide_word5(tgt[k], neighbours_general(src, H, M, W, k, c),
                                        valid_mask(k, M), (uint32_t)k, a);
        return;
    }
    const int64_t Wr = L / 128;
    for (int64_t i = 0; i < L; ++i)
        for (int64_t w = 0; w < Wr; ++w) {
            const bool left = ((i + c) & 1) == 0;
            const int64_t adjw = left ? (w == 0 ? Wr - 1 : w - 1) : (w == Wr - 1 ? 0 : w + 1);
            const int64_t idx = i * Wr + w;
            const uint64_t up = src[((i + L - 1) % L) * Wr + w], dn = src[((i + 1) % L) * Wr + w];
            if (rows5 == 2) {
                tgt[idx] = queued_word5(tgt[idx], up, dn, src[idx], src[i * Wr + adjw], left,
                                        (uint32_t)idx, a);
                continue;
            }
            const Neighbours nb{up, dn, src[idx], side_vector(src[idx], src[i * Wr + adjw], left)};
            tgt[idx] = rows::decide_word5(tgt[idx], nb, ~0ull, (uint32_t)idx, a);
        }
}

// The persistent batch kernel's per-lattice sequence: extended colour arrays
// refreshed after every half-sweep, neighbours by funnel shifts.
void emu_batch_lattice(uint64_t *words, int64_t L, double beta, double J, uint64_t seed,
                       uint32_t stream, int64_t nsweeps, uint64_t ctr, const uint64_t *T)
{
    (void)beta;
    const uint32_t H = (uint32_t)L / 2, M = (uint32_t)(L * L / 2), W = (M + 63) / 64;
    std::vector<uint64_t> E0(W + 2), E1(W + 2);
    for (uint32_t k = 0; k < W; ++k) {
        E0[k] = words[k];
        E1[k] = words[W + k];
    }
    auto refresh = [&](std::vector<uint64_t> &E) {
        uint64_t tail[3];
        ext_tail(E.data(), M, W, tail);
        E[W - 1] = tail[0];
        E[W] = tail[1];
        E[W + 1] = tail[2];
    };
    refresh(E0);
    refresh(E1);
    const Metro2 m = metro2_from_table(T, J < 0);
    for (int64_t sw = 0; sw < nsweeps; ++sw)
        for (int c = 0; c < 2; ++c) {
            const uint64_t t = 2 * (ctr + (uint64_t)sw) + (uint64_t)c;
            std::vector<uint64_t> &tgt = c ? E1 : E0;
            const std::vector<uint64_t> &src = c ? E0 : E1;
            const SweepArgs2 a{m, (uint32_t)t, (uint32_t)(t >> 32), stream, (uint32_t)seed,
                               (uint32_t)(seed >> 32)};
            for (uint32_t k = 0; k < W; ++k) {
                const Neighbours nb = neighbours_ext(src.data(), H, M, k, c);
                tgt[k] ^= rows::decide_word_any(tgt[k], nb, valid_mask(k, M), k, a);
            }
            refresh(tgt);
        }
    for (uint32_t k = 0; k < W; ++k) {
        words[k] = E0[k] & valid_mask(k, M);
        words[W + k] = E1[k] & valid_mask(k, M);
    }
}

} // extern "C"
