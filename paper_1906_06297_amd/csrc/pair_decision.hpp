// Per-block decisions for lanes that share one word's Philox blocks: the
// batch kernel's lane pairs compute alternate blocks and exchange what each
// decides.  Plain bit logic, compiled for the host in the tests too.
#pragma once

#include "ising_rows.hpp"

namespace ising {
namespace rows {

// What block q alone decides, whatever came before: per half, the spins
// whose compare ends within its two planes (d: the uniform's bit differs from
// the threshold's in one of them) and, of those, the ones whose uniform is
// the smaller at that first difference (f).  Applying the (d, f) of
// consecutive blocks in order to the pending spins gives the state that
// applying their planes one by one gives; a lane pair uses this to evaluate
// two blocks at once and exchange the results.
struct BlockDecision {
    uint32_t d[2], f[2];
};

__host__ __device__ __forceinline__ BlockDecision block_decision_lane(const State &s,
                                                                      const Block &x, uint32_t q,
                                                                      const Metro2 &m)
{
    const uint32_t b0 = 31 - 2 * q, b1 = 30 - 2 * q;
    const uint32_t mA0 = thr_mask(m.thrA, b0), mB0 = thr_mask(m.thrB, b0);
    const uint32_t mA1 = thr_mask(m.thrA, b1), mB1 = thr_mask(m.thrB, b1);
    BlockDecision r;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint32_t P0 = h ? x.x1 : x.x0, P1 = h ? x.x3 : x.x2;
        const uint32_t t0 = lop3<tt((kA & kB) | (~kA & kC))>(s.a[h], mA0, mB0);
        const uint32_t t1 = lop3<tt((kA & kB) | (~kA & kC))>(s.a[h], mA1, mB1);
        const uint32_t e0 = P0 ^ t0;
        const uint32_t g1 = lop3<tt((kA ^ kB) & kB)>(P1, t1, 0u); // ends in plane 1, below T
        r.d[h] = lop3<tt(kA | (kB ^ kC))>(e0, P1, t1);
        r.f[h] = lop3<tt((kA & kB) | (~kA & kC))>(e0, t0, g1);
    }
    return r;
}

__host__ __device__ __forceinline__ void apply_decision(State &s, const BlockDecision &r)
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        s.tf[h] = lop3<tt(kA ^ (kB & kC))>(s.tf[h], s.p[h], r.f[h]);
        s.p[h] = lop3<tt(kA & ~kB)>(s.p[h], r.d[h], 0u);
    }
}

} // namespace rows
} // namespace ising
