// C entry points over the batch planner header for the host tests.
#include <cstdint>
#include <vector>

#include "../paper_1906_06297_amd/csrc/batch_plan.hpp"

using namespace ising::plan;

namespace {
std::vector<std::vector<Option>> unpack(int n, const int *counts, const uint32_t *bundles,
                                        const double *ms)
{
    std::vector<std::vector<Option>> opts(n);
    int k = 0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < counts[i]; ++j, ++k)
            opts[i].push_back(Option{bundles[k], ms[k]});
    return opts;
}
} // namespace

extern "C" {

// Makespan, busy time and sum of squared workgroup loads of the choice pick
// (one option index per size).
void plan_estimate(int n, const int *counts, const uint32_t *bundles, const double *ms,
                   const int *pick, uint32_t slots, double *makespan, double *busy, double *sumsq)
{
    const auto opts = unpack(n, counts, bundles, ms);
    const std::vector<size_t> p(pick, pick + n);
    const Estimate e = estimate(opts, p, slots);
    *makespan = e.makespan;
    *busy = e.busy;
    *sumsq = e.sumsq;
}

// The improved choice from start, written to pick.
void plan_choose(int n, const int *counts, const uint32_t *bundles, const double *ms,
                 const int *start, uint32_t slots, int *pick)
{
    const auto opts = unpack(n, counts, bundles, ms);
    const auto p = choose(opts, std::vector<size_t>(start, start + n), slots);
    for (int i = 0; i < n; ++i)
        pick[i] = (int)p[i];
}
}
