// Host-side choice of the tile of every lattice size of a batch, for the
// makespan of one persistent launch rather than for each size on its own.
//
// Each size has a few tile options, each timed alone on the GPU and each
// splitting the size's lattices into some number of bundles (one workgroup
// each).  A size timed alone on an otherwise idle chip finishes fastest with
// the most bundles, but the whole batch has only as many resident workgroups
// as the compute units hold; bundles beyond that wait for a workgroup to free
// up and run a second round.  The estimate below schedules every bundle of a
// choice of options longest first on the resident workgroups (the order in
// which the persistent kernel takes them) and reports the makespan; the
// choice is improved one size at a time while the makespan falls, and among
// equal makespans while the sizes' bundle durations, longest first, fall
// (every size as fast as the workgroups left over allow).  Plain C++ with no
// HIP calls, so it is tested on the host.
#pragma once

#include <algorithm>
#include <cstdint>
#include <functional>
#include <queue>
#include <vector>

namespace ising {
namespace plan {

struct Option {
    uint32_t bundles; // workgroups the size needs with this tile
    double ms;        // the size alone, one launch, on `slots` workgroups
};

struct Estimate {
    double makespan = 0.0;        // longest workgroup
    double busy = 0.0;            // sum over bundles of their durations
    std::vector<double> per_size; // bundle duration of each size, longest first
};

// Duration of one bundle: the size alone ran ceil(bundles / slots) rounds.
inline double bundle_ms(const Option &o, uint32_t slots)
{
    const uint32_t s = std::max(1u, slots);
    const uint32_t rounds = std::max(1u, (o.bundles + s - 1) / s);
    return o.ms / (double)rounds;
}

// Longest-first list schedule of every bundle of the choice `pick` (one
// option index per size) on `slots` workgroups.
inline Estimate estimate(const std::vector<std::vector<Option>> &opts,
                         const std::vector<size_t> &pick, uint32_t slots)
{
    std::vector<double> d;
    Estimate e;
    for (size_t i = 0; i < opts.size(); ++i) {
        const Option &o = opts[i][pick[i]];
        const double bm = bundle_ms(o, slots);
        d.insert(d.end(), o.bundles, bm);
        e.busy += bm * (double)o.bundles;
        e.per_size.push_back(bm);
    }
    std::sort(e.per_size.begin(), e.per_size.end(), std::greater<double>());
    std::sort(d.begin(), d.end(), std::greater<double>());
    std::priority_queue<double, std::vector<double>, std::greater<double>> load;
    for (uint32_t s = 0; s < std::max(1u, slots); ++s)
        load.push(0.0);
    for (double x : d) {
        const double t = load.top() + x;
        load.pop();
        load.push(t);
        e.makespan = std::max(e.makespan, t);
    }
    return e;
}

// Strict order: shorter makespan, then shorter bundle durations (longest
// first, lexicographic), then less busy time.
inline bool better(const Estimate &a, const Estimate &b)
{
    if (a.makespan != b.makespan)
        return a.makespan < b.makespan;
    if (a.per_size != b.per_size)
        return a.per_size < b.per_size;
    return a.busy < b.busy;
}

// From `start`, change one size's option at a time while the estimate gets
// strictly better (the order is strict, so this ends).
inline std::vector<size_t> improve(const std::vector<std::vector<Option>> &opts,
                                   std::vector<size_t> start, uint32_t slots)
{
    std::vector<size_t> pick = std::move(start);
    Estimate best = estimate(opts, pick, slots);
    for (bool improved = true; improved;) {
        improved = false;
        for (size_t i = 0; i < opts.size(); ++i)
            for (size_t j = 0; j < opts[i].size(); ++j) {
                if (j == pick[i])
                    continue;
                std::vector<size_t> trial = pick;
                trial[i] = j;
                const Estimate e = estimate(opts, trial, slots);
                if (better(e, best)) {
                    pick = std::move(trial);
                    best = e;
                    improved = true;
                }
            }
    }
    return pick;
}

// The better of two local searches: one from the fastest option of each size
// alone (`fastest`), one from the option with the fewest bundles (the most
// lattices per workgroup, the highest throughput of a compute unit).
inline std::vector<size_t> choose(const std::vector<std::vector<Option>> &opts,
                                  const std::vector<size_t> &fastest, uint32_t slots)
{
    std::vector<size_t> fewest(opts.size(), 0);
    for (size_t i = 0; i < opts.size(); ++i)
        for (size_t j = 1; j < opts[i].size(); ++j) {
            const Option &a = opts[i][j], &c = opts[i][fewest[i]];
            if (a.bundles < c.bundles || (a.bundles == c.bundles && a.ms < c.ms))
                fewest[i] = j;
        }
    std::vector<size_t> p1 = improve(opts, fastest, slots);
    std::vector<size_t> p2 = improve(opts, fewest, slots);
    return better(estimate(opts, p2, slots), estimate(opts, p1, slots)) ? p2 : p1;
}

} // namespace plan
} // namespace ising
