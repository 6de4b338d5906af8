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
// equal makespans (to the nanosecond) while the sum of the squared workgroup
// loads falls: less work in all and less of it stacked on few workgroups,
// which is what lets a later move shorten the makespan.  Plain C++ with no
// HIP calls, so it is tested on the host.
#pragma once

#include <algorithm>
#include <cmath>
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
    double sumsq = 0.0;           // sum over workgroups of their load squared
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
    for (; !load.empty(); load.pop())
        e.sumsq += load.top() * load.top();
    return e;
}

// Makespan to the nanosecond (times in ms), so that sums taken in another
// order compare equal.
inline long long makespan_ns(const Estimate &e) { return std::llround(e.makespan * 1e6); }

// Strict order: shorter makespan (to the nanosecond), then a smaller sum of
// squared loads, then shorter bundle durations (longest first,
// lexicographic), then less busy time.
inline bool better(const Estimate &a, const Estimate &b)
{
    const long long ma = makespan_ns(a), mb = makespan_ns(b);
    if (ma != mb)
        return ma < mb;
    if (a.sumsq != b.sumsq)
        return a.sumsq < b.sumsq;
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

// The best of several local searches: from the fastest option of each size
// alone (`fastest`), from the option with the fewest bundles (the most
// lattices per workgroup, the highest throughput of a compute unit), and from
// `restarts` random choices drawn from a fixed splitmix64 stream (one search
// takes milliseconds; single-size moves alone stop short of the best plans).
inline std::vector<size_t> choose(const std::vector<std::vector<Option>> &opts,
                                  const std::vector<size_t> &fastest, uint32_t slots,
                                  int restarts = 16)
{
    std::vector<size_t> fewest(opts.size(), 0);
    for (size_t i = 0; i < opts.size(); ++i)
        for (size_t j = 1; j < opts[i].size(); ++j) {
            const Option &a = opts[i][j], &c = opts[i][fewest[i]];
            if (a.bundles < c.bundles || (a.bundles == c.bundles && a.ms < c.ms))
                fewest[i] = j;
        }
    std::vector<size_t> best = improve(opts, fastest, slots);
    Estimate be = estimate(opts, best, slots);
    auto consider = [&](std::vector<size_t> start) {
        std::vector<size_t> p = improve(opts, std::move(start), slots);
        const Estimate e = estimate(opts, p, slots);
        if (better(e, be)) {
            best = std::move(p);
            be = e;
        }
    };
    consider(fewest);
    // each search costs sizes x options x bundles; batches of many sizes keep
    // to the two deterministic starts
    if (opts.size() > 32)
        restarts = 0;
    uint64_t z = 0x5EED5EED5EED5EEDull;
    auto next = [&z]() {
        uint64_t x = (z += 0x9E3779B97F4A7C15ull);
        x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
        x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
        return x ^ (x >> 31);
    };
    for (int r = 0; r < restarts; ++r) {
        std::vector<size_t> start(opts.size());
        for (size_t i = 0; i < opts.size(); ++i)
            start[i] = (size_t)(next() % opts[i].size());
        consider(std::move(start));
    }
    return best;
}

} // namespace plan
} // namespace ising
