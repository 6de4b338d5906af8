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
#include <climits>
#include <cstdint>
#include <functional>
#include <queue>
#include <utility>
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

// ------------------------------------------------------ mixed-size bundles
// Lattices of different sizes may also share a workgroup.  Two models of a
// workgroup's duration, each fitted to the bundles of one kind (a size with
// its tile) timed alone, neither right everywhere:
//  - additive: a bundle of n lattices takes a + n b; a workgroup of several
//    kinds max a + sum b.  Close where lattices are small and the half-sweep
//    is the latency of one word's decision chain.
//  - rounds: a half-sweep is bound by vector-ALU issue on the busiest of the
//    compute unit's four SIMDs, which run the workgroup's wavefronts round
//    robin: a bundle filling W wavefronts takes a + b ceil(W / 4); several
//    kinds, threads back to back, max a + max b ceil(W / 4).  Close where
//    lattices fill wavefronts.
// The autotuner packs with both and times the results.
enum Model { kAdditive = 0, kRounds = 1 };

struct Kind {
    double a = 0.0, b = 0.0; // ms for the sweeps the model was timed on
    uint32_t threads = 0;    // threads a lattice takes in the workgroup layout
    uint32_t lds_words = 0;  // LDS words a lattice takes
    bool exclusive = false;  // shares a workgroup only with lattices of its own kind
};

// Wavefronts per SIMD of a workgroup with `threads` threads.
inline uint32_t simd_waves(uint32_t threads) { return ((threads + 63) / 64 + 3) / 4; }

// Model duration of a workgroup: its largest a, largest and summed b, threads.
inline double group_time(Model m, double a, double bmax, double bsum, uint32_t threads)
{
    return m == kRounds ? a + bmax * (double)simd_waves(threads) : a + bsum;
}

// (a, b) from bundle durations t of n lattices of `threads` threads each: the
// line through the points with the smallest and the largest x (x = n, or the
// SIMD rounds of n lattices), a >= 0, b > 0.  With one x, a defaults to
// a_default, at most 0.8 t.
inline void fit_kind(const std::vector<std::pair<uint32_t, double>> &pts, uint32_t threads,
                     Model m, double a_default, double *a, double *b)
{
    uint32_t x0 = UINT32_MAX, x1 = 0;
    double t0 = 0.0, t1 = 0.0;
    for (const auto &p : pts) {
        const uint32_t x = m == kRounds ? simd_waves(p.first * threads) : p.first;
        if (x < x0 || (x == x0 && p.second < t0)) {
            x0 = x;
            t0 = p.second;
        }
        if (x > x1 || (x == x1 && p.second < t1)) {
            x1 = x;
            t1 = p.second;
        }
    }
    if (x1 > x0) {
        *b = std::max((t1 - t0) / (double)(x1 - x0), 0.02 * t1 / (double)x1);
        *a = std::max(0.0, t0 - *b * (double)x0);
    } else {
        *a = std::min(a_default, 0.8 * t0);
        *b = (t0 - *a) / (double)std::max(1u, x0);
    }
}

struct Packing {
    std::vector<std::vector<uint32_t>> groups; // item indices per workgroup (none empty)
    std::vector<double> est;                   // model duration per workgroup
    double makespan = 0.0;
    bool ok = false;
};

// Places the items in `use` (kinds in item_kind) on at most `slots`
// workgroups of max_threads threads and max_lds LDS words: the largest
// (threads x b under kRounds, b otherwise) first, each on the workgroup whose
// model duration after adding it is smallest, among equals the fullest.  Not
// ok if some item fits nowhere.
inline Packing lpt_pack(const std::vector<Kind> &kinds, const std::vector<uint32_t> &item_kind,
                        const std::vector<uint32_t> &use, uint32_t slots, uint32_t max_threads,
                        uint32_t max_lds, Model model)
{
    std::vector<uint32_t> order = use;
    auto weight = [&](uint32_t i) {
        const Kind &k = kinds[item_kind[i]];
        return model == kRounds ? k.b * k.threads : k.b;
    };
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t x, uint32_t y) { return weight(x) > weight(y); });
    struct Load {
        double a = 0.0, bmax = 0.0, bsum = 0.0;
        uint32_t threads = 0, lds = 0;
    };
    Packing p;
    const uint32_t g = slots;
    std::vector<Load> load(g);
    std::vector<std::vector<uint32_t>> groups(g);
    for (uint32_t i : order) {
        const Kind &k = kinds[item_kind[i]];
        int best = -1;
        double best_t = 0.0;
        for (uint32_t w = 0; w < g; ++w) {
            const Load &l = load[w];
            if (l.threads + k.threads > max_threads || l.lds + k.lds_words > max_lds)
                continue;
            const double t = group_time(model, std::max(l.a, k.a), std::max(l.bmax, k.b),
                                        l.bsum + k.b, l.threads + k.threads);
            if (best < 0 || t < best_t - 1e-12 ||
                (t <= best_t + 1e-12 && l.threads > load[(size_t)best].threads)) {
                best = (int)w;
                best_t = t;
            }
        }
        if (best < 0)
            return p;
        Load &l = load[(size_t)best];
        l.a = std::max(l.a, k.a);
        l.bmax = std::max(l.bmax, k.b);
        l.bsum += k.b;
        l.threads += k.threads;
        l.lds += k.lds_words;
        groups[(size_t)best].push_back(i);
    }
    for (uint32_t w = 0; w < g; ++w)
        if (!groups[w].empty()) {
            p.groups.push_back(std::move(groups[w]));
            p.est.push_back(group_time(model, load[w].a, load[w].bmax, load[w].bsum,
                                       load[w].threads));
            p.makespan = std::max(p.makespan, p.est.back());
        }
    p.ok = true;
    return p;
}

// All items on at most `slots` workgroups.  Without exclusive kinds, one
// largest-first pass (lpt_pack).  With them, a makespan bound T is searched
// by bisection: each exclusive kind fills workgroups of its own with as many
// lattices as keep its model duration <= T (within threads and LDS), and the
// other items go largest first onto the workgroups left; T is feasible if
// those end by T.
inline Packing pack_mixed(const std::vector<Kind> &kinds, const std::vector<uint32_t> &item_kind,
                          uint32_t slots, uint32_t max_threads, uint32_t max_lds, Model model)
{
    slots = std::max(1u, slots);
    std::vector<uint32_t> mix;
    std::vector<std::vector<uint32_t>> excl(kinds.size());
    for (uint32_t i = 0; i < (uint32_t)item_kind.size(); ++i)
        (kinds[item_kind[i]].exclusive ? excl[item_kind[i]] : mix).push_back(i);
    bool any_excl = false;
    for (const auto &e : excl)
        any_excl = any_excl || !e.empty();
    if (!any_excl)
        return lpt_pack(kinds, item_kind, mix, slots, max_threads, max_lds, model);
    auto own_time = [&](const Kind &kd, uint32_t m) {
        return group_time(model, kd.a, kd.b, kd.b * (double)m, m * kd.threads);
    };
    // lattices per workgroup of exclusive kind k under bound T (0: none fits)
    auto per_wg = [&](size_t k, double T) -> uint32_t {
        const Kind &kd = kinds[k];
        uint32_t m = 0;
        while (m < excl[k].size() && (m + 1) * kd.threads <= max_threads &&
               (m + 1) * kd.lds_words <= max_lds && own_time(kd, m + 1) <= T)
            ++m;
        return m;
    };
    auto attempt = [&](double T, Packing *out) -> bool {
        uint32_t used = 0;
        for (size_t k = 0; k < kinds.size(); ++k)
            if (!excl[k].empty()) {
                const uint32_t m = per_wg(k, T);
                if (m == 0)
                    return false;
                used += (uint32_t)((excl[k].size() + m - 1) / m);
            }
        if (used > slots || (used == slots && !mix.empty()))
            return false;
        Packing p;
        if (!mix.empty()) {
            p = lpt_pack(kinds, item_kind, mix, slots - used, max_threads, max_lds, model);
            if (!p.ok || p.makespan > T)
                return false;
        }
        for (size_t k = 0; k < kinds.size(); ++k) {
            if (excl[k].empty())
                continue;
            const uint32_t m = per_wg(k, T);
            for (size_t s0 = 0; s0 < excl[k].size(); s0 += m) {
                const size_t cnt = std::min<size_t>(m, excl[k].size() - s0);
                p.groups.emplace_back(excl[k].begin() + (long)s0,
                                      excl[k].begin() + (long)(s0 + cnt));
                p.est.push_back(own_time(kinds[k], (uint32_t)cnt));
                p.makespan = std::max(p.makespan, p.est.back());
            }
        }
        p.ok = true;
        *out = std::move(p);
        return true;
    };
    double lo = 0.0, hi = 0.0;
    for (uint32_t i = 0; i < (uint32_t)item_kind.size(); ++i)
        hi += own_time(kinds[item_kind[i]], 1);
    Packing best;
    if (!attempt(hi, &best))
        return Packing{};
    for (int it = 0; it < 50; ++it) {
        const double mid = 0.5 * (lo + hi);
        Packing p;
        if (attempt(mid, &p)) {
            hi = mid;
            best = std::move(p);
        } else {
            lo = mid;
        }
    }
    return best;
}

} // namespace plan
} // namespace ising
