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

// Line fit of one kind's bundle durations t at lattice counts n.
void plan_fit_kind(int npts, const uint32_t *n, const double *t, uint32_t threads, int model,
                   double a_default, double *a, double *b)
{
    std::vector<std::pair<uint32_t, double>> pts;
    for (int i = 0; i < npts; ++i)
        pts.emplace_back(n[i], t[i]);
    fit_kind(pts, threads, (Model)model, a_default, a, b);
}

// Mixed packing of items (kinds per item) on `slots` workgroups: the
// workgroup of each item (-1 if the packing failed) and the model makespan.
double plan_pack_mixed(int nkinds, const double *a, const double *b, const uint32_t *threads,
                       const uint32_t *lds, const int *exclusive, int nitems,
                       const uint32_t *item_kind, uint32_t slots, uint32_t max_threads,
                       uint32_t max_lds, int model, int *group_of)
{
    std::vector<Kind> kinds(nkinds);
    for (int k = 0; k < nkinds; ++k) {
        kinds[k].a = a[k];
        kinds[k].b = b[k];
        kinds[k].threads = threads[k];
        kinds[k].lds_words = lds[k];
        kinds[k].exclusive = exclusive[k] != 0;
    }
    const Packing p = pack_mixed(kinds, std::vector<uint32_t>(item_kind, item_kind + nitems),
                                 slots, max_threads, max_lds, (Model)model);
    for (int i = 0; i < nitems; ++i)
        group_of[i] = -1;
    if (!p.ok)
        return -1.0;
    for (size_t g = 0; g < p.groups.size(); ++g)
        for (uint32_t i : p.groups[g])
            group_of[i] = (int)g;
    return p.makespan;
}
}
