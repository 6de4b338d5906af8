// C ABI of batched lattices (include/ising.h): planning bundles for the
// persistent kernel, the captured HIP graph of one batch sweep, the
// autotuner of words per thread, and per-lattice observables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ising.h"
#include "batch.hpp"
#include "batch_plan.hpp"
#include "host_common.hpp"

using namespace ising;

extern "C" int64_t ising_batch_words(int32_t n, const int64_t *Ls);

namespace {
struct Tile {
    uint32_t wpt;     // words per lane group
    uint32_t lpw;     // lanes per word (1 or 2)
    uint32_t cap = 0; // most lattices per bundle, 0 = as many as the workgroup holds
};
} // namespace

struct ising_batch {
    int32_t n = 0;
    std::vector<int64_t> Ls;
    std::vector<BatchLattice> lats; // host copy
    uint64_t *words = nullptr;      // caller's buffer
    size_t bytes = 0;
    std::map<int64_t, Tile> tiles;   // per lattice size
    std::map<int64_t, double> est_ms; // tuned duration of one bundle per size, if known
    // mixed-size bundles (chosen by the autotuner): the duration model of
    // every size with its tile; otherwise bundles hold one size each
    bool mixed = false;
    plan::Model model = plan::kAdditive;
    std::map<int64_t, plan::Kind> kinds;
    // the mixed plan's workgroup loads as the autotuner left them (lattice
    // indices); empty: packed from `kinds`
    std::vector<std::vector<uint32_t>> groups;
    // the installed plan per size: most lattices in one workgroup, workgroups
    std::map<int64_t, std::pair<uint32_t, uint32_t>> plan_stats;
    // device state owned by the batch
    BatchLattice *d_lats = nullptr;
    BatchSlot *d_slots = nullptr;
    BatchBundle *d_bundles = nullptr;
    uint32_t *d_next = nullptr;
    uint64_t *d_counter = nullptr;
    int64_t *d_spin_off = nullptr; // offset of lattice q in an int8 spin array
    uint32_t nbundles = 0, grid = 0;
    size_t lds_bytes = 0;
    // captured sweep
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t exec_nsweeps = -1;
};

namespace {

constexpr size_t kMaxBundleLds = 64 * 1024; // LDS of one workgroup
constexpr uint32_t kMaxBatchL = 722;        // two extended colour arrays within 64 KiB of LDS

uint32_t words_of(int64_t L) { return (uint32_t)((L * L / 2 + 63) / 64); }

uint32_t threads_per_lattice(uint32_t W, Tile t) { return ((W + t.wpt - 1) / t.wpt) * t.lpw; }

// Lattices of W words per colour that one workgroup takes: limited by its
// threads, by 64 KiB of LDS and by the tile's cap.
uint32_t lattices_per_bundle(uint32_t W, Tile t)
{
    const uint32_t lds_per = (uint32_t)(kMaxBundleLds / ((size_t)batch_lds_words(W) * 8));
    uint32_t per = std::max(1u, std::min((uint32_t)kBatchThreads / threads_per_lattice(W, t),
                                         lds_per));
    return t.cap ? std::min(per, t.cap) : per;
}

bool tile_ok(uint32_t W, Tile t)
{
    return t.wpt >= 1 && t.wpt <= W && (t.lpw == 1 || t.lpw == 2) &&
           threads_per_lattice(W, t) <= (uint32_t)kBatchThreads;
}

// Without tuning: a lane pair per word when the lattice leaves room for it,
// and as few words per lane group as the workgroup allows.
Tile default_tile(uint32_t W)
{
    for (uint32_t lpw : {2u, 1u})
        for (uint32_t wpt = 1; wpt <= W; ++wpt)
            if (tile_ok(W, Tile{wpt, lpw}))
                return Tile{wpt, lpw};
    return Tile{W, 1};
}

struct Plan {
    std::vector<BatchSlot> slots;
    std::vector<BatchBundle> bundles;
    size_t lds_bytes = 0;
};

// Appends a bundle of lattices `ids` with their tiles, threads and LDS back
// to back.  `mixed`: lane-pair lattices first (so pairs start at even
// threads), then one-lane ones, each group largest first, so that a
// wavefront rarely serves lattices of different sizes.
void add_bundle(Plan &p, const ising_batch *b, std::vector<std::pair<uint32_t, Tile>> items,
                bool mixed)
{
    auto threads = [&](const std::pair<uint32_t, Tile> &it) {
        return threads_per_lattice(b->lats[it.first].W, it.second);
    };
    if (mixed)
        std::stable_sort(items.begin(), items.end(), [&](const auto &x, const auto &y) {
            if (x.second.lpw != y.second.lpw)
                return x.second.lpw > y.second.lpw;
            return b->lats[x.first].L > b->lats[y.first].L;
        });
    BatchBundle bd{(uint32_t)p.slots.size(), (uint32_t)items.size(), 0, 0};
    uint32_t thread = 0, lds = 0;
    for (const auto &it : items) {
        const BatchLattice &lt = b->lats[it.first];
        const uint32_t tpl = threads(it);
        p.slots.push_back(BatchSlot{it.first, thread, tpl, slot_tile(it.second.wpt, it.second.lpw),
                                    lds});
        thread += tpl;
        lds += batch_lds_words(lt.W);
        if (!((lt.M & 63) == 0 && lt.W >= 2))
            bd.refresh = 1;
    }
    p.bundles.push_back(bd);
    p.lds_bytes = std::max(p.lds_bytes, (size_t)lds * 8);
}

// Bundles of same-size lattices, largest work first.  `only_L` restricts the
// plan to one size (autotuning) with tile `only`, 0 = all sizes, own tiles.
Plan make_plan(const ising_batch *b, int64_t only_L, Tile only)
{
    std::map<int64_t, std::vector<uint32_t>> by_size;
    for (int32_t q = 0; q < b->n; ++q)
        if (!only_L || b->Ls[q] == only_L)
            by_size[b->Ls[q]].push_back((uint32_t)q);
    // bundles start longest first: by their tuned durations when every size
    // has one, else by spins
    bool have_est = !only_L;
    for (auto &kv : by_size)
        have_est = have_est && b->est_ms.count(kv.first);
    struct Item {
        double work;
        Tile tile;
        std::vector<uint32_t> ids;
    };
    std::vector<Item> items;
    for (auto &kv : by_size) {
        const int64_t L = kv.first;
        const uint32_t W = words_of(L);
        const Tile tile = only_L ? only : b->tiles.at(L);
        const uint32_t per = lattices_per_bundle(W, tile);
        for (size_t i = 0; i < kv.second.size(); i += per) {
            Item it;
            const uint32_t cnt = (uint32_t)std::min<size_t>(per, kv.second.size() - i);
            it.ids.assign(kv.second.begin() + i, kv.second.begin() + i + cnt);
            it.tile = tile;
            it.work = have_est ? b->est_ms.at(L) : (double)cnt * (double)(L * L);
            items.push_back(std::move(it));
        }
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const Item &a, const Item &c) { return a.work > c.work; });
    Plan p;
    for (auto &it : items) {
        std::vector<std::pair<uint32_t, Tile>> v;
        for (uint32_t q : it.ids)
            v.emplace_back(q, it.tile);
        add_bundle(p, b, std::move(v), false);
    }
    return p;
}

// What the persistent kernel relies on, checked on the host before a plan
// is launched: every lattice in at most one slot (`all`: in exactly one); in
// each bundle, slots in increasing, disjoint thread ranges within the
// workgroup, lane pairs at even threads, the slot's threads matching its
// tile, and its LDS range within the launch's LDS and apart from the others.
int check_plan(const BatchLattice *lats, int32_t n, const BatchSlot *slots, size_t nslots,
               const BatchBundle *bundles, size_t nbundles, size_t lds_bytes, bool all = true)
{
    std::vector<uint8_t> seen((size_t)n, 0);
    size_t used = 0;
    for (size_t bi = 0; bi < nbundles; ++bi) {
        const BatchBundle &bd = bundles[bi];
        if (bd.count == 0 || (size_t)bd.first + bd.count > nslots)
            return host::fail(ISING_E_HIP, "batch plan: bundle %zu has no slots in range", bi);
        uint32_t thread_end = 0, lds_end = 0;
        bool refresh = false;
        for (uint32_t i = 0; i < bd.count; ++i) {
            const BatchSlot &sl = slots[bd.first + i];
            const uint32_t wpt = sl.tile & 0xFFFFu, lpw = sl.tile >> 16;
            if (sl.lat >= (uint32_t)n || seen[sl.lat])
                return host::fail(ISING_E_HIP, "batch plan: lattice %u missing or repeated",
                                  sl.lat);
            seen[sl.lat] = 1;
            ++used;
            const BatchLattice &lt = lats[sl.lat];
            if (wpt < 1 || (lpw != 1 && lpw != 2) ||
                sl.tpl != threads_per_lattice(lt.W, Tile{wpt, lpw}) ||
                (lpw == 2 && (sl.thread0 & 1)) || sl.thread0 < thread_end ||
                sl.thread0 + sl.tpl > (uint32_t)kBatchThreads || sl.lds_off < lds_end ||
                ((size_t)sl.lds_off + batch_lds_words(lt.W)) * 8 > lds_bytes)
                return host::fail(ISING_E_HIP, "batch plan: slot %u of bundle %zu does not fit", i,
                                  bi);
            thread_end = sl.thread0 + sl.tpl;
            lds_end = sl.lds_off + batch_lds_words(lt.W);
            refresh = refresh || !((lt.M & 63) == 0 && lt.W >= 2);
        }
        if (refresh && !bd.refresh)
            return host::fail(ISING_E_HIP, "batch plan: bundle %zu needs the refresh barrier", bi);
    }
    if (all && used != (size_t)n)
        return host::fail(ISING_E_HIP, "batch plan: %zu of %d lattices placed", used, (int)n);
    return ISING_OK;
}

// Threads a lattice of W words takes in a mixed bundle.
uint32_t mixed_threads(uint32_t W, Tile t) { return threads_per_lattice(W, t); }

// Mixed-size bundles from the duration model of every size (b->kinds, with
// the tiles in b->tiles) on `slots` workgroups, longest estimate first.
// Workgroup loads that hold every lattice of b exactly once, each within a
// workgroup's threads and LDS (a cached plan is checked before use).
bool valid_groups(const ising_batch *b, const std::vector<std::vector<uint32_t>> &groups)
{
    std::vector<uint8_t> seen((size_t)b->n, 0);
    size_t used = 0;
    for (const auto &g : groups) {
        uint32_t threads = 0, lds = 0;
        for (uint32_t q : g) {
            if (q >= (uint32_t)b->n || seen[q])
                return false;
            seen[q] = 1;
            ++used;
            threads += threads_per_lattice(b->lats[q].W, b->tiles.at(b->Ls[q]));
            lds += batch_lds_words(b->lats[q].W);
        }
        if (g.empty() || threads > (uint32_t)kBatchThreads || (size_t)lds * 8 > kMaxBundleLds)
            return false;
    }
    return used == (size_t)b->n;
}

// A plan of mixed bundles from workgroup loads (lattice indices), in order.
Plan plan_from_groups(const ising_batch *b, const std::vector<std::vector<uint32_t>> &groups)
{
    Plan p;
    for (const auto &g : groups) {
        std::vector<std::pair<uint32_t, Tile>> v;
        for (uint32_t q : g)
            v.emplace_back(q, b->tiles.at(b->Ls[q]));
        add_bundle(p, b, std::move(v), true);
    }
    return p;
}

bool make_mixed_plan(const ising_batch *b, uint32_t slots, Plan *out, double *makespan,
                     std::vector<std::vector<uint32_t>> *groups_out = nullptr)
{
    std::vector<plan::Kind> kinds;
    std::map<int64_t, uint32_t> kind_of;
    for (auto &kv : b->tiles) {
        auto it = b->kinds.find(kv.first);
        if (it == b->kinds.end())
            return false;
        plan::Kind k = it->second;
        const uint32_t W = words_of(kv.first);
        k.threads = mixed_threads(W, kv.second);
        k.lds_words = batch_lds_words(W);
        kind_of[kv.first] = (uint32_t)kinds.size();
        kinds.push_back(k);
    }
    std::vector<uint32_t> item_kind((size_t)b->n);
    for (int32_t q = 0; q < b->n; ++q)
        item_kind[(size_t)q] = kind_of.at(b->Ls[(size_t)q]);
    const plan::Packing pk = plan::pack_mixed(kinds, item_kind, slots, (uint32_t)kBatchThreads,
                                              (uint32_t)(kMaxBundleLds / 8), b->model);
    if (!pk.ok)
        return false;
    std::vector<size_t> order(pk.groups.size());
    for (size_t i = 0; i < order.size(); ++i)
        order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return pk.est[x] > pk.est[y]; });
    std::vector<std::vector<uint32_t>> groups;
    for (size_t gi : order)
        groups.push_back(pk.groups[gi]);
    *out = plan_from_groups(b, groups);
    if (makespan)
        *makespan = pk.makespan;
    if (groups_out)
        *groups_out = std::move(groups);
    return true;
}

void free_plan_buffers(ising_batch *b)
{
    if (b->d_slots)
        (void)hipFree(b->d_slots);
    if (b->d_bundles)
        (void)hipFree(b->d_bundles);
    b->d_slots = nullptr;
    b->d_bundles = nullptr;
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->exec_nsweeps = -1;
}

// Workgroups of the persistent kernel the chip holds at once: compute units
// times what one holds with lds_bytes of LDS each.
int resident_slots(size_t lds_bytes, uint32_t *slots)
{
    int dev = 0, cus = 0, occ = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || cus <= 0)
        return host::fail(ISING_E_HIP, "cannot query the number of compute units");
    e = batch_sweep_blocks_per_cu(lds_bytes, &occ);
    if (e != hipSuccess || occ <= 0)
        return host::fail(ISING_E_HIP, "the batch kernel does not fit a compute unit with %zu B "
                          "of LDS", lds_bytes);
    *slots = (uint32_t)cus * (uint32_t)occ;
    return ISING_OK;
}

// Workgroups of the persistent kernel: all resident at once, never more than
// bundles; further bundles go to whichever workgroup finishes first.
int persistent_grid(size_t lds_bytes, uint32_t nbundles, uint32_t *grid)
{
    uint32_t slots = 0;
    if (int rc = resident_slots(lds_bytes, &slots))
        return rc;
    *grid = std::max(1u, std::min(nbundles, slots));
    return ISING_OK;
}

int install_plan(ising_batch *b, const Plan &p)
{
    if (int rc = check_plan(b->lats.data(), b->n, p.slots.data(), p.slots.size(),
                            p.bundles.data(), p.bundles.size(), p.lds_bytes))
        return rc;
    free_plan_buffers(b);
    hipError_t e = hipMalloc(&b->d_slots, std::max<size_t>(1, p.slots.size()) * sizeof(BatchSlot));
    if (e == hipSuccess)
        e = hipMalloc(&b->d_bundles, std::max<size_t>(1, p.bundles.size()) * sizeof(BatchBundle));
    if (e == hipSuccess && !p.slots.empty())
        e = hipMemcpy(b->d_slots, p.slots.data(), p.slots.size() * sizeof(BatchSlot),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !p.bundles.empty())
        e = hipMemcpy(b->d_bundles, p.bundles.data(), p.bundles.size() * sizeof(BatchBundle),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return host::hip_fail(e, "batch plan upload");
    b->nbundles = (uint32_t)p.bundles.size();
    b->lds_bytes = p.lds_bytes;
    b->plan_stats.clear();
    for (const BatchBundle &bd : p.bundles) {
        std::map<int64_t, uint32_t> here;
        for (uint32_t i = 0; i < bd.count; ++i)
            ++here[b->Ls[p.slots[bd.first + i].lat]];
        for (auto &kv : here) {
            auto &st = b->plan_stats[kv.first];
            st.first = std::max(st.first, kv.second);
            ++st.second;
        }
    }
    return persistent_grid(p.lds_bytes, b->nbundles, &b->grid);
}

// The plan the batch's settings call for: mixed-size bundles when the
// autotuner chose them, else one size per bundle.
int install_current_plan(ising_batch *b)
{
    if (b->mixed && !b->groups.empty())
        return install_plan(b, plan_from_groups(b, b->groups));
    if (b->mixed) {
        uint32_t slots = 0;
        if (int rc = resident_slots(kMaxBundleLds, &slots))
            return rc;
        Plan p;
        if (make_mixed_plan(b, slots, &p, nullptr))
            return install_plan(b, p);
        b->mixed = false;
    }
    return install_plan(b, make_plan(b, 0, Tile{1, 1}));
}

int check_batch(const ising_batch *b)
{
    if (!b)
        return host::fail(ISING_E_BADARG, "null batch");
    return ISING_OK;
}

// Descriptors of the n lattices (offsets back to back, colour 0 then 1), with
// default tiles per size; the batch's device state is not touched.
int fill_lattices(ising_batch *b, int32_t n, const int64_t *Ls, const double *betas, double J,
                  const uint64_t *seeds, const uint32_t *stream_ids)
{
    b->n = n;
    uint64_t off = 0;
    for (int32_t q = 0; q < n; ++q) {
        if (!std::isfinite(betas[q]) || betas[q] < 0.0 || stream_ids[q] >= (1u << 24))
            return host::fail(ISING_E_BADARG, "lattice %d: beta must be finite and >= 0, "
                              "stream id < 2^24", (int)q);
        BatchLattice lt{};
        lt.word_off = off;
        lt.L = (uint32_t)Ls[q];
        lt.H = lt.L / 2;
        lt.M = lt.L * lt.L / 2;
        lt.W = words_of(Ls[q]);
        lt.m = host::metro2_params(betas[q], J);
        lt.key0 = (uint32_t)seeds[q];
        lt.key1 = (uint32_t)(seeds[q] >> 32);
        lt.stream_id = stream_ids[q];
        b->lats.push_back(lt);
        b->Ls.push_back(Ls[q]);
        if (!b->tiles.count(Ls[q]))
            b->tiles[Ls[q]] = default_tile(lt.W);
        off += 2 * (uint64_t)lt.W;
    }
    return ISING_OK;
}

// Arguments shared by ising_batch_create and ising_batch_sweep_noalloc.
int check_batch_args(int32_t n, const int64_t *Ls, const double *betas, double J,
                     const uint64_t *seeds, const uint32_t *stream_ids, const uint64_t *d_words,
                     size_t bytes)
{
    if (n <= 0 || !Ls || !betas || !seeds || !stream_ids || !d_words)
        return host::fail(ISING_E_BADARG, "empty batch or null pointer");
    if (!std::isfinite(J))
        return host::fail(ISING_E_BADARG, "J must be finite");
    const int64_t need = ising_batch_words(n, Ls);
    if (need < 0)
        return host::fail(ISING_E_SIZE, "every L must be even, >= 4 and <= %u", kMaxBatchL);
    if (bytes < (size_t)need * 8)
        return host::fail(ISING_E_SIZE, "buffer of %zu bytes is smaller than the %lld needed",
                          bytes, (long long)(need * 8));
    return ISING_OK;
}

// ---------------------------------------------------- sweeps without allocation
// ising_batch_sweep_noalloc keeps the persistent kernel's descriptors, bundle
// list, work-queue counter and sweep counter in this fixed device array
// instead of memory it allocates.  Each device holds its own copy at its own
// address, taken once per device with hipGetSymbolAddress; host code uses
// that address, never the array's name.
constexpr int32_t kNoAllocMaxLattices = 4096;
constexpr size_t kNoAllocScratchBytes = 512 * 1024;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
unsigned char *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

int scratch_of_current_device(unsigned char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return host::hip_fail(e, "current device");
    if (dev < 0 || dev >= kMaxDevices)
        return host::fail(ISING_E_HIP, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return host::hip_fail(e, "address of the batch scratch array");
        g_scratch[dev] = (unsigned char *)ptr;
    }
    *out = g_scratch[dev];
    return ISING_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// The plan of ising_batch_sweep_noalloc, built in fixed arrays (no heap):
// lattices grouped by size, default tiles, bundles of as many lattices as a
// workgroup takes, largest work (lattices x L^2) first, ties in creation
// order -- the untuned plan of a batch handle.
struct NoAllocPlan {
    BatchLattice lats[kNoAllocMaxLattices];
    uint32_t order[kNoAllocMaxLattices];
    BatchSlot slots[kNoAllocMaxLattices];
    BatchBundle bundles[kNoAllocMaxLattices];
    Tile tile_of[kNoAllocMaxLattices]; // tile of each bundle
    double work[kNoAllocMaxLattices];
    uint32_t border[kNoAllocMaxLattices];
    uint32_t nbundles = 0;
    size_t lds_bytes = 0;
    unsigned char stage[kNoAllocScratchBytes]; // host image of the scratch array

    int build(int32_t n, const int64_t *Ls, const double *betas, double J, const uint64_t *seeds,
              const uint32_t *stream_ids)
    {
        uint64_t off = 0;
        for (int32_t q = 0; q < n; ++q) {
            if (!std::isfinite(betas[q]) || betas[q] < 0.0 || stream_ids[q] >= (1u << 24))
                return host::fail(ISING_E_BADARG, "lattice %d: beta must be finite and >= 0, "
                                  "stream id < 2^24", (int)q);
            BatchLattice &lt = lats[q];
            lt = BatchLattice{};
            lt.word_off = off;
            lt.L = (uint32_t)Ls[q];
            lt.H = lt.L / 2;
            lt.M = lt.L * lt.L / 2;
            lt.W = words_of(Ls[q]);
            lt.m = host::metro2_params(betas[q], J);
            lt.key0 = (uint32_t)seeds[q];
            lt.key1 = (uint32_t)(seeds[q] >> 32);
            lt.stream_id = stream_ids[q];
            off += 2 * (uint64_t)lt.W;
            order[q] = (uint32_t)q;
        }
        std::sort(order, order + n, [this](uint32_t a, uint32_t b) {
            return lats[a].L != lats[b].L ? lats[a].L < lats[b].L : a < b;
        });
        // bundles, members still in `order`
        nbundles = 0;
        lds_bytes = 0;
        for (int32_t g0 = 0; g0 < n;) {
            const uint32_t L = lats[order[g0]].L, W = lats[order[g0]].W;
            int32_t g1 = g0;
            while (g1 < n && lats[order[g1]].L == L)
                ++g1;
            const Tile tile = default_tile(W);
            const uint32_t per = lattices_per_bundle(W, tile);
            const uint32_t refresh = ((lats[order[g0]].M & 63) == 0 && W >= 2) ? 0u : 1u;
            for (int32_t k = g0; k < g1; k += (int32_t)per) {
                const uint32_t cnt = (uint32_t)std::min<int32_t>((int32_t)per, g1 - k);
                bundles[nbundles] = BatchBundle{(uint32_t)k, cnt, refresh, 0};
                tile_of[nbundles] = Tile{tile.wpt, tile.lpw};
                work[nbundles] = (double)cnt * (double)L * (double)L;
                border[nbundles] = nbundles;
                lds_bytes = std::max(lds_bytes, (size_t)cnt * batch_lds_words(W) * 8);
                ++nbundles;
            }
            g0 = g1;
        }
        std::sort(border, border + nbundles, [this](uint32_t a, uint32_t b) {
            return work[a] != work[b] ? work[a] > work[b] : a < b;
        });
        // bundles in that order, each with its lattices' slots contiguous
        // (threads and LDS back to back, as a batch handle's one-size bundles)
        uint32_t m = 0;
        BatchBundle *sorted = (BatchBundle *)stage; // reuse the stage as room to permute
        for (uint32_t k = 0; k < nbundles; ++k) {
            BatchBundle bd = bundles[border[k]];
            const Tile t = tile_of[border[k]];
            for (uint32_t c = 0; c < bd.count; ++c) {
                const uint32_t q = order[bd.first + c];
                const uint32_t tpl = threads_per_lattice(lats[q].W, t);
                slots[m + c] = BatchSlot{q, c * tpl, tpl, slot_tile(t.wpt, t.lpw),
                                         c * batch_lds_words(lats[q].W)};
            }
            bd.first = m;
            m += bd.count;
            sorted[k] = bd;
        }
        std::memcpy(bundles, sorted, (size_t)nbundles * sizeof(BatchBundle));
        return ISING_OK;
    }
};

NoAllocPlan g_noalloc_plan; // static storage; callers take g_noalloc_mu
std::mutex g_noalloc_mu;


// ---------------------------------------------------------------- cache file
std::string cache_key() { return "gfx950/batch-sweep-v11"; }

// Tiles per size ([wpt, lpw, cap, a, b, exclusive]: a and b the duration
// model of the size with that tile, for mixed-size bundles, and whether its
// lattices keep workgroups of their own), whether bundles mix sizes and
// under which duration model they were packed.
struct CacheEntry {
    Tile tile{1, 1};
    plan::Kind kind;
};

// The batch a cached workgroup plan belongs to: its lattice count and an
// FNV-1a hash of the sizes in order (the plan lists lattice indices).
std::string batch_fingerprint(const ising_batch *b)
{
    uint64_t h = 0xcbf29ce484222325ull;
    for (int64_t L : b->Ls)
        for (int k = 0; k < 8; ++k) {
            h ^= (uint64_t)(L >> (8 * k)) & 0xFF;
            h *= 0x100000001b3ull;
        }
    char buf[48];
    std::snprintf(buf, sizeof buf, "%d:%016llx", (int)b->n, (unsigned long long)h);
    return buf;
}

bool read_cache(const char *path, std::map<int64_t, CacheEntry> &out, bool *mixed,
                plan::Model *model, const ising_batch *b,
                std::vector<std::vector<uint32_t>> *groups)
{
    std::ifstream f(path);
    if (!f)
        return false;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    const std::string tag = "\"key\": \"" + cache_key() + "\"";
    if (s.find(tag) == std::string::npos)
        return false;
    *mixed = s.find("\"mixed\": 1") != std::string::npos;
    *model = s.find("\"model\": 1") != std::string::npos ? plan::kRounds : plan::kAdditive;
    size_t pos = s.find("\"tiles\"");
    if (pos == std::string::npos)
        return false;
    pos = s.find('{', pos);
    const size_t end = s.find('}', pos);
    if (pos == std::string::npos || end == std::string::npos)
        return false;
    std::string body = s.substr(pos + 1, end - pos - 1);
    for (char &ch : body)
        if (ch == '"' || ch == ',' || ch == ':' || ch == '[' || ch == ']')
            ch = ' ';
    std::istringstream in(body);
    long long L;
    unsigned w, l, c;
    double a, bb;
    unsigned excl;
    while (in >> L >> w >> l >> c >> a >> bb >> excl) {
        CacheEntry e;
        e.tile = Tile{w, l, c};
        e.kind.a = a;
        e.kind.b = bb;
        e.kind.exclusive = excl != 0;
        out[(int64_t)L] = e;
    }
    // the workgroup plan, if it was tuned for this very batch
    groups->clear();
    const std::string fp = "\"groups_for\": \"" + batch_fingerprint(b) + "\"";
    size_t g = s.find("\"groups\": [");
    if (s.find(fp) != std::string::npos && g != std::string::npos) {
        int depth = 0;
        std::vector<uint32_t> cur;
        for (size_t i = s.find('[', g); i < s.size(); ++i) {
            const char ch = s[i];
            if (ch == '[') {
                ++depth;
                cur.clear();
            } else if (ch == ']') {
                if (depth == 2)
                    groups->push_back(cur);
                if (--depth == 0)
                    break;
            } else if (ch >= '0' && ch <= '9') {
                uint32_t v = 0;
                while (i < s.size() && s[i] >= '0' && s[i] <= '9')
                    v = v * 10 + (uint32_t)(s[i++] - '0');
                --i;
                cur.push_back(v);
            }
        }
        if (depth != 0)
            groups->clear();
    }
    return true;
}

bool write_cache(const char *path, const ising_batch *b)
{
    std::ofstream f(path);
    if (!f)
        return false;
    f.precision(17);
    f << "{\"key\": \"" << cache_key() << "\", \"mixed\": " << (b->mixed ? 1 : 0)
      << ", \"model\": " << (int)b->model << ", \"tiles\": {";
    bool first = true;
    for (auto &kv : b->tiles) {
        auto k = b->kinds.find(kv.first);
        const bool have = k != b->kinds.end();
        f << (first ? "" : ", ") << "\"" << kv.first << "\": [" << kv.second.wpt << ", "
          << kv.second.lpw << ", " << kv.second.cap << ", " << (have ? k->second.a : 0.0)
          << ", " << (have ? k->second.b : 0.0) << ", " << (have && k->second.exclusive ? 1 : 0)
          << "]";
        first = false;
    }
    f << "}";
    if (b->mixed && !b->groups.empty()) {
        f << ", \"groups_for\": \"" << batch_fingerprint(b) << "\", \"groups\": [";
        for (size_t g = 0; g < b->groups.size(); ++g) {
            f << (g ? ", [" : "[");
            for (size_t i = 0; i < b->groups[g].size(); ++i)
                f << (i ? ", " : "") << b->groups[g][i];
            f << "]";
        }
        f << "]";
    }
    f << "}\n";
    return (bool)f;
}

// ------------------------------------------------------------------ tuner
// The autotuner's state: a scratch copy of the lattices and counter (tuning
// never changes the batch), the reference result every timed plan must
// reproduce bit for bit, and the timings of every size alone.
class Tuner {
  public:
    Tuner(ising_batch *b, int64_t sweeps, hipStream_t s)
        : b_(b), sweeps_(sweeps), s_(s), log_(std::getenv("ISING_AUTOTUNE_LOG") != nullptr)
    {
    }
    ~Tuner()
    {
        for (void *p : {(void *)slot_buf_, (void *)bundles_, (void *)clk_, (void *)scratch_,
                        (void *)ctr_, (void *)next_})
            if (p)
                (void)hipFree(p);
        if (e0_)
            (void)hipEventDestroy(e0_);
        if (e1_)
            (void)hipEventDestroy(e1_);
    }

    int start()
    {
        nbytes_ = (size_t)ising_batch_words(b_->n, b_->Ls.data()) * 8;
        hipError_t e = hipMalloc(&scratch_, nbytes_);
        if (e == hipSuccess)
            e = hipMalloc(&ctr_, 8);
        if (e == hipSuccess)
            e = hipMalloc(&next_, 4);
        if (e == hipSuccess)
            e = hipEventCreate(&e0_);
        if (e == hipSuccess)
            e = hipEventCreate(&e1_);
        return e == hipSuccess ? ISING_OK : host::hip_fail(e, "autotune");
    }

    // Runs plan p for the tuning sweeps on the scratch copy, from the batch's
    // lattices and counter 0 every time; best of two launches in *best, the
    // lattices in out and (per_bundle) each bundle's duration in the second
    // launch, in ms.  `all`: the plan must hold every lattice.
    int time_plan(const Plan &p, float *best, std::vector<uint64_t> &out,
                  std::vector<double> *per_bundle = nullptr, bool all = true)
    {
        uint32_t grid = 0;
        if (int rc = check_plan(b_->lats.data(), b_->n, p.slots.data(), p.slots.size(),
                                p.bundles.data(), p.bundles.size(), p.lds_bytes, all))
            return rc;
        if (int rc = persistent_grid(p.lds_bytes, (uint32_t)p.bundles.size(), &grid))
            return rc;
        for (void *q : {(void *)slot_buf_, (void *)bundles_})
            if (q)
                (void)hipFree(q);
        slot_buf_ = nullptr;
        bundles_ = nullptr;
        hipError_t e = hipMalloc(&slot_buf_, p.slots.size() * sizeof(BatchSlot));
        if (e == hipSuccess)
            e = hipMalloc(&bundles_, p.bundles.size() * sizeof(BatchBundle));
        if (e == hipSuccess)
            e = hipMemcpy(slot_buf_, p.slots.data(), p.slots.size() * sizeof(BatchSlot),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(bundles_, p.bundles.data(), p.bundles.size() * sizeof(BatchBundle),
                          hipMemcpyHostToDevice);
        if (per_bundle && e == hipSuccess && clk_n_ < 2 * p.bundles.size()) {
            if (clk_)
                (void)hipFree(clk_);
            clk_ = nullptr;
            clk_n_ = 2 * p.bundles.size();
            e = hipMalloc(&clk_, clk_n_ * sizeof(uint64_t));
        }
        if (per_bundle && e == hipSuccess && wall_khz_ <= 0.0) {
            int dev = 0, khz = 0;
            e = hipGetDevice(&dev);
            if (e == hipSuccess)
                e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
            wall_khz_ = khz > 0 ? (double)khz : 1.0e5;
        }
        *best = 1e30f;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
            const uint64_t zero = 0;
            float ms = 0.f;
            e = hipMemcpyAsync(scratch_, b_->words, nbytes_, hipMemcpyDeviceToDevice, s_);
            if (e == hipSuccess)
                e = hipMemcpyAsync(ctr_, &zero, 8, hipMemcpyHostToDevice, s_);
            if (e == hipSuccess)
                e = hipEventRecord(e0_, s_);
            if (e == hipSuccess)
                e = launch_batch_sweep(b_->d_lats, slot_buf_, bundles_, (uint32_t)p.bundles.size(),
                                       grid, p.lds_bytes, next_, scratch_, ctr_, sweeps_, s_,
                                       (per_bundle && rep == 1) ? clk_ : nullptr);
            if (e == hipSuccess)
                e = hipEventRecord(e1_, s_);
            if (e == hipSuccess)
                e = hipEventSynchronize(e1_);
            if (e == hipSuccess)
                e = hipEventElapsedTime(&ms, e0_, e1_);
            *best = std::min(*best, ms);
        }
        if (e == hipSuccess) {
            out.resize(nbytes_ / 8);
            e = hipMemcpy(out.data(), scratch_, nbytes_, hipMemcpyDeviceToHost);
        }
        if (per_bundle && e == hipSuccess) {
            std::vector<uint64_t> t(2 * p.bundles.size());
            e = hipMemcpy(t.data(), clk_, t.size() * sizeof(uint64_t), hipMemcpyDeviceToHost);
            per_bundle->assign(p.bundles.size(), 0.0);
            for (size_t i = 0; i < p.bundles.size() && e == hipSuccess; ++i)
                (*per_bundle)[i] = (double)(t[2 * i + 1] - t[2 * i]) / wall_khz_;
        }
        return e == hipSuccess ? ISING_OK : host::hip_fail(e, "autotune");
    }

    // Every tile candidate of each size -- each also with a half and a
    // quarter of the lattices per bundle -- timed with that size alone; all
    // must reproduce the same lattices.
    int time_sizes()
    {
        for (auto &kv : b_->tiles) {
            const int64_t L = kv.first;
            const uint32_t W = words_of(L);
            std::vector<Tile> cands;
            for (uint32_t lpw : {1u, 2u})
                for (uint32_t w : {1u, 2u, 3u, 4u, 6u, 8u, 12u, 16u}) {
                    const Tile t{w, lpw};
                    if (!tile_ok(W, t))
                        continue;
                    bool dup = false;
                    for (const Tile &c : cands)
                        dup = dup || (c.lpw == lpw && threads_per_lattice(W, c) ==
                                                          threads_per_lattice(W, t));
                    if (!dup)
                        cands.push_back(t);
                }
            // half-empty workgroups run their lattices' sweeps sooner, on
            // compute units the batch leaves idle
            const size_t nbase = cands.size();
            for (size_t i = 0; i < nbase; ++i) {
                const uint32_t full = make_plan(b_, L, cands[i]).bundles.front().count;
                for (uint32_t cap : {full / 2, full / 4})
                    if (cap >= 1 && cap < full)
                        cands.push_back(Tile{cands[i].wpt, cands[i].lpw, cap});
            }
            std::vector<plan::Option> o;
            std::vector<Tile> ot;
            std::vector<uint32_t> op;
            size_t fi = 0;
            std::vector<uint64_t> ref, out;
            for (const Tile &w : cands) {
                const Plan p = make_plan(b_, L, w);
                uint32_t held = 0;
                if (int rc = resident_slots(p.lds_bytes, &held))
                    return rc;
                slots_ = slots_ ? std::min(slots_, held) : held;
                float ms = 0.f;
                if (int rc = time_plan(p, &ms, o.empty() ? ref : out, nullptr, false))
                    return rc;
                if (!o.empty() && out != ref)
                    return host::fail(ISING_E_HIP, "autotune: tile (%u, %u, %u) of L=%lld changed "
                                      "the lattice", w.wpt, w.lpw, w.cap, (long long)L);
                o.push_back(plan::Option{(uint32_t)p.bundles.size(), (double)ms});
                ot.push_back(w);
                op.push_back(p.bundles.front().count);
                if (o.back().ms < o[fi].ms)
                    fi = o.size() - 1;
            }
            sizes_.push_back(L);
            opts_.push_back(std::move(o));
            opt_tiles_.push_back(std::move(ot));
            opt_per_.push_back(std::move(op));
            fastest_.push_back(fi);
        }
        return ISING_OK;
    }

    // One size per bundle: the jointly estimated best tiles, kept only if the
    // whole batch, timed both ways, runs faster with them than with the
    // fastest tile of every size alone.
    int choose_one_size()
    {
        pick_ = plan::choose(opts_, fastest_, slots_);
        apply(fastest_);
        if (int rc = time_plan(make_plan(b_, 0, Tile{1, 1}), &ms_best_, ref_))
            return rc;
        if (pick_ != fastest_) {
            float ms_pick = 0.f;
            apply(pick_);
            if (int rc = time_plan(make_plan(b_, 0, Tile{1, 1}), &ms_pick, out_))
                return rc;
            if (out_ != ref_)
                return host::fail(ISING_E_HIP, "autotune: the joint tiles changed the lattices");
            if (ms_fast_wins(ms_pick))
                pick_ = fastest_;
            else
                ms_best_ = ms_pick;
        }
        apply(pick_);
        return ISING_OK;
    }

    // Mixed-size bundles.  For each duration model, (a, b) per size and tile
    // from the single-size timings; tiles per size by one of two rules -- the
    // cheapest per lattice among the tiles whose single lattice fits the
    // one-size plan's makespan, or the one-size plan's own tiles -- each with
    // every size mixing, or with the sizes whose colour rows are not whole
    // 32-bit halves (general neighbour extraction, long per-word chains) in
    // workgroups of their own.  Each packing is timed on the whole batch; the
    // fastest is refined by measurement and replaces the one-size plan if
    // faster.
    int choose_mixed()
    {
        if (sizes_.empty())
            return ISING_OK;
        const double hom_est = plan::estimate(opts_, pick_, slots_).makespan;
        if (log_)
            std::fprintf(stderr, "[autotune] one-size plan: estimated %.4f ms, timed %.4f ms, "
                         "%u workgroups\n", hom_est, (double)ms_best_, slots_);
        const std::map<int64_t, Tile> hom_tiles = b_->tiles;
        float ms_keep = 0.f;
        Choice keep;
        for (plan::Model model : {plan::kAdditive, plan::kRounds}) {
            Fits f = fit_models(model);
            for (int rule = 0; rule < 4; ++rule) {
                Choice c = tiles_by_rule(f, model, rule, hom_tiles, hom_est);
                b_->tiles = c.tiles;
                b_->kinds = c.kinds;
                b_->model = model;
                Plan p;
                double est = 0.0;
                const bool packed = make_mixed_plan(b_, slots_, &p, &est, &c.groups);
                if (log_)
                    log_choice(c, model, rule, packed, est);
                if (!packed)
                    continue;
                float ms = 0.f;
                if (int rc = time_plan(p, &ms, out_))
                    return rc;
                if (log_)
                    std::fprintf(stderr, "[autotune]   timed %.4f ms\n", (double)ms);
                if (out_ != ref_)
                    return host::fail(ISING_E_HIP, "autotune: mixed-size bundles changed the "
                                      "lattices");
                if (ms < ms_best_ && (keep.tiles.empty() || ms < ms_keep)) {
                    ms_keep = ms;
                    keep = std::move(c);
                    keep.model = model;
                }
            }
        }
        if (keep.tiles.empty()) {
            b_->tiles = hom_tiles;
            b_->kinds.clear();
            b_->model = plan::kAdditive;
            b_->mixed = false;
            return ISING_OK;
        }
        b_->tiles = keep.tiles;
        b_->kinds = keep.kinds;
        b_->model = keep.model;
        b_->mixed = true;
        std::vector<std::vector<uint32_t>> groups = keep.groups;
        float ms = ms_keep;
        if (int rc = refine(groups, &ms))
            return rc;
        b_->groups = ms < ms_keep ? groups : keep.groups;
        return ISING_OK;
    }

  private:
    struct Fits { // per size: (a, b) of each tile, the tile, fitted through two x
        std::vector<std::vector<plan::Kind>> kinds;
        std::vector<std::vector<Tile>> tiles;
        std::vector<std::vector<bool>> two;
    };
    struct Choice {
        std::map<int64_t, Tile> tiles;
        std::map<int64_t, plan::Kind> kinds;
        std::vector<std::vector<uint32_t>> groups;
        plan::Model model = plan::kAdditive;
    };

    void apply(const std::vector<size_t> &pick)
    {
        for (size_t i = 0; i < sizes_.size(); ++i) {
            b_->tiles[sizes_[i]] = opt_tiles_[i][pick[i]];
            b_->est_ms[sizes_[i]] = plan::bundle_ms(opts_[i][pick[i]], slots_);
        }
    }
    bool ms_fast_wins(float ms_pick) const { return ms_best_ < ms_pick; }

    // (a, b) of every size and tile under `model`; a one-x fit takes the
    // median intercept of the two-x fits.
    Fits fit_models(plan::Model model) const
    {
        Fits f;
        f.kinds.resize(sizes_.size());
        f.tiles.resize(sizes_.size());
        f.two.resize(sizes_.size());
        std::vector<double> intercepts;
        for (int pass = 0; pass < 2; ++pass) {
            double a_def = 0.0;
            if (pass == 1 && !intercepts.empty()) {
                std::sort(intercepts.begin(), intercepts.end());
                a_def = intercepts[intercepts.size() / 2];
            }
            for (size_t i = 0; i < sizes_.size(); ++i) {
                std::map<std::pair<uint32_t, uint32_t>, std::vector<std::pair<uint32_t, double>>>
                    pts;
                for (size_t j = 0; j < opts_[i].size(); ++j)
                    pts[{opt_tiles_[i][j].wpt, opt_tiles_[i][j].lpw}].emplace_back(
                        opt_per_[i][j], plan::bundle_ms(opts_[i][j], slots_));
                f.kinds[i].clear();
                f.tiles[i].clear();
                f.two[i].clear();
                for (auto &kv : pts) {
                    const Tile t{kv.first.first, kv.first.second};
                    const uint32_t tpl = threads_per_lattice(words_of(sizes_[i]), t);
                    plan::Kind k;
                    plan::fit_kind(kv.second, tpl, model, a_def, &k.a, &k.b);
                    auto x = [&](uint32_t n) {
                        return model == plan::kRounds ? plan::simd_waves(n * tpl) : n;
                    };
                    bool two = false;
                    for (auto &pt : kv.second)
                        two = two || x(pt.first) != x(kv.second.front().first);
                    if (pass == 0 && two)
                        intercepts.push_back(k.a);
                    f.kinds[i].push_back(k);
                    f.tiles[i].push_back(t);
                    f.two[i].push_back(two);
                }
            }
        }
        return f;
    }

    Choice tiles_by_rule(const Fits &f, plan::Model model, int rule,
                         const std::map<int64_t, Tile> &hom_tiles, double hom_est) const
    {
        Choice c;
        for (size_t i = 0; i < sizes_.size(); ++i) {
            auto tpl = [&](size_t j) { return threads_per_lattice(words_of(sizes_[i]), f.tiles[i][j]); };
            // per-lattice share of the compute unit, and one lattice alone
            auto cost = [&](size_t j) {
                return model == plan::kRounds ? f.kinds[i][j].b * (double)tpl(j) : f.kinds[i][j].b;
            };
            auto alone = [&](size_t j) {
                return plan::group_time(model, f.kinds[i][j].a, f.kinds[i][j].b, f.kinds[i][j].b,
                                        tpl(j));
            };
            bool any_two = false;
            for (size_t j = 0; j < f.kinds[i].size(); ++j)
                any_two = any_two || f.two[i][j];
            size_t pick = SIZE_MAX;
            for (size_t j = 0; j < f.kinds[i].size(); ++j) {
                if (rule % 2 == 1) {
                    const Tile &h = hom_tiles.at(sizes_[i]);
                    if (f.tiles[i][j].wpt == h.wpt && f.tiles[i][j].lpw == h.lpw)
                        pick = j;
                } else if ((!any_two || f.two[i][j]) && alone(j) <= hom_est &&
                           (pick == SIZE_MAX || cost(j) < cost(pick) ||
                            (cost(j) == cost(pick) && f.kinds[i][j].a < f.kinds[i][pick].a))) {
                    pick = j; // (a one-x fit only guesses its split into a and b)
                }
            }
            if (pick == SIZE_MAX)
                pick = 0;
            c.tiles[sizes_[i]] = f.tiles[i][pick];
            c.kinds[sizes_[i]] = f.kinds[i][pick];
            c.kinds[sizes_[i]].exclusive = rule >= 2 && (sizes_[i] % 64) != 0;
        }
        return c;
    }

    void log_choice(const Choice &c, plan::Model model, int rule, bool packed, double est) const
    {
        std::fprintf(stderr, "[autotune] %s model, rule %d: %s, estimated %.4f ms\n",
                     model == plan::kRounds ? "rounds" : "additive", rule,
                     packed ? "packed" : "does not pack", est);
        for (auto &kv : c.tiles) {
            const plan::Kind &k = c.kinds.at(kv.first);
            std::fprintf(stderr, "[autotune]   L=%lld tile (%u, %u) a=%.4f b=%.5f%s\n",
                         (long long)kv.first, kv.second.wpt, kv.second.lpw, k.a, k.b,
                         k.exclusive ? " own workgroups" : "");
        }
    }

    void log_bundles(const char *what, const std::vector<std::vector<uint32_t>> &groups,
                     const std::vector<double> &dur) const
    {
        if (!log_ || dur.size() < groups.size())
            return;
        std::vector<size_t> o(groups.size());
        for (size_t i = 0; i < o.size(); ++i)
            o[i] = i;
        std::stable_sort(o.begin(), o.end(), [&](size_t x, size_t y) { return dur[x] > dur[y]; });
        for (size_t k = 0; k < o.size(); ++k) {
            if (k >= 8 && k + 4 < o.size())
                continue;
            std::map<int64_t, int> comp;
            for (uint32_t q : groups[o[k]])
                ++comp[b_->Ls[q]];
            std::string c;
            for (auto &kv : comp)
                c += " " + std::to_string(kv.first) + "x" + std::to_string(kv.second);
            std::fprintf(stderr, "[autotune]   %s #%zu %.4f ms:%s\n", what, k, dur[o[k]], c.c_str());
        }
    }

    bool fits(const std::vector<uint32_t> &g, uint32_t q) const
    {
        uint32_t threads = 0, lds = 0;
        for (uint32_t x : g) {
            threads += mixed_threads(b_->lats[x].W, b_->tiles.at(b_->Ls[x]));
            lds += batch_lds_words(b_->lats[x].W);
        }
        threads += mixed_threads(b_->lats[q].W, b_->tiles.at(b_->Ls[q]));
        lds += batch_lds_words(b_->lats[q].W);
        return threads <= (uint32_t)kBatchThreads && (size_t)lds * 8 <= kMaxBundleLds;
    }

    // Measured refinement of a mixed packing: time every bundle and move one
    // lattice at a time out of the slowest workgroup onto one of the four
    // least loaded it fits.  Many workgroups end within a few per cent of
    // each other, so a move is kept unless the whole launch gets slower
    // (beyond 0.3 %, the timing noise): the slowest ones come down one by
    // one.  At most 96 moves and 256 timed trials; `groups` and *ms end as
    // the fastest plan seen.
    int refine(std::vector<std::vector<uint32_t>> &groups, float *ms)
    {
        std::vector<double> dur;
        float cur = 0.f;
        if (int rc = time_plan(plan_from_groups(b_, groups), &cur, out_, &dur))
            return rc;
        if (out_ != ref_)
            return host::fail(ISING_E_HIP, "autotune: a mixed plan changed the lattices");
        log_bundles("kept", groups, dur);
        std::vector<std::vector<uint32_t>> best = groups;
        float best_ms = cur;
        int moves = 0, trials = 0;
        for (int it = 0; it < 96 && trials < 256; ++it) {
            if (groups.size() < slots_)
                groups.emplace_back(); // an idle workgroup is a target too
            dur.resize(groups.size(), 0.0);
            std::vector<size_t> order(groups.size());
            for (size_t i = 0; i < order.size(); ++i)
                order[i] = i;
            std::stable_sort(order.begin(), order.end(),
                             [&](size_t x, size_t y) { return dur[x] > dur[y]; });
            const size_t sw = order.front();
            // one lattice of each size in the slowest workgroup, largest first
            std::vector<uint32_t> cand;
            for (uint32_t q : groups[sw]) {
                bool seen = false;
                for (uint32_t c : cand)
                    seen = seen || b_->Ls[c] == b_->Ls[q];
                if (!seen)
                    cand.push_back(q);
            }
            std::stable_sort(cand.begin(), cand.end(),
                             [&](uint32_t x, uint32_t y) { return b_->Ls[x] > b_->Ls[y]; });
            bool moved = false;
            for (uint32_t q : cand) {
                if (moved || groups[sw].size() < 2)
                    break;
                std::vector<size_t> targets; // least loaded first
                for (size_t k = order.size(); k-- > 1 && targets.size() < 4;)
                    if (fits(groups[order[k]], q))
                        targets.push_back(order[k]);
                for (size_t tw : targets) {
                    if (++trials > 256)
                        break;
                    std::vector<std::vector<uint32_t>> trial = groups;
                    trial[sw].erase(std::find(trial[sw].begin(), trial[sw].end(), q));
                    trial[tw].push_back(q);
                    std::vector<std::vector<uint32_t>> nonempty;
                    for (auto &g : trial)
                        if (!g.empty())
                            nonempty.push_back(g);
                    float ms_t = 0.f;
                    std::vector<double> dur_t;
                    if (int rc = time_plan(plan_from_groups(b_, nonempty), &ms_t, out_, &dur_t))
                        return rc;
                    if (out_ != ref_)
                        return host::fail(ISING_E_HIP, "autotune: a refined plan changed the "
                                          "lattices");
                    if (ms_t < cur * 1.003f) {
                        groups = std::move(nonempty);
                        dur = std::move(dur_t);
                        cur = ms_t;
                        moved = true;
                        ++moves;
                        if (cur < best_ms) {
                            best_ms = cur;
                            best = groups;
                        }
                        break;
                    }
                }
            }
            if (!groups.empty() && groups.back().empty())
                groups.pop_back();
            if (!moved)
                break;
        }
        if (log_) {
            std::fprintf(stderr, "[autotune] refined by %d moves: %.4f ms (best %.4f)\n", moves,
                         (double)cur, (double)best_ms);
            log_bundles("refined", groups, dur);
        }
        groups = std::move(best);
        *ms = best_ms;
        return ISING_OK;
    }

    ising_batch *b_;
    int64_t sweeps_;
    hipStream_t s_;
    bool log_;
    size_t nbytes_ = 0;
    uint64_t *scratch_ = nullptr, *ctr_ = nullptr, *clk_ = nullptr;
    uint32_t *next_ = nullptr;
    BatchSlot *slot_buf_ = nullptr;
    BatchBundle *bundles_ = nullptr;
    size_t clk_n_ = 0;
    double wall_khz_ = 0.0;
    hipEvent_t e0_ = nullptr, e1_ = nullptr;
    uint32_t slots_ = 0;
    // per size: the options timed alone, their tiles, lattices in their
    // fullest bundle, and the fastest
    std::vector<int64_t> sizes_;
    std::vector<std::vector<plan::Option>> opts_;
    std::vector<std::vector<Tile>> opt_tiles_;
    std::vector<std::vector<uint32_t>> opt_per_;
    std::vector<size_t> fastest_;
    std::vector<size_t> pick_;
    float ms_best_ = 0.f;              // the one-size plan's timing
    std::vector<uint64_t> ref_, out_; // the whole batch: reference result, latest result
};

} // namespace

extern "C" {

int64_t ising_batch_words(int32_t n, const int64_t *Ls)
{
    if (n < 0 || (n > 0 && !Ls))
        return -1;
    int64_t total = 0;
    for (int32_t q = 0; q < n; ++q) {
        if (Ls[q] < 4 || (Ls[q] & 1) || Ls[q] > (int64_t)kMaxBatchL)
            return -1;
        total += 2 * (int64_t)words_of(Ls[q]);
    }
    return total;
}

int ising_batch_create(ising_batch **out, int32_t n, const int64_t *Ls, const double *betas,
                       double J, const uint64_t *seeds, const uint32_t *stream_ids,
                       uint64_t *d_words, size_t bytes)
{
    if (!out)
        return host::fail(ISING_E_BADARG, "null output");
    *out = nullptr;
    if (int r = check_batch_args(n, Ls, betas, J, seeds, stream_ids, d_words, bytes))
        return r;
    ising_batch *b = new ising_batch();
    b->words = d_words;
    b->bytes = bytes;
    if (int r = fill_lattices(b, n, Ls, betas, J, seeds, stream_ids)) {
        delete b;
        return r;
    }
    hipError_t e = hipMalloc(&b->d_lats, b->lats.size() * sizeof(BatchLattice));
    if (e == hipSuccess)
        e = hipMalloc(&b->d_next, 4);
    if (e == hipSuccess)
        e = hipMalloc(&b->d_counter, 8);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_lats, b->lats.data(), b->lats.size() * sizeof(BatchLattice),
                      hipMemcpyHostToDevice);
    const uint64_t zero = 0;
    if (e == hipSuccess)
        e = hipMemcpy(b->d_counter, &zero, 8, hipMemcpyHostToDevice);
    std::vector<int64_t> spin_off((size_t)n);
    int64_t so = 0;
    for (int32_t q = 0; q < n; ++q) {
        spin_off[(size_t)q] = so;
        so += Ls[q] * Ls[q];
    }
    if (e == hipSuccess)
        e = hipMalloc(&b->d_spin_off, (size_t)n * 8);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_spin_off, spin_off.data(), (size_t)n * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        ising_batch_destroy(b);
        return host::hip_fail(e, "batch allocation");
    }
    if (int r = install_plan(b, make_plan(b, 0, Tile{1, 1}))) {
        ising_batch_destroy(b);
        return r;
    }
    *out = b;
    return host::ok();
}

int ising_batch_destroy(ising_batch *b)
{
    if (!b)
        return host::ok();
    free_plan_buffers(b);
    if (b->d_lats)
        (void)hipFree(b->d_lats);
    if (b->d_next)
        (void)hipFree(b->d_next);
    if (b->d_counter)
        (void)hipFree(b->d_counter);
    if (b->d_spin_off)
        (void)hipFree(b->d_spin_off);
    if (b->capture_stream)
        (void)hipStreamDestroy(b->capture_stream);
    delete b;
    return host::ok();
}

int ising_batch_lattice(const ising_batch *b, int32_t q, ising_lattice *out)
{
    if (int e = check_batch(b))
        return e;
    if (!out || q < 0 || q >= b->n)
        return host::fail(ISING_E_BADARG, "lattice index out of range");
    const BatchLattice &lt = b->lats[(size_t)q];
    out->words = b->words + lt.word_off;
    out->L = lt.L;
    out->seed = ((uint64_t)lt.key1 << 32) | lt.key0;
    out->stream_id = lt.stream_id;
    out->reserved = 0;
    return host::ok();
}

int ising_batch_init(ising_batch *b, void *hip_stream)
{
    if (int e = check_batch(b))
        return e;
    hipError_t e = launch_batch_init(b->d_lats, (uint32_t)b->n, b->words, (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return host::hip_fail(e, "batch init launch");
    return host::ok();
}

int ising_batch_set_counter(ising_batch *b, uint64_t rng_counter, void *hip_stream)
{
    if (int e = check_batch(b))
        return e;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipMemcpyAsync(b->d_counter, &rng_counter, 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return host::hip_fail(e, "set batch counter");
    return host::ok();
}

int ising_batch_get_counter(const ising_batch *b, uint64_t *rng_counter, void *hip_stream)
{
    if (int e = check_batch(b))
        return e;
    if (!rng_counter)
        return host::fail(ISING_E_BADARG, "null output");
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipMemcpyAsync(rng_counter, b->d_counter, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return host::hip_fail(e, "get batch counter");
    return host::ok();
}

int ising_batch_sweep(ising_batch *b, int64_t nsweeps, void *hip_stream)
{
    if (int e = check_batch(b))
        return e;
    if (nsweeps < 0)
        return host::fail(ISING_E_BADARG, "nsweeps must be >= 0");
    if (nsweeps == 0)
        return host::ok();
    hipStream_t s = (hipStream_t)hip_stream;
    if (!b->exec || b->exec_nsweeps != nsweeps) {
        if (b->exec)
            (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t le = launch_batch_sweep(b->d_lats, b->d_slots, b->d_bundles, b->nbundles,
                                               b->grid, b->lds_bytes, b->d_next, b->words,
                                               b->d_counter, nsweeps, b->capture_stream);
            e = hipStreamEndCapture(b->capture_stream, &graph);
            if (le != hipSuccess)
                e = le;
        }
        if (e == hipSuccess)
            e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
        if (graph)
            (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            b->exec = nullptr;
            return host::hip_fail(e, "batch sweep graph capture");
        }
        b->exec_nsweeps = nsweeps;
    }
    hipError_t e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess)
        return host::hip_fail(e, "batch sweep graph launch");
    return host::ok();
}

int ising_batch_observables(const ising_batch *b, int64_t *d_bond, int64_t *d_mag,
                            void *hip_stream)
{
    if (int e = check_batch(b))
        return e;
    if (!d_bond || !d_mag)
        return host::fail(ISING_E_BADARG, "null output pointer");
    hipError_t e = launch_batch_observables(b->d_lats, (uint32_t)b->n, b->words, d_bond, d_mag,
                                            (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return host::hip_fail(e, "batch observables launch");
    return host::ok();
}

int ising_batch_get_spins_dev(const ising_batch *b, int8_t *d_spins, void *hip_stream)
{
    if (int e = check_batch(b))
        return e;
    if (!d_spins)
        return host::fail(ISING_E_BADARG, "null spins");
    hipError_t e = launch_batch_to_spins(b->d_lats, (uint32_t)b->n, b->words, b->d_spin_off,
                                         d_spins, (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return host::hip_fail(e, "batch to spins");
    return host::ok();
}

int ising_batch_set_spins_dev(ising_batch *b, const int8_t *d_spins, void *hip_stream)
{
    if (int e = check_batch(b))
        return e;
    if (!d_spins)
        return host::fail(ISING_E_BADARG, "null spins");
    hipError_t e = launch_batch_from_spins(b->d_lats, (uint32_t)b->n, b->words, b->d_spin_off,
                                           d_spins, (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return host::hip_fail(e, "spins to batch");
    return host::ok();
}

int ising_batch_get_tiles(const ising_batch *b, int64_t L, uint32_t *wpt, uint32_t *lpw)
{
    if (int e = check_batch(b))
        return e;
    auto it = b->tiles.find(L);
    if (!wpt || !lpw || it == b->tiles.end())
        return host::fail(ISING_E_BADARG, "no lattice of that size in the batch");
    *wpt = it->second.wpt;
    *lpw = it->second.lpw;
    return host::ok();
}

int ising_batch_get_plan(const ising_batch *b, int64_t L, uint32_t *lattices_per_workgroup,
                         uint32_t *workgroups)
{
    if (int e = check_batch(b))
        return e;
    auto it = b->tiles.find(L);
    if (!lattices_per_workgroup || !workgroups || it == b->tiles.end())
        return host::fail(ISING_E_BADARG, "no lattice of that size in the batch");
    auto st = b->plan_stats.find(L);
    *lattices_per_workgroup = st == b->plan_stats.end() ? 0 : st->second.first;
    *workgroups = st == b->plan_stats.end() ? 0 : st->second.second;
    return host::ok();
}

int ising_batch_set_bundles(ising_batch *b, int32_t nbundles, const int32_t *counts,
                            const int32_t *lattices)
{
    if (int e = check_batch(b))
        return e;
    if (nbundles <= 0 || !counts || !lattices)
        return host::fail(ISING_E_BADARG, "no bundles or null pointer");
    Plan p;
    int64_t at = 0;
    std::vector<uint8_t> seen((size_t)b->n, 0);
    for (int32_t i = 0; i < nbundles; ++i) {
        if (counts[i] <= 0 || at + counts[i] > b->n)
            return host::fail(ISING_E_BADARG, "bundle %d: count %d out of range", (int)i,
                              (int)counts[i]);
        std::vector<std::pair<uint32_t, Tile>> v;
        uint32_t threads = 0, lds = 0;
        for (int32_t c = 0; c < counts[i]; ++c, ++at) {
            const int32_t q = lattices[at];
            if (q < 0 || q >= b->n || seen[(size_t)q])
                return host::fail(ISING_E_BADARG, "lattice %d missing, repeated or out of range",
                                  (int)q);
            seen[(size_t)q] = 1;
            const Tile t = b->tiles.at(b->Ls[(size_t)q]);
            threads += mixed_threads(b->lats[(size_t)q].W, t);
            lds += batch_lds_words(b->lats[(size_t)q].W);
            v.emplace_back((uint32_t)q, t);
        }
        if (threads > (uint32_t)kBatchThreads || (size_t)lds * 8 > kMaxBundleLds)
            return host::fail(ISING_E_BADARG, "bundle %d needs %u threads and %u B of LDS (at most "
                              "%d and %zu)", (int)i, threads, lds * 8, kBatchThreads,
                              kMaxBundleLds);
        add_bundle(p, b, std::move(v), true);
    }
    if (at != b->n)
        return host::fail(ISING_E_BADARG, "the bundles hold %lld of %d lattices", (long long)at,
                          (int)b->n);
    if (int rc = install_plan(b, p))
        return rc;
    b->mixed = true;
    b->groups.clear(); // the caller's plan stands until the batch is replanned
    b->est_ms.clear();
    return host::ok();
}

int ising_batch_get_mixed(const ising_batch *b, int32_t *mixed)
{
    if (int e = check_batch(b))
        return e;
    if (!mixed)
        return host::fail(ISING_E_BADARG, "null output");
    *mixed = b->mixed ? 1 : 0;
    return host::ok();
}

int ising_batch_set_tiles(ising_batch *b, int64_t L, uint32_t wpt, uint32_t lpw)
{
    if (int e = check_batch(b))
        return e;
    auto it = b->tiles.find(L);
    if (it == b->tiles.end())
        return host::fail(ISING_E_BADARG, "no lattice of that size in the batch");
    if (!tile_ok(words_of(L), Tile{wpt, lpw}))
        return host::fail(ISING_E_BADARG, "tile (%u words, %u lanes per word) does not fit a "
                          "workgroup of %d threads", wpt, lpw, kBatchThreads);
    it->second = Tile{wpt, lpw};
    b->est_ms.erase(L); // bundles go back to ordering by spins
    b->mixed = false;   // and to one size each
    b->groups.clear();
    return install_plan(b, make_plan(b, 0, Tile{1, 1}));
}

int ising_batch_autotune(ising_batch *b, int64_t tune_sweeps, const char *cache_path,
                         void *hip_stream)
{
    if (int e = check_batch(b))
        return e;
    if (tune_sweeps <= 0)
        return host::fail(ISING_E_BADARG, "tune_sweeps must be > 0");
    b->est_ms.clear();
    b->kinds.clear();
    b->groups.clear();
    b->mixed = false;
    std::map<int64_t, CacheEntry> cached;
    bool cached_mixed = false;
    plan::Model cached_model = plan::kAdditive;
    std::vector<std::vector<uint32_t>> cached_groups;
    if (cache_path &&
        read_cache(cache_path, cached, &cached_mixed, &cached_model, b, &cached_groups)) {
        bool complete = true;
        for (auto &kv : b->tiles)
            complete = complete && cached.count(kv.first) &&
                       tile_ok(words_of(kv.first), cached[kv.first].tile);
        if (complete) {
            for (auto &kv : b->tiles) {
                kv.second = cached[kv.first].tile;
                b->kinds[kv.first] = cached[kv.first].kind;
            }
            b->mixed = cached_mixed;
            b->model = cached_model;
            if (cached_mixed && valid_groups(b, cached_groups))
                b->groups = std::move(cached_groups);
            return install_current_plan(b);
        }
    }
    int rc = ISING_OK;
    {
        Tuner t(b, tune_sweeps, (hipStream_t)hip_stream);
        if ((rc = t.start()) == ISING_OK && (rc = t.time_sizes()) == ISING_OK &&
            (rc = t.choose_one_size()) == ISING_OK)
            rc = t.choose_mixed();
    }
    if (rc != ISING_OK) {
        b->est_ms.clear();
        b->kinds.clear();
        b->groups.clear();
        b->mixed = false;
        return rc;
    }
    if (cache_path && !write_cache(cache_path, b))
        return host::fail(ISING_E_BADARG, "cannot write the autotune cache %s", cache_path);
    return install_current_plan(b);
}

int ising_batch_sweep_noalloc(int32_t n, const int64_t *Ls, const double *betas, double J,
                              const uint64_t *seeds, const uint32_t *stream_ids,
                              uint64_t *d_words, size_t bytes, int64_t nsweeps,
                              uint64_t rng_counter, void *hip_stream)
{
    if (int r = check_batch_args(n, Ls, betas, J, seeds, stream_ids, d_words, bytes))
        return r;
    if (n > kNoAllocMaxLattices)
        return host::fail(ISING_E_SIZE, "at most %d lattices without allocation (got %d)",
                          kNoAllocMaxLattices, (int)n);
    if (nsweeps < 0)
        return host::fail(ISING_E_BADARG, "nsweeps must be >= 0");
    if (nsweeps == 0)
        return host::ok();
    // host threads take turns: the plan and its host image are one static
    // buffer, consumed by the copy below before the lock is released (a copy
    // from pageable host memory returns once its source has been read)
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    NoAllocPlan &p = g_noalloc_plan;
    if (int r = p.build(n, Ls, betas, J, seeds, stream_ids))
        return r;
    if (int r = check_plan(p.lats, n, p.slots, (size_t)n, p.bundles, p.nbundles, p.lds_bytes))
        return r;
    uint32_t grid = 0;
    if (int r = persistent_grid(p.lds_bytes, p.nbundles, &grid))
        return r;
    // scratch layout: sweep counter, queue counter | lattices | slots | bundles
    const size_t o_lats = 256;
    const size_t o_slots = align256(o_lats + (size_t)n * sizeof(BatchLattice));
    const size_t o_bundles = align256(o_slots + (size_t)n * sizeof(BatchSlot));
    const size_t total = o_bundles + (size_t)p.nbundles * sizeof(BatchBundle);
    if (total > kNoAllocScratchBytes)
        return host::fail(ISING_E_SIZE, "descriptors need %zu bytes, the scratch array holds %zu",
                          total, kNoAllocScratchBytes);
    unsigned char *ptr = nullptr;
    if (int r = scratch_of_current_device(&ptr))
        return r;
    unsigned char *stage = p.stage;
    std::memset(stage, 0, o_lats);
    std::memcpy(stage, &rng_counter, sizeof(rng_counter));
    std::memcpy(stage + o_lats, p.lats, (size_t)n * sizeof(BatchLattice));
    std::memcpy(stage + o_slots, p.slots, (size_t)n * sizeof(BatchSlot));
    std::memcpy(stage + o_bundles, p.bundles, (size_t)p.nbundles * sizeof(BatchBundle));
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipMemcpyAsync(ptr, stage, total, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_batch_sweep((const BatchLattice *)(ptr + o_lats),
                               (const BatchSlot *)(ptr + o_slots),
                               (const BatchBundle *)(ptr + o_bundles), p.nbundles, grid,
                               p.lds_bytes, (uint32_t *)(ptr + 8), d_words, (uint64_t *)ptr,
                               nsweeps, s);
    if (e != hipSuccess)
        return host::hip_fail(e, "batch sweep without allocation");
    return host::ok();
}

} // extern "C"
