// C ABI of batched lattices (include/ising.h): planning bundles for the
// persistent kernel, the captured HIP graph of one batch sweep, the
// autotuner of words per thread, and per-lattice observables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
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
    // device state owned by the batch
    BatchLattice *d_lats = nullptr;
    uint32_t *d_members = nullptr;
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
    std::vector<uint32_t> members;
    std::vector<BatchBundle> bundles;
    size_t lds_bytes = 0;
};

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
        BatchBundle bd;
        std::vector<uint32_t> ids;
    };
    std::vector<Item> items;
    for (auto &kv : by_size) {
        const int64_t L = kv.first;
        const uint32_t W = words_of(L);
        const Tile tile = only_L ? only : b->tiles.at(L);
        const uint32_t tpl = threads_per_lattice(W, tile);
        const uint32_t per = lattices_per_bundle(W, tile);
        for (size_t i = 0; i < kv.second.size(); i += per) {
            Item it;
            const uint32_t cnt = (uint32_t)std::min<size_t>(per, kv.second.size() - i);
            it.ids.assign(kv.second.begin() + i, kv.second.begin() + i + cnt);
            it.bd = BatchBundle{0, cnt, tile.wpt, tpl, tile.lpw, 0};
            it.work = have_est ? b->est_ms.at(L) : (double)cnt * (double)(L * L);
            items.push_back(std::move(it));
        }
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const Item &a, const Item &c) { return a.work > c.work; });
    Plan p;
    for (auto &it : items) {
        it.bd.first = (uint32_t)p.members.size();
        p.members.insert(p.members.end(), it.ids.begin(), it.ids.end());
        p.bundles.push_back(it.bd);
        const uint32_t W = b->lats[it.ids[0]].W;
        p.lds_bytes = std::max(p.lds_bytes, (size_t)it.bd.count * batch_lds_words(W) * 8);
    }
    return p;
}

void free_plan_buffers(ising_batch *b)
{
    if (b->d_members)
        (void)hipFree(b->d_members);
    if (b->d_bundles)
        (void)hipFree(b->d_bundles);
    b->d_members = nullptr;
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
    free_plan_buffers(b);
    hipError_t e = hipMalloc(&b->d_members, std::max<size_t>(1, p.members.size()) * 4);
    if (e == hipSuccess)
        e = hipMalloc(&b->d_bundles, std::max<size_t>(1, p.bundles.size()) * sizeof(BatchBundle));
    if (e == hipSuccess && !p.members.empty())
        e = hipMemcpy(b->d_members, p.members.data(), p.members.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && !p.bundles.empty())
        e = hipMemcpy(b->d_bundles, p.bundles.data(), p.bundles.size() * sizeof(BatchBundle),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return host::hip_fail(e, "batch plan upload");
    b->nbundles = (uint32_t)p.bundles.size();
    b->lds_bytes = p.lds_bytes;
    return persistent_grid(p.lds_bytes, b->nbundles, &b->grid);
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
    uint32_t members[kNoAllocMaxLattices];
    BatchBundle bundles[kNoAllocMaxLattices];
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
            const uint32_t tpl = threads_per_lattice(W, tile), per = lattices_per_bundle(W, tile);
            for (int32_t k = g0; k < g1; k += (int32_t)per) {
                const uint32_t cnt = (uint32_t)std::min<int32_t>((int32_t)per, g1 - k);
                bundles[nbundles] = BatchBundle{(uint32_t)k, cnt, tile.wpt, tpl, tile.lpw, 0};
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
        // bundles in that order, each with its members contiguous
        uint32_t m = 0;
        BatchBundle *sorted = (BatchBundle *)stage; // reuse the stage as room to permute
        for (uint32_t k = 0; k < nbundles; ++k) {
            BatchBundle bd = bundles[border[k]];
            for (uint32_t c = 0; c < bd.count; ++c)
                members[m + c] = order[bd.first + c];
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
std::string cache_key() { return "gfx950/batch-sweep-v8"; }

bool read_cache(const char *path, std::map<int64_t, Tile> &out)
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
    while (in >> L >> w >> l >> c)
        out[(int64_t)L] = Tile{w, l, c};
    return true;
}

bool write_cache(const char *path, const std::map<int64_t, Tile> &tiles)
{
    std::ofstream f(path);
    if (!f)
        return false;
    f << "{\"key\": \"" << cache_key() << "\", \"tiles\": {";
    bool first = true;
    for (auto &kv : tiles) {
        f << (first ? "" : ", ") << "\"" << kv.first << "\": [" << kv.second.wpt << ", "
          << kv.second.lpw << ", " << kv.second.cap << "]";
        first = false;
    }
    f << "}}\n";
    return (bool)f;
}

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
            hipError_t le = launch_batch_sweep(b->d_lats, b->d_members, b->d_bundles, b->nbundles,
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
    const uint32_t n = (uint32_t)std::count(b->Ls.begin(), b->Ls.end(), L);
    const uint32_t per = lattices_per_bundle(words_of(L), it->second);
    *lattices_per_workgroup = std::min(per, n);
    *workgroups = (n + per - 1) / per;
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
    return install_plan(b, make_plan(b, 0, Tile{1, 1}));
}

int ising_batch_autotune(ising_batch *b, int64_t tune_sweeps, const char *cache_path,
                         void *hip_stream)
{
    if (int e = check_batch(b))
        return e;
    if (tune_sweeps <= 0)
        return host::fail(ISING_E_BADARG, "tune_sweeps must be > 0");
    hipStream_t s = (hipStream_t)hip_stream;
    b->est_ms.clear();
    std::map<int64_t, Tile> cached;
    if (cache_path && read_cache(cache_path, cached)) {
        bool complete = true;
        for (auto &kv : b->tiles)
            complete = complete && cached.count(kv.first) &&
                       tile_ok(words_of(kv.first), cached[kv.first]);
        if (complete) {
            for (auto &kv : b->tiles)
                kv.second = cached[kv.first];
            return install_plan(b, make_plan(b, 0, Tile{1, 1}));
        }
    }
    // Scratch copy of the lattices and counter: tuning never changes the batch.
    const size_t nbytes = (size_t)ising_batch_words(b->n, b->Ls.data()) * 8;
    uint64_t *scratch = nullptr, *ctr = nullptr;
    uint32_t *members = nullptr, *next = nullptr;
    BatchBundle *bundles = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&scratch, nbytes);
    if (e == hipSuccess)
        e = hipMalloc(&ctr, 8);
    if (e == hipSuccess)
        e = hipMalloc(&next, 4);
    if (e == hipSuccess)
        e = hipEventCreate(&e0);
    if (e == hipSuccess)
        e = hipEventCreate(&e1);
    int rc = ISING_OK;
    // Runs plan p for tune_sweeps sweeps on the scratch copy, from the batch's
    // lattices and counter 0 every time; best of two launches, lattices to out.
    auto time_plan = [&](const Plan &p, float *best, std::vector<uint64_t> &out) -> bool {
        uint32_t grid = 0;
        if ((rc = persistent_grid(p.lds_bytes, (uint32_t)p.bundles.size(), &grid)))
            return false;
        if (members)
            (void)hipFree(members);
        if (bundles)
            (void)hipFree(bundles);
        members = nullptr;
        bundles = nullptr;
        e = hipMalloc(&members, p.members.size() * 4);
        if (e == hipSuccess)
            e = hipMalloc(&bundles, p.bundles.size() * sizeof(BatchBundle));
        if (e == hipSuccess)
            e = hipMemcpy(members, p.members.data(), p.members.size() * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(bundles, p.bundles.data(), p.bundles.size() * sizeof(BatchBundle),
                          hipMemcpyHostToDevice);
        *best = 1e30f;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
            const uint64_t zero = 0;
            float ms = 0.f;
            e = hipMemcpyAsync(scratch, b->words, nbytes, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(ctr, &zero, 8, hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipEventRecord(e0, s);
            if (e == hipSuccess)
                e = launch_batch_sweep(b->d_lats, members, bundles, (uint32_t)p.bundles.size(),
                                       grid, p.lds_bytes, next, scratch, ctr, tune_sweeps, s);
            if (e == hipSuccess)
                e = hipEventRecord(e1, s);
            if (e == hipSuccess)
                e = hipEventSynchronize(e1);
            if (e == hipSuccess)
                e = hipEventElapsedTime(&ms, e0, e1);
            *best = std::min(*best, ms);
        }
        if (e == hipSuccess) {
            out.resize(nbytes / 8);
            e = hipMemcpy(out.data(), scratch, nbytes, hipMemcpyDeviceToHost);
        }
        return e == hipSuccess;
    };
    // Every tile candidate of each size, timed with that size alone.
    std::vector<int64_t> sizes;
    std::vector<std::vector<plan::Option>> opts;
    std::vector<std::vector<Tile>> opt_tiles;
    std::vector<size_t> fastest;
    uint32_t slots = 0;
    std::vector<uint64_t> out_ref, out_try;
    for (auto &kv : b->tiles) {
        if (e != hipSuccess || rc != ISING_OK)
            break;
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
        // and each with fewer lattices per bundle: half-empty workgroups run
        // their lattices' sweeps sooner, on compute units the batch leaves idle
        const size_t nbase = cands.size();
        for (size_t i = 0; i < nbase; ++i) {
            const uint32_t full = make_plan(b, L, cands[i]).bundles.front().count;
            for (uint32_t cap : {full / 2, full / 4})
                if (cap >= 1 && cap < full)
                    cands.push_back(Tile{cands[i].wpt, cands[i].lpw, cap});
        }
        std::vector<plan::Option> o;
        std::vector<Tile> ot;
        size_t fi = 0;
        for (const Tile &w : cands) {
            const Plan p = make_plan(b, L, w);
            uint32_t held = 0;
            if ((rc = resident_slots(p.lds_bytes, &held)))
                break;
            slots = slots ? std::min(slots, held) : held;
            float ms = 0.f;
            if (!time_plan(p, &ms, o.empty() ? out_ref : out_try))
                break;
            // every candidate must reproduce the same lattices bit for bit
            if (!o.empty() && out_try != out_ref) {
                rc = host::fail(ISING_E_HIP, "autotune: tile (%u, %u, %u) of L=%lld changed the "
                                "lattice", w.wpt, w.lpw, w.cap, (long long)L);
                break;
            }
            o.push_back(plan::Option{(uint32_t)p.bundles.size(), (double)ms});
            ot.push_back(w);
            if (o.back().ms < o[fi].ms)
                fi = o.size() - 1;
        }
        if (e != hipSuccess || rc != ISING_OK)
            break;
        sizes.push_back(L);
        opts.push_back(std::move(o));
        opt_tiles.push_back(std::move(ot));
        fastest.push_back(fi);
    }
    // The tiles for the whole launch: the estimated best, kept only if the
    // whole batch, timed both ways, runs faster with it than with the fastest
    // tile of every size alone.
    auto apply = [&](const std::vector<size_t> &pick) {
        for (size_t i = 0; i < sizes.size(); ++i) {
            b->tiles[sizes[i]] = opt_tiles[i][pick[i]];
            b->est_ms[sizes[i]] = plan::bundle_ms(opts[i][pick[i]], slots);
        }
    };
    if (e == hipSuccess && rc == ISING_OK) {
        std::vector<size_t> pick = plan::choose(opts, fastest, slots);
        if (pick != fastest) {
            float ms_fast = 0.f, ms_pick = 0.f;
            apply(fastest);
            if (time_plan(make_plan(b, 0, Tile{1, 1}), &ms_fast, out_ref)) {
                apply(pick);
                if (time_plan(make_plan(b, 0, Tile{1, 1}), &ms_pick, out_try)) {
                    if (out_try != out_ref)
                        rc = host::fail(ISING_E_HIP, "autotune: the joint tiles changed the "
                                        "lattices");
                    else if (ms_fast < ms_pick)
                        pick = fastest;
                }
            }
        }
        if (e == hipSuccess && rc == ISING_OK)
            apply(pick);
    }
    if (members)
        (void)hipFree(members);
    if (bundles)
        (void)hipFree(bundles);
    if (scratch)
        (void)hipFree(scratch);
    if (ctr)
        (void)hipFree(ctr);
    if (next)
        (void)hipFree(next);
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (rc != ISING_OK || e != hipSuccess)
        b->est_ms.clear();
    if (rc != ISING_OK)
        return rc;
    if (e != hipSuccess)
        return host::hip_fail(e, "autotune");
    if (cache_path && !write_cache(cache_path, b->tiles))
        return host::fail(ISING_E_BADARG, "cannot write the autotune cache %s", cache_path);
    return install_plan(b, make_plan(b, 0, Tile{1, 1}));
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
    uint32_t grid = 0;
    if (int r = persistent_grid(p.lds_bytes, p.nbundles, &grid))
        return r;
    // scratch layout: sweep counter, queue counter | lattices | members | bundles
    const size_t o_lats = 256;
    const size_t o_members = align256(o_lats + (size_t)n * sizeof(BatchLattice));
    const size_t o_bundles = align256(o_members + (size_t)n * sizeof(uint32_t));
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
    std::memcpy(stage + o_members, p.members, (size_t)n * sizeof(uint32_t));
    std::memcpy(stage + o_bundles, p.bundles, (size_t)p.nbundles * sizeof(BatchBundle));
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipMemcpyAsync(ptr, stage, total, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_batch_sweep((const BatchLattice *)(ptr + o_lats),
                               (const uint32_t *)(ptr + o_members),
                               (const BatchBundle *)(ptr + o_bundles), p.nbundles, grid,
                               p.lds_bytes, (uint32_t *)(ptr + 8), d_words, (uint64_t *)ptr,
                               nsweeps, s);
    if (e != hipSuccess)
        return host::hip_fail(e, "batch sweep without allocation");
    return host::ok();
}

} // extern "C"
