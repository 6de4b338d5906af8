// The C ABI of libising (declared in include/ising.h): argument checks,
// the host-side threshold table, and the sweep driver.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ising.h"
#include "glass.hpp"
#include "host_common.hpp"
#include "launch.hpp"

namespace ising {
namespace host {

namespace {
thread_local std::string g_error;
} // namespace

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int ok()
{
    g_error.clear();
    return ISING_OK;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(ISING_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

const char *last_error() { return g_error.c_str(); }

void threshold_table(double beta, double J, uint64_t T[5])
{
    for (int a = 0; a < 5; ++a) {
        const double dE = 4.0 * J * (double)(a - 2);
        if (dE <= 0.0)
            T[a] = 1ull << 32;
        else
            T[a] = (uint64_t)std::floor(std::exp(-(beta * dE)) * 4294967296.0);
    }
}

// Heat bath (Sec. 2): flip probability e^{-beta dE} / (e^{-beta dE} + 1),
// evaluated as 1 / (1 + e^{beta dE}) (no intermediate overflow).
void heatbath_table(double beta, double J, uint64_t T[5])
{
    for (int a = 0; a < 5; ++a) {
        const double dE = 4.0 * J * (double)(a - 2);
        T[a] = (uint64_t)std::floor(1.0 / (1.0 + std::exp(beta * dE)) * 4294967296.0);
    }
}

rows::Table5 table5(const uint64_t T[5])
{
    rows::Table5 tab{};
    for (int a = 0; a < 5; ++a) {
        if (T[a] >= (1ull << 32)) {
            tab.always |= 1u << a;
        } else if (T[a] > 0) {
            tab.random |= 1u << a;
            tab.thr[a] = (uint32_t)T[a];
        }
    }
    return tab;
}

Metro2 metro2_params(double beta, double J)
{
    uint64_t T[5];
    threshold_table(beta, J, T);
    Metro2 m{};
    m.anti = J < 0.0 ? 1u : 0u;
    const uint64_t tA = m.anti ? T[1] : T[3], tB = m.anti ? T[0] : T[4];
    m.alwaysA = tA >= (1ull << 32);
    m.alwaysB = tB >= (1ull << 32);
    m.randA = !m.alwaysA && tA > 0;
    m.randB = !m.alwaysB && tB > 0;
    m.thrA = m.randA ? (uint32_t)tA : 0u;
    m.thrB = m.randB ? (uint32_t)tB : 0u;
    return m;
}

int check_L(int64_t L)
{
    if (L < 4 || (L & 1))
        return fail(ISING_E_BADARG, "L must be even and >= 4 (got %lld)", (long long)L);
    if (L > kMaxL)
        return fail(ISING_E_SIZE, "L = %lld exceeds the supported maximum %lld", (long long)L,
                    (long long)kMaxL);
    return ISING_OK;
}

int check_lattice(const ising_lattice *lat)
{
    if (!lat)
        return fail(ISING_E_BADARG, "null lattice");
    if (int e = check_L(lat->L))
        return e;
    if (!lat->words)
        return fail(ISING_E_BADARG, "null lattice words");
    if (lat->stream_id >= (1u << 24))
        return fail(ISING_E_BADARG, "stream_id must be < 2^24");
    return ISING_OK;
}

int check_temperature(double beta, double J)
{
    if (!std::isfinite(beta) || beta < 0.0)
        return fail(ISING_E_BADARG, "beta must be finite and >= 0");
    if (!std::isfinite(J))
        return fail(ISING_E_BADARG, "J must be finite");
    return ISING_OK;
}

} // namespace host
} // namespace ising

namespace {

using ising::host::fail;
using ising::host::hip_fail;
using ising::host::ok;

// Half-sweep kernel selection (for tests and measurements; 0 = default).
int g_variant = 0;

// The default kernel for a half-sweep (Metropolis or heat bath).  The queued
// row kernel gives each wavefront a band of rows of 64 word columns and walks
// the rows in sequence, so a lattice with few bands leaves most of the 1024
// SIMDs idle.  Measured per Metropolis half-sweep at beta_c: with at least
// 16384 wavefronts of 16-row bands (L >= 49152) those are fastest, by ~3 %
// over 32 rows (L = 65536: 280 against 290 us); below that 8-row bands win
// (L = 16384: 27 us against 49 us with 32 rows, 53 us general); with fewer
// than 1024 wavefronts even then (L < 8192) the general kernel, one thread
// per word, is fastest (L = 2048: 6.5 us against 39 us).
int default_variant(int64_t L)
{
    if (L % 128 != 0)
        return ising::kVariantGeneral;
    const int64_t segs = (L / 128 + 63) / 64; // wavefronts across a row
    if (segs * ((L + 15) / 16) >= 16384)
        return ising::kVariantQueue16;
    if (segs * ((L + 7) / 8) >= 1024)
        return ising::kVariantQueue8;
    return ising::kVariantGeneral;
}

// Kernel for ising_glass_sweep (L % 128 == 0): the queued row kernel with
// 8-row bands, fastest at every size measured (L = 65536: 402 us against 423
// with 16 rows and 439 with 32 -- the bond and spin streams gain from the
// extra wavefronts in flight; L = 2048: 14 us against 42 with 32 rows); or
// the one the caller forced (1, 2: the per-word row kernel).
int glass_variant()
{
    switch (g_variant) {
    case 0:
    case 5:
        return ising::kVariantQueue8;
    case 3:
        return ising::kVariantDefault;
    case 4:
        return ising::kVariantQueue16;
    default:
        return g_variant;
    }
}

// Kernel for ising_sweep: the size-dependent default, or the one the caller
// forced (3, 4, 5: the queued row kernel with 32-, 16- or 8-row bands
// whatever the size).
int sweep_variant(int64_t L)
{
    switch (g_variant) {
    case 0:
        return default_variant(L);
    case 3:
        return ising::kVariantDefault;
    case 4:
        return ising::kVariantQueue16;
    case 5:
        return ising::kVariantQueue8;
    default:
        return g_variant;
    }
}

using ising::host::check_L;
using ising::host::check_lattice;
using ising::host::check_temperature;
using ising::host::kMaxL;

int64_t words_per_colour(int64_t L) { return (L * L / 2 + 63) / 64; }

int run_sweeps(const ising_lattice *lat, double beta, double J, int64_t nsweeps,
               uint64_t rng_counter, int64_t *d_bond, int64_t *d_mag, hipStream_t s)
{
    const ising::Metro2 m = ising::host::metro2_params(beta, J);
    for (int64_t sw = 0; sw < nsweeps; ++sw) {
        for (int c = 0; c < 2; ++c) {
            const uint64_t t = 2 * (rng_counter + (uint64_t)sw) + (uint64_t)c;
            hipError_t e = ising::launch_half_sweep(lat->words, lat->L, c, m, t, lat->seed,
                                                    lat->stream_id, s, sweep_variant(lat->L));
            if (e != hipSuccess)
                return hip_fail(e, "half-sweep launch");
        }
        if (d_bond) {
            hipError_t e = ising::launch_observables(lat->words, lat->L, d_bond + sw,
                                                     d_mag + sw, s);
            if (e != hipSuccess)
                return hip_fail(e, "observables launch");
        }
    }
    return ok();
}

// Sweeps under a rule other than Metropolis.
int run_sweeps5(const ising_lattice *lat, const uint64_t T[5], int64_t nsweeps,
                uint64_t rng_counter, hipStream_t s)
{
    const ising::rows::Table5 tab = ising::host::table5(T);
    for (int64_t sw = 0; sw < nsweeps; ++sw) {
        for (int c = 0; c < 2; ++c) {
            const uint64_t t = 2 * (rng_counter + (uint64_t)sw) + (uint64_t)c;
            hipError_t e = ising::launch_half_sweep5(lat->words, lat->L, c, tab, t, lat->seed,
                                                     lat->stream_id, s, sweep_variant(lat->L));
            if (e != hipSuccess)
                return hip_fail(e, "half-sweep launch");
        }
    }
    return ok();
}

} // namespace

extern "C" {

int64_t ising_words_per_colour(int64_t L)
{
    if (check_L(L) != ISING_OK)
        return -1;
    return words_per_colour(L);
}

int ising_thresholds(double beta, double J, uint64_t *T_out)
{
    if (!T_out)
        return fail(ISING_E_BADARG, "null output");
    if (int e = check_temperature(beta, J))
        return e;
    ising::host::threshold_table(beta, J, T_out);
    return ok();
}

int ising_init(ising_lattice *lat, uint64_t *d_words, size_t bytes, int64_t L, uint64_t seed,
               uint32_t stream_id, void *hip_stream)
{
    if (!lat || !d_words)
        return fail(ISING_E_BADARG, "null lattice or words");
    if (int e = check_L(L))
        return e;
    if (stream_id >= (1u << 24))
        return fail(ISING_E_BADARG, "stream_id must be < 2^24");
    const int64_t W = words_per_colour(L);
    if (bytes < (size_t)(2 * W) * sizeof(uint64_t))
        return fail(ISING_E_SIZE, "buffer of %zu bytes is smaller than the %lld needed", bytes,
                    (long long)(16 * W));
    lat->words = d_words;
    lat->L = L;
    lat->seed = seed;
    lat->stream_id = stream_id;
    lat->reserved = 0;
    hipError_t e = ising::launch_init(d_words, L, seed, stream_id, (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return hip_fail(e, "init launch");
    return ok();
}

int ising_sweep(const ising_lattice *lat, double beta, double J, int64_t nsweeps,
                uint64_t rng_counter, void *hip_stream)
{
    if (int e = check_lattice(lat))
        return e;
    if (int e = check_temperature(beta, J))
        return e;
    if (nsweeps < 0)
        return fail(ISING_E_BADARG, "nsweeps must be >= 0");
    return run_sweeps(lat, beta, J, nsweeps, rng_counter, nullptr, nullptr,
                      (hipStream_t)hip_stream);
}

int ising_thresholds_rule(double beta, double J, int rule, uint64_t *T_out)
{
    if (!T_out)
        return fail(ISING_E_BADARG, "null output");
    if (int e = check_temperature(beta, J))
        return e;
    if (rule == ISING_RULE_METROPOLIS)
        ising::host::threshold_table(beta, J, T_out);
    else if (rule == ISING_RULE_HEATBATH)
        ising::host::heatbath_table(beta, J, T_out);
    else
        return fail(ISING_E_BADARG, "unknown rule %d", rule);
    return ok();
}

int ising_sweep_rule(const ising_lattice *lat, double beta, double J, int rule, int64_t nsweeps,
                     uint64_t rng_counter, void *hip_stream)
{
    if (rule == ISING_RULE_METROPOLIS)
        return ising_sweep(lat, beta, J, nsweeps, rng_counter, hip_stream);
    if (rule != ISING_RULE_HEATBATH)
        return fail(ISING_E_BADARG, "unknown rule %d", rule);
    if (int e = check_lattice(lat))
        return e;
    if (int e = check_temperature(beta, J))
        return e;
    if (nsweeps < 0)
        return fail(ISING_E_BADARG, "nsweeps must be >= 0");
    uint64_t T[5];
    ising::host::heatbath_table(beta, J, T);
    return run_sweeps5(lat, T, nsweeps, rng_counter, (hipStream_t)hip_stream);
}

int ising_sweep_traced(const ising_lattice *lat, double beta, double J, int64_t nsweeps,
                       uint64_t rng_counter, int64_t *d_bond_trace, int64_t *d_mag_trace,
                       void *hip_stream)
{
    if (int e = check_lattice(lat))
        return e;
    if (int e = check_temperature(beta, J))
        return e;
    if (nsweeps < 0)
        return fail(ISING_E_BADARG, "nsweeps must be >= 0");
    if (nsweeps > 0 && (!d_bond_trace || !d_mag_trace))
        return fail(ISING_E_BADARG, "null trace pointer");
    return run_sweeps(lat, beta, J, nsweeps, rng_counter, d_bond_trace, d_mag_trace,
                      (hipStream_t)hip_stream);
}

int ising_observables(const ising_lattice *lat, int64_t *d_bond, int64_t *d_mag,
                      void *hip_stream)
{
    if (int e = check_lattice(lat))
        return e;
    if (!d_bond || !d_mag)
        return fail(ISING_E_BADARG, "null output pointer");
    hipError_t e =
        ising::launch_observables(lat->words, lat->L, d_bond, d_mag, (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return hip_fail(e, "observables launch");
    return ok();
}

int ising_get_spins(const ising_lattice *lat, int8_t *host_spins, void *hip_stream)
{
    if (int e = check_lattice(lat))
        return e;
    if (!host_spins)
        return fail(ISING_E_BADARG, "null host buffer");
    const int64_t L = lat->L, H = L / 2, W = words_per_colour(L);
    std::vector<uint64_t> w((size_t)(2 * W));
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipMemcpyAsync(w.data(), lat->words, w.size() * sizeof(uint64_t),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "copy to host");
    for (int64_t i = 0; i < L; ++i)
        for (int64_t j = 0; j < L; ++j) {
            const int c = (int)((i + j) & 1);
            const int64_t n = i * H + (j >> 1);
            const uint64_t bit = (w[(size_t)(c * W + (n >> 6))] >> (n & 63)) & 1u;
            host_spins[i * L + j] = bit ? 1 : -1;
        }
    return ok();
}

int ising_set_spins(const ising_lattice *lat, const int8_t *host_spins, void *hip_stream)
{
    if (int e = check_lattice(lat))
        return e;
    if (!host_spins)
        return fail(ISING_E_BADARG, "null host buffer");
    const int64_t L = lat->L, H = L / 2, W = words_per_colour(L);
    std::vector<uint64_t> w((size_t)(2 * W), 0);
    for (int64_t i = 0; i < L; ++i)
        for (int64_t j = 0; j < L; ++j) {
            const int8_t v = host_spins[i * L + j];
            if (v != 1 && v != -1)
                return fail(ISING_E_BADARG, "spin (%lld, %lld) is %d, not +1/-1", (long long)i,
                            (long long)j, (int)v);
            if (v == 1) {
                const int c = (int)((i + j) & 1);
                const int64_t n = i * H + (j >> 1);
                w[(size_t)(c * W + (n >> 6))] |= 1ull << (n & 63);
            }
        }
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipMemcpyAsync(lat->words, w.data(), w.size() * sizeof(uint64_t),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "copy to device");
    return ok();
}

// ------------------------------------------------------------ +-J spin glass
namespace {

int check_glass(int64_t L)
{
    if (int e = check_L(L))
        return e;
    if (L % 128 != 0)
        return fail(ISING_E_SIZE, "the spin-glass sweep needs L %% 128 == 0 (L = %lld)",
                    (long long)L);
    return ISING_OK;
}

int check_bonds(const void *d_bonds, size_t bytes, int64_t L)
{
    if (!d_bonds)
        return fail(ISING_E_BADARG, "null bond array");
    if ((uintptr_t)d_bonds % 16 != 0) // the sweep reads two words at a time
        return fail(ISING_E_BADARG, "bond array must be 16-byte aligned");
    if (bytes < (size_t)(4 * words_per_colour(L)) * sizeof(uint64_t))
        return fail(ISING_E_SIZE, "bond array needs %lld bytes",
                    (long long)(4 * words_per_colour(L) * 8));
    return ISING_OK;
}

} // namespace

int ising_glass_bonds_init(uint64_t *d_bonds, size_t bytes, int64_t L, uint64_t seed,
                           uint32_t stream_id, void *hip_stream)
{
    if (int e = check_glass(L))
        return e;
    if (int e = check_bonds(d_bonds, bytes, L))
        return e;
    if (stream_id >= (1u << 24))
        return fail(ISING_E_BADARG, "stream_id must be < 2^24");
    hipError_t e = ising::launch_glass_bonds_init(d_bonds, L, seed, stream_id,
                                                  (hipStream_t)hip_stream);
    return e == hipSuccess ? ok() : hip_fail(e, "bond init launch");
}

int ising_glass_set_bonds(uint64_t *d_bonds, size_t bytes, int64_t L, const int8_t *host_right,
                          const int8_t *host_down, void *hip_stream)
{
    if (int e = check_glass(L))
        return e;
    if (int e = check_bonds(d_bonds, bytes, L))
        return e;
    if (!host_right || !host_down)
        return fail(ISING_E_BADARG, "null host bond array");
    const int64_t H = L / 2, W = words_per_colour(L);
    std::vector<uint64_t> w((size_t)(4 * W), 0);
    for (int64_t i = 0; i < L; ++i)
        for (int64_t j = 0; j < L; ++j) {
            const int8_t r = host_right[i * L + j], d = host_down[i * L + j];
            if ((r != 1 && r != -1) || (d != 1 && d != -1))
                return fail(ISING_E_BADARG, "bond at (%lld, %lld) is not +1/-1", (long long)i,
                            (long long)j);
            const int c = (int)((i + j) & 1);
            const int64_t n = i * H + (j >> 1);
            if (r < 0) // interleaved: word k of array x at 4 k + x
                w[(size_t)(4 * (n >> 6) + c)] |= 1ull << (n & 63);
            if (d < 0)
                w[(size_t)(4 * (n >> 6) + 2 + c)] |= 1ull << (n & 63);
        }
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipMemcpyAsync(d_bonds, w.data(), w.size() * sizeof(uint64_t),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    return e == hipSuccess ? ok() : hip_fail(e, "copy to device");
}

int ising_glass_sweep(const ising_lattice *lat, const uint64_t *d_bonds, size_t bond_bytes,
                      double beta, double J, int64_t nsweeps, uint64_t rng_counter,
                      void *hip_stream)
{
    if (int e = check_lattice(lat))
        return e;
    if (int e = check_glass(lat->L))
        return e;
    if (int e = check_bonds(d_bonds, bond_bytes, lat->L))
        return e;
    if (int e = check_temperature(beta, J))
        return e;
    if (nsweeps < 0)
        return fail(ISING_E_BADARG, "nsweeps must be >= 0");
    const ising::Metro2 m = ising::host::metro2_params(beta, J);
    hipStream_t s = (hipStream_t)hip_stream;
    for (int64_t sw = 0; sw < nsweeps; ++sw)
        for (int c = 0; c < 2; ++c) {
            const uint64_t t = 2 * (rng_counter + (uint64_t)sw) + (uint64_t)c;
            hipError_t e = ising::launch_glass_half_sweep(lat->words, d_bonds, lat->L, c, m, t,
                                                          lat->seed, lat->stream_id, s,
                                                          glass_variant());
            if (e != hipSuccess)
                return hip_fail(e, "half-sweep launch");
        }
    return ok();
}

int ising_glass_observables(const ising_lattice *lat, const uint64_t *d_bonds, size_t bond_bytes,
                            int64_t *d_bond, int64_t *d_mag, void *hip_stream)
{
    if (int e = check_lattice(lat))
        return e;
    if (int e = check_glass(lat->L))
        return e;
    if (int e = check_bonds(d_bonds, bond_bytes, lat->L))
        return e;
    if (!d_bond || !d_mag)
        return fail(ISING_E_BADARG, "null pointer");
    hipError_t e = ising::launch_glass_observables(lat->words, d_bonds, lat->L, d_bond, d_mag,
                                                   (hipStream_t)hip_stream);
    return e == hipSuccess ? ok() : hip_fail(e, "observables launch");
}

int ising_philox_rate(uint64_t nwords, uint32_t blocks_per_word, uint64_t seed,
                      uint32_t stream_id, uint64_t t, uint32_t *d_sink, uint32_t sink_words,
                      void *hip_stream)
{
    if (!d_sink || sink_words < 256 || sink_words % 256 != 0 || blocks_per_word < 1 ||
        blocks_per_word > 16 || nwords > (1ull << 32))
        return fail(ISING_E_BADARG, "need a sink of a multiple of 256 words, 1..16 blocks per "
                    "word and at most 2^32 words");
    hipError_t e = ising::launch_philox_rate(nwords, blocks_per_word, seed, stream_id, t, d_sink,
                                             sink_words, (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return hip_fail(e, "generator throughput launch");
    return ok();
}

int ising_set_sweep_kernel(int variant)
{
    if (variant < 0 || variant > 5)
        return fail(ISING_E_BADARG, "sweep kernel variant must be 0 to 5");
    g_variant = variant;
    return ok();
}

const char *ising_last_error(void) { return ising::host::last_error(); }

} // extern "C"
