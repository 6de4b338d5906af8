// C ABI of the matrix-multiply formulation (declared in include/ising.h).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ising.h"
#include "host_common.hpp"
#include "matmul.hpp"

namespace {

using ising::host::fail;
using ising::host::hip_fail;
using ising::host::ok;

int check_mm_L(int64_t L)
{
    if (int e = ising::host::check_L(L))
        return e;
    if (L % 256 != 0)
        return fail(ISING_E_SIZE, "the matrix-multiply sweep needs L %% 256 == 0 (L = %lld)",
                    (long long)L);
    return ISING_OK;
}

int check_buffer(const void *p, size_t bytes, int64_t need, const char *what)
{
    if (!p)
        return fail(ISING_E_BADARG, "null %s buffer", what);
    if ((uintptr_t)p % 16 != 0)
        return fail(ISING_E_BADARG, "%s buffer must be 16-byte aligned", what);
    if (bytes < (size_t)need)
        return fail(ISING_E_SIZE, "%s buffer needs %lld bytes", what, (long long)need);
    return ISING_OK;
}

} // namespace

extern "C" {

int64_t ising_mm_lattice_bytes(int64_t L)
{
    if (check_mm_L(L) != ISING_OK)
        return -1;
    return 2 * L * L;
}

int64_t ising_mm_sums_bytes(int64_t L)
{
    if (check_mm_L(L) != ISING_OK)
        return -1;
    return L * L;
}

int ising_mm_from_words(const ising_lattice *lat, uint16_t *d_spins, size_t bytes,
                        void *hip_stream)
{
    if (int e = ising::host::check_lattice(lat))
        return e;
    if (int e = check_mm_L(lat->L))
        return e;
    if (int e = check_buffer(d_spins, bytes, 2 * lat->L * lat->L, "spin"))
        return e;
    hipError_t e = ising::mm::launch_from_words(lat->words, d_spins, lat->L,
                                                (hipStream_t)hip_stream);
    return e == hipSuccess ? ok() : hip_fail(e, "layout conversion launch");
}

int ising_mm_to_words(const ising_lattice *lat, const uint16_t *d_spins, size_t bytes,
                      void *hip_stream)
{
    if (int e = ising::host::check_lattice(lat))
        return e;
    if (int e = check_mm_L(lat->L))
        return e;
    if (int e = check_buffer(d_spins, bytes, 2 * lat->L * lat->L, "spin"))
        return e;
    hipError_t e = ising::mm::launch_to_words(d_spins, lat->words, lat->L,
                                              (hipStream_t)hip_stream);
    return e == hipSuccess ? ok() : hip_fail(e, "layout conversion launch");
}

int ising_mm_sweep(int64_t L, uint64_t seed, uint32_t stream_id, uint16_t *d_spins,
                   size_t spin_bytes, uint16_t *d_sums, size_t sum_bytes, double beta, double J,
                   int64_t nsweeps, uint64_t rng_counter, int fused, void *hip_stream)
{
    if (int e = check_mm_L(L))
        return e;
    if (stream_id >= (1u << 24))
        return fail(ISING_E_BADARG, "stream_id must be < 2^24");
    if (int e = check_buffer(d_spins, spin_bytes, 2 * L * L, "spin"))
        return e;
    if (fused != 0 && fused != 1)
        return fail(ISING_E_BADARG, "fused must be 0 or 1");
    if (!fused)
        if (int e = check_buffer(d_sums, sum_bytes, L * L, "sum"))
            return e;
    if (int e = ising::host::check_temperature(beta, J))
        return e;
    if (nsweeps < 0)
        return fail(ISING_E_BADARG, "nsweeps must be >= 0");
    const ising::Metro2 m = ising::host::metro2_params(beta, J);
    hipStream_t s = (hipStream_t)hip_stream;
    for (int64_t sw = 0; sw < nsweeps; ++sw)
        for (int c = 0; c < 2; ++c) {
            const uint64_t t = 2 * (rng_counter + (uint64_t)sw) + (uint64_t)c;
            hipError_t e = ising::mm::launch_half_sweep(d_spins, d_sums, L, c, m, t, seed,
                                                        stream_id, fused != 0, s);
            if (e != hipSuccess)
                return hip_fail(e, "half-sweep launch");
        }
    return ok();
}

} // extern "C"
