// The random-number generator alone, for measurement (internal to libising).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"
#include "ising_rows.hpp"
#include "launch.hpp"

namespace ising {

// ------------------------------------------------- generator throughput
// The generator alone, with the sweep's counter layout (the lane-varying word
// index in counter word 3, every other word shared by the wavefront): each
// thread computes blocks q = 0..nq-1 for the word indices it is given and
// folds the outputs into one word, so no block is optimised away.  Its rate
// bounds every kernel that draws with the exact lazy compare.
__global__ __launch_bounds__(256) void k_philox_rate(uint64_t nwords, uint32_t nq, uint32_t key0,
                                                     uint32_t key1, uint32_t stream_id,
                                                     uint32_t t_lo, uint32_t t_hi,
                                                     uint32_t *__restrict__ sink)
{
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nthreads = (uint64_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    for (uint64_t k = tid; k < nwords; k += nthreads)
        for (uint32_t q = 0; q < nq; ++q) {
            const Block x = rows::philox_fast<rows::kCtrUniform>(
                ctr_word0(stream_id, kDomainSweep, q), t_lo, t_hi, (uint32_t)k, key0, key1);
            acc ^= rows::xor3(x.x0, x.x1, x.x2) ^ x.x3;
        }
    sink[tid] = acc;
}

hipError_t launch_philox_rate(uint64_t nwords, uint32_t nq, uint64_t seed, uint32_t stream_id,
                              uint64_t t, uint32_t *sink, uint32_t sink_words, hipStream_t s)
{
    hipLaunchKernelGGL(k_philox_rate, dim3(sink_words / 256), dim3(256), 0, s, nwords, nq,
                       (uint32_t)seed, (uint32_t)(seed >> 32), stream_id, (uint32_t)t,
                       (uint32_t)(t >> 32), sink);
    return hipGetLastError();
}

} // namespace ising
