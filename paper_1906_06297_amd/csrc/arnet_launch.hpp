// Host-side launchers of the autoregressive-proposal kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "arnet.hpp"

namespace ising {
namespace arnet {

hipError_t launch_pack(const NetDev &net, hipStream_t s);
hipError_t launch_forward(const NetDev &net, const int8_t *x, int B, bf16 *const h[6],
                          float *logits, float *logq, hipStream_t s);
hipError_t launch_sample(const NetDev &net, int B, bf16 *const h[6], int8_t *x, float *logq,
                         uint64_t seed, uint32_t stream_base, uint64_t round, hipStream_t s);
hipError_t launch_backward(const NetDev &net, const int8_t *x, int B, bf16 *const h[6],
                           const float *logits, float *dlogit, bf16 *dpre_a, bf16 *dpre_b,
                           float *grad, float *loss, hipStream_t s);
hipError_t launch_adam(float *params, const float *grad, float *m, float *v, int64_t n, float lr,
                       float beta1, float beta2, float eps, int64_t step, hipStream_t s);
hipError_t launch_spins_observables(const int8_t *x, int B, int L, int64_t *bond, int64_t *mag,
                                    hipStream_t s);
hipError_t launch_mh(int n, int N, int8_t *state, float *logq_cur, int64_t *bond_cur,
                     const int8_t *prop, const float *logq_prop, const int64_t *bond_prop,
                     const float *betaJ, uint64_t seed, uint32_t stream_base, uint64_t round,
                     int32_t *accepted, hipStream_t s);

} // namespace arnet
} // namespace ising
