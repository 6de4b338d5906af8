// Host-side launchers of the autoregressive-proposal kernels (internal).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "arnet.hpp"

namespace ising {
namespace arnet {

// log q~ (and the logits if `logits` is not null) of B configurations with
// every layer's activations in LDS, one workgroup per configuration; only
// where eval_supported() (two [L*L][C] bf16 buffers, the logits and the spins
// fit one workgroup's LDS).  Same results as launch_forward(), bit for bit.
bool eval_supported(int L, int C);
hipError_t launch_eval(const NetDev &net, const int8_t *x, int B, float *logits, float *logq,
                       hipStream_t s);

// Largest lattice the sampler takes: its longest anti-diagonal (ceil(L/2)
// sites) must fit four 16-row tiles.
constexpr int kSamplerMaxL = 128;

hipError_t launch_pack(const NetDev &net, hipStream_t s);
hipError_t launch_forward(const NetDev &net, const int8_t *x, int B, bf16 *const h[6],
                          float *logits, float *logq, hipStream_t s);
// LDS available to one workgroup on the current device.
size_t lds_limit();
// Whether the sampler can hold one configuration of an L x L, C-channel
// network in LDS (L <= kSamplerMaxL and the ring fits).
bool sampler_supported(int L, int C);
// Draws B configurations; `zout` receives their logits (B * L * L floats).
hipError_t launch_sample(const NetDev &net, int B, int8_t *x, float *zout, float *logq,
                         uint64_t seed, uint32_t stream_base, uint64_t round, hipStream_t s);
// Gradient of the mean NLL into `grad` and the loss into `loss`; `partial`
// holds kGradBlocks x (parameters + 1) floats.
hipError_t launch_backward(const NetDev &net, const int8_t *x, int B, bf16 *const h[6],
                           const float *logits, float *dlogit, float *dpre_a, float *dpre_b,
                           float *partial, float *grad, float *loss, hipStream_t s);
hipError_t launch_adam(float *params, const float *grad, float *m, float *v, int64_t n, float lr,
                       float beta1, float beta2, float eps, int64_t step, hipStream_t s);
hipError_t launch_spins_observables(const int8_t *x, int B, int L, int64_t *bond, int64_t *mag,
                                    hipStream_t s);
hipError_t launch_minibatch(const int8_t *pool, int64_t P, int L, int B, int8_t *out,
                           uint64_t seed, uint32_t stream_base, uint64_t round, hipStream_t s);
hipError_t launch_mh(int n, int N, int8_t *state, float *logq_cur, int64_t *bond_cur,
                     const int8_t *prop, const float *logq_prop, const int64_t *bond_prop,
                     const float *betaJ, uint64_t seed, uint32_t stream_base, uint64_t round,
                     int32_t *accepted, hipStream_t s);

} // namespace arnet
} // namespace ising
