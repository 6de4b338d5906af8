// C ABI of the learned global proposal (include/ising.h): the network object
// and its workspace, evaluation, gradients and Adam training, sampling, and
// the independence Metropolis-Hastings step.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/ising.h"
#include "arnet.hpp"
#include "arnet_launch.hpp"
#include "host_common.hpp"

using namespace ising;
using namespace ising::arnet;

struct ising_arnet {
    NetDev net{};
    int max_batch = 0;
    bf16 *h[6] = {};
    float *dpre_a = nullptr, *dpre_b = nullptr; // float32 backward signal
    float *partial = nullptr;                   // kGradBlocks x (parameters + 1)
    float *logits = nullptr, *dlogit = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    int64_t step = 0;
    int eval_mode = ISING_ARNET_EVAL_AUTO;
};

namespace {

void release(ising_arnet *a)
{
    void *ptrs[] = {a->net.params, a->net.w1, a->net.w6, a->net.w6p, a->dpre_a, a->dpre_b,
                    a->partial, a->logits, a->dlogit, a->grad, a->m, a->v};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    for (int l = 0; l < 6; ++l) {
        if (a->net.wf[l])
            (void)hipFree(a->net.wf[l]);
        if (a->net.wb[l])
            (void)hipFree(a->net.wb[l]);
        if (a->h[l])
            (void)hipFree(a->h[l]);
    }
}

int check_net(const ising_arnet *a) { return a ? ISING_OK : host::fail(ISING_E_BADARG, "null net"); }

int check_batch_size(const ising_arnet *a, int32_t B)
{
    if (B < 1 || B > a->max_batch)
        return host::fail(ISING_E_SIZE, "batch %d outside 1..%d", (int)B, a->max_batch);
    return ISING_OK;
}

// One Adam step on the master parameters with gradient g, then the packed
// weight copies.
int adam_and_pack(ising_arnet *a, const float *g, float lr, hipStream_t s)
{
    a->step += 1;
    hipError_t e = launch_adam(a->net.params, g, a->m, a->v, param_layout(a->net.C).total, lr,
                               0.9f, 0.999f, 1e-8f, a->step, s);
    if (e == hipSuccess)
        e = launch_pack(a->net, s);
    if (e != hipSuccess)
        return host::hip_fail(e, "Adam step");
    return host::ok();
}

} // namespace

extern "C" {

int64_t ising_arnet_num_params(int32_t channels)
{
    if (channels != 32 && channels != 64)
        return -1;
    return param_layout(channels).total;
}

int ising_arnet_create(ising_arnet **out, int32_t L, int32_t channels, int32_t max_batch)
{
    if (!out)
        return host::fail(ISING_E_BADARG, "null output");
    *out = nullptr;
    if (channels != 32 && channels != 64)
        return host::fail(ISING_E_BADARG, "channels must be 32 or 64");
    if (L < 2 || L > 1024 || max_batch < 1)
        return host::fail(ISING_E_BADARG, "need 2 <= L <= 1024 and max_batch >= 1");
    if ((int64_t)max_batch * L * L * channels >= (int64_t)1 << 31)
        return host::fail(ISING_E_SIZE, "max_batch * L^2 * channels must stay below 2^31");
    ising_arnet *a = new ising_arnet();
    a->net.L = L;
    a->net.N = L * L;
    a->net.C = channels;
    a->max_batch = max_batch;
    const int C = channels;
    const int64_t P = param_layout(C).total;
    const size_t act = (size_t)max_batch * a->net.N * C * sizeof(bf16);
    const size_t sig = (size_t)max_batch * a->net.N * C * sizeof(float);
    const size_t rowsf = (size_t)max_batch * a->net.N * sizeof(float);
    hipError_t e = hipMalloc(&a->net.params, P * 4);
    if (e == hipSuccess)
        e = hipMemset(a->net.params, 0, P * 4);
    if (e == hipSuccess)
        e = hipMalloc(&a->net.w1, 4 * C * 4);
    if (e == hipSuccess)
        e = hipMalloc(&a->net.w6, 5 * C * 4);
    if (e == hipSuccess)
        e = hipMalloc(&a->net.w6p, 16 * 5 * C * sizeof(bf16));
    for (int l = 2; l <= 5 && e == hipSuccess; ++l) {
        e = hipMalloc(&a->net.wf[l], 5 * C * C * sizeof(bf16));
        if (e == hipSuccess)
            e = hipMalloc(&a->net.wb[l], 5 * C * C * sizeof(bf16));
    }
    for (int l = 1; l <= 5 && e == hipSuccess; ++l)
        e = hipMalloc(&a->h[l], act);
    if (e == hipSuccess)
        e = hipMalloc(&a->dpre_a, sig);
    if (e == hipSuccess)
        e = hipMalloc(&a->dpre_b, sig);
    if (e == hipSuccess)
        e = hipMalloc(&a->partial, (size_t)kGradBlocks * (P + 1) * sizeof(float));
    if (e == hipSuccess)
        e = hipMalloc(&a->logits, rowsf);
    if (e == hipSuccess)
        e = hipMalloc(&a->dlogit, rowsf);
    if (e == hipSuccess)
        e = hipMalloc(&a->grad, P * 4);
    if (e == hipSuccess)
        e = hipMalloc(&a->m, P * 4);
    if (e == hipSuccess)
        e = hipMalloc(&a->v, P * 4);
    if (e == hipSuccess)
        e = hipMemset(a->m, 0, P * 4);
    if (e == hipSuccess)
        e = hipMemset(a->v, 0, P * 4);
    if (e == hipSuccess)
        e = launch_pack(a->net, nullptr);
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        release(a);
        delete a;
        return host::hip_fail(e, "network allocation");
    }
    *out = a;
    return host::ok();
}

int ising_arnet_destroy(ising_arnet *a)
{
    if (!a)
        return host::ok();
    release(a);
    delete a;
    return host::ok();
}

int ising_arnet_set_params(ising_arnet *a, const float *d_params, void *hip_stream)
{
    if (int e = check_net(a))
        return e;
    if (!d_params)
        return host::fail(ISING_E_BADARG, "null parameters");
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t P = param_layout(a->net.C).total;
    hipError_t e = hipMemcpyAsync(a->net.params, d_params, P * 4, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = launch_pack(a->net, s);
    if (e != hipSuccess)
        return host::hip_fail(e, "set parameters");
    return host::ok();
}

int ising_arnet_get_params(const ising_arnet *a, float *d_params, void *hip_stream)
{
    if (int e = check_net(a))
        return e;
    if (!d_params)
        return host::fail(ISING_E_BADARG, "null output");
    const int64_t P = param_layout(a->net.C).total;
    hipError_t e = hipMemcpyAsync(d_params, a->net.params, P * 4, hipMemcpyDeviceToDevice,
                                  (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return host::hip_fail(e, "get parameters");
    return host::ok();
}

int ising_arnet_log_prob(ising_arnet *a, const int8_t *d_spins, int32_t B, float *d_logq,
                         float *d_logits, void *hip_stream)
{
    if (int e = check_net(a))
        return e;
    if (int e = check_batch_size(a, B))
        return e;
    if (!d_spins || !d_logq)
        return host::fail(ISING_E_BADARG, "null pointer");
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e;
    if (a->eval_mode == ISING_ARNET_EVAL_AUTO && eval_supported(a->net.L, a->net.C)) {
        e = launch_eval(a->net, d_spins, B, d_logits, d_logq, s);
    } else {
        e = launch_forward(a->net, d_spins, B, a->h, a->logits, d_logq, s);
        if (e == hipSuccess && d_logits)
            e = hipMemcpyAsync(d_logits, a->logits, (size_t)B * a->net.N * 4,
                               hipMemcpyDeviceToDevice, s);
    }
    if (e != hipSuccess)
        return host::hip_fail(e, "log-probability");
    return host::ok();
}

int ising_arnet_set_eval_mode(ising_arnet *a, int32_t mode)
{
    if (int e = check_net(a))
        return e;
    if (mode != ISING_ARNET_EVAL_AUTO && mode != ISING_ARNET_EVAL_LAYERS)
        return host::fail(ISING_E_BADARG, "evaluation mode %d", (int)mode);
    a->eval_mode = mode;
    return host::ok();
}

int ising_arnet_gradient(ising_arnet *a, const int8_t *d_spins, int32_t B, float *d_grad,
                         float *d_loss, void *hip_stream)
{
    if (int e = check_net(a))
        return e;
    if (int e = check_batch_size(a, B))
        return e;
    if (!d_spins || !d_loss)
        return host::fail(ISING_E_BADARG, "null pointer");
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = launch_forward(a->net, d_spins, B, a->h, a->logits, nullptr, s);
    if (e == hipSuccess)
        e = launch_backward(a->net, d_spins, B, a->h, a->logits, a->dlogit, a->dpre_a, a->dpre_b,
                            a->partial, a->grad, d_loss, s);
    if (e == hipSuccess && d_grad)
        e = hipMemcpyAsync(d_grad, a->grad, param_layout(a->net.C).total * 4,
                           hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess)
        return host::hip_fail(e, "gradient");
    return host::ok();
}

int ising_arnet_gradient_at(ising_arnet *a, const int8_t *d_spins, int32_t B,
                            const uint16_t *d_acts, const float *d_logits, float *d_grad,
                            float *d_loss, void *hip_stream)
{
    if (int e = check_net(a))
        return e;
    if (int e = check_batch_size(a, B))
        return e;
    if (!d_spins || !d_acts || !d_logits || !d_loss)
        return host::fail(ISING_E_BADARG, "null pointer");
    hipStream_t s = (hipStream_t)hip_stream;
    const size_t per = (size_t)B * a->net.N * a->net.C;
    hipError_t e = hipSuccess;
    for (int l = 1; l <= 5 && e == hipSuccess; ++l)
        e = hipMemcpyAsync(a->h[l], d_acts + (size_t)(l - 1) * per, per * sizeof(bf16),
                           hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(a->logits, d_logits, (size_t)B * a->net.N * sizeof(float),
                           hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = launch_backward(a->net, d_spins, B, a->h, a->logits, a->dlogit, a->dpre_a, a->dpre_b,
                            a->partial, a->grad, d_loss, s);
    if (e == hipSuccess && d_grad)
        e = hipMemcpyAsync(d_grad, a->grad, param_layout(a->net.C).total * 4,
                           hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess)
        return host::hip_fail(e, "gradient at given activations");
    return host::ok();
}

int ising_arnet_train_step(ising_arnet *a, const int8_t *d_spins, int32_t B, float lr,
                           float *d_loss, void *hip_stream)
{
    if (!(lr > 0.f) || !std::isfinite(lr))
        return host::fail(ISING_E_BADARG, "learning rate must be finite and > 0");
    if (int e = ising_arnet_gradient(a, d_spins, B, nullptr, d_loss, hip_stream))
        return e;
    return adam_and_pack(a, a->grad, lr, (hipStream_t)hip_stream);
}

int ising_arnet_adam(ising_arnet *a, const float *d_grad, float lr, void *hip_stream)
{
    if (int e = check_net(a))
        return e;
    if (!d_grad)
        return host::fail(ISING_E_BADARG, "null gradient");
    if (!(lr > 0.f) || !std::isfinite(lr))
        return host::fail(ISING_E_BADARG, "learning rate must be finite and > 0");
    return adam_and_pack(a, d_grad, lr, (hipStream_t)hip_stream);
}

int ising_arnet_sample(ising_arnet *a, int32_t B, uint64_t seed, uint32_t stream_base,
                       uint64_t round, int8_t *d_spins, float *d_logq, void *hip_stream)
{
    if (int e = check_net(a))
        return e;
    if (int e = check_batch_size(a, B))
        return e;
    if (!d_spins || !d_logq)
        return host::fail(ISING_E_BADARG, "null pointer");
    if ((uint64_t)stream_base + (uint64_t)B > (1ull << 24))
        return host::fail(ISING_E_BADARG, "stream_base + B must not exceed 2^24");
    if (!sampler_supported(a->net.L, a->net.C))
        return host::fail(ISING_E_SIZE,
                          "the sampler holds a configuration in LDS: L <= %d and %zu bytes (L = %d, "
                          "C = %d needs %zu)",
                          kSamplerMaxL, lds_limit(), a->net.L, a->net.C,
                          sampler_lds_bytes(a->net.L, a->net.C));
    hipError_t e = launch_sample(a->net, B, d_spins, a->logits, d_logq, seed, stream_base, round,
                                 (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return host::hip_fail(e, "sample");
    return host::ok();
}

int ising_spins_observables(const int8_t *d_spins, int32_t B, int64_t L, int64_t *d_bond,
                            int64_t *d_mag, void *hip_stream)
{
    if (!d_spins || !d_bond || !d_mag || B < 1 || L < 2 || L > 65536)
        return host::fail(ISING_E_BADARG, "null pointer or bad size");
    hipError_t e = launch_spins_observables(d_spins, B, (int)L, d_bond, d_mag,
                                            (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return host::hip_fail(e, "observables of configurations");
    return host::ok();
}

int ising_spins_minibatch(const int8_t *d_pool, int64_t P, int64_t L, int32_t B, uint64_t seed,
                          uint32_t stream_base, uint64_t round, int8_t *d_out, void *hip_stream)
{
    if (!d_pool || !d_out || P < 1 || B < 1 || L < 2 || L > 1024)
        return host::fail(ISING_E_BADARG, "null pointer or bad size");
    if ((uint64_t)stream_base + (uint64_t)B > (1ull << 24))
        return host::fail(ISING_E_BADARG, "stream_base + B must not exceed 2^24");
    hipError_t e = launch_minibatch(d_pool, P, (int)L, B, d_out, seed, stream_base, round,
                                    (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return host::hip_fail(e, "minibatch");
    return host::ok();
}

int ising_mh_independence(int32_t n, int64_t L, int8_t *d_state, float *d_logq, int64_t *d_bond,
                          const int8_t *d_prop, const float *d_logq_prop,
                          const int64_t *d_bond_prop, const float *d_betaJ, uint64_t seed,
                          uint32_t stream_base, uint64_t round, int32_t *d_accepted,
                          void *hip_stream)
{
    if (n < 1 || L < 2 || L > 65536 || !d_state || !d_logq || !d_bond || !d_prop ||
        !d_logq_prop || !d_bond_prop || !d_betaJ || !d_accepted)
        return host::fail(ISING_E_BADARG, "null pointer or bad size");
    if ((uint64_t)stream_base + (uint64_t)n > (1ull << 24))
        return host::fail(ISING_E_BADARG, "stream_base + n must not exceed 2^24");
    hipError_t e = launch_mh(n, (int)(L * L), d_state, d_logq, d_bond, d_prop, d_logq_prop,
                             d_bond_prop, d_betaJ, seed, stream_base, round, d_accepted,
                             (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return host::hip_fail(e, "Metropolis-Hastings step");
    return host::ok();
}

} // extern "C"
