// Masked-convolution autoregressive network over Ising configurations (the
// learned global proposal), gfx950: shared definitions of the kernels and the
// host side (internal to libising).
//
// Sites in raster order p = i*L + j.  Layer 1: 3x3 mask A (strictly earlier
// sites), 1 -> C, ReLU; layers 2..5: mask B (with the centre), C -> C, ReLU;
// layer 6: mask B, C -> 1 logit; zero padding.  q(x_p = +1 | x_<p) =
// sigmoid(logit_p).  Weights are stored in bfloat16, activations between
// layers in bfloat16, every sum in float32 (MFMA accumulators for layers
// 2..6).  The backward signal is float32; it enters the MFMA products as the
// sum of two bfloat16 halves (hi = bf16(v), lo = bf16(v - hi)).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ising {
namespace arnet {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Tap offsets (dy, dx); the first four form mask A, all five mask B.
__host__ __device__ inline int tap_dy(int t) { return t < 3 ? -1 : 0; }
__host__ __device__ inline int tap_dx(int t) { return t < 3 ? t - 1 : (t == 3 ? -1 : 0); }

// Offsets of the parameter blocks in the flat float32 vector
// W1[4][C], b1[C], (W_l[5][C][C], b_l[C]) l = 2..5, W6[5][C], b6.
struct ParamLayout {
    int64_t W1, b1, W[6], b[6], W6, b6, total;
};

__host__ __device__ inline ParamLayout param_layout(int C)
{
    ParamLayout p{};
    int64_t o = 0;
    p.W1 = o;
    o += 4 * C;
    p.b1 = o;
    o += C;
    for (int l = 2; l <= 5; ++l) {
        p.W[l] = o;
        o += 5 * (int64_t)C * C;
        p.b[l] = o;
        o += C;
    }
    p.W6 = o;
    o += 5 * C;
    p.b6 = o;
    o += 1;
    p.total = o;
    return p;
}

// Workgroups of the weight-gradient kernels (each a contiguous range of
// 64-row chunks); their per-workgroup sums are added in workgroup order by a
// separate kernel, so a gradient does not depend on scheduling.
constexpr int kGradBlocks = 256;

// Device-side network state: master float32 parameters and the packed
// copies the kernels read.
struct NetDev {
    int L, N, C;
    float *params;  // master parameters (ParamLayout)
    float *w1, *w6; // bf16-rounded first and last layer weights, float32 [4][C], [5][C]
    bf16 *wf[6];    // layer l forward operand: wf[l][co][t*C + ci] = W_l[t][ci][co]
    bf16 *wb[6];    // layer l data-gradient operand: wb[l][ci][t*C + co] = W_l[t][ci][co]
    bf16 *w6p;      // layer 6 as an MFMA operand of 16 columns: w6p[0][t*C + ci] = W6[t][ci], rest 0
};

// LDS bytes of one configuration in the sampler: a ring of ceil(L/2) + 2 rows
// x 4 column slots x 5 layers x C activations, and the L*L spins.
__host__ __device__ inline int sampler_ring_rows(int L) { return (L + 1) / 2 + 2; }
__host__ __device__ inline size_t sampler_lds_bytes(int L, int C)
{
    return (size_t)sampler_ring_rows(L) * 4 * 5 * C * sizeof(bf16) + (((size_t)L * L + 15) / 16) * 16;
}

} // namespace arnet
} // namespace ising
