// gfx950 kernels of the masked-convolution autoregressive proposal: forward
// evaluation (log q of given configurations), ancestral sampling along
// anti-diagonals, backward pass and Adam, independence Metropolis-Hastings,
// and the observables of int8 configurations.
//
// Layers 2..6 run on bf16 MFMA (v_mfma_f32_16x16x32_bf16, float32
// accumulators) through one routine, conv_mfma(), which computes 16 rows x
// NOUT outputs of a masked 3x3 convolution from the five taps of each row; a
// row is a (configuration, site) pair.  The evaluator feeds it 16 consecutive
// sites, the sampler 16 sites of one anti-diagonal of one configuration, and
// an MFMA output element depends only on its own row of operands, so every
// conditional the sampler draws from is bit for bit the evaluator's -- the
// Metropolis-Hastings ratio then uses the exact probability with which a
// proposal was drawn.
//
// The backward pass keeps its signal in float32 and feeds it to the MFMA
// products as two bfloat16 halves; weight gradients are summed per workgroup
// over fixed row ranges and the workgroup sums added in workgroup order, so
// training is reproducible run to run.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "arnet.hpp"
#include "arnet_launch.hpp"
#include "ising_device.hpp"

namespace ising {
namespace arnet {

__device__ __forceinline__ float round_bf16(float v) { return (float)(bf16)v; }

// ------------------------------------------------------------ weight packing
__global__ __launch_bounds__(256) void k_pack(NetDev net)
{
    const int C = net.C;
    const ParamLayout pl = param_layout(C);
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < 16 * 5 * C) { // the 15 zero columns of layer 6's MFMA operand
        const int n = (int)(g / (5 * C));
        if (n > 0)
            net.w6p[g] = (bf16)0.f;
    }
    if (g >= pl.total)
        return;
    const float v = net.params[g];
    if (g >= pl.W1 && g < pl.W1 + 4 * C) {
        net.w1[g - pl.W1] = round_bf16(v);
        return;
    }
    if (g >= pl.W6 && g < pl.W6 + 5 * C) {
        net.w6[g - pl.W6] = round_bf16(v);
        net.w6p[g - pl.W6] = (bf16)v; // row 0: [t*C + ci]
        return;
    }
    for (int l = 2; l <= 5; ++l) {
        if (g >= pl.W[l] && g < pl.W[l] + 5 * (int64_t)C * C) {
            const int64_t idx = g - pl.W[l];
            const int t = (int)(idx / ((int64_t)C * C));
            const int ci = (int)((idx / C) % C), co = (int)(idx % C);
            const bf16 h = (bf16)v;
            net.wf[l][(int64_t)co * 5 * C + t * C + ci] = h;
            net.wb[l][(int64_t)ci * 5 * C + t * C + co] = h;
            return;
        }
    }
}

// ------------------------------------------------- per-row shared functions
// Layer 1 (mask A, one input channel): output channel c from the spins at the
// four mask-A taps (0 outside the lattice).
__device__ __forceinline__ float l1_from(const float (&xv)[4], const float *w1, const float *b1,
                                         int C, int c)
{
    float acc = 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        acc = fmaf(xv[t], w1[t * C + c], acc);
    return round_bf16(fmaxf(acc + b1[c], 0.f));
}

__device__ __forceinline__ float prob_plus(float z) { return 1.f / (1.f + expf(-z)); }

// Realised probability of +1 when x = +1 iff a 24-bit uniform u < P.
__device__ __forceinline__ float quantise(float P) { return ceilf(P * 16777216.f) * (1.f / 16777216.f); }

__device__ __forceinline__ double site_logq(float Pq, int xv)
{
    return xv > 0 ? log((double)Pq) : log1p(-(double)Pq);
}

// log q~ of one configuration from its logits, computed by a whole wavefront:
// lane l adds the sites p = l, l + 64, ... in increasing order, then the 64
// lane sums are combined by a butterfly (offsets 32, 16, .., 1).  Evaluator
// and sampler both use it, so their results agree bit for bit.
// The summation of config_logq() over terms given by term(p).
template <class Term>
__device__ __forceinline__ double wave_ordered_sum(int N, const Term &term)
{
    const int lane = threadIdx.x & 63;
    double acc = 0.0;
    for (int p = lane; p < N; p += 64)
        acc += term(p);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        acc += __shfl_xor(acc, off, 64);
    return acc;
}

__device__ __forceinline__ double site_term(const float *z, const int8_t *x, int p)
{
    return site_logq(quantise(prob_plus(z[p])), x[p]);
}

__device__ __forceinline__ double config_logq(const float *z, const int8_t *x, int N)
{
    return wave_ordered_sum(N, [&](int p) { return site_term(z, x, p); });
}

// ------------------------------------------------------------- MFMA tile
// Rows of a tile: a row is valid when b >= 0.  Row indices are below 2^31
// (a workspace holds at most 2^31 / C rows), so the division is 32-bit.
struct RowsOfSites { // 16 consecutive flattened (configuration, site) rows
    int64_t g0, total;
    int N;
    __device__ void operator()(int r, int64_t &b, int &p) const
    {
        const int64_t g = g0 + r;
        if (g >= total) {
            b = -1;
            p = 0;
            return;
        }
        const uint32_t bq = (uint32_t)g / (uint32_t)N;
        b = bq;
        p = (int)((uint32_t)g - bq * (uint32_t)N);
    }
};

// The four rows of a tile that one lane writes in conv_mfma()'s epilogue
// (kq*4 + q, q = 0..3), found once per tile rather than at every output
// block.
struct LaneRows {
    int64_t b[4];
    int p[4];
    template <class Rows>
    __device__ LaneRows(const Rows &rows, int kq)
    {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            rows(kq * 4 + q, b[q], p[q]);
    }
    __device__ void operator()(int row, int64_t &bb, int &pp) const
    {
        bb = b[row & 3];
        pp = p[row & 3];
    }
};

// The MFMA part of a masked 3x3 convolution tile: with the A operands of the
// five taps in registers (a[t][kc]: row lane & 15, k = kc*32 + (lane >> 4)*8
// + e), acc(row, n) = sum_t sum_k a[t][k] * w[n][t*C + k], accumulated over
// t = 0..4 and 32-wide k chunks in that order, then handed to the epilogue,
// for NOUT output columns in blocks of 16.  `bop(n0, t, kc)` yields the B
// operand (weights) of that step.
template <int C, int NOUT, class BOp, class Rows, class Epi>
__device__ __forceinline__ void conv_mfma(const bf16x8 (&a)[5][C / 32], const BOp &bop,
                                          const Rows &rows, const Epi &epi)
{
    constexpr int KC = C / 32;
    const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int n0 = 0; n0 < NOUT; n0 += 16) {
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 5; ++t)
#pragma unroll
            for (int kc = 0; kc < KC; ++kc)
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[t][kc], bop(n0, t, kc), acc, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int64_t bb;
            int pp;
            rows(kq * 4 + q, bb, pp);
            if (bb >= 0)
                epi(kq * 4 + q, bb, pp, n0 + r, acc[q]);
        }
    }
}

// The same contraction with each A operand the sum of two bf16 halves
// (backward signal): per step the high half, then the low half.
template <int C, int NOUT, class BOp, class Rows, class Epi>
__device__ __forceinline__ void conv_mfma_split(const bf16x8 (&ah)[5][C / 32],
                                                const bf16x8 (&al)[5][C / 32], const BOp &bop,
                                                const Rows &rows, const Epi &epi)
{
    constexpr int KC = C / 32;
    const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int n0 = 0; n0 < NOUT; n0 += 16) {
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 5; ++t)
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                const bf16x8 w = bop(n0, t, kc);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[t][kc], w, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[t][kc], w, acc, 0, 0, 0);
            }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int64_t bb;
            int pp;
            rows(kq * 4 + q, bb, pp);
            if (bb >= 0)
                epi(kq * 4 + q, bb, pp, n0 + r, acc[q]);
        }
    }
}

// B operands read from packed weights ([n][t*C + k], 5C per column n).
template <int C>
struct WeightsGlobal {
    const bf16 *wk;
    __device__ bf16x8 operator()(int n0, int t, int kc) const
    {
        const int lane = threadIdx.x & 63;
        return *(const bf16x8 *)(wk + (int64_t)(n0 + (lane & 15)) * 5 * C + (lane >> 4) * 8 + t * C +
                                 kc * 32);
    }
};

// The same operands held in registers (NOUT / 16 x 5 x C / 32 per lane).
template <int C, int NOUT>
struct WeightsRegs {
    bf16x8 w[NOUT / 16][5][C / 32];
    __device__ void load(const bf16 *wk)
    {
        const WeightsGlobal<C> g{wk};
#pragma unroll
        for (int n = 0; n < NOUT / 16; ++n)
#pragma unroll
            for (int t = 0; t < 5; ++t)
#pragma unroll
                for (int kc = 0; kc < C / 32; ++kc)
                    w[n][t][kc] = g(16 * n, t, kc);
    }
    __device__ bf16x8 operator()(int n0, int t, int kc) const { return w[n0 / 16][t][kc]; }
};

__device__ __forceinline__ void zero8(bf16x8 &v)
{
#pragma unroll
    for (int e = 0; e < 8; ++e)
        v[e] = (bf16)0.f;
}

// Eight bf16 values from p, or zeros where !ok, moved as one 128-bit integer
// vector (as bf16 elements the compiler rebuilds the vector 16 bits at a
// time around the branch).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ bf16x8 load8_or_zero(bool ok, const bf16 *p)
{
    u32x4 v = {0u, 0u, 0u, 0u};
    if (ok)
        v = *(const u32x4 *)p;
    return __builtin_bit_cast(bf16x8, v);
}

// A operand of tap t of a tile row (configuration b, site (ii, jj) of the
// tap) from an activation array: zero outside the lattice (zero padding).
template <int C>
__device__ __forceinline__ void load_tap(bf16x8 (&at)[C / 32], const bf16 *__restrict__ in,
                                         int64_t b, int N, int L, int ii, int jj, int kq)
{
    const bool ok = b >= 0 && ii >= 0 && ii < L && jj >= 0 && jj < L;
#pragma unroll
    for (int kc = 0; kc < C / 32; ++kc)
        at[kc] = load8_or_zero(ok, in + ((int64_t)b * N + ii * L + jj) * C + kc * 32 + kq * 8);
}

// The same from a float32 backward signal, split into bf16 halves.
template <int C>
__device__ __forceinline__ void load_tap_split(bf16x8 (&hi)[C / 32], bf16x8 (&lo)[C / 32],
                                               const float *__restrict__ in, int64_t b, int N, int L,
                                               int ii, int jj, int kq)
{
    const bool ok = b >= 0 && ii >= 0 && ii < L && jj >= 0 && jj < L;
#pragma unroll
    for (int kc = 0; kc < C / 32; ++kc) {
        if (ok) {
            const float *src = in + ((int64_t)b * N + ii * L + jj) * C + kc * 32 + kq * 8;
            const float4 v0 = *(const float4 *)src, v1 = *(const float4 *)(src + 4);
            const float v[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const bf16 h = (bf16)v[e];
                hi[kc][e] = h;
                lo[kc][e] = (bf16)(v[e] - (float)h);
            }
        } else {
            zero8(hi[kc]);
            zero8(lo[kc]);
        }
    }
}

struct EpiForward { // post-ReLU bf16 activation
    bf16 *out;
    const float *bias;
    int N, C;
    __device__ void operator()(int, int64_t b, int p, int col, float v) const
    {
        out[((int64_t)b * N + p) * C + col] = (bf16)fmaxf(v + bias[col], 0.f);
    }
};

struct EpiLogit { // layer 6: column 0 of the padded product is the logit
    float *z;
    float b6;
    int N;
    __device__ void operator()(int, int64_t b, int p, int col, float v) const
    {
        if (col == 0)
            z[(int64_t)b * N + p] = v + b6;
    }
};

struct EpiBackward { // float32 data gradient masked by the ReLU of the layer below
    float *out;
    const bf16 *act;
    int N, C;
    __device__ void operator()(int, int64_t b, int p, int col, float v) const
    {
        const int64_t o = ((int64_t)b * N + p) * C + col;
        out[o] = (float)act[o] > 0.f ? v : 0.f;
    }
};

// ---------------------------------------------------------------- forward
// Layer 1: one thread per (row, 8 output channels), one 16-byte store.
__global__ __launch_bounds__(256) void k_l1_fwd(NetDev net, const int8_t *__restrict__ x,
                                                bf16 *__restrict__ h1, int64_t rows_total)
{
    const int C = net.C, CG = C / 8;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= rows_total * CG)
        return;
    const int N = net.N, L = net.L;
    const int64_t row = g / CG;
    const int c0 = (int)(g - row * CG) * 8;
    const int64_t b = row / N;
    const int p = (int)(row - b * N), i = p / L, j = p - (p / L) * L;
    float xv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int ii = i + tap_dy(t), jj = j + tap_dx(t);
        xv[t] = (ii >= 0 && jj >= 0 && jj < L) ? (float)x[b * N + ii * L + jj] : 0.f;
    }
    const float *b1 = net.params + param_layout(C).b1;
    bf16x8 out;
#pragma unroll
    for (int e = 0; e < 8; ++e)
        out[e] = (bf16)l1_from(xv, net.w1, b1, C, c0 + e);
    *(bf16x8 *)(h1 + row * C + c0) = out;
}

template <int C>
__global__ __launch_bounds__(256) void k_conv_fwd(const bf16 *__restrict__ in, bf16 *__restrict__ out,
                                                  const bf16 *__restrict__ wk,
                                                  const float *__restrict__ bias, int L, int N,
                                                  int64_t rows_total)
{
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile * 16 >= rows_total)
        return;
    const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
    const RowsOfSites rows{tile * 16, rows_total, N};
    int64_t b;
    int p;
    rows(r, b, p);
    const int i = p / L, j = p - (p / L) * L;
    bf16x8 a[5][C / 32];
#pragma unroll
    for (int t = 0; t < 5; ++t)
        load_tap<C>(a[t], in, b, N, L, i + tap_dy(t), j + tap_dx(t), kq);
    conv_mfma<C, C>(a, WeightsGlobal<C>{wk}, LaneRows(rows, kq), EpiForward{out, bias, N, C});
}

// Layer 6 on MFMA: the weights as one 16-column operand whose column 0 is W6.
template <int C>
__global__ __launch_bounds__(256) void k_l6_fwd(NetDev net, const bf16 *__restrict__ h5,
                                                float *__restrict__ logits, int64_t rows_total)
{
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile * 16 >= rows_total)
        return;
    const int N = net.N, L = net.L;
    const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
    const RowsOfSites rows{tile * 16, rows_total, N};
    int64_t b;
    int p;
    rows(r, b, p);
    const int i = p / L, j = p - (p / L) * L;
    bf16x8 a[5][C / 32];
#pragma unroll
    for (int t = 0; t < 5; ++t)
        load_tap<C>(a[t], h5, b, N, L, i + tap_dy(t), j + tap_dx(t), kq);
    const float b6 = net.params[param_layout(C).b6];
    conv_mfma<C, 16>(a, WeightsGlobal<C>{net.w6p}, LaneRows(rows, kq), EpiLogit{logits, b6, N});
}

// Exact log-probability of each configuration under the sampler, one
// wavefront per configuration.
__global__ __launch_bounds__(256) void k_logq(const int8_t *__restrict__ x,
                                              const float *__restrict__ logits, int N, int B,
                                              float *__restrict__ logq)
{
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (b >= B)
        return;
    const double lq = config_logq(logits + (int64_t)b * N, x + (int64_t)b * N, N);
    if ((threadIdx.x & 63) == 0)
        logq[b] = (float)lq;
}

// ------------------------------------------------------- fused evaluator
// log q~ of whole configurations, one workgroup per configuration with every
// layer's activations in LDS (two [N][C] bf16 buffers, the logits and the
// spins): the seven launches of the evaluator above move each layer's
// activations through HBM, this one reads the spins and writes log q~ (and
// the logits if asked).  The per-element arithmetic is the evaluator's:
// layer 1 by l1_from(), layers 2..6 by conv_mfma() over 16-site tiles with the
// same operands (the weights loaded once per layer into registers from the
// same packed arrays), the epilogues' bias, ReLU and bf16 rounding, and
// config_logq() on the logits -- so its results equal the evaluator's, and
// the sampler's, bit for bit.

// Tile rows within one configuration: sites p0 .. p0 + 15 (valid below N).
struct CfgRows {
    int p0, N;
    __device__ void operator()(int r, int64_t &b, int &p) const
    {
        p = p0 + r;
        b = p < N ? 0 : -1;
        if (b < 0)
            p = 0;
    }
};

// A operand of tap t from the configuration's activations in LDS.
template <int C>
__device__ __forceinline__ void load_tap_lds(bf16x8 (&at)[C / 32], const bf16 *act, bool valid,
                                             int L, int ii, int jj, int kq)
{
    const bool ok = valid && ii >= 0 && ii < L && jj >= 0 && jj < L;
#pragma unroll
    for (int kc = 0; kc < C / 32; ++kc)
        at[kc] = load8_or_zero(ok, act + (ii * L + jj) * C + kc * 32 + kq * 8);
}

// As EpiForward, into the LDS buffer of the next layer, with the lane's
// biases in registers (a lane's output columns are n0 + (lane & 15)).
template <int C>
struct EpiForwardLds {
    bf16 *out;
    float bias[C / 16]; // bias[col >> 4] of this lane's column col
    __device__ void operator()(int, int64_t, int p, int col, float v) const
    {
        out[p * C + col] = (bf16)fmaxf(v + bias[col >> 4], 0.f);
    }
};

struct EpiLogitLds { // as EpiLogit, into the LDS logits
    float *z;
    float b6;
    __device__ void operator()(int, int64_t, int p, int col, float v) const
    {
        if (col == 0)
            z[p] = v + b6;
    }
};

// LDS of one configuration: two [N][C] bf16 activation buffers, the logits
// (float), the spins (padded to 16 bytes) and the per-site log q terms
// (double).
__host__ __device__ inline size_t eval_terms_offset(int N, int C)
{
    return ((2 * (size_t)N * C * sizeof(bf16) + (size_t)N * sizeof(float) + (size_t)N + 15) / 16) * 16;
}

__host__ __device__ inline size_t eval_lds_bytes(int N, int C)
{
    return eval_terms_offset(N, C) + (size_t)N * sizeof(double);
}

// One configuration's evaluation by the workgroup: spins xs (staged in LDS),
// activations act[0], act[1], logits z; layer weights from `wl(l)`.
template <int C, int W, class WL>
__device__ __forceinline__ void eval_config(const NetDev &net, const int8_t *xs, bf16 *const (&act)[2],
                                            float *z, const WL &wl)
{
    const int N = net.N, L = net.L;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, r = lane & 15, kq = lane >> 4;
    const ParamLayout pl = param_layout(C);
    // layer 1: one thread per (site, 8 output channels)
    const float *b1 = net.params + pl.b1;
    for (int g = tid; g < N * (C / 8); g += 64 * W) {
        const int p = g / (C / 8), c0 = (g - p * (C / 8)) * 8;
        const int i = p / L, j = p - (p / L) * L;
        float xv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int ii = i + tap_dy(t), jj = j + tap_dx(t);
            xv[t] = (ii >= 0 && jj >= 0 && jj < L) ? (float)xs[ii * L + jj] : 0.f;
        }
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e)
            o[e] = (bf16)l1_from(xv, net.w1, b1, C, c0 + e);
        *(bf16x8 *)(act[0] + p * C + c0) = o;
    }
    __syncthreads();
    const int tiles = (N + 15) / 16;
    // layers 2..5: act[(l - 2) & 1] -> act[(l - 1) & 1]
#pragma unroll
    for (int l = 2; l <= 5; ++l) {
        const bf16 *in = act[(l - 2) & 1];
        EpiForwardLds<C> epi;
        epi.out = act[(l - 1) & 1];
#pragma unroll
        for (int k = 0; k < C / 16; ++k)
            epi.bias[k] = net.params[pl.b[l] + 16 * k + r];
        const auto &w = wl(l);
        for (int tile = wv; tile < tiles; tile += W) {
            const CfgRows rows{tile * 16, N};
            int64_t bb;
            int p;
            rows(r, bb, p);
            const int i = p / L, j = p - (p / L) * L;
            bf16x8 a[5][C / 32];
#pragma unroll
            for (int t = 0; t < 5; ++t)
                load_tap_lds<C>(a[t], in, bb >= 0, L, i + tap_dy(t), j + tap_dx(t), kq);
            conv_mfma<C, C>(a, w, rows, epi);
        }
        __syncthreads();
    }
    // layer 6 from act[0] (layer 5's output)
    const EpiLogitLds epi6{z, net.params[pl.b6]};
    WeightsRegs<C, 16> w6;
    w6.load(net.w6p);
    for (int tile = wv; tile < tiles; tile += W) {
        const CfgRows rows{tile * 16, N};
        int64_t bb;
        int p;
        rows(r, bb, p);
        const int i = p / L, j = p - (p / L) * L;
        bf16x8 a[5][C / 32];
#pragma unroll
        for (int t = 0; t < 5; ++t)
            load_tap_lds<C>(a[t], act[0], bb >= 0, L, i + tap_dy(t), j + tap_dx(t), kq);
        conv_mfma<C, 16>(a, w6, rows, epi6);
    }
    __syncthreads();
}

// Weights of layers 2..5 held in registers for the whole launch (C = 32:
// 160 of them per lane) ...
template <int C>
struct HeldWeights {
    WeightsRegs<C, C> w[4];
    __device__ void load(const NetDev &net)
    {
#pragma unroll
        for (int l = 2; l <= 5; ++l)
            w[l - 2].load(net.wf[l]);
    }
    __device__ const WeightsRegs<C, C> &operator()(int l) const { return w[l - 2]; }
};

// ... or read from the packed arrays at each use (C = 64).
template <int C>
struct GlobalWeights {
    const bf16 *wf[6];
    __device__ WeightsGlobal<C> operator()(int l) const { return WeightsGlobal<C>{wf[l]}; }
};

// Persistent: workgroup g evaluates configurations g, g + grid, ...
template <int C, int W>
__global__ __launch_bounds__(64 * W) void k_eval(NetDev net, const int8_t *__restrict__ x, int B,
                                                 float *__restrict__ logits, float *__restrict__ logq)
{
    extern __shared__ __align__(16) unsigned char eval_lds[];
    const int N = net.N;
    bf16 *const act[2] = {(bf16 *)eval_lds, (bf16 *)eval_lds + (size_t)N * C};
    float *z = (float *)(act[1] + (size_t)N * C);
    int8_t *xs = (int8_t *)(z + N);
    double *terms = (double *)(eval_lds + eval_terms_offset(N, C));
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    constexpr bool kHold = C == 32;
    HeldWeights<kHold ? C : 32> held;
    if constexpr (kHold)
        held.load(net);
    for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
        for (int p = tid; p < N; p += 64 * W)
            xs[p] = x[b * N + p];
        __syncthreads();
        if constexpr (kHold)
            eval_config<C, W>(net, xs, act, z, held);
        else
            eval_config<C, W>(net, xs, act, z,
                              GlobalWeights<C>{{net.wf[0], net.wf[1], net.wf[2], net.wf[3], net.wf[4],
                                                net.wf[5]}});
        // log q~: the per-site terms of config_logq() by every wavefront, then
        // its summation, in its order, by one
        for (int p = tid; p < N; p += 64 * W) {
            terms[p] = site_term(z, xs, p);
            if (logits)
                logits[b * N + p] = z[p];
        }
        __syncthreads();
        if (wv == 0) {
            const double lq = wave_ordered_sum(N, [&](int p) { return terms[p]; });
            if (lane == 0)
                logq[b] = (float)lq;
        }
        __syncthreads(); // z, xs and the terms are rewritten by the next configuration
    }
}

// --------------------------------------------------------------- sampling
// Ancestral sampling along anti-diagonals.  Through the masks, every layer's
// output at site (i, j) depends only on sites (i-1, j-1..j+1) and (i, j-1) of
// the layer below (and (i, j) itself for mask B), so the six layers and the
// draw of (i, j) need exactly the sites (i-1, j+1) and (i, j-1) finished:
// at step t the kernel draws every site with j + 2i = t, all of whose
// prerequisites belong to step t-1.  A configuration takes 3L - 2 steps
// instead of L^2.
//
// One workgroup per configuration, W wavefronts, each a 16-row MFMA tile of
// sites of the current diagonal.  Activations live in LDS in a ring of rows
// (row i at slot i mod R, R = ceil(L/2) + 2 rows: the active diagonal spans
// at most ceil(L/2) rows plus the one above) with 4 column slots (j mod 4):
// at step t row i writes column j while its own step and row i+1's read
// columns j-3 .. j-1, so column j-4 is free.  Spins are kept whole in LDS.
// Each site draws with a 24-bit uniform of Philox domain 3,
//   counter (stream<<8 | 3<<4, round lo, round hi, p>>2), word p&3;
// its logit goes to `zout` and log q~ is summed from there as by the
// evaluator.
template <int C>
struct SamplerRows { // tile row -> (configuration, index on the diagonal)
    int64_t b;
    int s0, nsites;
    __device__ void operator()(int r, int64_t &bb, int &s) const
    {
        s = s0 + r;
        bb = s < nsites ? b : -1;
    }
};

// Post-ReLU bf16 activation into the ring: `slot[q]` is the element offset
// in `ring` of the entry of this lane's output row kq*4 + q (32-bit offsets,
// not pointers: half the registers), `bias[n]` the bias of its column
// n*16 + r.
template <int C>
struct EpiRing {
    bf16 *ring;
    const int (&slot)[4];
    const float (&bias)[C / 16];
    int layer;
    __device__ void operator()(int row, int64_t, int, int col, float v) const
    {
        ring[slot[row & 3] + layer * C + col] = (bf16)fmaxf(v + bias[col >> 4], 0.f);
    }
};

struct EpiZ { // logit of the diagonal's site s
    float *zs;
    float b6;
    __device__ void operator()(int, int64_t, int s, int col, float v) const
    {
        if (col == 0)
            zs[s] = v + b6;
    }
};

// Orders LDS accesses between the steps of the sampler: a wavefront's own
// LDS operations complete in order, so one wavefront needs only the fence;
// several meet at a barrier.  Global stores are not waited for.
template <int W>
__device__ __forceinline__ void lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    if (W > 1)
        __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int C, int W>
__global__ __launch_bounds__(64 * W) void k_sample(NetDev net, int8_t *__restrict__ x,
                                                   float *__restrict__ zout, float *__restrict__ logq,
                                                   uint32_t key0, uint32_t key1,
                                                   uint32_t stream_base, uint32_t round_lo,
                                                   uint32_t round_hi)
{
    constexpr int KC = C / 32;
    constexpr bool kRegW = C == 32; // the five layers' weights fit in registers
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ float zs[16 * W];
    __shared__ float w1s[4 * C], b1s[C];
    const int L = net.L, N = net.N, R = sampler_ring_rows(L);
    bf16 *ring = (bf16 *)smem; // [R][4][5][C]
    int8_t *sp = (int8_t *)(smem + (size_t)R * 4 * 5 * C * sizeof(bf16));
    const int64_t b = blockIdx.x;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
    const ParamLayout pl = param_layout(C);
    const float b6 = net.params[pl.b6];
    WeightsRegs<32, 32> wreg[kRegW ? 4 : 1];
    WeightsRegs<32, 16> w6reg;
    if constexpr (kRegW) {
#pragma unroll
        for (int l = 2; l <= 5; ++l)
            wreg[l - 2].load(net.wf[l]);
        w6reg.load(net.w6p);
    }
    float bias[4][C / 16]; // layers 2..5, this lane's output columns
#pragma unroll
    for (int l = 2; l <= 5; ++l)
#pragma unroll
        for (int n = 0; n < C / 16; ++n)
            bias[l - 2][n] = net.params[pl.b[l] + n * 16 + r];
    for (int e = threadIdx.x; e < 4 * C; e += 64 * W)
        w1s[e] = net.w1[e];
    for (int e = threadIdx.x; e < C; e += 64 * W)
        b1s[e] = net.params[pl.b1 + e];
    for (int e = threadIdx.x; e < N; e += 64 * W)
        sp[e] = 0;
    __syncthreads();
    const int steps = 3 * L - 2;
    // ring row of i: i mod R, carried along with i (i_lo never decreases)
    for (int t = 0; t < steps; ++t) {
        const int i_lo = t > L - 1 ? (t - L + 2) >> 1 : 0;
        const int i_hi = (t >> 1) < L - 1 ? (t >> 1) : L - 1;
        const int nsites = i_hi - i_lo + 1;
        // this lane's tile row: site s of the diagonal
        const int s = 16 * wave + r;
        const bool valid = s < nsites;
        const int i = i_lo + s, j = t - 2 * i;
        // ring rows of i, i-1 (i < L <= 2R - 4, so i mod R is one conditional subtraction)
        const int ri = valid ? (i >= R ? i - R : i) : 0, rup = ri == 0 ? R - 1 : ri - 1;
        // layer 1 (mask A) at the row's site, 8 channels per 16-byte group
        if (valid) {
            float xv[4];
#pragma unroll
            for (int tt = 0; tt < 3; ++tt) {
                const int jj = j + tap_dx(tt);
                xv[tt] = (i > 0 && jj >= 0 && jj < L) ? (float)sp[(i - 1) * L + jj] : 0.f;
            }
            xv[3] = j > 0 ? (float)sp[i * L + j - 1] : 0.f;
            bf16 *dst = ring + ((ri * 4 + (j & 3)) * 5 + 0) * C;
#pragma unroll
            for (int g = 0; g < KC; ++g) {
                const int c0 = (kq * KC + g) * 8;
                bf16x8 v;
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    v[e] = (bf16)l1_from(xv, w1s, b1s, C, c0 + e);
                *(bf16x8 *)(dst + c0) = v;
            }
        }
        // ring entries of the five taps of this lane's row, and of the four
        // output rows this lane writes in the epilogues
        int tap_base[5]; // element offsets in `ring`
        bool tap_ok[5];
#pragma unroll
        for (int tt = 0; tt < 5; ++tt) {
            const int jj = j + tap_dx(tt);
            tap_ok[tt] = valid && (tap_dy(tt) == 0 || i > 0) && jj >= 0 && jj < L;
            tap_base[tt] = (((tap_dy(tt) == 0 ? ri : rup) * 4 + (jj & 3)) * 5) * C + kq * 8;
        }
        int slot[4]; // element offsets in `ring`
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int so = 16 * wave + kq * 4 + q;
            const int io = i_lo + so, jo = t - 2 * io;
            slot[q] = (((so < nsites ? (io >= R ? io - R : io) : 0) * 4 + (jo & 3)) * 5) * C;
        }
        lds_sync<W>();
        const SamplerRows<C> rows{b, 16 * wave, nsites};
#pragma unroll
        for (int l = 2; l <= 6; ++l) {
            bf16x8 a[5][KC];
#pragma unroll
            for (int tt = 0; tt < 5; ++tt)
#pragma unroll
                for (int kc = 0; kc < KC; ++kc)
                    a[tt][kc] = load8_or_zero(tap_ok[tt], ring + tap_base[tt] + (l - 2) * C + kc * 32);
            if (l <= 5) {
                const EpiRing<C> epi{ring, slot, bias[l - 2], l - 1};
                if constexpr (kRegW)
                    conv_mfma<C, C>(a, wreg[kRegW ? l - 2 : 0], rows, epi);
                else
                    conv_mfma<C, C>(a, WeightsGlobal<C>{net.wf[l]}, rows, epi);
            } else {
                const EpiZ epi{zs, b6};
                if constexpr (kRegW)
                    conv_mfma<C, 16>(a, w6reg, rows, epi);
                else
                    conv_mfma<C, 16>(a, WeightsGlobal<C>{net.w6p}, rows, epi);
            }
            lds_sync<W>();
        }
        // the draws of this wavefront's sites
        if (lane < 16 && valid) {
            const int p = i * L + j;
            const float z = zs[s];
            const float Pq = quantise(prob_plus(z));
            const Block u = philox4x32_10(ctr_word0(stream_base + (uint32_t)b, 3u, 0u), round_lo,
                                          round_hi, (uint32_t)(p >> 2), key0, key1);
            const uint32_t w = (p & 3) == 0 ? u.x0 : (p & 3) == 1 ? u.x1 : (p & 3) == 2 ? u.x2 : u.x3;
            const float uf = (float)(w >> 8) * (1.f / 16777216.f);
            const int8_t xv = uf < Pq ? 1 : -1;
            sp[p] = xv;
            x[b * N + p] = xv;
            zout[b * N + p] = z;
        }
        lds_sync<W>();
    }
    __syncthreads(); // the logits in `zout` of every wavefront
    if (wave == 0) {
        const double lq = config_logq(zout + b * N, sp, N);
        if (lane == 0)
            logq[b] = (float)lq;
    }
}

// --------------------------------------------------------------- backward
// Rows [0, rows_total) are cut into 64-row chunks; workgroup g of a weight
// gradient kernel takes chunks [g*cpb, (g+1)*cpb) and writes its sums to row
// g of `partial` (pstride floats per row, the parameter vector plus the loss).
struct ChunkRange {
    int64_t c0, c1;
    __device__ ChunkRange(int64_t nchunks, int64_t cpb)
    {
        c0 = (int64_t)blockIdx.x * cpb;
        c1 = c0 + cpb < nchunks ? c0 + cpb : nchunks;
    }
};

// Fixed-order sum over the 256 threads of a workgroup (thread 0 adds the 256
// values in thread order); every thread gets the total.
__device__ __forceinline__ float block_sum_ordered(float v, float *red)
{
    __syncthreads();
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int k = 0; k < 256; ++k)
            s += red[k];
        red[256] = s;
    }
    __syncthreads();
    return red[256];
}

// Rows of a 64-row chunk as the staging loops need them: flattened site index
// of the row (configuration * N + site) and its lattice coordinates, or -1.
struct ChunkRows {
    int64_t base[64];
    int16_t i[64], j[64];
};

__device__ __forceinline__ void chunk_rows(ChunkRows &cr, int64_t row0, int64_t rows_total, int N,
                                           int L)
{
    const int k = threadIdx.x;
    if (k < 64) {
        const int64_t g = row0 + k;
        if (g < rows_total) {
            const int64_t b = g / N;
            const int p = (int)(g - b * N);
            cr.base[k] = b * N;
            cr.i[k] = (int16_t)(p / L);
            cr.j[k] = (int16_t)(p - (p / L) * L);
        } else {
            cr.base[k] = -1;
            cr.i[k] = 0;
            cr.j[k] = 0;
        }
    }
}

// The five mask-B taps of a chunk's 64 rows, transposed into LDS
// (sA[t][c][k] = act[row k shifted by tap t][c], 0 outside the lattice):
// items of 4 rows x 8 channels of one tap, four 16-byte loads and eight
// 8-byte LDS writes each.
template <int C>
__device__ __forceinline__ void stage_taps(bf16 (&sA)[5][C][64], const bf16 *__restrict__ act,
                                           const ChunkRows &cr, int L)
{
    constexpr int CG = C / 8;
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    for (int e = threadIdx.x; e < 5 * 16 * CG; e += blockDim.x) {
        const int cg = e % CG, k4 = (e / CG) % 16, t = e / (CG * 16);
        bf16x8 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = 4 * k4 + u;
            const int ii = cr.i[k] + tap_dy(t), jj = cr.j[k] + tap_dx(t);
            if (cr.base[k] >= 0 && ii >= 0 && jj >= 0 && jj < L)
                v[u] = *(const bf16x8 *)(act + (cr.base[k] + ii * L + jj) * C + cg * 8);
            else
                zero8(v[u]);
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const bf16x4 w = {v[0][c], v[1][c], v[2][c], v[3][c]};
            *(bf16x4 *)&sA[t][cg * 8 + c][4 * k4] = w;
        }
    }
}

// d(mean NLL)/d logit = -s sigmoid(-s z) / B (float32, written out), the mean
// NLL, and the layer-6 weight and bias gradients:
//   dW6[t][ci] = sum_rows h5[row shifted by tap t][ci] * dlogit[row]
// on MFMA: rows as the reduction dimension, 64 at a time transposed in LDS,
// dlogit as columns 0 (high half) and 1 (low half) of the B operand.
template <int C>
__global__ __launch_bounds__(256) void k_l6_back(NetDev net, const int8_t *__restrict__ x,
                                                 const float *__restrict__ logits,
                                                 const bf16 *__restrict__ h5,
                                                 float *__restrict__ dlogit, int64_t rows_total,
                                                 int64_t nchunks, int64_t cpb, float invB,
                                                 float *__restrict__ partial, int64_t pstride)
{
    constexpr int MT = C / 16, TILES = 5 * MT, TPW = (TILES + 3) / 4;
    __shared__ __align__(16) bf16 sA[5][C][64];
    __shared__ __align__(16) bf16 sD[16][64];
    __shared__ float red[257];
    const int N = net.N, L = net.L;
    const ParamLayout pl = param_layout(C);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, kq = lane >> 4;
    floatx4 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q)
        acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int e = tid; e < 14 * 64; e += 256)
        sD[2 + e / 64][e % 64] = (bf16)0.f;
    float lsum = 0.f, dsum = 0.f;
    __shared__ ChunkRows crow;
    const ChunkRange rng(nchunks, cpb);
    for (int64_t ch = rng.c0; ch < rng.c1; ++ch) {
        const int64_t row0 = ch * 64;
        __syncthreads();
        chunk_rows(crow, row0, rows_total, N, L);
        __syncthreads();
        stage_taps<C>(sA, h5, crow, L);
        if (tid < 64) {
            const int64_t g = row0 + tid;
            float d = 0.f;
            if (g < rows_total) {
                const float s = (float)x[g], z = logits[g], sz = s * z;
                d = -s / (1.f + expf(sz)) * invB;
                lsum += (fmaxf(-sz, 0.f) + log1pf(expf(-fabsf(sz)))) * invB;
                dlogit[g] = d;
            }
            dsum += d;
            const bf16 h = (bf16)d;
            sD[0][tid] = h;
            sD[1][tid] = (bf16)(d - (float)h);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int tile = wave + 4 * q;
            if (tile < TILES) {
                const int t = tile / MT, m = tile % MT;
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const bf16x8 av = *(const bf16x8 *)&sA[t][m * 16 + r][ks * 32 + kq * 8];
                    const bf16x8 bv = *(const bf16x8 *)&sD[r][ks * 32 + kq * 8];
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[q], 0, 0, 0);
                }
            }
        }
    }
    float *out = partial + (int64_t)blockIdx.x * pstride;
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int tile = wave + 4 * q;
        if (tile < TILES) { // wave-uniform
            const int t = tile / MT, m = tile % MT;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float lo = __shfl_down(acc[q][e], 1, 64); // column 1 of the same row
                if (r == 0)
                    out[pl.W6 + t * C + m * 16 + kq * 4 + e] = acc[q][e] + lo;
            }
        }
    }
    const float db = block_sum_ordered(dsum, red);
    const float ls = block_sum_ordered(lsum, red);
    if (tid == 0) {
        out[pl.b6] = db;
        out[pl.total] = ls;
    }
}

// Data gradient into layer 5, masked by its ReLU, float32:
//   dpre5[row][ci] = [h5 > 0] sum_t W6[t][ci] dlogit[row - tap t],
// one thread per (row, 8 channels).
__global__ __launch_bounds__(256) void k_l6_dgrad(NetDev net, const bf16 *__restrict__ h5,
                                                  const float *__restrict__ dlogit,
                                                  float *__restrict__ dpre, int64_t rows_total)
{
    const int C = net.C, CG = C / 8, N = net.N, L = net.L;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= rows_total * CG)
        return;
    const int64_t row = g / CG;
    const int c0 = (int)(g - row * CG) * 8;
    const int64_t b = row / N;
    const int p = (int)(row - b * N), i = p / L, j = p - (p / L) * L;
    float dh[8];
#pragma unroll
    for (int e = 0; e < 8; ++e)
        dh[e] = 0.f;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
        const int ii = i - tap_dy(t), jj = j - tap_dx(t);
        if (ii >= 0 && ii < L && jj >= 0 && jj < L) {
            const float d = dlogit[b * N + ii * L + jj];
#pragma unroll
            for (int e = 0; e < 8; ++e)
                dh[e] = fmaf(net.w6[t * C + c0 + e], d, dh[e]);
        }
    }
    const bf16x8 h = *(const bf16x8 *)(h5 + row * C + c0);
    float *o = dpre + row * C + c0;
    *(float4 *)o = float4{(float)h[0] > 0.f ? dh[0] : 0.f, (float)h[1] > 0.f ? dh[1] : 0.f,
                          (float)h[2] > 0.f ? dh[2] : 0.f, (float)h[3] > 0.f ? dh[3] : 0.f};
    *(float4 *)(o + 4) = float4{(float)h[4] > 0.f ? dh[4] : 0.f, (float)h[5] > 0.f ? dh[5] : 0.f,
                                (float)h[6] > 0.f ? dh[6] : 0.f, (float)h[7] > 0.f ? dh[7] : 0.f};
}

// Data gradient through a C -> C layer (the transposed convolution: taps at
// negated offsets), float32 signal split into bf16 halves, ReLU mask of the
// layer below.
template <int C>
__global__ __launch_bounds__(256) void k_conv_dgrad(const float *__restrict__ dpre_above,
                                                    float *__restrict__ dpre_below,
                                                    const bf16 *__restrict__ act_below,
                                                    const bf16 *__restrict__ wk, int L, int N,
                                                    int64_t rows_total)
{
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile * 16 >= rows_total)
        return;
    const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
    const RowsOfSites rows{tile * 16, rows_total, N};
    int64_t b;
    int p;
    rows(r, b, p);
    const int i = p / L, j = p - (p / L) * L;
    bf16x8 ah[5][C / 32], al[5][C / 32];
#pragma unroll
    for (int t = 0; t < 5; ++t)
        load_tap_split<C>(ah[t], al[t], dpre_above, b, N, L, i - tap_dy(t), j - tap_dx(t), kq);
    conv_mfma_split<C, C>(ah, al, WeightsGlobal<C>{wk}, LaneRows(rows, kq),
                          EpiBackward{dpre_below, act_below, N, C});
}

// Weight and bias gradients of a C -> C layer:
//   dW[t][ci][co] = sum_rows act_below[row shifted by tap t][ci] * dpre[row][co]
// on MFMA, rows as the reduction dimension, 64 rows at a time transposed in
// LDS, dpre as two bf16 halves; db[co] = sum_rows dpre[row][co] in float32.
// Weight and bias gradients of a C -> C layer:
//   dW[t][ci][co] = sum_rows act_below[row shifted by tap t][ci] * dpre[row][co]
// on MFMA, rows as the reduction dimension, 64 rows at a time transposed in
// LDS (a thread takes 4 rows x 8 channels: four 16-byte loads, eight 8-byte
// LDS writes), dpre as two bf16 halves; db[co] = sum_rows dpre[row][co] in
// float32, each thread adding its rows in order, the threads of a channel in
// thread order.
template <int C>
__global__ __launch_bounds__(256) void k_conv_wgrad(const bf16 *__restrict__ act_below,
                                                    const float *__restrict__ dpre, int L, int N,
                                                    int64_t rows_total, int64_t nchunks, int64_t cpb,
                                                    float *__restrict__ pW, float *__restrict__ pb,
                                                    int64_t pstride)
{
    constexpr int MT = C / 16, TILES = 5 * MT * MT, TPW = TILES / 4, CG = C / 8;
    __shared__ __align__(16) bf16 sA[5][C][64];
    __shared__ __align__(16) bf16 sDh[C][64];
    __shared__ __align__(16) bf16 sDl[C][64];
    __shared__ ChunkRows cr;
    __shared__ float red[256];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, kq = lane >> 4;
    floatx4 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q)
        acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
    float bacc[8] = {}; // channels cg*8 .. +7 of the dpre items this thread stages
    const ChunkRange rng(nchunks, cpb);
    for (int64_t ch = rng.c0; ch < rng.c1; ++ch) {
        const int64_t row0 = ch * 64;
        __syncthreads();
        chunk_rows(cr, row0, rows_total, N, L);
        __syncthreads();
        stage_taps<C>(sA, act_below, cr, L);
        // backward signal: items (4-row group, 8-channel group), fixed per thread
        if (tid < 16 * CG) {
            const int cg = tid % CG, k4 = tid / CG;
            float d[4][8];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t g = row0 + 4 * k4 + u;
                if (g < rows_total) {
                    const float4 a0 = *(const float4 *)(dpre + g * C + cg * 8);
                    const float4 a1 = *(const float4 *)(dpre + g * C + cg * 8 + 4);
                    const float t8[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        d[u][c] = t8[c];
                } else {
#pragma unroll
                    for (int c = 0; c < 8; ++c)
                        d[u][c] = 0.f;
                }
            }
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
                bf16x4 hi, lo;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    bacc[c] += d[u][c];
                    const bf16 h = (bf16)d[u][c];
                    hi[u] = h;
                    lo[u] = (bf16)(d[u][c] - (float)h);
                }
                *(bf16x4 *)&sDh[cg * 8 + c][4 * k4] = hi;
                *(bf16x4 *)&sDl[cg * 8 + c][4 * k4] = lo;
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int tile = wave * TPW + q;
            const int t = tile / (MT * MT), m = (tile / MT) % MT, n = tile % MT;
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const bf16x8 av = *(const bf16x8 *)&sA[t][m * 16 + r][ks * 32 + kq * 8];
                const bf16x8 bh = *(const bf16x8 *)&sDh[n * 16 + r][ks * 32 + kq * 8];
                const bf16x8 bl = *(const bf16x8 *)&sDl[n * 16 + r][ks * 32 + kq * 8];
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bh, acc[q], 0, 0, 0);
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bl, acc[q], 0, 0, 0);
            }
        }
    }
    float *oW = pW + (int64_t)blockIdx.x * pstride;
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int tile = wave * TPW + q;
        const int t = tile / (MT * MT), m = (tile / MT) % MT, n = tile % MT;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ci = m * 16 + kq * 4 + e, co = n * 16 + r;
            oW[((int64_t)t * C + ci) * C + co] = acc[q][e];
        }
    }
    // bias: thread tid < 16 CG holds channels (tid % CG)*8 .. +7 over its row
    // groups; the 16 threads of a channel group are added in thread order
    for (int c = 0; c < 8; ++c) {
        __syncthreads();
        red[tid] = bacc[c];
        __syncthreads();
        if (tid < CG) {
            float s = 0.f;
            for (int k4 = 0; k4 < 16; ++k4)
                s += red[k4 * CG + tid];
            pb[(int64_t)blockIdx.x * pstride + tid * 8 + c] = s;
        }
    }
}

// Weight and bias gradients of layer 1 on MFMA: A = the four mask-A spins of
// each row (rows 0..3) and a row of ones (row 4, the bias), B = dpre1 as two
// bf16 halves; dW1[t][c] = sum_rows x[row shifted by tap t] dpre1[row][c].
template <int C>
__global__ __launch_bounds__(256) void k_l1_wgrad(NetDev net, const int8_t *__restrict__ x,
                                                  const float *__restrict__ dpre1,
                                                  int64_t rows_total, int64_t nchunks, int64_t cpb,
                                                  float *__restrict__ partial, int64_t pstride)
{
    constexpr int NT = C / 16; // 16-column tiles, one or two per wavefront
    __shared__ __align__(16) bf16 sX[16][64];
    __shared__ __align__(16) bf16 sDh[C][64];
    __shared__ __align__(16) bf16 sDl[C][64];
    const int N = net.N, L = net.L;
    const ParamLayout pl = param_layout(C);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, kq = lane >> 4;
    floatx4 acc[2] = {floatx4{0.f, 0.f, 0.f, 0.f}, floatx4{0.f, 0.f, 0.f, 0.f}};
    for (int e = tid; e < 11 * 64; e += 256)
        sX[5 + e / 64][e % 64] = (bf16)0.f;
    const ChunkRange cr(nchunks, cpb);
    for (int64_t ch = cr.c0; ch < cr.c1; ++ch) {
        const int64_t row0 = ch * 64;
        __syncthreads();
        for (int e = tid; e < 64 * C; e += 256) {
            const int k = e / C, c = e % C;
            const int64_t g = row0 + k;
            const float d = g < rows_total ? dpre1[g * C + c] : 0.f;
            const bf16 h = (bf16)d;
            sDh[c][k] = h;
            sDl[c][k] = (bf16)(d - (float)h);
        }
        if (tid < 64) {
            const int64_t g = row0 + tid;
            const bool valid = g < rows_total;
            const int64_t b = valid ? g / N : 0;
            const int p = valid ? (int)(g - b * N) : 0, i = p / L, j = p - (p / L) * L;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int ii = i + tap_dy(t), jj = j + tap_dx(t);
                const bool ok = valid && ii >= 0 && jj >= 0 && jj < L;
                sX[t][tid] = ok ? (bf16)(float)x[(int64_t)b * N + ii * L + jj] : (bf16)0.f;
            }
            sX[4][tid] = valid ? (bf16)1.f : (bf16)0.f;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int nt = wave + 4 * q;
            if (nt < NT) {
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const bf16x8 av = *(const bf16x8 *)&sX[r][ks * 32 + kq * 8];
                    const bf16x8 bh = *(const bf16x8 *)&sDh[nt * 16 + r][ks * 32 + kq * 8];
                    const bf16x8 bl = *(const bf16x8 *)&sDl[nt * 16 + r][ks * 32 + kq * 8];
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bh, acc[q], 0, 0, 0);
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bl, acc[q], 0, 0, 0);
                }
            }
        }
    }
    float *out = partial + (int64_t)blockIdx.x * pstride;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int nt = wave + 4 * q;
        if (nt < NT) {
            const int c = nt * 16 + r;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = kq * 4 + e; // 0..3: taps, 4: bias
                if (row < 4)
                    out[pl.W1 + row * C + c] = acc[q][e];
                else if (row == 4)
                    out[pl.b1 + c] = acc[q][e];
            }
        }
    }
}

// grad[e] = sum over workgroups of partial[g][e], the last slot the loss: a
// workgroup takes 64 slots, its four wavefronts the workgroups g = w, w + 4,
// w + 8, .. (each in increasing g), and the four sums are added as
// (s0 + s1) + (s2 + s3).  The order is fixed, so the result is too.
__global__ __launch_bounds__(256) void k_reduce_partials(const float *__restrict__ partial,
                                                         int64_t pstride, int nblk, int64_t P,
                                                         float *__restrict__ grad,
                                                         float *__restrict__ loss)
{
    __shared__ float part[4][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t e = (int64_t)blockIdx.x * 64 + lane;
    float s = 0.f;
    if (e <= P)
        for (int g = w; g < nblk; g += 4)
            s += partial[(int64_t)g * pstride + e];
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && e <= P) {
        const float t = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
        if (e < P)
            grad[e] = t;
        else
            *loss = t;
    }
}

// Adam (Kingma and Ba 2015) on the float32 master parameters.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ params,
                                              const float *__restrict__ grad, float *__restrict__ m,
                                              float *__restrict__ v, int64_t n, float lr,
                                              float beta1, float beta2, float eps, float bc1,
                                              float bc2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const float g = grad[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * g;
    const float vi = beta2 * v[i] + (1.f - beta2) * g * g;
    m[i] = mi;
    v[i] = vi;
    params[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// ------------------------------------------------------ configurations
// Bond sum and magnetisation of int8 configurations (periodic, each bond once).
__global__ __launch_bounds__(256) void k_spins_observables(const int8_t *__restrict__ x, int L,
                                                           int64_t *bond, int64_t *mag)
{
    __shared__ int64_t sb[256], sm[256];
    const int N = L * L;
    const int8_t *s = x + (int64_t)blockIdx.x * N;
    int64_t tb = 0, tm = 0;
    for (int p = threadIdx.x; p < N; p += blockDim.x) {
        const int i = p / L, j = p % L;
        const int v = s[p];
        tb += v * (s[((i + 1) % L) * L + j] + s[i * L + (j + 1) % L]);
        tm += v;
    }
    sb[threadIdx.x] = tb;
    sm[threadIdx.x] = tm;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sb[threadIdx.x] += sb[threadIdx.x + h];
            sm[threadIdx.x] += sm[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bond[blockIdx.x] = sb[0];
        mag[blockIdx.x] = sm[0];
    }
}

// Training minibatch: configuration b of the output is configuration k of a
// pool of P under a random symmetry of the periodic Boltzmann weight (global
// flip, translation by (di, dj)), all from Philox block (stream_base + b) of
// domain 5 at counter (stream<<8 | 5<<4, round lo, round hi, 0):
//   k = floor((x1:x0) P / 2^64), flip = x2 & 1, di = (x2 >> 1) mod L,
//   dj = x3 mod L,
//   out[b][i][j] = (flip ? -1 : 1) * pool[k][(i + di) mod L][(j + dj) mod L].
__global__ __launch_bounds__(256) void k_minibatch(const int8_t *__restrict__ pool, int64_t P,
                                                   int L, int8_t *__restrict__ out, uint32_t key0,
                                                   uint32_t key1, uint32_t stream_base,
                                                   uint32_t round_lo, uint32_t round_hi)
{
    __shared__ int64_t k_s;
    __shared__ int flip_s, di_s, dj_s;
    const int b = blockIdx.x, N = L * L;
    if (threadIdx.x == 0) {
        const Block u = philox4x32_10(ctr_word0(stream_base + (uint32_t)b, 5u, 0u), round_lo,
                                      round_hi, 0u, key0, key1);
        const uint64_t r64 = ((uint64_t)u.x1 << 32) | u.x0;
        k_s = (int64_t)__umul64hi(r64, (uint64_t)P);
        flip_s = (int)(u.x2 & 1u);
        di_s = (int)((u.x2 >> 1) % (uint32_t)L);
        dj_s = (int)(u.x3 % (uint32_t)L);
    }
    __syncthreads();
    const int8_t *src = pool + k_s * N;
    const int di = di_s, dj = dj_s;
    const int8_t sg = flip_s ? -1 : 1;
    for (int p = threadIdx.x; p < N; p += blockDim.x) {
        const int i = p / L, j = p - (p / L) * L;
        int ii = i + di, jj = j + dj;
        ii -= ii >= L ? L : 0;
        jj -= jj >= L ? L : 0;
        out[(int64_t)b * N + p] = (int8_t)(sg * src[ii * L + jj]);
    }
}

// Independence Metropolis-Hastings step per chain, in float32 with every
// operation rounded on its own:
//   log A = ((beta J * float(bond' - bond)) + log q(x)) - log q(x'),
// accepted iff log A >= 0 or u < exp(log A), u a 24-bit uniform of Philox
// domain 2 (counter (stream<<8 | 2<<4, round lo, round hi, 0), word 0).
__device__ __forceinline__ float mh_log_ratio(float betaJ, int64_t dB, float lq_cur, float lq_prop)
{
#pragma clang fp contract(off)
    const float e = betaJ * (float)dB;
    const float s = e + lq_cur;
    return s - lq_prop;
}

__global__ __launch_bounds__(256) void k_mh(int N, int8_t *__restrict__ state,
                                            float *__restrict__ logq_cur,
                                            int64_t *__restrict__ bond_cur,
                                            const int8_t *__restrict__ prop,
                                            const float *__restrict__ logq_prop,
                                            const int64_t *__restrict__ bond_prop,
                                            const float *__restrict__ betaJ, uint32_t key0,
                                            uint32_t key1, uint32_t stream_base, uint32_t round_lo,
                                            uint32_t round_hi, int32_t *__restrict__ accepted)
{
    __shared__ int acc;
    const int c = blockIdx.x;
    if (threadIdx.x == 0) {
        const float log_a = mh_log_ratio(betaJ[c], bond_prop[c] - bond_cur[c], logq_cur[c], logq_prop[c]);
        const Block u = philox4x32_10(ctr_word0(stream_base + (uint32_t)c, 2u, 0u), round_lo,
                                      round_hi, 0u, key0, key1);
        const float uf = (float)(u.x0 >> 8) * (1.f / 16777216.f);
        acc = (log_a >= 0.f || uf < expf(log_a)) ? 1 : 0;
        if (acc) {
            logq_cur[c] = logq_prop[c];
            bond_cur[c] = bond_prop[c];
        }
        accepted[c] = acc;
    }
    __syncthreads();
    if (acc)
        for (int p = threadIdx.x; p < N; p += blockDim.x)
            state[(int64_t)c * N + p] = prop[(int64_t)c * N + p];
}

// --------------------------------------------------------------- launches
static inline uint32_t nblocks(int64_t n, int per) { return (uint32_t)((n + per - 1) / per); }

hipError_t launch_pack(const NetDev &net, hipStream_t s)
{
    const int64_t total = param_layout(net.C).total;
    const int64_t n = total > 16 * 5 * net.C ? total : 16 * 5 * net.C;
    hipLaunchKernelGGL(k_pack, dim3(nblocks(n, 256)), dim3(256), 0, s, net);
    return hipGetLastError();
}

hipError_t launch_forward(const NetDev &net, const int8_t *x, int B, bf16 *const h[6],
                          float *logits, float *logq, hipStream_t s)
{
    const int64_t rows = (int64_t)B * net.N;
    const ParamLayout pl = param_layout(net.C);
    hipLaunchKernelGGL(k_l1_fwd, dim3(nblocks(rows * (net.C / 8), 256)), dim3(256), 0, s, net, x, h[1],
                       rows);
    const uint32_t tiles = nblocks(rows, 16);
    for (int l = 2; l <= 5; ++l) {
        if (net.C == 32)
            hipLaunchKernelGGL(k_conv_fwd<32>, dim3(nblocks(tiles, 4)), dim3(256), 0, s, h[l - 1],
                               h[l], net.wf[l], net.params + pl.b[l], net.L, net.N, rows);
        else
            hipLaunchKernelGGL(k_conv_fwd<64>, dim3(nblocks(tiles, 4)), dim3(256), 0, s, h[l - 1],
                               h[l], net.wf[l], net.params + pl.b[l], net.L, net.N, rows);
    }
    if (net.C == 32)
        hipLaunchKernelGGL(k_l6_fwd<32>, dim3(nblocks(tiles, 4)), dim3(256), 0, s, net, h[5], logits, rows);
    else
        hipLaunchKernelGGL(k_l6_fwd<64>, dim3(nblocks(tiles, 4)), dim3(256), 0, s, net, h[5], logits, rows);
    if (logq)
        hipLaunchKernelGGL(k_logq, dim3(nblocks(B, 4)), dim3(256), 0, s, x, logits, net.N, B, logq);
    return hipGetLastError();
}

// Evaluator waves per workgroup (one workgroup per configuration).
constexpr int kEvalWaves = 8;

bool eval_supported(int L, int C)
{
    return (C == 32 || C == 64) && eval_lds_bytes(L * L, C) <= lds_limit();
}

template <int C>
static hipError_t launch_eval_c(const NetDev &net, const int8_t *x, int B, float *logits,
                                float *logq, size_t lds, hipStream_t s)
{
    static size_t allowed = 0; // dynamic LDS granted to this instance so far
    if (lds > allowed) {
        const hipError_t e = hipFuncSetAttribute((const void *)k_eval<C, kEvalWaves>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) {
            (void)hipGetLastError(); // leave no sticky error behind for later calls
            return e;
        }
        allowed = lds;
    }
    static int ncu = 0;
    if (!ncu) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            ncu <= 0)
            ncu = 256;
    }
    // one resident workgroup per compute unit (the LDS of one configuration)
    const int grid = B < ncu ? B : ncu;
    hipLaunchKernelGGL((k_eval<C, kEvalWaves>), dim3(grid), dim3(64 * kEvalWaves), lds, s, net, x, B,
                       logits, logq);
    return hipGetLastError();
}

hipError_t launch_eval(const NetDev &net, const int8_t *x, int B, float *logits, float *logq,
                       hipStream_t s)
{
    if (!eval_supported(net.L, net.C) || !logq)
        return hipErrorInvalidValue;
    const size_t lds = eval_lds_bytes(net.N, net.C);
    return net.C == 32 ? launch_eval_c<32>(net, x, B, logits, logq, lds, s)
                       : launch_eval_c<64>(net, x, B, logits, logq, lds, s);
}

size_t lds_limit()
{
    static size_t limit = 0;
    if (!limit) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            limit = (size_t)v;
        else
            limit = 64 * 1024;
    }
    return limit;
}

int sampler_waves(int L)
{
    const int sites = (L + 1) / 2; // longest anti-diagonal
    return sites <= 16 ? 1 : sites <= 32 ? 2 : 4;
}

template <int C, int W>
static hipError_t launch_sample_cw(const NetDev &net, int B, int8_t *x, float *zout, float *logq,
                                   uint64_t seed, uint32_t stream_base, uint64_t round, size_t lds,
                                   hipStream_t s)
{
    static size_t allowed = 0; // dynamic LDS granted to this instance so far
    if (lds > allowed) {
        const hipError_t e = hipFuncSetAttribute((const void *)k_sample<C, W>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) {
            (void)hipGetLastError(); // leave no sticky error behind for later calls
            return e;
        }
        allowed = lds;
    }
    hipLaunchKernelGGL((k_sample<C, W>), dim3(B), dim3(64 * W), lds, s, net, x, zout, logq,
                       (uint32_t)seed, (uint32_t)(seed >> 32), stream_base, (uint32_t)round,
                       (uint32_t)(round >> 32));
    return hipGetLastError();
}

bool sampler_supported(int L, int C)
{
    // dynamic ring and spins, plus the kernel's static logits of one diagonal
    return L <= kSamplerMaxL &&
           sampler_lds_bytes(L, C) + 16 * sampler_waves(L) * sizeof(float) <= lds_limit();
}

hipError_t launch_sample(const NetDev &net, int B, int8_t *x, float *zout, float *logq,
                         uint64_t seed, uint32_t stream_base, uint64_t round, hipStream_t s)
{
    if (!sampler_supported(net.L, net.C))
        return hipErrorInvalidValue;
    const size_t lds = sampler_lds_bytes(net.L, net.C);
    const int W = sampler_waves(net.L);
    if (net.C == 32) {
        if (W == 1)
            return launch_sample_cw<32, 1>(net, B, x, zout, logq, seed, stream_base, round, lds, s);
        if (W == 2)
            return launch_sample_cw<32, 2>(net, B, x, zout, logq, seed, stream_base, round, lds, s);
        return launch_sample_cw<32, 4>(net, B, x, zout, logq, seed, stream_base, round, lds, s);
    }
    if (W == 1)
        return launch_sample_cw<64, 1>(net, B, x, zout, logq, seed, stream_base, round, lds, s);
    if (W == 2)
        return launch_sample_cw<64, 2>(net, B, x, zout, logq, seed, stream_base, round, lds, s);
    return launch_sample_cw<64, 4>(net, B, x, zout, logq, seed, stream_base, round, lds, s);
}

hipError_t launch_backward(const NetDev &net, const int8_t *x, int B, bf16 *const h[6],
                           const float *logits, float *dlogit, float *dpre_a, float *dpre_b,
                           float *partial, float *grad, float *loss, hipStream_t s)
{
    const int64_t rows = (int64_t)B * net.N;
    const int C = net.C;
    const ParamLayout pl = param_layout(C);
    const int64_t pstride = pl.total + 1;
    const int64_t nchunks = (rows + 63) / 64;
    const int nblk = (int)(nchunks < kGradBlocks ? nchunks : kGradBlocks);
    const int64_t cpb = (nchunks + nblk - 1) / nblk;
    const uint32_t tiles = nblocks(rows, 16);
    if (C == 32)
        hipLaunchKernelGGL(k_l6_back<32>, dim3(nblk), dim3(256), 0, s, net, x, logits, h[5], dlogit,
                           rows, nchunks, cpb, 1.f / (float)B, partial, pstride);
    else
        hipLaunchKernelGGL(k_l6_back<64>, dim3(nblk), dim3(256), 0, s, net, x, logits, h[5], dlogit,
                           rows, nchunks, cpb, 1.f / (float)B, partial, pstride);
    hipLaunchKernelGGL(k_l6_dgrad, dim3(nblocks(rows * (C / 8), 256)), dim3(256), 0, s, net, h[5],
                       dlogit, dpre_a, rows);
    float *above = dpre_a, *below = dpre_b;
    for (int l = 5; l >= 2; --l) {
        if (C == 32) {
            hipLaunchKernelGGL(k_conv_wgrad<32>, dim3(nblk), dim3(256), 0, s, h[l - 1], above,
                               net.L, net.N, rows, nchunks, cpb, partial + pl.W[l], partial + pl.b[l],
                               pstride);
            hipLaunchKernelGGL(k_conv_dgrad<32>, dim3(nblocks(tiles, 4)), dim3(256), 0, s, above,
                               below, h[l - 1], net.wb[l], net.L, net.N, rows);
        } else {
            hipLaunchKernelGGL(k_conv_wgrad<64>, dim3(nblk), dim3(256), 0, s, h[l - 1], above,
                               net.L, net.N, rows, nchunks, cpb, partial + pl.W[l], partial + pl.b[l],
                               pstride);
            hipLaunchKernelGGL(k_conv_dgrad<64>, dim3(nblocks(tiles, 4)), dim3(256), 0, s, above,
                               below, h[l - 1], net.wb[l], net.L, net.N, rows);
        }
        float *tmp = above;
        above = below;
        below = tmp;
    }
    if (C == 32)
        hipLaunchKernelGGL(k_l1_wgrad<32>, dim3(nblk), dim3(256), 0, s, net, x, above, rows, nchunks,
                           cpb, partial, pstride);
    else
        hipLaunchKernelGGL(k_l1_wgrad<64>, dim3(nblk), dim3(256), 0, s, net, x, above, rows, nchunks,
                           cpb, partial, pstride);
    hipLaunchKernelGGL(k_reduce_partials, dim3(nblocks(pl.total + 1, 64)), dim3(256), 0, s, partial,
                       pstride, nblk, pl.total, grad, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *params, const float *grad, float *m, float *v, int64_t n, float lr,
                       float beta1, float beta2, float eps, int64_t step, hipStream_t s)
{
    // bias corrections of the float32 constants, formed in double (1 - beta^t
    // cancels badly in float32 for beta2 near 1)
    const float bc1 = (float)(1.0 - pow((double)beta1, (double)step));
    const float bc2 = (float)(1.0 - pow((double)beta2, (double)step));
    hipLaunchKernelGGL(k_adam, dim3(nblocks(n, 256)), dim3(256), 0, s, params, grad, m, v, n, lr,
                       beta1, beta2, eps, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_spins_observables(const int8_t *x, int B, int L, int64_t *bond, int64_t *mag,
                                    hipStream_t s)
{
    hipLaunchKernelGGL(k_spins_observables, dim3(B), dim3(256), 0, s, x, L, bond, mag);
    return hipGetLastError();
}

hipError_t launch_minibatch(const int8_t *pool, int64_t P, int L, int B, int8_t *out,
                           uint64_t seed, uint32_t stream_base, uint64_t round, hipStream_t s)
{
    hipLaunchKernelGGL(k_minibatch, dim3(B), dim3(256), 0, s, pool, P, L, out, (uint32_t)seed,
                       (uint32_t)(seed >> 32), stream_base, (uint32_t)round, (uint32_t)(round >> 32));
    return hipGetLastError();
}

hipError_t launch_mh(int n, int N, int8_t *state, float *logq_cur, int64_t *bond_cur,
                     const int8_t *prop, const float *logq_prop, const int64_t *bond_prop,
                     const float *betaJ, uint64_t seed, uint32_t stream_base, uint64_t round,
                     int32_t *accepted, hipStream_t s)
{
    hipLaunchKernelGGL(k_mh, dim3(n), dim3(256), 0, s, N, state, logq_cur, bond_cur, prop, logq_prop,
                       bond_prop, betaJ, (uint32_t)seed, (uint32_t)(seed >> 32), stream_base,
                       (uint32_t)round, (uint32_t)(round >> 32), accepted);
    return hipGetLastError();
}

} // namespace arnet
} // namespace ising
