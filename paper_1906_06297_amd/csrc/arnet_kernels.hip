// gfx950 kernels of the masked-convolution autoregressive proposal: forward
// evaluation (log q of given configurations), incremental ancestral sampling,
// backward pass and Adam, independence Metropolis-Hastings, and conversions
// between bit-packed lattices and int8 spin arrays.
//
// The C -> C layers run on bf16 MFMA (v_mfma_f32_16x16x32_bf16, float32
// accumulators) through one routine, conv_tile(), which computes 16 rows x C
// outputs of a masked 3x3 convolution; a row is a (configuration, site)
// pair.  The evaluator feeds it 16 sites of one configuration, the sampler 16
// configurations at one site, so every output element is produced by the same
// instruction sequence in both and the sampler's conditionals are bit for bit
// those of the evaluator -- the Metropolis-Hastings ratio then uses the exact
// probability with which a proposal was drawn.
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
    if (g >= pl.total)
        return;
    const float v = net.params[g];
    if (g >= pl.W1 && g < pl.W1 + 4 * C) {
        net.w1[g - pl.W1] = round_bf16(v);
        return;
    }
    if (g >= pl.W6 && g < pl.W6 + 5 * C) {
        net.w6[g - pl.W6] = round_bf16(v);
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

// Layer 1 at site (i, j) of a configuration x.
__device__ __forceinline__ float l1_value(const int8_t *x, int L, int i, int j, const float *w1,
                                          const float *b1, int C, int c)
{
    float xv[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int ii = i + tap_dy(t), jj = j + tap_dx(t);
        xv[t] = (ii >= 0 && jj >= 0 && jj < L) ? (float)x[ii * L + jj] : 0.f;
    }
    return l1_from(xv, w1, b1, C, c);
}

// Layer 6 (mask B, C -> 1) from the five tap rows of h5 (nullptr: outside the
// lattice), summed tap by tap, channel by channel.
__device__ __forceinline__ float l6_from_rows(const bf16 *const (&row)[5], int C, const float *w6,
                                              float b6)
{
    float acc = 0.f;
    for (int t = 0; t < 5; ++t) {
        if (row[t] == nullptr)
            continue;
        for (int ci = 0; ci < C; ++ci)
            acc = fmaf((float)row[t][ci], w6[t * C + ci], acc);
    }
    return acc + b6;
}

// Layer 6: the logit of site (i, j) of configuration b.
__device__ __forceinline__ float l6_logit(const bf16 *h5, int N, int L, int C, int64_t b, int i,
                                          int j, const float *w6, float b6)
{
    const bf16 *row[5];
    for (int t = 0; t < 5; ++t) {
        const int ii = i + tap_dy(t), jj = j + tap_dx(t);
        row[t] = (ii < 0 || jj < 0 || jj >= L) ? nullptr : h5 + ((int64_t)b * N + ii * L + jj) * C;
    }
    return l6_from_rows(row, C, w6, b6);
}

__device__ __forceinline__ float prob_plus(float z) { return 1.f / (1.f + expf(-z)); }

// Realised probability of +1 when x = +1 iff a 24-bit uniform u < P.
__device__ __forceinline__ float quantise(float P) { return ceilf(P * 16777216.f) * (1.f / 16777216.f); }

__device__ __forceinline__ double site_logq(float Pq, int xv)
{
    return xv > 0 ? log((double)Pq) : log1p(-(double)Pq);
}

// ------------------------------------------------------------- MFMA tile
// Rows of a tile: a row is valid when b >= 0.
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
        b = g / N;
        p = (int)(g - b * N);
    }
};

struct RowsOfConfigs { // 16 configurations at one site
    int64_t b0, B;
    int p;
    __device__ void operator()(int r, int64_t &b, int &pp) const
    {
        b = (b0 + r < B) ? b0 + r : -1;
        pp = p;
    }
};

// The MFMA part of a masked 3x3 convolution tile: with the A operands of the
// five taps in registers (a[t][kc]: row lane & 15, k = kc*32 + (lane >> 4)*8
// + e), acc(row, n) = sum_t sum_k a[t][k] * wk[n][t*C + k], accumulated over
// t = 0..4 and 32-wide k chunks in that order, then handed to the epilogue.
// `bop(n0, t, kc)` yields the B operand (weights) of that step.
template <int C, class BOp, class Rows, class Epi>
__device__ __forceinline__ void conv_mfma_b(const bf16x8 (&a)[5][C / 32], const BOp &bop,
                                            const Rows &rows, const Epi &epi)
{
    constexpr int KC = C / 32;
    const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int n0 = 0; n0 < C; n0 += 16) {
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

// B operands read from the packed weights of a layer.
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

template <int C, class Rows, class Epi>
__device__ __forceinline__ void conv_mfma(const bf16x8 (&a)[5][C / 32],
                                          const bf16 *__restrict__ wk, const Rows &rows,
                                          const Epi &epi)
{
    conv_mfma_b<C>(a, WeightsGlobal<C>{wk}, rows, epi);
}

// A operand of tap t of a tile row (configuration b, site (i, j)) from an
// activation array: zero outside the lattice (zero padding).
template <int C>
__device__ __forceinline__ void load_tap(bf16x8 (&at)[C / 32], const bf16 *__restrict__ in,
                                         int64_t b, int N, int L, int ii, int jj, int kq)
{
    const bool ok = b >= 0 && ii >= 0 && ii < L && jj >= 0 && jj < L;
#pragma unroll
    for (int kc = 0; kc < C / 32; ++kc) {
        if (ok) {
            at[kc] = *(const bf16x8 *)(in + ((int64_t)b * N + ii * L + jj) * C + kc * 32 + kq * 8);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                at[kc][e] = (bf16)0.f;
        }
    }
}

// out[rows, 0..C) of a masked 3x3 convolution with all five mask-B taps, the
// taps read at offset sign * (dy, dx) (sign -1: the transposed convolution of
// the backward pass).
template <int C, class Rows, class Epi>
__device__ __forceinline__ void conv_tile(const bf16 *__restrict__ in, const bf16 *__restrict__ wk,
                                          int L, int N, int sign, const Rows &rows, const Epi &epi)
{
    const int lane = threadIdx.x & 63, r = lane & 15, kq = lane >> 4;
    int64_t b;
    int p;
    rows(r, b, p);
    const int i = p / L, j = p - (p / L) * L;
    bf16x8 a[5][C / 32];
#pragma unroll
    for (int t = 0; t < 5; ++t)
        load_tap<C>(a[t], in, b, N, L, i + sign * tap_dy(t), j + sign * tap_dx(t), kq);
    conv_mfma<C>(a, wk, rows, epi);
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

// The sampler's epilogue: the activation also goes to an LDS tile (row =
// configuration within the 16, C channels), the next layer's centre tap.
struct EpiSample {
    bf16 *out;
    bf16 *tile;
    const float *bias;
    int N, C;
    __device__ void operator()(int row, int64_t b, int p, int col, float v) const
    {
        const bf16 h = (bf16)fmaxf(v + bias[col], 0.f);
        out[((int64_t)b * N + p) * C + col] = h;
        tile[row * C + col] = h;
    }
};

struct EpiBackward { // data gradient masked by the ReLU of the layer below
    bf16 *out;
    const bf16 *act;
    int N, C;
    __device__ void operator()(int, int64_t b, int p, int col, float v) const
    {
        const int64_t o = ((int64_t)b * N + p) * C + col;
        out[o] = (bf16)((float)act[o] > 0.f ? v : 0.f);
    }
};

// ---------------------------------------------------------------- forward
__global__ __launch_bounds__(256) void k_l1_fwd(NetDev net, const int8_t *__restrict__ x,
                                                bf16 *__restrict__ h1, int64_t rows_total)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= rows_total)
        return;
    const int N = net.N, L = net.L, C = net.C;
    const int64_t b = g / N;
    const int p = (int)(g - b * N), i = p / L, j = p % L;
    const ParamLayout pl = param_layout(C);
    for (int c = 0; c < C; ++c)
        h1[g * C + c] = (bf16)l1_value(x + b * N, L, i, j, net.w1, net.params + pl.b1, C, c);
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
    conv_tile<C>(in, wk, L, N, +1, RowsOfSites{tile * 16, rows_total, N},
                 EpiForward{out, bias, N, C});
}

__global__ __launch_bounds__(256) void k_l6_fwd(NetDev net, const bf16 *__restrict__ h5,
                                                float *__restrict__ logits, int64_t rows_total)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= rows_total)
        return;
    const int N = net.N, L = net.L;
    const int64_t b = g / N;
    const int p = (int)(g - b * N);
    const ParamLayout pl = param_layout(net.C);
    logits[g] = l6_logit(h5, N, L, net.C, b, p / L, p % L, net.w6, net.params[pl.b6]);
}

// Exact log-probability of each configuration under the sampler: sites in
// raster order, summed in double.
__global__ __launch_bounds__(256) void k_logq(const int8_t *__restrict__ x,
                                              const float *__restrict__ logits, int N, int B,
                                              float *__restrict__ logq)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B)
        return;
    double lq = 0.0;
    for (int p = 0; p < N; ++p)
        lq += site_logq(quantise(prob_plus(logits[(int64_t)b * N + p])), x[(int64_t)b * N + p]);
    logq[b] = (float)lq;
}

// --------------------------------------------------------------- sampling
// One wavefront draws 16 configurations site by site.  At site p it computes
// layer 1 .. 5 activations and the logit of p only (earlier sites are already
// final: every activation at a site depends on strictly earlier spins), then
// draws the spin with a 24-bit uniform of Philox domain 3,
//   counter (stream<<8 | 3<<4, round lo, round hi, p>>2), word p&3.
// The operands from the previous row (three taps of every layer) are loaded
// from the activation arrays at the start of the site, all at once; the
// outputs and spins of the current and previous site, the other two taps,
// are kept in LDS, so within a row no site waits on a store to memory (one
// memory fence per row).  The arithmetic is conv_mfma()'s and l1_from()'s,
// as in the evaluator.
// B operands of one layer held in registers for the whole kernel (C == 32:
// 10 operands per lane and layer).
template <int C>
struct WeightsRegs {
    bf16x8 w[C / 16][5][C / 32];
    __device__ void load(const bf16 *wk)
    {
        const WeightsGlobal<C> g{wk};
#pragma unroll
        for (int n = 0; n < C / 16; ++n)
#pragma unroll
            for (int t = 0; t < 5; ++t)
#pragma unroll
                for (int kc = 0; kc < C / 32; ++kc)
                    w[n][t][kc] = g(16 * n, t, kc);
    }
    __device__ bf16x8 operator()(int n0, int t, int kc) const { return w[n0 / 16][t][kc]; }
};

// A operand of a tap from an LDS tile of 16 rows x C (zero when !ok).
template <int C>
__device__ __forceinline__ void lds_tap(bf16x8 (&at)[C / 32], const bf16 *tile, bool ok, int r,
                                        int kq)
{
#pragma unroll
    for (int kc = 0; kc < C / 32; ++kc) {
        if (ok) {
            at[kc] = *(const bf16x8 *)(tile + r * C + kc * 32 + kq * 8);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                at[kc][e] = (bf16)0.f;
        }
    }
}

// Orders the wavefront's LDS accesses (one wavefront per workgroup) without
// waiting for its global stores.
__device__ __forceinline__ void lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int C>
__global__ __launch_bounds__(64) void k_sample(NetDev net, bf16 *h1, bf16 *h2, bf16 *h3, bf16 *h4,
                                               bf16 *h5, int8_t *__restrict__ x,
                                               float *__restrict__ logq, int B, uint32_t key0,
                                               uint32_t key1, uint32_t stream_base,
                                               uint32_t round_lo, uint32_t round_hi)
{
    constexpr int KC = C / 32;
    constexpr bool kRegW = C == 32; // the four layers' weights fit in registers
    // layer outputs (1..5) and spins at the last two sites, by site parity
    __shared__ __align__(16) bf16 hist[6][2][16 * C];
    __shared__ int8_t xs[2][16];
    const int N = net.N, L = net.L;
    const ParamLayout pl = param_layout(C);
    const int lane = threadIdx.x, r = lane & 15, kq = lane >> 4;
    const int64_t b0 = (int64_t)blockIdx.x * 16;
    bf16 *hs[6] = {nullptr, h1, h2, h3, h4, h5};
    WeightsRegs<(kRegW ? C : 32)> wreg[kRegW ? 4 : 1];
    if (kRegW)
#pragma unroll
        for (int l = 2; l <= 5; ++l)
            wreg[kRegW ? l - 2 : 0].load(net.wf[l]);
    double lq = 0.0;
    const int64_t b = (b0 + r < B) ? b0 + r : -1; // this lane's tile row
    const RowsOfConfigs rows_p{b0, B, 0};
    for (int p = 0; p < N; ++p) {
        const int i = p / L, j = p - (p / L) * L;
        const int cur = p & 1, prv = cur ^ 1;
        const bool left = j > 0; // tap (0, -1) inside the lattice
        // previous-row taps (dy = -1: t = 0, 1, 2) of layers 2..5 and 6, and spins
        bf16x8 pre[4][3][KC];
#pragma unroll
        for (int l = 2; l <= 5; ++l)
#pragma unroll
            for (int t = 0; t < 3; ++t)
                load_tap<C>(pre[l - 2][t], hs[l - 1], b, N, L, i + tap_dy(t), j + tap_dx(t), kq);
        bf16x8 r6[3][C / 8];
        bool in6[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int ii = i + tap_dy(t), jj = j + tap_dx(t);
            in6[t] = !(ii < 0 || jj < 0 || jj >= L);
            if (lane < 16 && b >= 0 && in6[t]) {
                const bf16 *src = h5 + (b * N + ii * L + jj) * C;
#pragma unroll
                for (int v = 0; v < C / 8; ++v)
                    r6[t][v] = *(const bf16x8 *)(src + v * 8);
            }
        }
        // layer 1 at p (mask A: earlier spins only)
        if (b >= 0) {
            float xv[4];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const int ii = i + tap_dy(t), jj = j + tap_dx(t);
                xv[t] = (ii >= 0 && jj >= 0 && jj < L) ? (float)x[b * N + ii * L + jj] : 0.f;
            }
            xv[3] = left ? (float)xs[prv][r] : 0.f;
            for (int c = kq; c < C; c += 4) {
                const bf16 h = (bf16)l1_from(xv, net.w1, net.params + pl.b1, C, c);
                h1[(b * N + p) * C + c] = h;
                hist[1][cur][r * C + c] = h;
            }
        }
        lds_sync();
        RowsOfConfigs rows = rows_p;
        rows.p = p;
#pragma unroll
        for (int l = 2; l <= 5; ++l) {
            bf16x8 a[5][KC];
#pragma unroll
            for (int t = 0; t < 3; ++t)
#pragma unroll
                for (int kc = 0; kc < KC; ++kc)
                    a[t][kc] = pre[l - 2][t][kc];
            lds_tap<C>(a[3], hist[l - 1][prv], b >= 0 && left, r, kq);
            lds_tap<C>(a[4], hist[l - 1][cur], b >= 0, r, kq);
            const EpiSample epi{hs[l], hist[l][cur], net.params + pl.b[l], N, C};
            if constexpr (kRegW)
                conv_mfma_b<C>(a, wreg[l - 2], rows, epi);
            else
                conv_mfma<C>(a, net.wf[l], rows, epi);
            lds_sync();
        }
        if (lane < 16 && b >= 0) {
            // layer 6, in l6_from_rows()'s order: taps 0..4, channels 0..C-1
            const float *w6 = net.w6;
            float acc = 0.f;
#pragma unroll
            for (int t = 0; t < 3; ++t)
                if (in6[t])
#pragma unroll
                    for (int v = 0; v < C / 8; ++v)
#pragma unroll
                        for (int e = 0; e < 8; ++e)
                            acc = fmaf((float)r6[t][v][e], w6[t * C + v * 8 + e], acc);
            if (left) {
                const bf16 *w = hist[5][prv] + r * C;
                for (int ci = 0; ci < C; ++ci)
                    acc = fmaf((float)w[ci], w6[3 * C + ci], acc);
            }
            const bf16 *centre = hist[5][cur] + r * C;
            for (int ci = 0; ci < C; ++ci)
                acc = fmaf((float)centre[ci], w6[4 * C + ci], acc);
            const float z = acc + net.params[pl.b6];
            const float Pq = quantise(prob_plus(z));
            const Block u = philox4x32_10(ctr_word0(stream_base + (uint32_t)b, 3u, 0u), round_lo,
                                          round_hi, (uint32_t)(p >> 2), key0, key1);
            const uint32_t w = (p & 3) == 0 ? u.x0 : (p & 3) == 1 ? u.x1 : (p & 3) == 2 ? u.x2 : u.x3;
            const float uf = (float)(w >> 8) * (1.f / 16777216.f);
            const int xv = uf < Pq ? 1 : -1;
            x[b * N + p] = (int8_t)xv;
            xs[cur][r] = (int8_t)xv;
            lq += site_logq(Pq, xv);
        }
        // the next row reads this row's activations and spins from memory
        if (j == L - 1)
            __syncthreads();
        else
            lds_sync();
    }
    if (lane < 16 && b >= 0)
        logq[b] = (float)lq;
}

// --------------------------------------------------------------- backward
__device__ __forceinline__ float block_sum(float v, float *scratch)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        scratch[w] = v;
    __syncthreads();
    float t = 0.f;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q)
        t += scratch[q];
    return t;
}

// d(mean NLL)/d logit = -s sigmoid(-s z) / B, and the mean NLL itself.
__global__ __launch_bounds__(256) void k_dlogit(const int8_t *__restrict__ x,
                                                const float *__restrict__ logits,
                                                float *__restrict__ dlogit, int64_t rows_total,
                                                float invB, float *loss)
{
    __shared__ float scratch[4];
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (g < rows_total) {
        const float s = (float)x[g], z = logits[g], sz = s * z;
        dlogit[g] = -s / (1.f + expf(sz)) * invB;
        l = (fmaxf(-sz, 0.f) + log1pf(expf(-fabsf(sz)))) * invB;
    }
    const float t = block_sum(l, scratch);
    if (threadIdx.x == 0)
        atomicAdd(loss, t);
}

// Weight and bias gradients of layer 6 over a chunk of rows per block.
__global__ __launch_bounds__(256) void k_l6_wgrad(NetDev net, const bf16 *__restrict__ h5,
                                                  const float *__restrict__ dlogit,
                                                  int64_t rows_total, int rows_per_block,
                                                  float *__restrict__ grad)
{
    __shared__ float scratch[4];
    const int N = net.N, L = net.L, C = net.C;
    const ParamLayout pl = param_layout(C);
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = r0 + rows_per_block < rows_total ? r0 + rows_per_block : rows_total;
    for (int e = threadIdx.x; e < 5 * C; e += blockDim.x) {
        const int t = e / C, ci = e % C;
        float acc = 0.f;
        for (int64_t g = r0; g < r1; ++g) {
            const int64_t b = g / N;
            const int p = (int)(g - b * N), ii = p / L + tap_dy(t), jj = p % L + tap_dx(t);
            if (ii >= 0 && jj >= 0 && jj < L)
                acc = fmaf((float)h5[((int64_t)b * N + ii * L + jj) * C + ci], dlogit[g], acc);
        }
        atomicAdd(&grad[pl.W6 + e], acc);
    }
    float db = 0.f;
    for (int64_t g = r0 + threadIdx.x; g < r1; g += blockDim.x)
        db += dlogit[g];
    db = block_sum(db, scratch);
    if (threadIdx.x == 0)
        atomicAdd(&grad[pl.b6], db);
}

// Data gradient into layer 5, masked by its ReLU: dpre5 = bf16(dh5 * [h5 > 0]).
__global__ __launch_bounds__(256) void k_l6_dgrad(NetDev net, const bf16 *__restrict__ h5,
                                                  const float *__restrict__ dlogit,
                                                  bf16 *__restrict__ dpre, int64_t rows_total)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int N = net.N, L = net.L, C = net.C;
    if (e >= rows_total * C)
        return;
    const int64_t g = e / C;
    const int ci = (int)(e % C);
    const int64_t b = g / N;
    const int p = (int)(g - b * N), i = p / L, j = p % L;
    float dh = 0.f;
    for (int t = 0; t < 5; ++t) {
        const int ii = i - tap_dy(t), jj = j - tap_dx(t);
        if (ii >= 0 && ii < L && jj >= 0 && jj < L)
            dh = fmaf(net.w6[t * C + ci], dlogit[(int64_t)b * N + ii * L + jj], dh);
    }
    dpre[e] = (bf16)((float)h5[e] > 0.f ? dh : 0.f);
}

template <int C>
__global__ __launch_bounds__(256) void k_conv_dgrad(const bf16 *__restrict__ dpre_above,
                                                    bf16 *__restrict__ dpre_below,
                                                    const bf16 *__restrict__ act_below,
                                                    const bf16 *__restrict__ wk, int L, int N,
                                                    int64_t rows_total)
{
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile * 16 >= rows_total)
        return;
    conv_tile<C>(dpre_above, wk, L, N, -1, RowsOfSites{tile * 16, rows_total, N},
                 EpiBackward{dpre_below, act_below, N, C});
}

// Weight and bias gradients of a C -> C layer:
//   dW[t][ci][co] = sum_rows act_below[row shifted by tap t][ci] * dpre[row][co]
// on MFMA, rows as the reduction dimension, 64 rows at a time transposed in LDS.
template <int C>
__global__ __launch_bounds__(256) void k_conv_wgrad(const bf16 *__restrict__ act_below,
                                                    const bf16 *__restrict__ dpre, int L, int N,
                                                    int64_t rows_total, int chunks_per_block,
                                                    float *__restrict__ gW, float *__restrict__ gb)
{
    constexpr int MT = C / 16, TILES = 5 * MT * MT, TPW = TILES / 4;
    __shared__ __align__(16) bf16 sA[5][C][64];
    __shared__ __align__(16) bf16 sD[C][64];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, kq = lane >> 4;
    floatx4 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q)
        acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
    float bacc = 0.f;
    for (int ch = 0; ch < chunks_per_block; ++ch) {
        const int64_t row0 = ((int64_t)blockIdx.x * chunks_per_block + ch) * 64;
        if (row0 >= rows_total)
            break;
        __syncthreads();
        for (int e = tid; e < 64 * C; e += 256) {
            const int k = e / C, c = e % C;
            const int64_t g = row0 + k;
            const bool valid = g < rows_total;
            const int64_t b = valid ? g / N : 0;
            const int p = valid ? (int)(g - b * N) : 0, i = p / L, j = p % L;
            sD[c][k] = valid ? dpre[g * C + c] : (bf16)0.f;
#pragma unroll
            for (int t = 0; t < 5; ++t) {
                const int ii = i + tap_dy(t), jj = j + tap_dx(t);
                const bool ok = valid && ii >= 0 && jj >= 0 && jj < L;
                sA[t][c][k] = ok ? act_below[((int64_t)b * N + ii * L + jj) * C + c] : (bf16)0.f;
            }
        }
        __syncthreads();
        if (tid < C)
            for (int k = 0; k < 64; ++k)
                bacc += (float)sD[tid][k];
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int tile = wave * TPW + q;
            const int t = tile / (MT * MT), m = (tile / MT) % MT, n = tile % MT;
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const bf16x8 av = *(const bf16x8 *)&sA[t][m * 16 + r][ks * 32 + kq * 8];
                const bf16x8 bv = *(const bf16x8 *)&sD[n * 16 + r][ks * 32 + kq * 8];
                acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[q], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int tile = wave * TPW + q;
        const int t = tile / (MT * MT), m = (tile / MT) % MT, n = tile % MT;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ci = m * 16 + kq * 4 + e, co = n * 16 + r;
            atomicAdd(&gW[((int64_t)t * C + ci) * C + co], acc[q][e]);
        }
    }
    if (tid < C)
        atomicAdd(&gb[tid], bacc);
}

// Weight and bias gradients of layer 1 over a chunk of rows per block.
__global__ __launch_bounds__(256) void k_l1_wgrad(NetDev net, const int8_t *__restrict__ x,
                                                  const bf16 *__restrict__ dpre1,
                                                  int64_t rows_total, int rows_per_block,
                                                  float *__restrict__ grad)
{
    const int N = net.N, L = net.L, C = net.C;
    const ParamLayout pl = param_layout(C);
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = r0 + rows_per_block < rows_total ? r0 + rows_per_block : rows_total;
    for (int e = threadIdx.x; e < 5 * C; e += blockDim.x) {
        const int t = e / C, c = e % C; // t == 4: bias
        float acc = 0.f;
        for (int64_t g = r0; g < r1; ++g) {
            const float d = (float)dpre1[g * C + c];
            if (t == 4) {
                acc += d;
                continue;
            }
            const int64_t b = g / N;
            const int p = (int)(g - b * N), ii = p / L + tap_dy(t), jj = p % L + tap_dx(t);
            if (ii >= 0 && jj >= 0 && jj < L)
                acc = fmaf((float)x[(int64_t)b * N + ii * L + jj], d, acc);
        }
        atomicAdd(&grad[t == 4 ? pl.b1 + c : pl.W1 + t * C + c], acc);
    }
}

__global__ __launch_bounds__(256) void k_fill_f32(float *p, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
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

// Independence Metropolis-Hastings step per chain, in float32:
//   log A = beta J (bond' - bond) + log q(x) - log q(x'),
// accepted iff log A >= 0 or u < exp(log A), u a 24-bit uniform of Philox
// domain 2 (counter (stream<<8 | 2<<4, round lo, round hi, 0)).
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
        const float log_a = betaJ[c] * (float)(bond_prop[c] - bond_cur[c]) + logq_cur[c] - logq_prop[c];
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
    hipLaunchKernelGGL(k_pack, dim3(nblocks(total, 256)), dim3(256), 0, s, net);
    return hipGetLastError();
}

hipError_t launch_forward(const NetDev &net, const int8_t *x, int B, bf16 *const h[6],
                          float *logits, float *logq, hipStream_t s)
{
    const int64_t rows = (int64_t)B * net.N;
    const ParamLayout pl = param_layout(net.C);
    hipLaunchKernelGGL(k_l1_fwd, dim3(nblocks(rows, 256)), dim3(256), 0, s, net, x, h[1], rows);
    const uint32_t tiles = nblocks(rows, 16);
    for (int l = 2; l <= 5; ++l) {
        if (net.C == 32)
            hipLaunchKernelGGL(k_conv_fwd<32>, dim3(nblocks(tiles, 4)), dim3(256), 0, s, h[l - 1],
                               h[l], net.wf[l], net.params + pl.b[l], net.L, net.N, rows);
        else
            hipLaunchKernelGGL(k_conv_fwd<64>, dim3(nblocks(tiles, 4)), dim3(256), 0, s, h[l - 1],
                               h[l], net.wf[l], net.params + pl.b[l], net.L, net.N, rows);
    }
    hipLaunchKernelGGL(k_l6_fwd, dim3(nblocks(rows, 256)), dim3(256), 0, s, net, h[5], logits, rows);
    if (logq)
        hipLaunchKernelGGL(k_logq, dim3(nblocks(B, 256)), dim3(256), 0, s, x, logits, net.N, B, logq);
    return hipGetLastError();
}

hipError_t launch_sample(const NetDev &net, int B, bf16 *const h[6], int8_t *x, float *logq,
                         uint64_t seed, uint32_t stream_base, uint64_t round, hipStream_t s)
{
    const uint32_t grid = nblocks(B, 16);
    if (net.C == 32)
        hipLaunchKernelGGL(k_sample<32>, dim3(grid), dim3(64), 0, s, net, h[1], h[2], h[3], h[4],
                           h[5], x, logq, B, (uint32_t)seed, (uint32_t)(seed >> 32), stream_base,
                           (uint32_t)round, (uint32_t)(round >> 32));
    else
        hipLaunchKernelGGL(k_sample<64>, dim3(grid), dim3(64), 0, s, net, h[1], h[2], h[3], h[4],
                           h[5], x, logq, B, (uint32_t)seed, (uint32_t)(seed >> 32), stream_base,
                           (uint32_t)round, (uint32_t)(round >> 32));
    return hipGetLastError();
}

hipError_t launch_backward(const NetDev &net, const int8_t *x, int B, bf16 *const h[6],
                           const float *logits, float *dlogit, bf16 *dpre_a, bf16 *dpre_b,
                           float *grad, float *loss, hipStream_t s)
{
    const int64_t rows = (int64_t)B * net.N;
    const int C = net.C;
    const ParamLayout pl = param_layout(C);
    hipLaunchKernelGGL(k_fill_f32, dim3(nblocks(pl.total, 256)), dim3(256), 0, s, grad, pl.total, 0.f);
    hipLaunchKernelGGL(k_fill_f32, dim3(1), dim3(64), 0, s, loss, (int64_t)1, 0.f);
    hipLaunchKernelGGL(k_dlogit, dim3(nblocks(rows, 256)), dim3(256), 0, s, x, logits, dlogit, rows,
                       1.f / (float)B, loss);
    const int rpb = 1024;
    hipLaunchKernelGGL(k_l6_wgrad, dim3(nblocks(rows, rpb)), dim3(256), 0, s, net, h[5], dlogit, rows,
                       rpb, grad);
    hipLaunchKernelGGL(k_l6_dgrad, dim3(nblocks(rows * C, 256)), dim3(256), 0, s, net, h[5], dlogit,
                       dpre_a, rows);
    bf16 *above = dpre_a, *below = dpre_b;
    const int cpb = 16; // 64-row chunks per workgroup
    const uint32_t tiles = nblocks(rows, 16);
    for (int l = 5; l >= 2; --l) {
        if (C == 32) {
            hipLaunchKernelGGL(k_conv_wgrad<32>, dim3(nblocks(rows, 64 * cpb)), dim3(256), 0, s,
                               h[l - 1], above, net.L, net.N, rows, cpb, grad + pl.W[l],
                               grad + pl.b[l]);
            hipLaunchKernelGGL(k_conv_dgrad<32>, dim3(nblocks(tiles, 4)), dim3(256), 0, s, above,
                               below, h[l - 1], net.wb[l], net.L, net.N, rows);
        } else {
            hipLaunchKernelGGL(k_conv_wgrad<64>, dim3(nblocks(rows, 64 * cpb)), dim3(256), 0, s,
                               h[l - 1], above, net.L, net.N, rows, cpb, grad + pl.W[l],
                               grad + pl.b[l]);
            hipLaunchKernelGGL(k_conv_dgrad<64>, dim3(nblocks(tiles, 4)), dim3(256), 0, s, above,
                               below, h[l - 1], net.wb[l], net.L, net.N, rows);
        }
        bf16 *tmp = above;
        above = below;
        below = tmp;
    }
    hipLaunchKernelGGL(k_l1_wgrad, dim3(nblocks(rows, rpb)), dim3(256), 0, s, net, x, above, rows,
                       rpb, grad);
    return hipGetLastError();
}

hipError_t launch_adam(float *params, const float *grad, float *m, float *v, int64_t n, float lr,
                       float beta1, float beta2, float eps, int64_t step, hipStream_t s)
{
    const float bc1 = 1.f - powf(beta1, (float)step), bc2 = 1.f - powf(beta2, (float)step);
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
