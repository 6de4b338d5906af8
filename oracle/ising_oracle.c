/*
 * Plain CPU oracle for the checkerboard Metropolis simulation of the 2D
 * ferromagnetic Ising model (Romero, Bisson, Fatica, Bernaschi,
 * "A Performance study of the 2D Ising model on GPUs", arXiv:1906.06297).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the GPU library.
 *
 * The lattice is a full L x L array of int8 spins (+1/-1), row-major, periodic
 * in both directions -- the straightforward representation the paper's basic
 * implementation starts from (Sec. 3.1), without the colour compaction or any
 * bit packing.  Every site of one colour is updated from the other colour
 * (Sec. 2, checkerboard decomposition); the Metropolis rule is Sec. 2: accept
 * a flip whose energy change is not positive, otherwise accept it with
 * probability exp(-beta*dE).
 *
 * Readings of the paper that this file fixes (the paper is silent on them):
 *  - Colour of site (i,j) is (i+j)&1, 0 = "black"; black is updated first in
 *    every sweep (Sec. 3.3 launches one kernel per colour without naming the
 *    order).
 *  - The energy of Eq. (1) counts each nearest-neighbour bond once, so the
 *    change from flipping sigma with neighbour sum nn is dE = 2*J*sigma*nn,
 *    as in the update kernels of Fig. 2.
 *  - dE = 0 is accepted (exp(0) = 1 exceeds any uniform in [0,1)).
 *  - +-J spin glass (the extension the conclusions name): couplings
 *    J * Jr, J * Jd with bond signs +1/-1 from Philox domain 4, one draw per
 *    bond; the field h replaces the neighbour sum in a = (4 + sigma h) / 2.
 *  - Heat bath (Sec. 2, the other local rule named there): the flip
 *    probability e^{-beta dE} / (e^{-beta dE} + 1) is evaluated as
 *    1 / (1 + e^{beta dE}) (no intermediate overflow) and quantised the same
 *    way, T[a] = floor(p * 2^32); every class then draws a random number.
 *  - The acceptance probability is quantised to 32 bits: the flip is taken
 *    iff r < T[a], r a uniform 32-bit integer, a = number of neighbours
 *    aligned with sigma, T[a] = 2^32 when dE <= 0 and
 *    floor(exp(-beta*dE) * 2^32) otherwise (IEEE double, libm exp).
 *  - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 *    random numbers: as easy as 1, 2, 3", SC'11), the counter-based generator
 *    the paper uses (Sec. 3.2, Sec. 3.3), addressed without stored state as
 *    the paper does with its seed/sequence/offset triple:
 *       key     = (seed mod 2^32, seed >> 32)
 *       counter = (stream<<8 | domain<<4 | q,  t mod 2^32,  t >> 32,  k)
 *    where k is the 64-spin chunk of the site in colour-linear order
 *    (n = i*(L/2) + j/2, k = n>>6, bit b = n&63), t the half-sweep index
 *    2*(rng_counter + sweep) + colour, domain 0 for sweeps and 1 for the
 *    initial state.  Block q = 0..15 yields bit-planes 2q = x1:x0 and
 *    2q+1 = x3:x2 (high:low 32-bit halves); plane p supplies bit 31-p of the
 *    32-bit r of the spin at bit b.  This oracle always builds all 32 planes.
 *  - Initial state: sigma = +1 iff bit b of plane 0 of the domain-1 block
 *    with t = colour, q = 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, written from the SC'11 description: ten rounds of two      */
/* 32x32->64 multiplies; the key is bumped by the Weyl constants between     */
/* rounds.                                                                   */
/* ------------------------------------------------------------------------ */
#define ORC_PHILOX_MUL_A 0xD2511F53u
#define ORC_PHILOX_MUL_B 0xCD9E8D57u
#define ORC_PHILOX_WEYL_A 0x9E3779B9u
#define ORC_PHILOX_WEYL_B 0xBB67AE85u

void orc_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += ORC_PHILOX_WEYL_A;
            k1 += ORC_PHILOX_WEYL_B;
        }
        uint64_t prod_a = (uint64_t)ORC_PHILOX_MUL_A * x0;
        uint64_t prod_b = (uint64_t)ORC_PHILOX_MUL_B * x2;
        uint32_t y0 = (uint32_t)(prod_b >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)prod_b;
        uint32_t y2 = (uint32_t)(prod_a >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)prod_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

enum { ORC_DOMAIN_SWEEP = 0, ORC_DOMAIN_INIT = 1, ORC_DOMAIN_COUPLINGS = 4 };

/* One Philox block at the canonical address. */
static void orc_block(uint64_t seed, uint32_t stream, uint32_t domain, uint32_t q,
                      uint64_t t, uint64_t chunk, uint32_t out[4])
{
    uint32_t ctr[4];
    uint32_t key[2];
    ctr[0] = (stream << 8) | (domain << 4) | q;
    ctr[1] = (uint32_t)t;
    ctr[2] = (uint32_t)(t >> 32);
    ctr[3] = (uint32_t)chunk;
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    orc_philox4x32_10(ctr, key, out);
}

/* All 32 bit-planes of one chunk at one half-sweep. */
static void orc_planes(uint64_t seed, uint32_t stream, uint64_t t, uint64_t chunk,
                       uint64_t planes[32])
{
    for (uint32_t q = 0; q < 16; ++q) {
        uint32_t x[4];
        orc_block(seed, stream, ORC_DOMAIN_SWEEP, q, t, chunk, x);
        planes[2 * q] = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
        planes[2 * q + 1] = (uint64_t)x[2] | ((uint64_t)x[3] << 32);
    }
}

/* The 32-bit uniform of the spin at bit b: plane p is bit 31-p. */
static uint32_t orc_r_from_planes(const uint64_t planes[32], int b)
{
    uint32_t r = 0;
    for (int p = 0; p < 32; ++p)
        r |= (uint32_t)((planes[p] >> b) & 1u) << (31 - p);
    return r;
}

/* Exported for tests: the uniform of colour-linear site n at half-sweep t. */
uint32_t orc_site_uniform(uint64_t seed, uint32_t stream, uint64_t t, int64_t n)
{
    uint64_t planes[32];
    orc_planes(seed, stream, t, (uint64_t)(n >> 6), planes);
    return orc_r_from_planes(planes, (int)(n & 63));
}

/* ------------------------------------------------------------------------ */
/* Acceptance thresholds (Sec. 2 Metropolis rule; dE from Eq. (1)).          */
/* a = number of the 4 neighbours equal to sigma, so sigma*nn = 2a - 4.      */
/* ------------------------------------------------------------------------ */
void orc_thresholds(double beta, double J, uint64_t *T)
{
    for (int a = 0; a <= 4; ++a) {
        int sigma_nn = 2 * a - 4;
        double dE = 2.0 * J * sigma_nn;
        if (dE <= 0.0) {
            T[a] = (uint64_t)1 << 32;
        } else {
            double p = exp(-(beta * dE));
            T[a] = (uint64_t)floor(p * 4294967296.0);
        }
    }
}

/* Heat-bath thresholds (Sec. 2: a spin flips with probability               */
/* e^{-beta dE} / (e^{-beta dE} + 1)), written as 1 / (1 + e^{beta dE}) so    */
/* that no intermediate overflows; T[a] = floor(p * 2^32), 2^32 when p rounds */
/* to 1.                                                                     */
void orc_thresholds_heatbath(double beta, double J, uint64_t *T)
{
    for (int a = 0; a <= 4; ++a) {
        int sigma_nn = 2 * a - 4;
        double dE = 2.0 * J * sigma_nn;
        double p = 1.0 / (1.0 + exp(beta * dE));
        T[a] = (uint64_t)floor(p * 4294967296.0);
    }
}

/* ------------------------------------------------------------------------ */
/* Lattice helpers.                                                          */
/* ------------------------------------------------------------------------ */
static inline int64_t orc_wrap(int64_t x, int64_t L)
{
    x %= L;
    return x < 0 ? x + L : x;
}

/* Colour-linear index of site (i,j) within its colour array. */
static inline int64_t orc_colour_linear(int64_t i, int64_t j, int64_t L)
{
    return i * (L / 2) + (j >> 1);
}

/* Sum of the four nearest neighbours of (i,j), periodic. */
static inline int orc_neighbour_sum(const int8_t *s, int64_t L, int64_t i, int64_t j)
{
    int64_t up = orc_wrap(i - 1, L), down = orc_wrap(i + 1, L);
    int64_t left = orc_wrap(j - 1, L), right = orc_wrap(j + 1, L);
    return s[up * L + j] + s[down * L + j] + s[i * L + left] + s[i * L + right];
}

/* The Metropolis decision for one site given its uniform. */
static inline int8_t orc_site_update(int8_t sigma, int nn, uint32_t r, const uint64_t *T)
{
    int a = (4 + sigma * nn) / 2;
    return ((uint64_t)r < T[a]) ? (int8_t)-sigma : sigma;
}

/* Initial state. */
void orc_init(int8_t *s, int64_t L, uint64_t seed, uint32_t stream)
{
    int64_t H = L / 2, M = L * L / 2;
    int64_t nchunks = (M + 63) / 64;
    for (int c = 0; c < 2; ++c) {
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < nchunks; ++k) {
            uint32_t x[4];
            orc_block(seed, stream, ORC_DOMAIN_INIT, 0, (uint64_t)c, (uint64_t)k, x);
            uint64_t plane0 = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
            for (int b = 0; b < 64; ++b) {
                int64_t n = 64 * k + b;
                if (n >= M)
                    break;
                int64_t i = n / H, jc = n % H;
                int64_t j = 2 * jc + ((i + c) & 1);
                s[i * L + j] = ((plane0 >> b) & 1u) ? 1 : -1;
            }
        }
    }
}

/* One half-sweep: every site of colour c, each from the other colour only. */
static void orc_half_sweep_impl(int8_t *s, int64_t L, int c, const uint64_t *T, uint64_t seed,
                                uint32_t stream, uint64_t t, int parallel)
{
    int64_t H = L / 2, M = L * L / 2;
    int64_t nchunks = (M + 63) / 64;
#pragma omp parallel for schedule(static) if (parallel)
    for (int64_t k = 0; k < nchunks; ++k) {
        uint64_t planes[32];
        orc_planes(seed, stream, t, (uint64_t)k, planes);
        for (int b = 0; b < 64; ++b) {
            int64_t n = 64 * k + b;
            if (n >= M)
                break;
            int64_t i = n / H, jc = n % H;
            int64_t j = 2 * jc + ((i + c) & 1);
            int8_t sigma = s[i * L + j];
            int nn = orc_neighbour_sum(s, L, i, j);
            s[i * L + j] = orc_site_update(sigma, nn, orc_r_from_planes(planes, b), T);
        }
    }
}

void orc_half_sweep(int8_t *s, int64_t L, int c, const uint64_t *T, uint64_t seed,
                    uint32_t stream, uint64_t t)
{
    orc_half_sweep_impl(s, L, c, T, seed, stream, t, 1);
}

/* Energy (as the bond sum: E = -J * bond) and magnetisation; Eq. (1) with
 * each bond counted once. */
static void orc_observables_impl(const int8_t *s, int64_t L, int64_t *bond, int64_t *mag,
                                 int parallel)
{
    int64_t b = 0, m = 0;
#pragma omp parallel for reduction(+ : b, m) schedule(static) if (parallel)
    for (int64_t i = 0; i < L; ++i) {
        int64_t down = orc_wrap(i + 1, L);
        for (int64_t j = 0; j < L; ++j) {
            int64_t right = orc_wrap(j + 1, L);
            int sigma = s[i * L + j];
            b += sigma * (s[down * L + j] + s[i * L + right]);
            m += sigma;
        }
    }
    *bond = b;
    *mag = m;
}

void orc_observables(const int8_t *s, int64_t L, int64_t *bond, int64_t *mag)
{
    orc_observables_impl(s, L, bond, mag, 1);
}

/* nsweeps full sweeps (black then white) starting at sweep counter
 * rng_counter; optional per-sweep trace of (bond sum, magnetisation). */
static void orc_sweeps_table_impl(int8_t *s, int64_t L, const uint64_t *T, uint64_t seed,
                                  uint32_t stream, int64_t nsweeps, uint64_t rng_counter,
                                  int64_t *bond_trace, int64_t *mag_trace, int parallel)
{
    for (int64_t sw = 0; sw < nsweeps; ++sw) {
        for (int c = 0; c < 2; ++c) {
            uint64_t t = 2 * (rng_counter + (uint64_t)sw) + (uint64_t)c;
            orc_half_sweep_impl(s, L, c, T, seed, stream, t, parallel);
        }
        if (bond_trace && mag_trace)
            orc_observables_impl(s, L, &bond_trace[sw], &mag_trace[sw], parallel);
    }
}

static void orc_sweeps_impl(int8_t *s, int64_t L, double beta, double J, uint64_t seed,
                            uint32_t stream, int64_t nsweeps, uint64_t rng_counter,
                            int64_t *bond_trace, int64_t *mag_trace, int parallel)
{
    uint64_t T[5];
    orc_thresholds(beta, J, T);
    orc_sweeps_table_impl(s, L, T, seed, stream, nsweeps, rng_counter, bond_trace, mag_trace,
                          parallel);
}

void orc_sweeps(int8_t *s, int64_t L, double beta, double J, uint64_t seed, uint32_t stream,
                int64_t nsweeps, uint64_t rng_counter, int64_t *bond_trace, int64_t *mag_trace)
{
    orc_sweeps_impl(s, L, beta, J, seed, stream, nsweeps, rng_counter, bond_trace, mag_trace, 1);
}

/* Sweeps under any acceptance table T[a] (flip iff r < T[a]). */
void orc_sweeps_table(int8_t *s, int64_t L, const uint64_t *T, uint64_t seed, uint32_t stream,
                      int64_t nsweeps, uint64_t rng_counter, int64_t *bond_trace,
                      int64_t *mag_trace)
{
    orc_sweeps_table_impl(s, L, T, seed, stream, nsweeps, rng_counter, bond_trace, mag_trace, 1);
}

/* ------------------------------------------------------------------------ */
/* +-J spin glass (the extension named in the paper's conclusions): bond     */
/* couplings J * Jr[i][j] between (i,j) and (i,j+1) and J * Jd[i][j] between */
/* (i,j) and (i+1,j), Jr, Jd = +1/-1.  The local field is h = sum over the   */
/* four bonds of the bond sign times the neighbour, dE = 2 J sigma h, and     */
/* a = (4 + sigma h) / 2 takes the Metropolis table of (beta, J) as before.   */
/* ------------------------------------------------------------------------ */
static inline int orc_glass_field(const int8_t *s, const int8_t *Jr, const int8_t *Jd,
                                  int64_t L, int64_t i, int64_t j)
{
    int64_t up = orc_wrap(i - 1, L), down = orc_wrap(i + 1, L);
    int64_t left = orc_wrap(j - 1, L), right = orc_wrap(j + 1, L);
    return Jd[up * L + j] * s[up * L + j] + Jd[i * L + j] * s[down * L + j] +
           Jr[i * L + left] * s[i * L + left] + Jr[i * L + j] * s[i * L + right];
}

static void orc_glass_half_sweep(int8_t *s, const int8_t *Jr, const int8_t *Jd, int64_t L,
                                 int c, const uint64_t *T, uint64_t seed, uint32_t stream,
                                 uint64_t t)
{
    int64_t H = L / 2, M = L * L / 2;
    int64_t nchunks = (M + 63) / 64;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nchunks; ++k) {
        uint64_t planes[32];
        orc_planes(seed, stream, t, (uint64_t)k, planes);
        for (int b = 0; b < 64; ++b) {
            int64_t n = 64 * k + b;
            if (n >= M)
                break;
            int64_t i = n / H, jc = n % H;
            int64_t j = 2 * jc + ((i + c) & 1);
            int8_t sigma = s[i * L + j];
            int h = orc_glass_field(s, Jr, Jd, L, i, j);
            s[i * L + j] = orc_site_update(sigma, h, orc_r_from_planes(planes, b), T);
        }
    }
}

/* Random bond signs (probability 1/2 each), one Philox block per 64 bonds:
 * the bond to the right (array x = c) and the bond below (x = 2 + c) of the
 * colour-c site at colour-linear index n take bit n & 63 of x0 | x1 << 32 of
 * block (stream << 8 | 4 << 4 | x, 0, 0, n >> 6); bit 1 means -1. */
void orc_glass_couplings(int8_t *Jr, int8_t *Jd, int64_t L, uint64_t seed, uint32_t stream)
{
    int64_t H = L / 2, M = L * L / 2;
    int64_t nchunks = (M + 63) / 64;
    for (uint32_t x = 0; x < 4; ++x) {
        int c = (int)(x & 1);
        int8_t *dst = x < 2 ? Jr : Jd;
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < nchunks; ++k) {
            uint32_t w[4];
            orc_block(seed, stream, ORC_DOMAIN_COUPLINGS, x, 0, (uint64_t)k, w);
            uint64_t bits = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
            for (int b = 0; b < 64; ++b) {
                int64_t n = 64 * k + b;
                if (n >= M)
                    break;
                int64_t i = n / H, jc = n % H;
                int64_t j = 2 * jc + ((i + c) & 1);
                dst[i * L + j] = ((bits >> b) & 1u) ? -1 : 1;
            }
        }
    }
}

/* Bond sum sum_<ij> J_ij/J sigma_i sigma_j (energy E = -J * bond) and M. */
void orc_glass_observables(const int8_t *s, const int8_t *Jr, const int8_t *Jd, int64_t L,
                           int64_t *bond, int64_t *mag)
{
    int64_t b = 0, m = 0;
#pragma omp parallel for reduction(+ : b, m) schedule(static)
    for (int64_t i = 0; i < L; ++i) {
        int64_t down = orc_wrap(i + 1, L);
        for (int64_t j = 0; j < L; ++j) {
            int64_t right = orc_wrap(j + 1, L);
            int sigma = s[i * L + j];
            b += sigma * (Jd[i * L + j] * s[down * L + j] + Jr[i * L + j] * s[i * L + right]);
            m += sigma;
        }
    }
    *bond = b;
    *mag = m;
}

void orc_glass_sweeps(int8_t *s, const int8_t *Jr, const int8_t *Jd, int64_t L, double beta,
                      double J, uint64_t seed, uint32_t stream, int64_t nsweeps,
                      uint64_t rng_counter, int64_t *bond_trace, int64_t *mag_trace)
{
    uint64_t T[5];
    orc_thresholds(beta, J, T);
    for (int64_t sw = 0; sw < nsweeps; ++sw) {
        for (int c = 0; c < 2; ++c) {
            uint64_t t = 2 * (rng_counter + (uint64_t)sw) + (uint64_t)c;
            orc_glass_half_sweep(s, Jr, Jd, L, c, T, seed, stream, t);
        }
        if (bond_trace && mag_trace)
            orc_glass_observables(s, Jr, Jd, L, &bond_trace[sw], &mag_trace[sw]);
    }
}

/* Many independent lattices, one per thread at a time.  Lattice q occupies
 * spins[offsets[q] .. offsets[q] + Ls[q]^2). */
void orc_batch_sweeps(int8_t *spins, const int64_t *offsets, const int64_t *Ls,
                      const double *betas, int32_t nlat, double J, const uint64_t *seeds,
                      const uint32_t *streams, int64_t nsweeps, uint64_t rng_counter)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t q = 0; q < nlat; ++q)
        orc_sweeps_impl(spins + offsets[q], Ls[q], betas[q], J, seeds[q], streams[q], nsweeps,
                        rng_counter, NULL, NULL, 0);
}

/* ------------------------------------------------------------------------ */
/* Windowed evolution, to check large lattices on a sample of sites.        */
/* win is an h x w block of the periodic L x L lattice whose top-left site  */
/* is (i0, j0).  Its initial contents are the initial state of those sites. */
/* Each half-sweep updates only the window sites whose four neighbours lie  */
/* inside the window, with the global colour and random-number address of   */
/* the site.  Sites at distance d from the window edge are exact for        */
/* d >= (number of half-sweeps done) + 1.                                    */
/* ------------------------------------------------------------------------ */
void orc_window_init(int8_t *win, int64_t L, int64_t i0, int64_t j0, int64_t h, int64_t w,
                     uint64_t seed, uint32_t stream)
{
#pragma omp parallel for schedule(static)
    for (int64_t di = 0; di < h; ++di) {
        int64_t i = orc_wrap(i0 + di, L);
        for (int64_t dj = 0; dj < w; ++dj) {
            int64_t j = orc_wrap(j0 + dj, L);
            int c = (int)((i + j) & 1);
            int64_t n = orc_colour_linear(i, j, L);
            uint32_t x[4];
            orc_block(seed, stream, ORC_DOMAIN_INIT, 0, (uint64_t)c, (uint64_t)(n >> 6), x);
            uint64_t plane0 = (uint64_t)x[0] | ((uint64_t)x[1] << 32);
            win[di * w + dj] = ((plane0 >> (n & 63)) & 1u) ? 1 : -1;
        }
    }
}

void orc_window_sweeps(int8_t *win, int64_t L, int64_t i0, int64_t j0, int64_t h, int64_t w,
                       double beta, double J, uint64_t seed, uint32_t stream, int64_t nsweeps,
                       uint64_t rng_counter)
{
    uint64_t T[5];
    orc_thresholds(beta, J, T);
    for (int64_t sw = 0; sw < nsweeps; ++sw) {
        for (int c = 0; c < 2; ++c) {
            uint64_t t = 2 * (rng_counter + (uint64_t)sw) + (uint64_t)c;
#pragma omp parallel for schedule(static)
            for (int64_t di = 1; di < h - 1; ++di) {
                int64_t i = orc_wrap(i0 + di, L);
                for (int64_t dj = 1; dj < w - 1; ++dj) {
                    int64_t j = orc_wrap(j0 + dj, L);
                    if ((int)((i + j) & 1) != c)
                        continue;
                    int8_t sigma = win[di * w + dj];
                    int nn = win[(di - 1) * w + dj] + win[(di + 1) * w + dj] +
                             win[di * w + dj - 1] + win[di * w + dj + 1];
                    uint32_t r = orc_site_uniform(seed, stream, t, orc_colour_linear(i, j, L));
                    win[di * w + dj] = orc_site_update(sigma, nn, r, T);
                }
            }
        }
    }
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
