/*
 * ising.h -- C ABI of libising.so, a gfx950 (MI355X) implementation of the
 * checkerboard Metropolis simulation of the 2D ferromagnetic Ising model
 * (Romero, Bisson, Fatica, Bernaschi, "A Performance study of the 2D Ising
 * model on GPUs", arXiv:1906.06297).
 *
 * Model (Sec. 2, Eq. (1)): spins sigma = +/-1 on a periodic L x L square
 * lattice, H = -J * sum over nearest-neighbour bonds (each bond once) of
 * sigma_i sigma_j.  A sweep updates all sites of one checkerboard colour in
 * parallel from the other colour, then the other colour (Sec. 2), each site
 * by the Metropolis rule (Sec. 2): a flip with energy change dE <= 0 is
 * accepted, otherwise with probability exp(-beta * dE).
 *
 * Conventions shared by every entry point
 *  - Colour of site (i, j) is (i + j) & 1; colour 0 ("black") is updated
 *    first in each sweep.
 *  - Layout (Sec. 3.1 / Sec. 3.3 compact the two colours into separate
 *    arrays along the rows; here at one bit per spin): colour c is the bit
 *    string of its L*L/2 spins in colour-linear order n = i*(L/2) + j/2, bit
 *    n&63 of 64-bit word n>>6, least significant bit first, bit 1 <=> +1.
 *    A lattice occupies 2 * ising_words_per_colour(L) words, colour 0 first.
 *    Bits past the last spin of a colour are zero and stay zero.
 *  - Acceptance is exact in integers: the flip of a site with a aligned
 *    neighbours is taken iff r < T[a], r a 32-bit uniform and
 *    T[a] = 2^32 if dE <= 0, floor(exp(-beta*dE) * 2^32) otherwise, with
 *    dE = 4*J*(a - 2), evaluated on the host in IEEE double precision.
 *  - Random numbers: Philox4x32-10 (Salmon et al., SC'11), the generator the
 *    paper uses (Sec. 3.2, 3.3), addressed statelessly as the paper does with
 *    seed/sequence/offset: key = seed, counter = (stream_id<<8 | domain<<4 | q,
 *    t mod 2^32, t >> 32, n>>6), t = 2*(rng_counter + sweep) + colour.
 *    Block q gives bit-planes 2q (words x1:x0) and 2q+1 (x3:x2); plane p is
 *    bit 31-p of the spin's r.  The initial state uses domain 1, t = colour,
 *    q = 0: sigma = +1 iff the spin's bit of plane 0 is set.
 *  - Device pointers are HIP device memory owned by the caller.  Host
 *    pointers are ordinary host memory owned by the caller.
 *  - hip_stream is a hipStream_t (0 = the null stream).  Work is enqueued
 *    asynchronously on it unless stated otherwise.
 *  - Every function returns ISING_OK or a negative code and, on error,
 *    enqueues no work; ising_last_error() then describes the failure.
 */
#ifndef ISING_H
#define ISING_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ISING_OK = 0,
    ISING_E_BADARG = -1, /* invalid value or null pointer */
    ISING_E_SIZE = -2,   /* buffer too small, or size outside the supported range */
    ISING_E_HIP = -3     /* a HIP runtime call or kernel launch failed */
};

/* Local update rules (Sec. 2). */
enum {
    ISING_RULE_METROPOLIS = 0, /* flip with probability min(1, e^{-beta dE}) */
    ISING_RULE_HEATBATH = 1    /* flip with probability e^{-beta dE} / (e^{-beta dE} + 1) */
};

/* A lattice: plain data, owned by the caller, as is the memory it points to. */
typedef struct ising_lattice {
    uint64_t *words;    /* device: 2 * ising_words_per_colour(L) words */
    int64_t L;          /* linear size: even, 4 <= L, with L*L/128 < 2^32 */
    uint64_t seed;      /* Philox key */
    uint32_t stream_id; /* counter field that separates lattices sharing a seed; < 2^24 */
    uint32_t reserved;  /* zero */
} ising_lattice;

/* Words per colour, ceil(L*L/128); -1 if L is not a supported size. */
int64_t ising_words_per_colour(int64_t L);

/* The threshold table T[0..4] for (beta, J) (Sec. 2 Metropolis rule with
 * dE from Eq. (1)); host only, no GPU work.  beta >= 0 and J finite. */
int ising_thresholds(double beta, double J, uint64_t *T_out);

/* Fills *lat and writes the initial state into d_words (bytes >= 16 *
 * ising_words_per_colour(L)).  Asynchronous. */
int ising_init(ising_lattice *lat, uint64_t *d_words, size_t bytes, int64_t L, uint64_t seed,
               uint32_t stream_id, void *hip_stream);

/* nsweeps checkerboard sweeps at (beta, J), black then white half-sweep,
 * sweep s using t = 2*(rng_counter + s) + colour (Sec. 2; the counter plays the
 * role of the paper's Philox offset, Sec. 3.2).  Splitting a run into calls
 * with consecutive rng_counter gives the same lattice.  Asynchronous. */
int ising_sweep(const ising_lattice *lat, double beta, double J, int64_t nsweeps,
                uint64_t rng_counter, void *hip_stream);

/* The threshold table T[0..4] of a rule (ISING_RULE_*): flip iff r < T[a],
 * r a uniform 32-bit integer, a the number of neighbours aligned with the
 * spin; T[a] = floor(p * 2^32) of the rule's flip probability p (heat bath
 * evaluated as 1 / (1 + e^{beta dE})), 2^32 when p = 1.  Host only.
 * ISING_E_BADARG for an unknown rule, beta < 0 or a non-finite J. */
int ising_thresholds_rule(double beta, double J, int rule, uint64_t *T_out);

/* As ising_sweep under rule `rule` (Sec. 2: the checkerboard decomposition
 * serves any local rule; heat bath draws for all five classes).  Same
 * counters and planes as ising_sweep, so ISING_RULE_METROPOLIS is
 * ising_sweep.  Asynchronous; ISING_E_BADARG for an unknown rule. */
int ising_sweep_rule(const ising_lattice *lat, double beta, double J, int rule, int64_t nsweeps,
                     uint64_t rng_counter, void *hip_stream);

/* As ising_sweep, and after sweep s writes the bond sum and magnetisation of
 * the lattice to d_bond_trace[s] and d_mag_trace[s] (device, nsweeps int64
 * each).  Asynchronous. */
int ising_sweep_traced(const ising_lattice *lat, double beta, double J, int64_t nsweeps,
                       uint64_t rng_counter, int64_t *d_bond_trace, int64_t *d_mag_trace,
                       void *hip_stream);

/* Writes the bond sum B = sum over bonds of sigma_i sigma_j (energy
 * E = -J * B, Eq. (1)) and the magnetisation M = sum of sigma (Sec. 5.3) to
 * the device int64 pointers d_bond and d_mag.  Asynchronous. */
int ising_observables(const ising_lattice *lat, int64_t *d_bond, int64_t *d_mag,
                      void *hip_stream);

/* +-J spin glass (the extension named in the paper's conclusions): couplings
 * J_ij = J * (1 - 2 b_ij) with one sign bit b_ij per bond.  The bond array
 * (device, caller-owned, 4 * ising_words_per_colour(L) uint64 words) holds
 * four bit arrays x in the colour-compact layout of the spins: x = 0, 1 the
 * bond to the right of every colour-0, colour-1 site, x = 2, 3 the bond below
 * every colour-0, colour-1 site; padding bits 0.  Interleaved word by word:
 * word k of array x is word 4 k + x of the bond array, so that the four bond
 * words of spin word k are one 32-byte chunk; the array must be 16-byte
 * aligned (ISING_E_BADARG otherwise; hipMalloc's alignment suffices).  Only row-aligned
 * sizes (L % 128 == 0; ISING_E_SIZE otherwise).  Every call takes the array's
 * size in bytes and returns ISING_E_SIZE if it is too small.
 *
 * Random signs, each -1 with probability 1/2: bit n of array x is bit n & 63
 * of x0 | x1 << 32 of Philox4x32-10 block (stream_id << 8 | 4 << 4 | x, 0, 0,
 * n >> 6) under key seed.  Asynchronous. */
int ising_glass_bonds_init(uint64_t *d_bonds, size_t bytes, int64_t L, uint64_t seed,
                           uint32_t stream_id, void *hip_stream);

/* Bond array from host L x L int8 arrays of +1/-1: host_right[i*L + j] on the
 * bond (i, j)-(i, j+1), host_down[i*L + j] on (i, j)-(i+1, j), periodic.
 * ISING_E_BADARG for other values.  Synchronises hip_stream. */
int ising_glass_set_bonds(uint64_t *d_bonds, size_t bytes, int64_t L, const int8_t *host_right,
                          const int8_t *host_down, void *hip_stream);

/* As ising_sweep with the couplings of d_bonds: the Metropolis rule of Sec. 2
 * with dE = 2 J sigma h, h the sum over the four bonds of sign times neighbour.
 * Same counters and planes as ising_sweep (all-ferromagnetic bonds give
 * ising_sweep's lattice).  Asynchronous. */
int ising_glass_sweep(const ising_lattice *lat, const uint64_t *d_bonds, size_t bond_bytes,
                      double beta, double J, int64_t nsweeps, uint64_t rng_counter,
                      void *hip_stream);

/* Bond sum sum over bonds of (J_ij / J) sigma_i sigma_j (energy E = -J * that)
 * and magnetisation to the device int64 pointers.  Asynchronous. */
int ising_glass_observables(const ising_lattice *lat, const uint64_t *d_bonds, size_t bond_bytes,
                            int64_t *d_bond, int64_t *d_mag, void *hip_stream);

/* Matrix-multiply formulation of the sweep (Sec. 3.2: the bidiagonal kernel
 * matrix K and the four block equations for the neighbour sums of the black
 * and white blocks), kept as a measured negative control beside the
 * bit-packed kernels; L % 256 == 0 (ISING_E_SIZE otherwise).
 *
 * Spin buffer (device, caller-owned, 16-byte aligned, ising_mm_lattice_bytes
 * = 2 L^2 bytes): one IEEE binary16 per spin (+1 = 0x3C00, -1 = 0xBC00); the
 * lattice as 256 x 256 sub-lattices (row-major over sub-lattices), each as
 * four 128 x 128 row-major blocks sigma_ab, block index 2a + b, holding the
 * sites (2r + a, 2q + b) of the sub-lattice.  Sum buffer (device, 16-byte
 * aligned, ising_mm_sums_bytes = L^2 bytes): the fp16 neighbour sums of one
 * colour, used by the unfused form only.  Both return -1 for an unsupported
 * L. */
int64_t ising_mm_lattice_bytes(int64_t L);
int64_t ising_mm_sums_bytes(int64_t L);

/* Converts the bit-packed lattice `lat` into the fp16 block layout, or back
 * (the words of `lat` are overwritten).  Asynchronous. */
int ising_mm_from_words(const ising_lattice *lat, uint16_t *d_spins, size_t bytes,
                        void *hip_stream);
int ising_mm_to_words(const ising_lattice *lat, const uint16_t *d_spins, size_t bytes,
                      void *hip_stream);

/* nsweeps sweeps of the fp16 lattice (seed and stream_id as in
 * ising_lattice).  Per half-sweep the neighbour sums of the colour are
 * nn = P M1 + M2 Q per target block (P, Q: the blocks holding its horizontal
 * and vertical neighbours; M1, M2: K or its transpose) on fp16 MFMA, plus the
 * edge neighbours from the adjacent sub-lattices, then each run of 64
 * same-colour spins of a row is decided with the Philox counters, planes and
 * exact compare of ising_sweep -- the same lattice, bit for bit, as
 * ising_sweep from the same start.  fused = 0: the paper's three steps
 * (products writing the sums to d_sums, a boundary kernel, an update kernel);
 * fused = 1: one kernel per half-sweep with the sums kept on chip (d_sums may
 * be NULL).  Asynchronous. */
int ising_mm_sweep(int64_t L, uint64_t seed, uint32_t stream_id, uint16_t *d_spins,
                   size_t spin_bytes, uint16_t *d_sums, size_t sum_bytes, double beta, double J,
                   int64_t nsweeps, uint64_t rng_counter, int fused, void *hip_stream);

/* Copies the lattice to host_spins as an L x L row-major int8 array of
 * +1/-1.  Synchronises hip_stream. */
int ising_get_spins(const ising_lattice *lat, int8_t *host_spins, void *hip_stream);

/* Overwrites the lattice from an L x L row-major int8 array of +1/-1 (any
 * other value is rejected).  Synchronises hip_stream. */
int ising_set_spins(const ising_lattice *lat, const int8_t *host_spins, void *hip_stream);

/* ------------------------------------------------------------------------
 * Batches of independent lattices (each L <= 722, so that a lattice fits in
 * LDS), all advanced by one persistent kernel launch.  Each lattice follows
 * exactly the single-lattice rules above with its own seed, stream id and
 * beta; J is shared.  Lattice q occupies 2 * ising_words_per_colour(L_q)
 * words of one caller-owned device buffer, lattices in order, so any lattice
 * can also be used with the single-lattice calls (ising_batch_lattice).
 * The batch object is owned by the library (ising_batch_destroy); it keeps
 * the batch's sweep counter on the device.  Calls on one batch must not
 * overlap from several host threads.
 * ------------------------------------------------------------------------ */
typedef struct ising_batch ising_batch;

/* Total words of a batch buffer; -1 if some L is unsupported. */
int64_t ising_batch_words(int32_t n, const int64_t *Ls);

/* Creates a batch over d_words (bytes >= 8 * ising_batch_words(n, Ls)).
 * Ls, betas, seeds, stream_ids: host arrays of n entries.  Synchronous;
 * allocates the batch's device descriptors and sets its counter to 0. */
int ising_batch_create(ising_batch **out, int32_t n, const int64_t *Ls, const double *betas,
                       double J, const uint64_t *seeds, const uint32_t *stream_ids,
                       uint64_t *d_words, size_t bytes);

/* Frees what ising_batch_create allocated (not the caller's buffer). */
int ising_batch_destroy(ising_batch *b);

/* A single-lattice view of lattice q (words inside the batch buffer). */
int ising_batch_lattice(const ising_batch *b, int32_t q, ising_lattice *out);

/* Initial state of every lattice (same rule as ising_init).  Asynchronous. */
int ising_batch_init(ising_batch *b, void *hip_stream);

/* nsweeps sweeps of every lattice, sweep s of lattice q with
 * t = 2*(counter + s) + colour, then counter += nsweeps; the counter is the
 * batch's own, on the device, so consecutive calls continue every chain
 * exactly as one longer call.  The three kernels of one call (queue reset,
 * persistent sweep, counter advance) are captured once per nsweeps value as a
 * HIP graph and replayed.  Asynchronous. */
int ising_batch_sweep(ising_batch *b, int64_t nsweeps, void *hip_stream);

/* Sets / reads the batch's sweep counter.  Synchronise hip_stream. */
int ising_batch_set_counter(ising_batch *b, uint64_t rng_counter, void *hip_stream);
int ising_batch_get_counter(const ising_batch *b, uint64_t *rng_counter, void *hip_stream);

/* Bond sum and magnetisation of every lattice into device arrays of n int64
 * (E_q = -J * bond[q]).  Asynchronous. */
int ising_batch_observables(const ising_batch *b, int64_t *d_bond, int64_t *d_mag,
                            void *hip_stream);

/* Tile of lattices of size L in the persistent kernel: lpw (1 or 2) lanes per
 * word -- a pair of lanes computes alternate Philox blocks of one word and
 * both apply them in order -- and wpt words per lane group, so a lattice of W
 * words per colour takes ceil(W / wpt) * lpw threads and floor(1024 / that)
 * lattices share a workgroup (the autotuner may also cap that number).  set
 * replans the batch and lifts the cap for L; results never depend on the
 * tile. */
int ising_batch_get_tiles(const ising_batch *b, int64_t L, uint32_t *wpt, uint32_t *lpw);
int ising_batch_set_tiles(ising_batch *b, int64_t L, uint32_t wpt, uint32_t lpw);

/* The current plan for the lattices of size L: the most of them that share
 * one workgroup of the persistent kernel and how many workgroups hold some
 * (with mixed-size bundles, beside lattices of other sizes).  BADARG if the
 * batch has no lattice of size L or an output pointer is NULL. */
int ising_batch_get_plan(const ising_batch *b, int64_t L, uint32_t *lattices_per_workgroup,
                         uint32_t *workgroups);

/* *mixed = 1 if the current plan has bundles that may mix lattice sizes (the
 * autotuner chose them, or ising_batch_set_bundles set them), else 0. */
int ising_batch_get_mixed(const ising_batch *b, int32_t *mixed);

/* Sets the plan explicitly: nbundles workgroup loads in launch order, bundle
 * i holding the counts[i] lattices listed next in `lattices` (indices into
 * the batch; every lattice exactly once), each with its size's current tile,
 * threads back to back (lane-pair tiles first).  BADARG if a bundle
 * needs more than 1024 threads or 64 KiB of LDS, or the list is not a
 * permutation of the batch.  Results never depend on the plan. */
int ising_batch_set_bundles(ising_batch *b, int32_t nbundles, const int32_t *counts,
                            const int32_t *lattices);

/* Times every tile candidate of every lattice size in the batch -- each tile
 * also with a half and a quarter of the lattices per workgroup -- over
 * tune_sweeps sweeps of a scratch copy, each size alone (the batch itself is
 * unchanged), and requires all candidates to produce identical lattices.  The
 * tiles kept are chosen together for the whole launch: the workgroups the
 * chip holds at once bound how many bundles start together, so the fastest
 * tile of each size alone can leave bundles for a second round.  From the
 * timings, a longest-first schedule on those workgroups estimates the
 * makespan of each choice; the best estimate is then timed on the whole
 * batch against the fastest tiles of each size and kept if faster.  Then
 * bundles that mix sizes: from the same timings, each size's tiles get a
 * duration model (two are tried: a bundle of n lattices takes a + n b, a
 * workgroup of several sizes max a + sum b; or a + b per round of wavefronts
 * on the compute unit's SIMDs), lattices are placed largest first where the
 * model's workgroup duration grows least (sizes whose rows are not whole
 * 32-bit halves optionally in workgroups of their own), and the fastest of
 * these plans, each timed on the whole batch, replaces the one-size bundles
 * if it is faster (again with identical lattices); it is then refined by
 * moving lattices out of the slowest workgroups, timed per workgroup on the
 * device clock.  cache_path (may be NULL) is a JSON file keyed by target and
 * kernel version: read if it covers every size, written after tuning (a
 * mixed plan read from it is the tuned one if the file was written for a
 * batch of the same sizes in the same order, else packed again from the
 * cached models).  With ISING_AUTOTUNE_LOG set in the environment
 * the estimates and timings go to stderr.  Synchronises hip_stream;
 * allocates scratch device memory while it runs. */
int ising_batch_autotune(ising_batch *b, int64_t tune_sweeps, const char *cache_path,
                         void *hip_stream);

/* Copies every lattice of the batch to / from device int8 spins (+1/-1), L_q x
 * L_q row-major per lattice, lattices back to back.  set rejects nothing: any
 * nonzero positive byte is +1.  Asynchronous. */
int ising_batch_get_spins_dev(const ising_batch *b, int8_t *d_spins, void *hip_stream);
int ising_batch_set_spins_dev(ising_batch *b, const int8_t *d_spins, void *hip_stream);

/* The batched sweep for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the inputs of
 * ising_batch_create (caller's lattice buffer, initialised as there, e.g. by a
 * batch handle's ising_batch_init) and of one ising_batch_sweep, with the
 * batch's sweep counter given as rng_counter; the lattices end exactly as
 * after ising_batch_set_counter(rng_counter) and ising_batch_sweep(nsweeps)
 * on a batch of the same lattices.  Allocates nothing: the persistent
 * kernel's descriptors, bundle list, work-queue counter and sweep counter go
 * to a fixed device array of 512 KiB per GPU (at most 4096 lattices;
 * ISING_E_SIZE beyond), which keeps the last call's contents; every call
 * rewrites what it uses.  The untuned tiles are used.  Calls from several
 * host threads take turns; calls whose work overlaps on one GPU (different
 * streams) share that array and race.  Asynchronous. */
int ising_batch_sweep_noalloc(int32_t n, const int64_t *Ls, const double *betas, double J,
                              const uint64_t *seeds, const uint32_t *stream_ids,
                              uint64_t *d_words, size_t bytes, int64_t nsweeps,
                              uint64_t rng_counter, void *hip_stream);

/* ------------------------------------------------------------------------
 * Learned global proposal.  The paper names critical slowing down of local
 * Metropolis updates and cluster moves (Sec. 2); here an autoregressive
 * masked-convolution network q(x) = prod_p q(x_p | x_<p) over sites in raster
 * order p = i*L + j proposes whole configurations, accepted by the
 * independence Metropolis-Hastings rule, so the chain keeps the Boltzmann
 * distribution of Eq. (1) exactly.
 *   layer 1: 3x3 mask A (offsets (-1,-1), (-1,0), (-1,+1), (0,-1)), 1 -> C, ReLU
 *   layers 2..5: 3x3 mask B (those and (0,0)), C -> C, ReLU
 *   layer 6: mask B, C -> 1 logit; zero padding; q(x_p = +1 | .) = sigmoid.
 * Parameters: one float32 vector (ising_arnet_num_params(C) entries) in the
 * order W1[4][C], b1[C], (W_l[5][C][C], b_l[C]) for l = 2..5, W6[5][C], b6,
 * W_l[t][ci][co] taking input channel ci at tap t to output co.  Weights are
 * used in bfloat16, activations stored in bfloat16, sums in float32 (MFMA
 * for layers 2..6).  The backward signal is float32 (in the MFMA products as
 * two bfloat16 halves) and gradients are summed in a fixed order, so they do
 * not vary from run to run.  Spins are device int8 arrays, one L x L raster
 * per configuration.  A sampled spin is +1 iff a 24-bit uniform (Philox domain 3)
 * is below sigmoid(logit), so its realised probability is P~ = ceil(P 2^24) /
 * 2^24; log-probabilities returned are the exact log prod_p (P~ or 1 - P~),
 * bit-identical between the sampler and the evaluator.
 * ------------------------------------------------------------------------ */
typedef struct ising_arnet ising_arnet;

/* Number of parameters for C channels (32 or 64); -1 otherwise. */
int64_t ising_arnet_num_params(int32_t channels);

/* Network for L x L configurations (2 <= L <= 1024), C = 32 or 64, and a
 * workspace for batches of up to max_batch configurations (max_batch * L^2 *
 * C < 2^31); parameters start at zero.  Synchronous. */
int ising_arnet_create(ising_arnet **out, int32_t L, int32_t channels, int32_t max_batch);
int ising_arnet_destroy(ising_arnet *net);

/* Copy parameters from / to a device float32 vector.  Asynchronous. */
int ising_arnet_set_params(ising_arnet *net, const float *d_params, void *hip_stream);
int ising_arnet_get_params(const ising_arnet *net, float *d_params, void *hip_stream);

/* log q~ of B configurations into d_logq[B]; d_logits[B][L*L] may be NULL.
 * Asynchronous.  Where two L*L x C bf16 activation buffers, the logits and
 * the spins fit one workgroup's LDS (L = 32 at C = 32 on gfx950), one kernel
 * evaluates each configuration with all layers on chip; otherwise one launch
 * per layer moves the activations through the workspace.  Both give the same
 * values bit for bit (the per-element MFMA sequence of the sampler, so the
 * log q~ of a sampled configuration equals what the sampler reported). */
int ising_arnet_log_prob(ising_arnet *net, const int8_t *d_spins, int32_t B, float *d_logq,
                         float *d_logits, void *hip_stream);

/* Evaluation path of ising_arnet_log_prob: ISING_ARNET_EVAL_AUTO (the
 * on-chip kernel where it fits, the default) or ISING_ARNET_EVAL_LAYERS (one
 * launch per layer always; for comparing the two).  ISING_E_BADARG for any
 * other value. */
#define ISING_ARNET_EVAL_AUTO 0
#define ISING_ARNET_EVAL_LAYERS 1
int ising_arnet_set_eval_mode(ising_arnet *net, int32_t mode);

/* Mean negative log-likelihood -1/B sum_b sum_p log sigmoid(x_bp logit_bp)
 * into d_loss[0] and its gradient into d_grad (may be NULL).  Asynchronous. */
int ising_arnet_gradient(ising_arnet *net, const int8_t *d_spins, int32_t B, float *d_grad,
                         float *d_loss, void *hip_stream);

/* The same backward pass at given forward values instead of the network's
 * own forward pass: d_acts holds the post-ReLU activations of layers 1..5 as
 * bfloat16 bit patterns, [5][B][L*L][C], d_logits the logits [B][L*L]
 * (float32); ReLU masks are d_acts > 0.  The backward pass alone is then a
 * function of its inputs (the forward pass's bf16 rounding decisions, which
 * float32 sums may take differently from other evaluations, are fixed), for
 * checking it element by element.  Asynchronous. */
int ising_arnet_gradient_at(ising_arnet *net, const int8_t *d_spins, int32_t B,
                            const uint16_t *d_acts, const float *d_logits, float *d_grad,
                            float *d_loss, void *hip_stream);

/* One Adam step (Kingma and Ba) on that loss: beta1, beta2 and eps are the
 * float32 values nearest 0.9, 0.999 and 1e-8, the bias corrections 1 -
 * beta^t of the network's step count t are formed in double and rounded, the
 * update itself is float32.  Asynchronous. */
int ising_arnet_train_step(ising_arnet *net, const int8_t *d_spins, int32_t B, float lr,
                           float *d_loss, void *hip_stream);

/* The same Adam step with a caller's gradient d_grad (num_params floats,
 * device).  Asynchronous. */
int ising_arnet_adam(ising_arnet *net, const float *d_grad, float lr, void *hip_stream);

/* Draws B configurations: sites along anti-diagonals j + 2i = t (each needs
 * only sites of diagonal t - 1 and earlier), each configuration held in LDS
 * by one workgroup; configuration b uses Philox stream id stream_base + b
 * (< 2^24) and counter word `round`.  Writes the spins and their log q~.
 * Needs L <= 128 and the configuration's activation ring within the
 * device's LDS per workgroup (ISING_E_SIZE otherwise).  Asynchronous. */
int ising_arnet_sample(ising_arnet *net, int32_t B, uint64_t seed, uint32_t stream_base,
                       uint64_t round, int8_t *d_spins, float *d_logq, void *hip_stream);

/* Bond sum and magnetisation of B int8 configurations (periodic, each bond
 * once).  Asynchronous. */
int ising_spins_observables(const int8_t *d_spins, int32_t B, int64_t L, int64_t *d_bond,
                            int64_t *d_mag, void *hip_stream);

/* Training minibatch of B configurations from a pool of P int8
 * configurations (L x L each, 2 <= L <= 1024), each under a random symmetry
 * of the periodic Boltzmann weight of Eq. (1) -- a global spin flip and a
 * translation -- all drawn from Philox block stream_base + b (< 2^24) of
 * domain 5 at counter word `round`, (x0..x3): configuration
 * k = floor((x1 2^32 + x0) P / 2^64), flipped iff x2 is odd, translated by
 * di = (x2 >> 1) mod L rows and dj = x3 mod L columns:
 * out[b][i][j] = +-pool[k][(i + di) mod L][(j + dj) mod L].  Asynchronous. */
int ising_spins_minibatch(const int8_t *d_pool, int64_t P, int64_t L, int32_t B, uint64_t seed,
                          uint32_t stream_base, uint64_t round, int8_t *d_out, void *hip_stream);

/* Independence Metropolis-Hastings step for n chains of L x L spins, in
 * float32, each operation rounded on its own:
 * log A = ((betaJ[c] (bond'[c] - bond[c])) + logq[c]) - logq'[c];
 * accepted iff log A >= 0 or u < exp(log A), u a 24-bit uniform of Philox
 * domain 2 (stream stream_base + c, counter word `round`).  Accepted chains
 * take the proposal's spins, log q and bond sum in place; d_accepted[c] is
 * 1 or 0.  Asynchronous. */
int ising_mh_independence(int32_t n, int64_t L, int8_t *d_state, float *d_logq, int64_t *d_bond,
                          const int8_t *d_prop, const float *d_logq_prop,
                          const int64_t *d_bond_prop, const float *d_betaJ, uint64_t seed,
                          uint32_t stream_base, uint64_t round, int32_t *d_accepted,
                          void *hip_stream);

/* The random-number generator alone, for measurement: blocks q = 0 ..
 * blocks_per_word-1 of Philox4x32-10 (Salmon et al., SC'11, the generator of
 * Sec. 3.3) for word indices 0 .. nwords-1 with the half-sweep's counter layout
 * (stream_id, half-sweep index t, key seed), spread over sink_words threads (a
 * multiple of 256), each folding its outputs into d_sink[thread].  Its rate
 * bounds any sweep that decides with the exact lazy compare.  Asynchronous. */
int ising_philox_rate(uint64_t nwords, uint32_t blocks_per_word, uint64_t seed,
                      uint32_t stream_id, uint64_t t, uint32_t *d_sink, uint32_t sink_words,
                      void *hip_stream);

/* Selects the half-sweep kernel for later calls in this process, for tests and
 * measurements.  0 = default, by size (Metropolis and heat bath): for
 * row-aligned sizes (L % 128 == 0) the streaming row kernel with its
 * per-wavefront work queue, with 16-row bands when that makes at least 16384
 * wavefronts (L >= 49152) and 8-row bands when those make at least 1024 (L >=
 * 8192); otherwise the general kernel, one thread per word.  1 = the
 * general-geometry kernel for every size, 2 = the row kernel without the work
 * queue, 3, 4, 5 = the queued row kernel with 32-, 16- or 8-row bands for
 * every row-aligned size.  ising_glass_sweep takes the queued row kernel
 * (default: 8-row bands at every size; 3, 4, 5 as above) and its per-word row
 * kernel for 1 and 2.
 * All choices give identical lattices.  Process-wide setting; not
 * synchronised with calls running on other threads. */
int ising_set_sweep_kernel(int variant);

/* Description of the last error on the calling thread ("" if none). */
const char *ising_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ISING_H */
