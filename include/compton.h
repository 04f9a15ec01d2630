/*
 * compton.h -- C ABI of libcompton.so: the per-pair Compton-scattering
 * Monte-Carlo step of a particle-in-cell code and the small network that
 * stands in for its inverse-CDF angle/energy sampler, on AMD MI355X (gfx950).
 *
 * Method (Badiali, Bilbao, Cruz, Silva, "Machine Learning-based models in
 * particle-in-cell codes for advanced physics extensions"):
 *   Sec. 3.1  particles are binned into collision cells and paired inside each
 *             cell; for every pair the interaction probability is compared
 *             with a random number; accepted collisions are resolved and both
 *             momenta updated.
 *   Sec. 3.2  the probability is a function of the macro-particle weights,
 *             momenta and a normalisation factor: the photon is boosted into
 *             the lepton rest frame, the Klein-Nishina cross-section is
 *             evaluated there and the rate is carried back to the lab frame;
 *             P_max = 2 sigma_T c dt max[w_e, w_gamma] bounds it.
 *   Sec. 2    a network object is loaded once and then run on any batch of
 *             inputs; Sec. 4: it can also be trained inside the simulation.
 *
 * Units: momenta in m_e c, energies in m_e c^2.  Cross-sections enter as
 * s(x) = sigma_KN(x) / sigma_T with x the rest-frame photon energy.
 *
 * Conventions shared by every call:
 *   - Every pointer to particle, offset, input or output data is DEVICE memory
 *     owned by the caller; it must stay valid until the work queued on
 *     `stream` has completed.  Particle arrays are updated in place.
 *   - Calls only queue work on `stream` (a hipStream_t passed as void*; NULL
 *     is the default stream) and return without synchronising, except the
 *     calls documented as synchronous.
 *   - Every call returns a cs_status; on failure nothing is queued and
 *     cs_last_error() describes the reason.  No C++ exception crosses the ABI.
 *   - Physical anomalies are not errors: they are counted in cs_stats.
 *   - One context per host thread and stream; contexts are not thread-safe.
 */
#ifndef COMPTON_H
#define COMPTON_H

#include <stdint.h>

/* Exported entry points (the library is built with hidden visibility). */
#if defined(__GNUC__)
#define CS_API __attribute__((visibility("default")))
#else
#define CS_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CS_OK = 0,
    CS_ERR_INVALID_ARG = 1, /* null pointer, bad size, dt <= 0, bad enum ...      */
    CS_ERR_LAYOUT = 2,      /* cell offsets not a valid layout (cs_check_layout) */
    CS_ERR_UNSUPPORTED = 3, /* valid request this library does not handle       */
    CS_ERR_HIP = 4,         /* the HIP runtime reported an error                */
    CS_ERR_IO = 5,          /* file missing, unreadable or corrupt              */
    CS_ERR_NOT_READY = 6    /* MLP sampler requested without a usable network   */
} cs_status;

/* Storage type of particle and sampler arrays.  Arithmetic is FP64 either way. */
typedef enum { CS_F32 = 0, CS_F64 = 1 } cs_dtype;

/* Angle/energy sampler used for accepted collisions. */
typedef enum {
    CS_SAMPLER_PLAIN = 0,    /* inverse CDF of the Klein-Nishina angular law, FP64 */
    CS_SAMPLER_MLP_F32 = 1,  /* network, FP32 arithmetic                          */
    CS_SAMPLER_MLP_BF16 = 2, /* network, BF16 MFMA hidden layers, FP32 accumulate */
    CS_SAMPLER_MLP_FP8 = 3   /* network, FP8 E4M3 MFMA, per-layer scales          */
} cs_sampler;

typedef enum { CS_LOSS_MSE = 0, CS_LOSS_MAE = 1 } cs_loss;

typedef struct cs_ctx cs_ctx;
typedef struct cs_mlp cs_mlp;

/* One particle species as structure of arrays: x, y, z momentum components
 * (m_e c) and macro-particle weight w, each n elements of the call's dtype. */
typedef struct {
    void* x;
    void* y;
    void* z;
    void* w;
    int64_t n;
} cs_species;

/* Per-step counters and sums, written to device memory by cs_compton_step.
 * 128 bytes. */
typedef struct {
    int64_t n_pairs;      /* candidate pairs formed                              */
    int64_t n_collided;   /* pairs with u < P                                    */
    int64_t n_clipped;    /* pairs whose P exceeded 1 and was clipped to 1       */
    int64_t n_invalid;    /* pairs skipped: non-finite input or negative weight  */
    int64_t n_fallback;   /* MLP sampler only: samples outside the network's x   */
                          /* range, resolved by the plain sampler                */
    int64_t layout_error; /* 1 when the offsets were not a valid layout; then    */
                          /* no particle was touched                             */
    int64_t overflow;     /* NTC steps only: 1 when the step drew more           */
                          /* candidates than it can hold (2^31 - 2, or a NTC     */
                          /* graph's capacity); then no particle was touched and */
                          /* n_pairs holds the count (at most 2^31 - 1)          */
    int64_t reserved_i;
    double sum_prob;      /* sum of P over valid pairs (fixed summation order)   */
    double energy_before; /* sum over collided pairs of gamma + eps before       */
    double energy_after;  /* ... and gamma' + eps' after (pre-storage rounding)  */
    double reserved_d[5];
} cs_stats;

/* ---------------------------------------------------------------- lifecycle */

/* Create a context on HIP device `device` (its workspace grows on demand). */
CS_API cs_status cs_create(cs_ctx** out, int device);
CS_API cs_status cs_destroy(cs_ctx* ctx);
/* Text of the last failure on this context (never NULL; "" after success).
 * With ctx == NULL: the last failure of cs_create. */
CS_API const char* cs_last_error(const cs_ctx* ctx);
/* Synchronous: wait for `stream` and report any asynchronous HIP error. */
CS_API cs_status cs_sync(cs_ctx* ctx, void* stream);

/* ------------------------------------------------------------ the step ---- */

/*
 * cs_compton_step -- one Monte-Carlo Compton step over every collision cell.
 *
 * Particles are sorted by cell: cell c owns electrons [off_e[c], off_e[c+1])
 * and photons [off_g[c], off_g[c+1]).  off_e / off_g are int64 device arrays
 * of n_cells + 1 entries; a valid layout starts at 0, never decreases and ends
 * at the species count.  An invalid layout is detected on the device: the step
 * then touches no particle and sets stats->layout_error (use cs_check_layout
 * for a synchronous check).
 *
 * Per cell with N_e electrons and N_g photons, min(N_e, N_g) pairs are formed:
 * the smaller species in storage order, the larger one through a keyed
 * pseudo-random bijection of its [0, N) drawn per (seed, cell, step), so no
 * particle is in two pairs.  With N_max = max(N_e, N_g), each pair collides
 * with probability
 *     P = dt * density_norm * N_max * max(w_e, w_g) * s(x) * (1 - beta . k_hat)
 * (clipped to 1), where density_norm = sigma_T c / V_cell in the caller's
 * units; P <= 2 dt density_norm N_max max(w) is the paper's P_max.
 * An accepted pair takes its rest-frame scattering cosine from `sampler`
 * (PLAIN: the inverse Klein-Nishina CDF), conserves momentum exactly
 * (p' = p + k - k'), and is written back in place; with unequal weights the
 * lighter particle always moves and the heavier with probability
 * w_min / w_max.  Random numbers come from Philox4x32-10 keyed by `seed`,
 * with counters built from (particle or cell index, step, purpose), so a
 * step is a pure function of (state, seed, step).
 *
 * dtype:   storage type of all eight particle arrays.
 * sampler: CS_SAMPLER_PLAIN with mlp == NULL, or an MLP sampler with a
 *          network prepared by cs_mlp_quantize for that precision.
 * stats:   nullable device pointer to one cs_stats, overwritten.
 * Errors:  CS_ERR_INVALID_ARG (null arrays with n > 0, n_cells < 0,
 *          dt <= 0 or non-finite, density_norm < 0, bad enums),
 *          CS_ERR_UNSUPPORTED (a species count >= 2^31),
 *          CS_ERR_NOT_READY (MLP sampler without prepared weights).
 */
CS_API cs_status cs_compton_step(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons,
                          const int64_t* off_e, const int64_t* off_g, int64_t n_cells, double dt,
                          double density_norm, uint64_t seed, uint64_t step, cs_sampler sampler,
                          const cs_mlp* mlp, cs_stats* stats, void* stream);

/*
 * cs_compton_step_noalloc -- cs_compton_step for callers that cannot
 * allocate device memory during the step (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): it calls no
 * hipMalloc, hipFree or allocating routine.  Same arguments, semantics,
 * results (bit for bit) and errors as cs_compton_step; it always runs the
 * fused strategy, whatever the context's options.
 *
 * Its workspace is a static device buffer of 8 MiB that the library holds on
 * every device it runs on until the process ends (looked up and initialised
 * once per device by cs_create).  That bounds the problem: about 24 bytes per
 * cell plus 4 per 256 pairs, i.e. roughly 340,000 cells of 256 pairs; larger
 * problems fail with CS_ERR_UNSUPPORTED (and cs_last_error says how much the
 * step would need) before anything is queued.
 *
 * Every call on one device shares that device's buffer, whatever the
 * context: calls on one stream (or otherwise ordered) are safe; calls that
 * overlap on one device -- concurrent streams, or threads -- race and give
 * undefined results.
 */
CS_API cs_status cs_compton_step_noalloc(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons,
                                  const int64_t* off_e, const int64_t* off_g, int64_t n_cells, double dt,
                                  double density_norm, uint64_t seed, uint64_t step, cs_sampler sampler,
                                  const cs_mlp* mlp, cs_stats* stats, void* stream);

/* Synchronous layout check of device offsets: CS_OK or CS_ERR_LAYOUT. */
CS_API cs_status cs_check_layout(cs_ctx* ctx, const int64_t* off, int64_t n_cells, int64_t n_particles,
                          void* stream);

/* cs_ntc_step -- one Compton step with no-time-counter candidate selection
 * (Bird's NTC method, named in Sec. 3.1 as the way the module shortens each
 * cell's pair list; probability and its bound from Sec. 3.2), in place of
 * the 1:1 pairing of cs_compton_step.  Same arrays, layout, units and
 * weight rule as cs_compton_step, plain inverse-CDF sampler.
 *
 * Per cell, with W the largest finite non-negative weight among its
 * electrons and photons: P_max = 2 dt density_norm W; N_e N_g P_max
 * candidates, rounded stochastically, each an electron and a photon picked
 * uniformly with replacement and accepted with probability P / P_max,
 * P = dt density_norm max(w_e, w_g) s(x) flux.  A cell's candidates are
 * taken in order, each on the momenta the earlier collisions of its cell
 * left; the GPU resolves candidates that share no particle in parallel, with
 * the same result.  Random numbers: Philox4x32-10 keyed by `seed`, counters
 * from (cell, candidate number, step, purpose).
 *
 * stats (nullable device pointer): n_pairs = candidates, n_collided,
 * n_invalid (candidates with a non-finite value or a negative weight),
 * n_clipped = candidates with P > P_max (none, by the bound), sum_prob = the
 * sum of P / P_max over valid candidates (the expected collision count),
 * energy sums as cs_compton_step.
 *
 * The call queues the whole step, then waits until the step's candidate
 * count is known on the device (the rest of the step runs meanwhile): the
 * launches are sized for the context's candidate capacity, and a step that
 * draws more candidates than that changes nothing, so the call grows the
 * capacity and queues the step again (this happens on the first call and
 * whenever the count grows past the capacity, which is then set 25% above
 * the count).  The context keeps the scratch: about 60 bytes per candidate
 * of capacity, 300 per cell, and 32 per particle (tags that persist
 * across calls).
 * Errors: CS_ERR_INVALID_ARG (NULL arrays with n > 0, NULL offsets,
 *         n_cells >= 2^31 - 1, dt <= 0 or non-finite, density_norm < 0),
 *         CS_ERR_UNSUPPORTED (a species count >= 2^31, or 2^31 - 1 or more
 *         candidates in the step; nothing was changed, stats->overflow = 1),
 *         CS_ERR_LAYOUT (offsets not a valid layout; nothing was changed,
 *         stats->layout_error = 1).
 */
CS_API cs_status cs_ntc_step(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons,
                             const int64_t* off_e, const int64_t* off_g, int64_t n_cells, double dt,
                             double density_norm, uint64_t seed, uint64_t step, cs_stats* stats, void* stream);

/*
 * cs_bin_particles -- group one species by collision cell, the staging that
 * precedes pairing (Sec. 3.1: the particles of each cell are collected
 * before pairs are formed), so that a caller need not sort on the host.
 *
 * cell[i] (int32, device) is particle i's cell.  The particles with a cell
 * in [0, n_cells) are written to `out` in cell order, stable (inside a cell
 * they keep their input order): out position off[c] + k holds the k-th
 * particle of cell c.  off (int64 device array of n_cells + 1) receives the
 * CSR offsets, off[n_cells] = number of such particles; `out` is then a
 * valid species for cs_compton_step with these offsets.  Particles whose id
 * lies outside [0, n_cells) belong to no cell: they are counted into
 * *n_invalid (int64 device scalar, may be NULL) and placed after the cells,
 * at out positions off[n_cells] .. n - 1, in input order.
 *
 * in and out: distinct device SoA arrays (x, y, z, w) of `dtype`, in.n =
 * out.n = n with 0 <= n < 2^31; 0 <= n_cells < 2^31 - 1.  Caller-owned; the
 * library keeps a scratch buffer in the context (about 40 n bytes, grown on
 * demand: a growth synchronises `stream` first).  Asynchronous on `stream`.
 * CS_ERR_INVALID_ARG for bad sizes, NULL or overlapping arrays.
 */
CS_API cs_status cs_bin_particles(cs_ctx* ctx, cs_dtype dtype, const int32_t* cell, cs_species in, cs_species out,
                          int64_t* off, int64_t n_cells, int64_t* n_invalid, void* stream);

/* Rest-frame photon energy x = gamma eps - p . k (in m_e c^2; the invariant
 * P.K of Sec. 3.2's boost to the lepton frame) of the n pairs (electron i,
 * photon i), i < n <= min(electrons.n, photons.n), evaluated in FP64 by the
 * step's own cancellation-free form; x_out: n doubles (device).  Weights are
 * not read.  For sampler inputs shaped like a plasma's pairs.
 * CS_ERR_INVALID_ARG on NULL arrays, a bad dtype or n out of range. */
CS_API cs_status cs_pair_x(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons, int64_t n,
                    double* x_out, void* stream);

/*
 * cs_sample_plain -- the conventional sampler on its own: for each i,
 * mu[i] = F^-1(u[i]; x[i]) with F the CDF of the rest-frame scattering cosine
 * under the Klein-Nishina law, and ratio[i] = eps'/eps = 1/(1 + x(1 - mu)).
 * Arrays of n elements of `dtype` (FP64 arithmetic either way); x >= 0,
 * u in [0, 1).  Used for training targets and the sampler-stage benchmark.
 */
CS_API cs_status cs_sample_plain(cs_ctx* ctx, cs_dtype dtype, const void* x, const void* u, int64_t n,
                          void* mu_out, void* ratio_out, void* stream);

/* ------------------------------------------- the probability network --- */

/*
 * The paper's own learned component (Sec. 3.2): a dense network that maps a
 * candidate pair to its probability of interaction against the cell's
 * majorant, y' = P / P_max, in place of the analytic evaluation.
 *
 * Inputs: CS_PNET_INPUTS FP32 values per pair, row-major [n][9]: photon
 * momentum k (3), lepton momentum p (3), the majorant P_max, the weights
 * w_e, w_g (code units).  Network 9 -> 9 -> 12 -> 9 -> 1, ReLU hidden layers,
 * sigmoid output.  Parameters: CS_PNET_PARAMS FP32 values, per layer the
 * weight matrix W[n_out][n_in] row-major, then the bias b[n_out].  All arrays
 * are caller-owned device memory; every call is asynchronous on `stream`;
 * CS_ERR_INVALID_ARG for NULL arrays or bad sizes.
 */
#define CS_PNET_INPUTS 9
#define CS_PNET_PARAMS 337

/* The analytic target of each pair: y = P / P_max = s(x) (1 - beta . k_hat)
 * / 2 with x the rest-frame photon energy and s = sigma_KN / sigma_T (FP64
 * arithmetic, Sec. 3.2), independent of P_max and the weights given that
 * P_max bounds the pair's P = tau w_max s(x) (1 - beta . k_hat). */
CS_API cs_status cs_pnet_target(cs_ctx* ctx, const float* in, int64_t n, float* y_out, void* stream);

/* y_out[i] = the network's y' for pair i. */
CS_API cs_status cs_pnet_forward(cs_ctx* ctx, const float* params, const float* in, int64_t n, float* y_out,
                          void* stream);

/* Gradient of the mean loss over the n pairs (MAE, the paper's, or MSE:
 * mean |y' - t|, mean (y' - t)^2 / 2) with respect to the parameters into
 * grad_out (CS_PNET_PARAMS), and the loss into *loss_out (device scalar, may
 * be NULL).  Per-pair contributions are summed in a fixed order (the result
 * does not depend on timing).  The context keeps a scratch of about 1.3 n
 * bytes, grown on demand (a growth synchronises `stream`). */
CS_API cs_status cs_pnet_grad(cs_ctx* ctx, const float* params, const float* in, const float* target, int64_t n,
                       cs_loss loss, float* grad_out, float* loss_out, void* stream);

/* One Adam step (Kingma & Ba: beta1 0.9, beta2 0.999, eps 1e-8, bias
 * corrected) on the CS_PNET_PARAMS parameters with moments m, v (zero before
 * step 1); t >= 1 the step number, lr > 0 (the paper's: 1e-3). */
CS_API cs_status cs_pnet_adam(cs_ctx* ctx, float* params, const float* grad, float* m, float* v, int64_t t, float lr,
                       void* stream);

/* ------------------------------------------------- the learned sampler --- */

/*
 * A small fully connected network standing in for the inverse-CDF sampler
 * (Sec. 2: the network object is loaded once and run on any batch; Sec. 3.2:
 * dense layers trained with Adam on data the conventional method produced;
 * Sec. 4: training can run inside the simulation).  Inputs (x, u): the
 * rest-frame photon energy x in [1e-4, 1e2] and a uniform u in [0, 1);
 * features f1 = (log10 x + 1)/3, f2 = 2u - 1.  Hidden layers use SiLU, the
 * output layer is linear and gives (mu_hat, r_hat) ~ (cos theta, eps'/eps).
 * The sampler reading is mu = clamp(mu_hat, -1, 1) and r = 1/(1 + x(1 - mu)),
 * so the Compton relation holds exactly; inputs with x outside the trained
 * range fall back to the plain sampler.
 *
 * Widths: the library's kernels take exactly {2, 64, 64, 64, 64, 2}
 * (12,802 parameters); other widths give CS_ERR_UNSUPPORTED.
 * Parameter layout (host and device, FP32): per layer the weight matrix
 * W[n_out][n_in] row-major, then the bias[n_out].
 * The network owns its device memory: FP32 master weights, Adam moments and
 * step count, and the BF16 / FP8 copies prepared by cs_mlp_quantize.
 */
#define CS_MLP_X_MIN 1e-4 /* default x range of a network (cs_mlp_set_domain) */
#define CS_MLP_X_MAX 1e2

CS_API cs_status cs_mlp_create(cs_ctx* ctx, const int32_t* widths, int32_t n_widths, const float* init_params_host,
                        cs_mlp** out); /* init_params_host: n_params floats, or NULL for zeros */
CS_API cs_status cs_mlp_destroy(cs_mlp* mlp);
CS_API int64_t cs_mlp_num_params(const cs_mlp* mlp); /* -1 for NULL */
/* Synchronous host copies of the FP32 master parameters.  Setting them
 * invalidates the BF16 / FP8 copies and keeps the Adam state. */
CS_API cs_status cs_mlp_set_params(cs_mlp* mlp, const float* host, int64_t n);
CS_API cs_status cs_mlp_get_params(const cs_mlp* mlp, float* host, int64_t n);
/* The x range [x_min, x_max] the network answers for (synchronous).  Its
 * first input feature is log10 x mapped linearly from [log10 x_min,
 * log10 x_max] onto [-1, 1]; samples with x outside the range (compared in
 * FP32) are answered by the plain sampler and counted as fallbacks.  Default
 * [CS_MLP_X_MIN, CS_MLP_X_MAX]; a network is trained for one range, so set it
 * before training.  Setting it invalidates the FP8 copy (its input scales
 * depend on the features).  CS_ERR_INVALID_ARG unless 0 < x_min < x_max,
 * both finite. */
CS_API cs_status cs_mlp_set_domain(cs_mlp* mlp, double x_min, double x_max);
CS_API cs_status cs_mlp_get_domain(const cs_mlp* mlp, double* x_min, double* x_max);
/* Save / load (synchronous): a versioned binary file with the widths, the
 * FP32 parameters, the Adam moments and step count, the x range, and a
 * checksum (files of the first version, without the x range, load with the
 * default range).  CS_ERR_IO on a missing, truncated or corrupt file. */
CS_API cs_status cs_mlp_save(const cs_mlp* mlp, const char* path);
CS_API cs_status cs_mlp_load(cs_ctx* ctx, const char* path, cs_mlp** out);

/* Prepare the reduced-precision copy used by `precision` (MLP_BF16: weights
 * rounded to BF16; MLP_FP8: weights and layer inputs scaled per layer by
 * amax/448 and rounded to OCP FP8 E4M3, the input scales calibrated on the n
 * device samples (calib_x, calib_u), which must lie in the trained range).
 * MLP_F32 needs no preparation.  Queues work on `stream`. */
CS_API cs_status cs_mlp_quantize(cs_ctx* ctx, cs_mlp* mlp, cs_sampler precision, const float* calib_x,
                          const float* calib_u, int64_t n, void* stream);

/* Raw network outputs y[2 i], y[2 i + 1] = (mu_hat, r_hat) for n device
 * inputs, in `precision` (F32 on the VALU; BF16 / FP8 on MFMA with FP32
 * accumulation; first and last layers FP32).  No range check. */
CS_API cs_status cs_mlp_forward(cs_ctx* ctx, const cs_mlp* mlp, cs_sampler precision, const float* x, const float* u,
                         int64_t n, float* y_out, void* stream);

/* Sampler: mu_out[i] = clamp(mu_hat, -1, 1), ratio_out[i] = 1/(1 + x(1 - mu));
 * where x is outside the network's x range (cs_mlp_set_domain) the plain
 * sampler answers and fallback_mask[i] = 1 (nullable mask, else 0). */
CS_API cs_status cs_mlp_sample(cs_ctx* ctx, const cs_mlp* mlp, cs_sampler precision, const float* x, const float* u,
                        int64_t n, float* mu_out, float* ratio_out, uint8_t* fallback_mask, void* stream);

/* Gradient of the loss (MSE: 1/(2n) sum (y - t)^2; MAE: 1/(2n) sum |y - t|)
 * over the n device samples with targets (mu_t, r_t), FP32, reduced over the
 * batch in a fixed order (bitwise reproducible).  grad_out: device,
 * n_params floats; loss_out: nullable device float. */
CS_API cs_status cs_mlp_grad(cs_ctx* ctx, const cs_mlp* mlp, const float* x, const float* u, const float* mu_t,
                      const float* r_t, int64_t n, cs_loss loss, float* grad_out, float* loss_out, void* stream);
/* One Adam update (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with
 * the given device gradient. */
CS_API cs_status cs_mlp_adam_step(cs_ctx* ctx, cs_mlp* mlp, const float* grad, float lr, void* stream);
/* cs_mlp_grad followed by cs_mlp_adam_step (the paper's learning rate is
 * 1e-3).  Invalidates the BF16 / FP8 copies. */
CS_API cs_status cs_mlp_train_step(cs_ctx* ctx, cs_mlp* mlp, const float* x, const float* u, const float* mu_t,
                            const float* r_t, int64_t n, float lr, cs_loss loss, float* loss_out, void* stream);

/* --------------------------------------------------------- options ------ */

/* Kernel strategies of cs_compton_step; all give bitwise-identical results. */
typedef enum {
    CS_STRATEGY_FUSED = 0,        /* scan + persistent step kernel with an LDS queue of    */
                                  /* accepted pairs drained in place (default)             */
    CS_STRATEGY_MULTI_KERNEL = 1, /* one kernel per stage (baseline)                       */
    CS_STRATEGY_COMPACT = 2,      /* scan + pair kernel compacting accepted pairs by       */
                                  /* decoupled look-back + dense collide kernel            */
    CS_STRATEGY_PER_CELL = 3      /* one workgroup per cell, collisions resolved in place  */
                                  /* without compaction (baseline; plain sampler only)     */
} cs_strategy;

typedef enum {
    CS_OPT_STRATEGY = 0,         /* a cs_strategy                                        */
    CS_OPT_CHUNKS_PER_BLOCK = 1, /* fused: 256-pair chunks per workgroup; compact: the  */
                                 /* pair kernel's chunks per workgroup (rounded up to a  */
                                 /* multiple of the pairs per lane, at most 32);         */
                                 /* 0 = automatic (compact: the fewest with which every  */
                                 /* pair workgroup is resident on the device at once)    */
    CS_OPT_PAIRS_PER_LANE = 2,   /* compact: chunks each lane of the pair kernel takes   */
                                 /* at a time (1, 2 or 4), 0 = automatic (1)             */
    CS_OPT_WIDE_INDEX = 3        /* compact: 0 (default) = the pair kernel reads the     */
                                 /* particles with 32-bit byte offsets whenever each     */
                                 /* species has at most 2^32 / element-size entries,     */
                                 /* 64-bit indexing otherwise; 1 = 64-bit indexing       */
                                 /* always (same results)                                */
} cs_option;

/* Set / read a context option.  CS_ERR_INVALID_ARG for unknown options or
 * out-of-range values (chunks per block in [0, 4096]; pairs per lane 0, 1, 2
 * or 4; wide index 0 or 1). */
CS_API cs_status cs_set_option(cs_ctx* ctx, cs_option opt, int64_t value);
CS_API cs_status cs_get_option(const cs_ctx* ctx, cs_option opt, int64_t* value);

/* ---------------------------------------------------------- autotune ---- */

#define CS_TUNE_MAX 16

typedef struct {
    int32_t n;                               /* candidates timed                   */
    int32_t best;                            /* index of the fastest               */
    int32_t strategy[CS_TUNE_MAX];           /* cs_strategy of candidate i         */
    int32_t chunks_per_block[CS_TUNE_MAX];   /* fused: chunks per workgroup        */
    int32_t pairs_per_lane[CS_TUNE_MAX];     /* compact: pairs per lane            */
    float ms[CS_TUNE_MAX];                   /* median step time, milliseconds     */
} cs_tune_result;

/* Pick the kernel strategy and its tile shape for this problem (the batching
 * of the Sec. 3.1 step over uneven cells): every candidate (fused with 4..32
 * chunks per workgroup, compact with 1 or 2 pairs per lane and several chunks
 * per workgroup, among them the fewest that keep the pair grid resident at
 * once) runs `reps` timed
 * steps on a private device copy of the particles, its result after one step
 * from the same state is checked to be bitwise identical to the first
 * candidate's (CS_ERR_HIP if not, which would be a library defect), and the
 * fastest is stored in the context (CS_OPT_STRATEGY, CS_OPT_CHUNKS_PER_BLOCK,
 * CS_OPT_PAIRS_PER_LANE).
 * The caller's particles are not modified.  Arguments as cs_compton_step
 * (stats are not written); reps in [1, 100].  Synchronous; allocates and
 * frees the private copy.  `out` may be NULL. */
CS_API cs_status cs_autotune(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons,
                      const int64_t* cell_off_e, const int64_t* cell_off_g, int64_t n_cells, double dt,
                      double density_norm, uint64_t seed, uint64_t step, cs_sampler sampler, const cs_mlp* mlp,
                      int32_t reps, cs_tune_result* out, void* stream);

/* ------------------------------------------------------------- graphs ---- */

typedef struct cs_graph cs_graph;

/* Capture one cs_compton_step with these arguments (and the context's current
 * strategy, which must be FUSED or COMPACT) into a HIP graph.  Replays take the
 * step index from a device counter owned by the graph: cs_graph_set_step sets
 * it, and every replay uses it and advances it by one, so that N replays
 * equal N cs_compton_step calls with steps s, s+1, ... .  The graph owns its
 * workspace; the particle, offset, stats and network data must stay at the
 * same addresses for as long as the graph is replayed.  `stream` must not be
 * NULL (the legacy stream cannot be captured).  The counter starts at 0. */
CS_API cs_status cs_graph_create(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons,
                          const int64_t* cell_off_e, const int64_t* cell_off_g, int64_t n_cells, double dt,
                          double density_norm, uint64_t seed, cs_sampler sampler, const cs_mlp* mlp,
                          cs_stats* stats, void* stream, cs_graph** out);
/* Capture one cs_ntc_step with these arguments into a HIP graph, for callers
 * that replay the NTC step without host involvement.  The graph's launches
 * are sized for `max_candidates` candidates per step (1 <= max_candidates <=
 * 2^31 - 2; about 60 bytes of device memory each, owned by the graph); a
 * replay whose step draws more changes no particle and writes a stats
 * record with overflow = 1 and n_pairs = its candidate count.  The step
 * index works as for cs_graph_create (cs_graph_set_step, advanced by each
 * replay); cs_graph_launch and cs_graph_destroy apply.  Errors as
 * cs_ntc_step's argument checks, CS_ERR_LAYOUT for particles without
 * cells; a bad device layout shows only in the stats record. */
CS_API cs_status cs_ntc_graph_create(cs_ctx* ctx, cs_dtype dtype, cs_species electrons, cs_species photons,
                                     const int64_t* cell_off_e, const int64_t* cell_off_g, int64_t n_cells,
                                     double dt, double density_norm, uint64_t seed, int64_t max_candidates,
                                     cs_stats* stats, void* stream, cs_graph** out);
/* Queue the step index of the next replay on `stream`. */
CS_API cs_status cs_graph_set_step(cs_graph* graph, uint64_t step, void* stream);
/* Queue one replay (one step) on `stream`. */
CS_API cs_status cs_graph_launch(cs_graph* graph, void* stream);
/* Synchronises the device, then frees the graph and its workspace. */
CS_API cs_status cs_graph_destroy(cs_graph* graph);

/* ------------------------------------------------------- measurement ---- */

/* Stages of cs_compton_step, in order. */
typedef enum {
    CS_STAGE_PREP = 0,     /* offsets check, pairs per cell, scans, chunk map   */
    CS_STAGE_PAIR = 1,     /* pairing, x, s(x), P, accept, compaction           */
    CS_STAGE_COMPACT = 2,  /* offsets of the accepted pairs                     */
    CS_STAGE_COLLIDE = 3,  /* sampling, scattering, write-back                  */
    CS_STAGE_FINALIZE = 4, /* stats reduction                                   */
    CS_STAGE_COUNT = 5
} cs_stage;

/* Enable (1) or disable (0) per-stage timing: while enabled, every
 * cs_compton_step records HIP events between its stages on its stream
 * (the Sec. 3.3 stage breakdown of the paper, measured on the device) into a
 * ring of 512 steps; no host synchronisation happens during the steps.
 * Either call restarts the count of timed steps. */
CS_API cs_status cs_set_stage_timing(cs_ctx* ctx, int enable);
/* Synchronous: wait for the last timed step and write up to n stage
 * durations in milliseconds (index = cs_stage), each the mean over the steps
 * timed since timing was enabled or since the previous read (the last 512 of
 * them at most); *n_written gets the count.  CS_ERR_NOT_READY when no step
 * was timed. */
CS_API cs_status cs_stage_times(cs_ctx* ctx, float* ms_out, int32_t n, int32_t* n_written);

#ifdef __cplusplus
}
#endif

#endif /* COMPTON_H */
