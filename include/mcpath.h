/*
 * mcpath.h -- C ABI of the MI355X (gfx950) Monte Carlo path engine.
 *
 * The engine estimates E[f(X_{0:T})] for an SDE dX = mu dt + sigma dW
 * (Eq. 1, Eq. 2) by the empirical mean over N simulated Euler-Maruyama paths
 * (Eq. 3; scheme of Sec. II-A.1, correlated form of Sec. II-A.2), together
 * with the estimator's standard error (variance term of the bias-variance
 * split, Sec. V-B) and pathwise greeks (Sec. I-A.3). Gaussian increments
 * come from the keyed counter-based Philox4x32-10 generator (Sec. IV-A)
 * through Box-Muller; every step of the computation runs in hand-written
 * HIP kernels on one GPU.
 *
 * Random-number layout (shared contract with any independent checker):
 *   normal k of path p in stream `tag` is slot (k mod 4) of the Philox block
 *   with counter (floor(k/4), p mod 2^32, p >> 32, tag) and key
 *   (seed mod 2^32, seed >> 32); a block's words (w0,w1,w2,w3) give
 *   normals r(w0)cos(2 pi u(w1)), r(w0)sin(2 pi u(w1)), r(w2)cos(2 pi u(w3)),
 *   r(w2)sin(2 pi u(w3)), with u(w) = (2 (w >> 9) + 1) 2^-24 and
 *   r(w) = sqrt(-2 ln u(w)). A model with d normals per time step uses
 *   k = i d + a at step i (GBM d = 1; Heston d = 2 with a = 0 the variance
 *   driver; basket d = number of assets). Tags: 0 main run, 1 pilot run,
 *   2 learned-hedge training set, tag + 16 l level l of a multilevel
 *   estimate; tag + 5 carries the Brownian-bridge uniforms of the
 *   continuously monitored barrier, tag + 6 the digital shifts of the
 *   randomised quasi-Monte Carlo replicates, tag + 7 the fresh paths of
 *   the out-of-sample Longstaff-Schwartz estimate.
 *
 * Conventions for every entry point:
 *   - Returns an mc_status; no exception or signal crosses the ABI.
 *   - On error nothing is written to the output structs; mc_last_error()
 *     gives a message.
 *   - Host pointers are read during the call only; the library keeps no
 *     pointer to caller memory after it returns.
 *   - Device pointers (workspace, checkpoint buffers) are owned by the
 *     caller and must stay valid until the call returns.
 *   - One context per host thread; calls on one context are serialised by
 *     the caller.
 *   - All pricing entry points block until the result is on the host.
 */
#ifndef MCPATH_H
#define MCPATH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MC_OK = 0,
    MC_ERR_INVALID_ARG = -1,   /* a NULL pointer, non-finite or out-of-range value */
    MC_ERR_NOT_PD = -2,        /* correlation matrix not positive definite */
    MC_ERR_NO_DEVICE = -3,     /* no HIP device, or the device index is out of range */
    MC_ERR_OOM = -4,           /* device allocation failed */
    MC_ERR_DEVICE = -5,        /* a HIP runtime call or kernel launch failed */
    MC_ERR_UNSUPPORTED = -6,   /* valid arguments, combination not offered */
    MC_ERR_WORKSPACE = -7      /* caller workspace smaller than required */
} mc_status;

typedef enum { MC_GBM = 1, MC_GBM_BASKET = 2, MC_HESTON = 3 } mc_model_kind;

/* GBM discretisation (Sec. II-A.1 applied to dS = r S dt + sigma S dW):
 * MC_LOG_EULER steps ln S, MC_EULER_S steps S itself. Heston always uses
 * full-truncation Euler on (ln S, v); the basket always uses log-Euler. */
typedef enum { MC_LOG_EULER = 0, MC_EULER_S = 1 } mc_scheme;

/* Arithmetic of the path state (Sec. V-A). MC_FP64: the whole path in
 * double. MC_FP32: single-precision path state and arithmetic, double
 * precision only for the cross-path sums. For the basket the correlated
 * increment Z L^T is a matrix product on the matrix cores: MC_FP32 uses
 * FP32 inputs, MC_BF16_GEMM / MC_FP16_GEMM round Z and L to bfloat16 /
 * half with FP32 accumulation, MC_BF16X2_GEMM splits L into two bfloat16
 * terms (hi + lo) to remove the systematic rounding of L. */
typedef enum {
    MC_FP64 = 0, MC_FP32 = 1, MC_BF16_GEMM = 2, MC_FP16_GEMM = 3, MC_BF16X2_GEMM = 4
} mc_precision;

typedef struct {
    mc_model_kind kind;
    uint32_t dim;              /* assets: 1 for MC_GBM and MC_HESTON */
    double r;                  /* risk-free rate (drift under Q) */
    double T;                  /* maturity in years, > 0 */
    const double *S0;          /* [dim] initial prices, host, > 0 */
    const double *sigma;       /* [dim] volatilities, host (GBM, basket), >= 0 */
    const double *corr;        /* [dim*dim] row-major correlation, host; basket only */
    double v0, kappa, theta, xi, rho;  /* Heston: v0 >= 0, kappa, theta, xi >= 0, |rho| < 1 */
    mc_scheme scheme;
} mc_model;

typedef enum {
    MC_EURO_CALL = 1,           /* (S_T - K)+ */
    MC_ASIAN_ARITH_CALL = 2,    /* (A - K)+, A = mean of S_{t_1..t_n} (S0 excluded) */
    MC_ASIAN_GEO_CALL = 3,      /* (exp(mean of ln S_{t_i}) - K)+ */
    MC_UO_BARRIER_CALL = 4,     /* (S_T - K)+ 1{S_{t_i} < B for i = 1..n} */
    MC_BASKET_CALL = 5,         /* (sum_a w_a S_T,a - K)+ */
    MC_UO_BRIDGE_CALL = 6       /* up-and-out call, continuous monitoring through the
                                   Brownian-bridge maximum between steps (Sec. VI-A.1) */
} mc_payoff_kind;

/* Control variates. MC_CV_GEO_ASIAN: Y = P_A - beta (P_G - C_G) with C_G the
 * discrete geometric-Asian closed form (GBM only). MC_CV_LEARNED: Y = payoff
 * - H, H the discounted P&L of a learned hedge (Heston Asian only). */
typedef enum { MC_CV_NONE = 0, MC_CV_GEO_ASIAN = 1, MC_CV_LEARNED = 2 } mc_cv_kind;

typedef struct {
    mc_payoff_kind kind;
    double K;                  /* strike, >= 0 */
    double B;                  /* barrier (barrier payoffs), > S0 */
    const double *weights;     /* [dim] basket weights, host; NULL = 1/dim each */
    mc_cv_kind cv;
} mc_payoff;

#define MC_GREEK_DELTA 1u      /* d price / d S0 (basket: of asset 0) */
#define MC_GREEK_VEGA 2u       /* GBM: d/d sigma; Heston: d/d v0 */

/* How mc_price computes the requested greeks (Sec. I-A.3).
 *   MC_GREEKS_PATHWISE: derivatives of each path's payoff (forward tangents;
 *     the adjoint for Heston); refused for discontinuous payoffs (barriers).
 *   MC_GREEKS_FD_CRN: central finite differences on common random numbers:
 *     the run is repeated with the parameter bumped up and down by the
 *     relative step fd_rel_step on the same paths (same seed, tag and path
 *     indices), and the greek is the mean of the per-path differences over
 *     2 h theta, with its standard error. Any GBM or Heston payoff, and the
 *     basket delta (S0 of asset 0). The greeks are those of the payoff
 *     without control variate. The bumped GBM and Heston runs use FP64
 *     paths whatever prec is (the price keeps prec): a difference over a
 *     relative bump h loses about -log10(h) digits.
 *   MC_GREEKS_TANGENT: pathwise derivatives in forward mode. GBM and basket
 *     pathwise greeks are forward tangents already (the same as
 *     MC_GREEKS_PATHWISE); for Heston the tangents of (ln S, v) with respect
 *     to v0 ride along the forward pass instead of the checkpointed reverse
 *     sweep: no checkpoint memory and about half the cost for the two
 *     inputs, in MC_FP32 or MC_FP64 paths. Same payoff restrictions as
 *     MC_GREEKS_PATHWISE. */
typedef enum {
    MC_GREEKS_PATHWISE = 0,
    MC_GREEKS_FD_CRN = 1,
    MC_GREEKS_TANGENT = 2
} mc_greeks_method;

#define MC_MLP_NPARAM 4545     /* 4-64-64-1 hedge network, FP32 */
/* mc_options.pilot_paths value: the geometric-Asian control variate's
 * coefficient beta = Cov(A, G) / Var(G) is taken from the paths it corrects
 * (the usual in-sample estimator: no pilot run, a bias of order 1/n_paths);
 * MC_ERR_UNSUPPORTED with the learned control variate, whose pilot decides
 * the fallback to plain Monte Carlo. */
#define MC_PILOT_IN_SAMPLE UINT64_MAX

typedef struct {
    mc_precision prec;         /* default MC_FP32 */
    uint32_t greeks;           /* MC_GREEK_* bits */
    uint64_t path_offset;      /* first global path index (sharding, resumption) */
    uint32_t stream_tag;       /* Philox stream tag, default 0 */
    void *hip_stream;          /* hipStream_t to run on; NULL = the context stream */
    void *workspace;           /* device scratch; NULL = context-owned */
    size_t workspace_bytes;
    const float *cv_weights;   /* [MC_MLP_NPARAM] host, for MC_CV_LEARNED */
    uint32_t cv_hedge_every;   /* learned hedge rebalanced every m steps (>= 1) */
    double cv_beta;            /* control-variate coefficient. Static CV: NaN = estimate
                                  on a pilot. Learned CV: Y = payoff - cv_beta H; NaN =
                                  1 with a pilot run deciding between the hedged
                                  estimator and plain MC (mc_result.cv_fallback);
                                  on fallback path_values are not written */
    uint64_t pilot_paths;      /* pilot size (tag 1) for beta / fallback; 0 = 2^16;
                                  MC_PILOT_IN_SAMPLE: the static CV's beta from the
                                  main run's own moments (no pilot) */
    double *path_values;       /* optional host [n_paths * mc_path_channels()]
                                  per-path values (testing and diagnostics) */
    uint32_t greeks_method;    /* mc_greeks_method, default MC_GREEKS_PATHWISE */
    double fd_rel_step;        /* MC_GREEKS_FD_CRN relative bump h, 0 < h < 0.5; default 1e-3 */
} mc_options;

typedef struct {
    double price, std_err, variance;   /* estimator (with the control variate, if any) */
    double delta, delta_se, vega, vega_se;
    double plain_price, plain_std_err; /* same paths without the control variate */
    double cv_beta;                    /* coefficient used (static CV) */
    double vrf;                        /* variance-reduction factor plain/CV */
    uint64_t n_paths, n_nonfinite;
    double kernel_ms;                  /* device time of the path kernel(s) */
    int cv_fallback;                   /* 1 when the learned CV lost to plain MC on the pilot */
    int greeks_method;                 /* mc_greeks_method that produced delta and vega */
} mc_result;

typedef struct mc_context mc_context;

/* Opens a context on HIP device `device` with its own stream. */
mc_status mc_create(mc_context **ctx, int device);
/* Frees the context, its stream and its device buffers. NULL is allowed. */
mc_status mc_destroy(mc_context *ctx);

/* Fills opts with defaults (MC_FP32, no greeks, tag 0, beta NaN, m = 1,
 * pathwise greeks, finite-difference step 1e-3). */
void mc_options_default(mc_options *opts);

/* Runs every argument check mc_price makes (values, model/payoff/precision
 * combination, positive definiteness of a basket correlation) without
 * touching a device. ctx may be NULL (then no message is kept). */
mc_status mc_validate(mc_context *ctx, const mc_model *model, const mc_payoff *payoff,
                      uint64_t n_paths, uint32_t n_steps, const mc_options *opts);

/* Bytes of device workspace one mc_price call needs (0 on bad arguments). */
size_t mc_workspace_bytes(const mc_model *model, const mc_payoff *payoff,
                          uint64_t n_paths, uint32_t n_steps, const mc_options *opts);

/* Estimates E[f(X_{0:T})] of Eq. (2) by Eq. (3) over n_paths paths of
 * n_steps Euler-Maruyama steps (Sec. II-A.1 / II-A.2), with standard error
 * and the requested pathwise greeks (Sec. I-A.3). Path p of the run uses
 * global index opts->path_offset + p in the counter, so disjoint path
 * ranges can be merged exactly. Requires n_paths >= 2, n_steps >= 1.
 * Pathwise greeks of a discontinuous payoff (barriers) are MC_ERR_UNSUPPORTED.
 * opts may be NULL (defaults). */
mc_status mc_price(mc_context *ctx, const mc_model *model, const mc_payoff *payoff,
                   uint64_t n_paths, uint32_t n_steps, uint64_t seed,
                   const mc_options *opts, mc_result *out);

/* Allocation-free pricing, for callers that cannot allocate device memory
 * during the call: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc. Same arguments, kernels and results as
 * mc_price (bit for bit: same grid, same fixed-order reductions), restricted
 * to what fits a fixed device scratch: models MC_GBM and MC_HESTON, payoffs
 * without the learned control variate (the geometric-Asian control variate
 * and its pilot are allowed), pathwise greeks only (GBM tangents; Heston
 * forward tangents, or the adjoint while its checkpoints fit on chip, i.e.
 * n_steps <= 256), no path_values; opts->workspace is ignored. The call performs no device or pinned-host allocation and no
 * free: the block moments and the reduced moments live in a static device
 * array of MC_NOALLOC_SCRATCH_BYTES, one per GPU, held until the process
 * ends, whose address the library looks up once per device in mc_create.
 * The moments come back through a fixed host array of the context.
 * Every call on one GPU shares that GPU's scratch and leaves its contents
 * there; each run overwrites all of it that it reads, so nothing needs
 * clearing. Calls that overlap on one GPU (two host threads, or two
 * contexts' streams at once) race on the scratch: serialise them.
 * The GBM kernel and the Heston price and tangent kernels run on
 * persistent grids (at most 8192 workgroups), so those runs need at most
 * 8192 moment vectors of at most 9 channels (3.7 MB) whatever n_paths is.
 * The Heston adjoint takes one path per thread: one 88-byte vector per 256
 * paths, so it fits up to about 1.2e7 paths.
 * Errors: those of mc_price; a model, payoff or option outside the list
 * above -> MC_ERR_UNSUPPORTED; a run whose moments would not fit the
 * scratch -> MC_ERR_WORKSPACE, before any launch. */
#define MC_NOALLOC_SCRATCH_BYTES (4u << 20)
size_t mc_noalloc_scratch_bytes(void);
mc_status mc_price_noalloc(mc_context *ctx, const mc_model *model, const mc_payoff *payoff,
                           uint64_t n_paths, uint32_t n_steps, uint64_t seed,
                           const mc_options *opts, mc_result *out);

/* Prices n_payoffs payoffs on the same simulated paths in one pass.
 * results[i] receives payoff i. GBM only. */
mc_status mc_price_multi(mc_context *ctx, const mc_model *model,
                         const mc_payoff *payoffs, uint32_t n_payoffs,
                         uint64_t n_paths, uint32_t n_steps, uint64_t seed,
                         const mc_options *opts, mc_result *results);

/* Number of per-path channels written to opts->path_values by mc_price for
 * this model/payoff/options, and the name of channel i ("euro", "asian",
 * "geo", "uo", "uo_bridge", "euro_delta", "euro_vega", "asian_delta",
 * "asian_vega", "basket", "basket_delta0", "hedge_pnl", ...). Every channel
 * is a discounted per-path value; a row is one path. Returns 0 / NULL on
 * bad arguments. */
uint32_t mc_path_channels(const mc_model *model, const mc_payoff *payoff,
                          const mc_options *opts);
const char *mc_path_channel_name(const mc_model *model, const mc_payoff *payoff,
                                 const mc_options *opts, uint32_t i);

/* Pathwise adjoint greeks (Sec. I-A.3, Sec. VI-A.2 basket delta by
 * back-propagation), Heston European or arithmetic-Asian call. The reverse
 * sweep restarts from checkpoints of (ln S, v) saved every `ckpt_every`
 * steps (even, 2..16) and regenerates the normals from Philox.
 *   MC_ADJ_FULL: forward + reverse in one launch; fills price, delta, vega
 *                (d/dv0) and their standard errors. With at most 16
 *                checkpoints (n_steps <= 16 ckpt_every) they stay in on-chip
 *                memory (LDS) and ckpt is ignored; above that ckpt is used,
 *                or the context workspace when ckpt is NULL.
 *   MC_ADJ_FWD:  forward only: price, and writes the checkpoints to ckpt.
 *   MC_ADJ_REV:  reverse only from the checkpoints of a previous FWD call
 *                with identical arguments; fills delta, vega scaled by
 *                grad_out (the upstream derivative of the loss w.r.t. price).
 * ckpt is a device buffer of mc_adjoint_ckpt_bytes() bytes, FP32, laid out
 * [checkpoint][component][path], then one row of the terminal statistic.
 * mc_adjoint_ckpt_bytes returns 0 for a period that is not even in 2..16.
 * Errors: another period -> MC_ERR_UNSUPPORTED; FWD/REV without ckpt ->
 * MC_ERR_INVALID_ARG; ckpt_bytes too small -> MC_ERR_WORKSPACE. */
typedef enum { MC_ADJ_FULL = 0, MC_ADJ_FWD = 1, MC_ADJ_REV = 2 } mc_adjoint_phase;
size_t mc_adjoint_ckpt_bytes(uint64_t n_paths, uint32_t n_steps, uint32_t ckpt_every);
mc_status mc_greeks_adjoint(mc_context *ctx, const mc_model *model,
                            const mc_payoff *payoff, uint64_t n_paths,
                            uint32_t n_steps, uint64_t seed, const mc_options *opts,
                            mc_adjoint_phase phase, uint32_t ckpt_every,
                            void *ckpt, size_t ckpt_bytes, double grad_out,
                            mc_result *out);

/* Adam settings for mc_cv_train (Kingma and Ba). The step size of Adam
 * step t (0-based) is lr * decay^floor(t / decay_every): a step decay of the
 * learning rate, the moment estimates carried across the drops; decay_every
 * = 0 keeps lr for every step (decay is then ignored). Zero-initialised
 * decay fields give the constant rate. MC_ERR_INVALID_ARG: lr, eps not
 * positive, beta1 or beta2 outside [0, 1), batch not a positive multiple of
 * 256, decay outside (0, 1] while decay_every > 0. */
typedef struct {
    double lr, beta1, beta2, eps;
    uint32_t steps;            /* Adam steps */
    uint64_t batch;            /* minibatch paths, multiple of 256 */
    uint32_t hedge_every;      /* rebalancing period m >= 1 */
    mc_precision prec;         /* MC_FP32 or MC_BF16_GEMM for the 64x64 layer */
    uint32_t decay_every;      /* steps between learning-rate drops, 0: none */
    double decay;              /* factor per drop, in (0, 1] when decay_every > 0 */
} mc_adam_cfg;

/* Trains the hedge network of the learned control variate on n_train paths
 * of stream tag 2 (cycled in minibatches) to minimise the batch variance of
 * Y = payoff - H. weights_inout: host [MC_MLP_NPARAM] FP32, initial weights
 * in, trained weights out. loss_log: host [steps] or NULL. Heston Asian
 * call only. The training paths are simulated once into a device cache of
 * the network's inputs, n_train * ceil(n_steps / hedge_every) * 20 bytes
 * plus 8 bytes per path (MC_ERR_OOM if it cannot be allocated). */
mc_status mc_cv_train(mc_context *ctx, const mc_model *model, const mc_payoff *payoff,
                      uint64_t n_train, uint32_t n_steps, uint64_t seed,
                      const mc_adam_cfg *cfg, float *weights_inout, float *loss_log);

/* Loss and gradient of the learned CV on one minibatch (paths path0 ..
 * path0+batch-1 of stream `tag`): grad_out host [MC_MLP_NPARAM] FP32. */
mc_status mc_cv_loss_grad(mc_context *ctx, const mc_model *model, const mc_payoff *payoff,
                          uint32_t n_steps, uint64_t seed, uint32_t tag, uint64_t path0,
                          uint64_t batch, const mc_adam_cfg *cfg, const float *weights,
                          double *loss_out, float *grad_out);

/* Multilevel Monte Carlo (Sec. V-B, Sec. VIII; Giles): the estimate of the
 * finest level's expectation as a telescoping sum of independent level
 * estimators,
 *     E[P_L] = E[P_0] + sum_{l=1..L-1} E[P_l - P_{l-1}],
 * where level l's correction is simulated with both the level's own
 * configuration ("fine") and the previous level's ("coarse") on the SAME
 * paths, so that its variance is small and few paths suffice. Two
 * couplings between consecutive levels:
 *   precision: equal n_steps, different prec. Fine and coarse use the same
 *              normals; this is the low-precision companion estimator whose
 *              bias a reference-precision level corrects (Sec. V-B). Any
 *              model.
 *   time:      equal prec, n_steps(l) = c n_steps(l-1) with c = 2 or 4. The
 *              coarse step k uses (z_{ck} + ... + z_{ck+c-1}) / sqrt(c) of the
 *              fine path's normals (the same Brownian path on the coarser
 *              grid). One-dimensional GBM, every payoff except the
 *              Brownian-bridge barrier.
 * Level l draws from stream tag opts->stream_tag + 16 l (paths from
 * opts->path_offset), so levels are independent. The payoff must have
 * cv = MC_CV_NONE; opts->greeks and opts->path_values must be 0 / NULL. The
 * per-path values of a correction level are kept on the device in chunks of
 * at most 2^20 paths and reduced there (FP64); n_paths per level is
 * otherwise unlimited. Errors: n_levels outside 1..MC_MLMC_MAX_LEVELS, a
 * level with n_paths < 2 or n_steps = 0 -> MC_ERR_INVALID_ARG; consecutive
 * levels that match neither coupling, or a model/payoff/precision that the
 * single-level mc_price rejects -> that error. */
#define MC_MLMC_MAX_LEVELS 8
typedef struct {
    uint32_t n_steps;          /* time steps of this level */
    mc_precision prec;         /* arithmetic of this level */
    uint64_t n_paths;          /* paths of this level's estimator, >= 2 */
} mc_level;

typedef enum { MC_COUPLE_NONE = 0, MC_COUPLE_PRECISION = 1, MC_COUPLE_TIME = 2 } mc_coupling;

typedef struct {
    double price;              /* sum of the level means */
    double std_err;            /* sqrt(sum_l variance[l] / n_paths[l]) */
    uint32_t n_levels;
    mc_coupling coupling[MC_MLMC_MAX_LEVELS];    /* level 0: MC_COUPLE_NONE */
    double mean[MC_MLMC_MAX_LEVELS];       /* Y_0 = P_0, Y_l = P_l - P_{l-1} */
    double variance[MC_MLMC_MAX_LEVELS];   /* sample variance of Y_l (N_l - 1) */
    double fine_mean[MC_MLMC_MAX_LEVELS];  /* mean of P_l on level l's paths */
    double coarse_mean[MC_MLMC_MAX_LEVELS];/* mean of P_{l-1} on the same paths */
    uint64_t n_paths[MC_MLMC_MAX_LEVELS];
    double kernel_ms[MC_MLMC_MAX_LEVELS];  /* device time of the level's kernels */
} mc_mlmc_result;

mc_status mc_price_mlmc(mc_context *ctx, const mc_model *model, const mc_payoff *payoff,
                        uint32_t n_levels, const mc_level *levels, uint64_t seed,
                        const mc_options *opts, mc_mlmc_result *out);

/* Path counts that minimise the total cost sum_l N_l cost[l] subject to
 * sum_l var[l] / N_l = target_se^2 (Lagrange multiplier; Giles):
 *     N_l = ceil(target_se^-2 sqrt(var[l] / cost[l]) sum_k sqrt(var[k] cost[k])),
 * at least 2. var and cost: host [n_levels], finite, var >= 0, cost > 0.
 * Host arithmetic only (no device). Errors: MC_ERR_INVALID_ARG. */
mc_status mc_mlmc_allocate(uint32_t n_levels, const double *var, const double *cost,
                           double target_se, uint64_t *n_paths_out);

/* Portfolio risk over a horizon (Sec. VI-B.1). The basket model's d assets
 * (dim a multiple of 16 up to 256, correlation, sigma) are simulated by
 * log-Euler under the real-world measure, with drift mu[a] in place of r,
 * to the horizon T = model->T in n_steps steps. The portfolio holds, on
 * every asset a, quantity[k] European calls of strike strike_mult[k] * S0_a
 * expiring at the horizon (k < n_strikes; negative quantities are short).
 * Per path
 *     PnL = sum_a sum_k quantity[k] (S_{T,a} - strike_mult[k] S0_a)^+ - V0,
 * V0 the Black-Scholes value at time 0 (rate r, volatility sigma_a) of the
 * holdings; the horizon value is not discounted. With k = floor(N (1 -
 * alpha)) + 1 and PnL_(k) the k-th smallest of the N path values,
 *     VaR_alpha  = -PnL_(k)  (the printed infimum read as the (1 - alpha)
 *                            quantile: -inf{x : P(PnL <= x) > 1 - alpha}),
 *     CVaR_alpha = -mean{PnL_i : PnL_i < PnL_(k)}  (-E[PnL | -PnL > VaR]).
 * The order statistic is exact over the simulated values (radix select on
 * the device). Options: prec MC_FP32, MC_BF16_GEMM or MC_FP16_GEMM;
 * stream_tag, path_offset, hip_stream; path_values (host [N], the P&L of
 * each path) optional; greeks must be 0. The per-path P&L is kept in
 * context-owned device memory (8 bytes per path). Errors: a NULL argument,
 * n_strikes outside 1..MC_MAX_STRIKES, a non-finite or negative strike,
 * non-finite quantity or drift, alpha outside (0, 1) or k < 2 (an empty
 * tail) -> MC_ERR_INVALID_ARG; a model the basket pricer rejects -> that
 * error. */
#define MC_MAX_STRIKES 8
typedef struct {
    uint32_t n_strikes;                    /* calls per asset, 1..MC_MAX_STRIKES */
    double strike_mult[MC_MAX_STRIKES];    /* strike of call k on asset a / S0_a */
    double quantity[MC_MAX_STRIKES];       /* holding of call k on each asset */
    const double *mu;                      /* [dim] real-world drifts; NULL: model->r */
    double alpha;                          /* confidence level, 0 < alpha < 1 */
} mc_portfolio;

typedef struct {
    double var;                /* VaR_alpha */
    double cvar;               /* CVaR_alpha */
    double quantile_pnl;       /* PnL_(k) = -VaR_alpha */
    double pnl_mean;           /* mean horizon P&L */
    double pnl_std_err;        /* its standard error */
    double premium;            /* V0 */
    uint64_t k;                /* rank of the order statistic */
    uint64_t n_tail;           /* paths strictly below PnL_(k) */
    uint64_t n_paths;
    double kernel_ms;          /* path kernel */
    double select_ms;          /* order statistic and tail sum */
} mc_risk_result;

mc_status mc_risk(mc_context *ctx, const mc_model *model, const mc_portfolio *portfolio,
                  uint64_t n_paths, uint32_t n_steps, uint64_t seed, const mc_options *opts,
                  mc_risk_result *out);

/* Randomised quasi-Monte Carlo for the basket (quasi-random numbers of
 * Sec. IV-B; the Sobol' experiment of Sec. VI-D). Path p is Sobol' point p
 * (path_offset + i, below 2^32) in n_steps * dim dimensions; normal k uses
 * dimension k. Sobol' construction: dimension 0 van der Corput; dimension
 * j >= 1 the j-th primitive polynomial over GF(2) (by degree, then bit
 * pattern) with initial direction integers m_i = 2 (h mod 2^(i-1)) + 1,
 * h = SplitMix64(64 j + i), then the Bratley-Fox recursion; direction word
 * of bit b: m_(b+1) << (31 - b). Replicate r xors dimension j's word with
 * word (j mod 4) of the Philox block (floor(j/4), r, stream_tag + 6) (a
 * random digital shift); the shifted words pass through the same uniform
 * and Box-Muller maps as Philox words. Each replicate's estimate is the
 * mean over its n_points paths; price and std_err are the mean of the
 * n_replicates estimates and their standard deviation / sqrt(n_replicates)
 * (NaN for one replicate). Model MC_GBM_BASKET, payoff MC_BASKET_CALL,
 * prec MC_FP32 or MC_FP16_GEMM, greeks 0; path_values (host
 * [n_points][3], the channels of mc_price) only with one replicate.
 * Precision: the QMC standard error falls below the bias of BF16 products
 * (L' rounded to 8 bits moves a 16-asset price by a few 1e-4 relative,
 * about 4 QMC standard errors at 16 x 2^16 points), so MC_BF16_GEMM and
 * MC_BF16X2_GEMM are MC_ERR_UNSUPPORTED here; FP16 products (11 bits) stay
 * within 0.1 standard errors of the FP64 estimate at that size.
 * Errors: n_replicates outside 1..MC_QMC_MAX_REPLICATES, point indices
 * reaching 2^32, or n_steps * dim above 2^16 dimensions ->
 * MC_ERR_INVALID_ARG; otherwise the errors of mc_price. */
#define MC_QMC_MAX_REPLICATES 64
typedef struct {
    double price;              /* basket call: mean of the replicate estimates */
    double std_err;
    double geo_price;          /* geometric basket call on the same points */
    double geo_std_err;
    uint32_t n_replicates;
    uint64_t n_points;
    double replicate_price[MC_QMC_MAX_REPLICATES];
    double replicate_geo[MC_QMC_MAX_REPLICATES];
    double kernel_ms;          /* path kernels of all replicates */
} mc_qmc_result;

mc_status mc_price_qmc(mc_context *ctx, const mc_model *model, const mc_payoff *payoff,
                       uint64_t n_points, uint32_t n_steps, uint64_t seed,
                       uint32_t n_replicates, const mc_options *opts, mc_qmc_result *out);

/* Longstaff-Schwartz pricing of a Bermudan option (chained least-squares
 * regressions for callable options, Sec. II-A.3; the American max-option
 * experiment of Sec. VI-C). Model MC_GBM (dim 1) or MC_GBM_BASKET with dim
 * 1..4 (S0, sigma, corr); every asset pays the continuous dividend yield
 * spec->dividend, so it drifts at r - q under the pricing measure. Paths are
 * simulated by log-Euler (steps_per_date steps between consecutive dates;
 * step i uses normals i dim + a) and may be exercised at the n_dates dates
 * t_j = j T / n_dates, j = 1..n_dates. Payoff f, with y_a = S_a / K and
 * equal weights 1/dim:
 *     MC_LSM_MAX_CALL    (max_a S_a - K)+
 *     MC_LSM_BASKET_PUT  (K - mean_a S_a)+
 *     MC_LSM_BASKET_CALL (mean_a S_a - K)+
 * Every path carries a discounted cash flow C, first e^{-rT} f(t_M). For
 * j = M-1 .. 1 the cash flows of the paths in the money at t_j are
 * regressed on the features of y(t_j) by least squares (Cholesky
 * factorisation of the FP64 Gram matrix); a path in the money whose
 * discounted exercise value e^{-r t_j} f is at least the fitted
 * continuation exercises, C = e^{-r t_j} f. price = mean of C (t = 0 is not
 * an exercise date). Features: all monomials of y_1..y_dim of total degree
 * <= spec->degree (1..3), by degree, then by the nondecreasing index tuple,
 * and f / K last for the max-call with dim >= 2; at most
 * MC_LSM_MAX_FEATURES. A date with fewer in-the-money paths than features,
 * or a Cholesky pivot <= 1e-12 times its diagonal entry, gets no regression
 * and no exercise (its beta row is NaN, beta_valid 0). The out-of-sample
 * estimate applies the fitted rule to n_paths_oos independent paths of
 * stream opts->stream_tag + 7 (a stopping rule, so its expectation is a
 * lower bound on the option's value).
 * Arithmetic: FP32 path state, stored exercise-date states and cash flows
 * (device memory: (n_dates - 1) * dim * n_paths * 4 + 5 n_paths bytes,
 * owned by the context); FP64 features, Gram matrices, solves and
 * decisions.
 * Options: prec MC_FP32 only; stream_tag, path_offset, hip_stream; greeks
 * 0. diag (optional) receives per-path results on the host.
 * Errors: NULL model/spec/out, dim outside 1..4, unknown payoff, K or
 * dividend not finite, K <= 0, n_dates outside 1..MC_LSM_MAX_DATES,
 * steps_per_date 0, degree outside 1..3, n_paths < 2 ->
 * MC_ERR_INVALID_ARG; more than MC_LSM_MAX_FEATURES features, another
 * precision, greeks -> MC_ERR_UNSUPPORTED; a correlation that is not
 * positive definite -> MC_ERR_NOT_PD. */
#define MC_LSM_MAX_DATES 64
#define MC_LSM_MAX_FEATURES 11
typedef enum {
    MC_LSM_MAX_CALL = 1, MC_LSM_BASKET_PUT = 2, MC_LSM_BASKET_CALL = 3
} mc_lsm_payoff;

typedef struct {
    mc_lsm_payoff payoff;
    double K;                  /* strike, > 0 */
    double dividend;           /* continuous dividend yield q of every asset */
    uint32_t n_dates;          /* exercise dates M, 1..MC_LSM_MAX_DATES */
    uint32_t steps_per_date;   /* Euler steps between consecutive dates, >= 1 */
    uint32_t degree;           /* total degree of the monomial features, 1..3 */
    uint64_t n_paths_oos;      /* fresh paths for the out-of-sample estimate; 0 = none */
} mc_lsm_spec;

typedef struct {
    double price, std_err;             /* in-sample estimate (mean of C) */
    double price_oos, std_err_oos;     /* out-of-sample estimate; NaN when not run */
    double european, european_se;      /* exercise at t_M only, same paths */
    uint32_t n_features;
    double beta[MC_LSM_MAX_DATES][MC_LSM_MAX_FEATURES];  /* row j-1: date j */
    int beta_valid[MC_LSM_MAX_DATES];
    uint64_t n_itm[MC_LSM_MAX_DATES];  /* paths in the money at date j (row j-1) */
    uint64_t n_paths, n_paths_oos;
    double sim_ms;                     /* path simulation and storage */
    double regress_ms;                 /* backward pass: solves and updates */
    double oos_ms;                     /* out-of-sample paths */
    double update_ms;                  /* the n_dates - 1 update kernels alone */
} mc_lsm_result;

typedef struct {
    double *cash_flow;          /* host [n_paths]: C of each in-sample path */
    int32_t *exercise_date;     /* host [n_paths]: j of the exercise, 0 = never */
    double *oos_value;          /* host [n_paths_oos]: discounted value of each fresh path */
    int32_t *oos_exercise_date; /* host [n_paths_oos] */
} mc_lsm_paths;

mc_status mc_price_lsm(mc_context *ctx, const mc_model *model, const mc_lsm_spec *spec,
                       uint64_t n_paths, uint64_t seed, const mc_options *opts,
                       mc_lsm_result *out, const mc_lsm_paths *diag);

/* Raw Philox4x32-10 blocks of sampled (path, block) pairs and the normals
 * of one path, computed by the same device functions the path kernels use
 * (bit-exact checks of the random-number layout). Host arrays. */
mc_status mc_philox_words(mc_context *ctx, uint64_t seed, uint32_t tag, uint64_t n,
                          const uint64_t *paths, const uint64_t *blocks, uint32_t *out4);
mc_status mc_normals(mc_context *ctx, uint64_t seed, uint32_t tag, uint64_t path,
                     uint64_t k0, uint64_t count, mc_precision prec, double *out);

const char *mc_status_str(mc_status st);
const char *mc_last_error(const mc_context *ctx);

#ifdef __cplusplus
}
#endif

#endif /* MCPATH_H */
