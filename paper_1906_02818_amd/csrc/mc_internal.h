// Internal interface between the C ABI (api.hip) and the kernel translation
// units. Host-side declarations only; no torch types anywhere.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcp {

constexpr int kBlock = 256;          // threads per path-kernel workgroup (4 waves)
#ifndef MCP_GBM_MAX_BLOCKS
#define MCP_GBM_MAX_BLOCKS 8192
#endif
// GBM grid cap: the persistent grid gives each thread several paths.
constexpr uint32_t kGbmMaxBlocks = MCP_GBM_MAX_BLOCKS;

// ---- GBM path functionals (bit mask -> per-path channels, in bit order) ----
enum : uint32_t {
  G_EURO = 1u << 0,     // "euro"
  G_ASIAN = 1u << 1,    // "asian"
  G_GEO = 1u << 2,      // "geo"
  G_UO = 1u << 3,       // "uo"
  G_UOBB = 1u << 4,     // "uo_bridge"
  G_EURO_G = 1u << 5,   // "euro_delta", "euro_vega"
  G_ASIAN_G = 1u << 6,  // "asian_delta", "asian_vega"
  G_ALL = 0x7Fu
};

__host__ __device__ constexpr int popcount_c(uint32_t m) {
  return m == 0 ? 0 : (int)(m & 1u) + popcount_c(m >> 1);
}
__host__ __device__ constexpr int gbm_channels(uint32_t mask) {
  return popcount_c(mask & 0x1Fu) + 2 * popcount_c(mask & 0x60u);
}
// Moment vector of C channels: [n_valid, n_nonfinite, mean y_c (C),
// co-moment sum (y_a - mean_a)(y_b - mean_b) (a <= b)]; block partials are
// block-major, [block][n_moments(C)] (device/reduce.h).
__host__ __device__ constexpr int n_moments(int C) { return 2 + C + C * (C + 1) / 2; }
constexpr int kMaxMomentChannels = 9;

struct GbmParams {
  uint64_t n_paths, path_offset;
  uint32_t n_steps, tag, k0, k1;
  int log_scheme;
  // Multilevel coupling: step i uses the normalised sum of normals
  // coarsen*i .. coarsen*i + coarsen - 1 (1, 2 or 4; 1 = plain).
  uint32_t coarsen;
  // Model constants, double on the host; kernels round them to their type.
  double S0, K, disc, T, dt, sdt, sigma;
  // Log scheme, in the kernel's log domain (log2 for FP32, ln for FP64):
  double drift_dom, vol_dom, barrier_dom, bridge_c;
  // Euler on S: increments of S/S0.
  double r_dt, vol_sdt, barrier_rel;
  double* partials;   // [n_blocks][n_moments]
  double* path_out;   // [n_paths][C] or nullptr
};

// Launches the GBM path kernel for the instantiated mask `mask` (must be one
// returned by gbm_pick_mask). Returns the number of blocks via *n_blocks.
hipError_t launch_gbm(const GbmParams& p, uint32_t mask, bool fp64, hipStream_t s,
                      uint32_t* n_blocks);
// Smallest instantiated mask containing `want` for this precision/scheme
// and coupling factor, or 0 when none does.
uint32_t gbm_pick_mask(uint32_t want, bool fp64, bool log_scheme, uint32_t coarsen = 1);

// Moments of [a[ca] - b[cb], a[ca], b[cb]] over n paths of two per-path
// tables with Ca and Cb channels (multilevel correction); returns the block
// count.
hipError_t launch_diff_moments(const double* a, uint32_t Ca, uint32_t ca, const double* b,
                               uint32_t Cb, uint32_t cb, uint64_t n, double* partials,
                               hipStream_t s, uint32_t* n_blocks);
constexpr uint32_t kDiffMaxBlocks = 1024;

// ---- Heston ----
enum : uint32_t { H_EURO = 1u << 0, H_ASIAN = 1u << 1 };

// Heston kernels run on a persistent grid of at most this many workgroups
// (each thread prices several paths); partials are one moment vector per
// workgroup.
constexpr uint32_t kHestonMaxBlocks = 8192;
uint32_t heston_blocks(uint64_t n_paths);

struct HestonParams {
  uint64_t n_paths, path_offset;
  uint32_t n_steps, tag, k0, k1;
  double S0, K, disc, dt, sdt, r, v0, kappa, theta, xi, rho, rho_c;
  double* partials;
  double* path_out;
};
hipError_t launch_heston(const HestonParams& p, uint32_t mask, bool fp64, hipStream_t s,
                         uint32_t* n_blocks);
// Price, pathwise delta and d/dv0 of one payoff by forward-mode tangents
// (channels: payoff, delta, d/dv0).
hipError_t launch_heston_tangent(const HestonParams& p, bool asian, bool fp64, hipStream_t s,
                                 uint32_t* n_blocks);

// Pathwise adjoint (reverse sweep with checkpoints every `every` steps:
// even, 2..kCkptMax; kCkpt by default). A full (one-launch) sweep with at
// most kLdsCkpt checkpoints keeps them in LDS (2 kLdsCkpt floats per path,
// 32 KB per 256-path block) and needs no device buffer.
constexpr int kCkpt = 16;
constexpr int kCkptMax = 16;
constexpr int kLdsCkpt = 16;
struct AdjointParams {
  HestonParams h;
  int asian;            // 1: arithmetic-Asian call, 0: European call
  int phase;            // 0 full, 1 forward (write checkpoints), 2 reverse
  float* ckpt;          // [2*n_ckpt + 1][n_paths]: (z, v) per checkpoint, then terminal;
                        // nullptr for a full sweep with checkpoints in LDS
  uint32_t n_ckpt;
  uint32_t every;       // checkpoint period
  double grad_out;
};
hipError_t launch_heston_adjoint(const AdjointParams& p, hipStream_t s, uint32_t* n_blocks);

// ---- Basket (correlated GBM, MFMA increments) ----
enum : int { BK_FP32 = 0, BK_BF16 = 1, BK_FP16 = 2, BK_BF16X2 = 3 };
struct BasketParams {
  uint64_t n_paths, path_offset;
  uint32_t n_steps, tag, k0, k1;
  uint32_t d;             // assets, multiple of 16, <= 256
  const void* Lblk;       // packed lower-triangular 32x16 blocks of L' (device)
  const void* Lblk_lo;    // BF16X2: the lo term, same layout
  const float* asset;     // device [4][256]: n*mu_a (log2), w_a*S0_a, w_a*ln 2, S0_a
  double disc, K, geo0, w0;
  // Call portfolio (risk mode): q_k calls of strike m_k S0_a on every asset;
  // the per-path value is sum_a S0_a sum_k q_k (S_a/S0_a - m_k)^+ - premium.
  uint32_t n_strikes;     // 0: basket-call mode
  float pm[8], pq[8];
  double premium;
  // Randomised quasi-Monte Carlo: when qV is set, normal block j of path p
  // comes from Sobol' point p (dimensions 4j..4j+3) shifted by qshift.
  const uint32_t* qV;     // [dims][32] direction words
  const uint32_t* qshift; // [dims], or [replicates][dims] with q_rep_blocks
  // Replicates in one launch: block b runs replicate b / q_rep_blocks with
  // shift row q_dims * replicate, and writes its moments to that
  // replicate's own [q_rep_blocks][moment] partials.
  uint32_t q_rep_blocks, q_dims;
  double* partials;
  double* path_out;       // [n_paths][3] (basket) or [n_paths] (portfolio), or nullptr
};
constexpr int kMaxStrikes = 8;
// Number of 32-wide asset blocks the kernel is instantiated for (1, 2, 4, 8).
uint32_t basket_blocks_nd(uint32_t d);
hipError_t launch_basket(const BasketParams& p, int prec, hipStream_t s, uint32_t* n_blocks);
// All n_rep randomised-QMC replicates of p in one launch (p.qshift holds
// n_rep rows of p.q_dims shifts); *blocks_per_rep = one replicate's blocks.
hipError_t launch_basket_qmc_batch(BasketParams p, int prec, uint32_t n_rep, hipStream_t s,
                                   uint32_t* blocks_per_rep);

// Digital shifts of one randomised-QMC replicate: shift[j] = word (j mod 4)
// of Philox block (floor(j/4), replicate, tag) under key (k0, k1).
// Digital shifts of replicates replicate0 .. replicate0 + n_rep - 1:
// shift [n_rep][n_dims].
hipError_t launch_qmc_shifts(uint32_t k0, uint32_t k1, uint32_t tag, uint64_t replicate0,
                             uint32_t n_rep, uint32_t n_dims, uint32_t* shift, hipStream_t s);

// ---- Order statistic and tail mean of per-path values (risk metrics) ----
// Exact k-th smallest (1-based) of x[0..n) by an 8-pass radix select on the
// order-preserving 64-bit keys of the doubles, then the count and sum of the
// values strictly below it. `state` and `hist` are small device scratch
// areas (kSelectStateBytes, 256 uint32); partials holds kDiffMaxBlocks x 2
// doubles. Everything is enqueued on s without host synchronisation.
constexpr size_t kSelectStateBytes = 64;
hipError_t launch_select_kth(const double* x, uint64_t n, uint64_t k, void* state, uint32_t* hist,
                             hipStream_t s);
hipError_t launch_tail_sum(const double* x, uint64_t n, const void* state, double* partials,
                           hipStream_t s, uint32_t* n_blocks);
// Host view of the selection state after the passes: the key of the k-th
// smallest value and the value itself.
double select_key_to_value(uint64_t key);

// ---- Longstaff-Schwartz regression (Bermudan options) ----
// d <= 4 correlated GBM assets with dividend yield, log-Euler in the log2
// domain: x_a = log2(S_a / K), so that y_a = S_a / K = exp2(x_a).
constexpr int kLsmMaxD = 4, kLsmMaxDates = 64, kLsmMaxFeat = 11;
// Moments per block: the upper triangle of u u^T, u = (features, cash flow),
// then the sum and the sum of squares of the cash flow and the number of
// paths in the money at the last date.
constexpr int kLsmMaxMom = (kLsmMaxFeat + 1) * (kLsmMaxFeat + 2) / 2 + 3;
constexpr uint32_t kLsmMaxBlocks = 2048;
enum : uint32_t { LSM_MAX_CALL = 1, LSM_BASKET_PUT = 2, LSM_BASKET_CALL = 3 };
struct LsmParams {
  uint64_t n_paths, path_offset;
  uint32_t tag, k0, k1;
  uint32_t d, degree, pay_feat;  // pay_feat: f/K appended to the features
  uint32_t kind, n_dates, spd;   // payoff, exercise dates, Euler steps per date
  uint32_t nf;                   // number of features
  float x0[kLsmMaxD];            // log2(S0_a / K)
  float drift[kLsmMaxD];         // (r - q - sigma_a^2 / 2) dt / ln 2
  float vol[kLsmMaxD][kLsmMaxD]; // sigma_a sqrt(dt) L_ab / ln 2 (lower triangle)
  double discK[kLsmMaxDates + 1];// K e^{-r t_j}, j = 0..n_dates
  uint64_t ystride;               // row stride of y and length of C: n_paths rounded up to 64
  float* y;                      // [n_dates][d][ystride]: S_a(t_j) / K
  float* C;                      // [ystride] discounted cash flow
  uint8_t* ex;                   // [n_paths] exercise date (0 = never), or nullptr
  const double* beta;            // [n_dates][kLsmMaxFeat]
  const int* valid;              // [n_dates]: 1 when date j has a regression
  double* partials;              // [n_mom][n_blocks]
  double* path_value;            // out-of-sample: [n_paths] values, or nullptr
};
// Moments the kernels of this feature set write (see kLsmMaxMom).
uint32_t lsm_n_moments(uint32_t nf);
uint32_t lsm_n_features(uint32_t d, uint32_t degree, uint32_t pay_feat);
// Simulation of the stored paths (cash flows at t_M, Gram matrix of date
// n_dates - 1 and the exercise-at-maturity moments), the update of date j
// (exercise rule of date j, then the Gram matrix of date j - 1, or the
// price moments when j = 1), the reduction of a stage's block partials into
// `out` followed by the Cholesky solve of date j (none when j = 0), and the
// out-of-sample estimate on fresh paths.
hipError_t launch_lsm_sim(const LsmParams& p, hipStream_t s, uint32_t* n_blocks);
hipError_t launch_lsm_update(const LsmParams& p, uint32_t j, hipStream_t s, uint32_t* n_blocks);
hipError_t launch_lsm_reduce_solve(const double* partials, uint32_t nb, uint32_t nmom,
                                  double* out, uint32_t nf, uint32_t j, double* beta, int* valid,
                                  hipStream_t s);
hipError_t launch_lsm_oos(const LsmParams& p, hipStream_t s, uint32_t* n_blocks);

// ---- Learned martingale control variate (Heston Asian) ----
// Hedge network 4 -> 64 -> 64 -> 1 with tanh, run on MFMA for 32 paths per
// wave. Host-packed per-lane fragments (see api.hip, pack_mlp):
constexpr int kMlpH = 64;
constexpr int kMlpNParam = 4545;
// Row stride of the per-block gradient partials: whole 128-byte lines.
constexpr int kGradStride = (kMlpNParam + 31) / 32 * 32;
struct CvParams {
  HestonParams h;
  uint32_t hedge_every;      // rebalancing period m
  int bf16;                  // 1: BF16 MFMA operands, 0: FP32 MFMA
  const float* theta;        // [4545] flat weights (b3 is read from here)
  const float* w1f;          // [2 mb][64 lane][8]   layer-1 A fragments (W1 | b1 | 0)
  const float* w2f;          // [2 mb][4 kb][64][8]  layer-2 A fragments (permuted W2)
  const float* w2tf;         // [2 mb][4 kb][64][8]  W2^T fragments for the backward pass
  const float* lanec;        // [2][8][64][4]: per-lane b2 * (-2 / ln 2), 2 W3 of the lane's units
  const float* dfac;         // [n_steps + 1]: e^{r t_i}
  // training
  uint32_t val_blocks;       // blocks of the hedged-value kernel whose moment vectors
                             // (in `partials`) the backward sums for Ybar
  const double* y_path;      // per-path values of that pass, [n_paths][3] (Y is channel 2)
  double g_scale;            // -2 / B
  float* grad_partials;      // [n_blocks][kGradStride]: FP64 wave sums rounded to FP32
  double* partials;
  double* path_out;
  // Feature cache of the training paths, one entry per hedge segment k (the
  // network's inputs do not depend on its weights, so each training path is
  // simulated once per training run, not once per Adam step).
  float* c_phi;              // [n_seg][4][c_stride] features at the segment's opening date
  float* c_dst;              // [n_seg][c_stride] discounted price change over the segment
  double* c_pay;             // [c_stride] discounted payoff
  uint64_t c_stride;         // paths held by the cache
  uint64_t c_first;          // the minibatch's first path within the cache
  uint32_t n_seg;            // ceil(n_steps / hedge_every)
  uint32_t seg_split;        // backward: waves per 32-path tile, each taking a
                             // contiguous range of segments (set by its launcher)
};
constexpr int kCvPathsPerBlock = 256;       // evaluation: 4 waves of 64 paths
constexpr int kCvTrainPathsPerBlock = 128;  // training: 4 waves of 32 paths (/ split)
// Fragment layout of the weights, built on the device from theta.
constexpr int kW1fFloats = 2 * 64 * 8, kW2fFloats = 2 * 4 * 64 * 8, kLanecFloats = 2 * 64 * 32;
hipError_t launch_cv_pack(const float* theta, float* w1f, float* w2f, float* w2tf, float* lanec,
                          hipStream_t s);
hipError_t launch_cv_price(const CvParams& p, hipStream_t s, uint32_t* n_blocks);
// Training on the feature cache: fill it (h.n_paths paths from h.path_offset),
// the network along every 32-path tile of the minibatch with the per-path
// hedged values and their moments, and the gradient partials.
hipError_t launch_cv_cache(const CvParams& p, hipStream_t s);
hipError_t launch_cv_values(const CvParams& p, hipStream_t s, uint32_t* n_blocks);
hipError_t launch_cv_backward(const CvParams& p, hipStream_t s, uint32_t* n_blocks);
// Workgroups of the backward (the rows of its gradient partials) and of the
// hedged-value kernel (the rows of its block moments) for a minibatch of
// n_paths with n_seg hedge segments; *split (if given) receives the waves
// per 32-path tile.
uint32_t cv_bwd_blocks(uint64_t n_paths, uint32_t n_seg, uint32_t* split);
uint32_t cv_values_blocks(uint64_t n_paths, uint32_t n_seg, uint32_t* split);
constexpr int kCvValSlab = 16;  // segments a wave of a split tile holds (values)
// The hedged-value kernel's moment vectors (one per workgroup) and where
// their fixed-order merge (the minibatch's loss) goes.
struct CvValMoments {
  const double* partials;
  uint32_t n_blocks;
  double* out;
};
// Reduces the per-block gradient partials [n_blocks][kMlpNParam], takes one
// Adam step and refreshes the packed fragments, in one launch; or only
// reduces them into grad (the same fixed order). A workgroup of its own in
// the same launch merges the hedged values' moments into vm.out.
hipError_t launch_adam_pack(const float* partials, uint32_t n_blocks, const CvValMoments& vm,
                            double* grad, float* theta, float* m, float* v, int t, double lr,
                            double b1, double b2, double eps, float* w1f, float* w2f, float* w2tf,
                            float* lanec, hipStream_t s);
hipError_t launch_grad_sum(const float* partials, uint32_t n_blocks, const CvValMoments& vm,
                           double* grad, hipStream_t s);

// ---- reductions and diagnostics ----
// Moment vectors of C channels (1..kMaxMomentChannels): n_batch independent
// merges of block-major partials [batch][n_blocks][n_moments(C)] into
// out [batch][n_moments(C)], in a fixed order. A single batch of more than
// 4096 vectors merges in two stages and overwrites the partials' chunk heads.
hipError_t launch_final_merge(double* partials, uint32_t n_blocks, uint32_t C,
                              uint32_t n_batch, double* out, hipStream_t s);
// Plain sums: partials [n_mom][n_blocks] -> out [n_mom]; the batch form takes
// partials [batch][n_mom][n_blocks] -> out [batch][n_mom].
hipError_t launch_final_reduce(const double* partials, uint32_t n_blocks, uint32_t n_mom,
                               double* out, hipStream_t s);
hipError_t launch_final_reduce_batch(const double* partials, uint32_t n_blocks, uint32_t n_mom,
                                     uint32_t n_batch, double* out, hipStream_t s);
hipError_t launch_philox_words(uint32_t k0, uint32_t k1, uint32_t tag, uint64_t n,
                               const uint64_t* paths, const uint64_t* blocks, uint32_t* out,
                               hipStream_t s);
hipError_t launch_normals(uint32_t k0, uint32_t k1, uint32_t tag, uint64_t path,
                          uint64_t k_first, uint64_t count, bool fp64, double* out,
                          hipStream_t s);

}  // namespace mcp
