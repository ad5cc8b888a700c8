// C ABI of the path engine (include/mcpath.h): argument validation, device
// workspace and stream plumbing, kernel dispatch and the estimator formulas
// (Eq. 3 and the variance term of Sec. V-B) applied to the block moments
// the kernels produce. Host code only; every per-path computation runs in
// the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mcpath.h"
#include "host_math.h"
#include "host_sobol.h"
#include "mc_internal.h"

struct mc_context {
  int device = 0;
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  double* pinned = nullptr;      // host staging for moments
  size_t pinned_count = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::string err;
  // Multilevel runs: when `sink` is set, run_moments writes the per-path
  // values there (device) instead of returning them to the host; `coarsen`
  // is the GBM coupling factor of the next run (1 = plain).
  double* sink = nullptr;
  uint32_t coarsen = 1;
  void* mlmc_buf = nullptr;
  size_t mlmc_bytes = 0;
  // Sobol' direction words of the last quasi-Monte Carlo call (device,
  // [qmc_dims][32]) followed by one replicate's shifts [qmc_dims].
  uint32_t* qmc_buf = nullptr;
  uint32_t qmc_dims = 0;
  // Longstaff-Schwartz: stored exercise-date states, cash flows and the
  // regression workspace of the last call (device, grown on demand).
  void* lsm_buf = nullptr;
  size_t lsm_bytes = 0;
  hipEvent_t ev2 = nullptr, ev3 = nullptr;
  // The correlation matrix of the last basket call and its Cholesky factor
  // (or that it is not positive definite): a repeated basket skips the
  // O(d^3) factorisation, which costs milliseconds on the host at d = 256.
  std::vector<double> chol_corr, chol_L;
  bool chol_pd = false;
  // Event pairs around each date's update kernel (created on first use).
  std::vector<hipEvent_t> lsm_ev;
  // Allocation-free calls (mc_price_noalloc): while `noalloc` is set, every
  // device buffer of the call comes from this device's static scratch array
  // (address from hipGetSymbolAddress at mc_create) and the reduced moments
  // come back into host_mom instead of pinned memory.
  void* scratch = nullptr;
  bool noalloc = false;
  double host_mom[256] = {};
};

// Device scratch of the allocation-free entry point: the block moment
// partials and the reduced moments of one run (MC_NOALLOC_SCRATCH_BYTES,
// one copy per GPU, held until the process ends). Host code never passes
// this name to a kernel or a copy: it uses the per-device address that
// scratch_address() obtained from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[MC_NOALLOC_SCRATCH_BYTES];

namespace {

using namespace mcp;

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Address of `scratch` on `device`, which must be the current device. The
// lookup runs once per device; later contexts on it reuse the address.
hipError_t scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxScratchDevices) return hipSuccess;   // no scratch there
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

mc_status fail(mc_context* ctx, mc_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

#define HIP_TRY(ctx, expr)                                                                \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(ctx, e_ == hipErrorOutOfMemory ? MC_ERR_OOM : MC_ERR_DEVICE, "%s: %s", \
                  #expr, hipGetErrorString(e_));                                          \
  } while (0)

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }
bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

mc_options defaults() {
  mc_options o;
  mc_options_default(&o);
  return o;
}

mc_status validate_common(mc_context* ctx, const mc_model* m, const mc_payoff* f,
                          uint64_t n_paths, uint32_t n_steps) {
  if (!m || !f) return fail(ctx, MC_ERR_INVALID_ARG, "model and payoff must not be NULL");
  if (n_paths < 2) return fail(ctx, MC_ERR_INVALID_ARG, "n_paths must be >= 2");
  if (n_steps == 0) return fail(ctx, MC_ERR_INVALID_ARG, "n_steps must be >= 1");
  if (n_paths > (1ull << 36)) return fail(ctx, MC_ERR_INVALID_ARG, "n_paths above 2^36");
  if (!finite_pos(m->T)) return fail(ctx, MC_ERR_INVALID_ARG, "T must be finite and > 0");
  if (!std::isfinite(m->r)) return fail(ctx, MC_ERR_INVALID_ARG, "r must be finite");
  if (!finite_nonneg(f->K)) return fail(ctx, MC_ERR_INVALID_ARG, "K must be finite and >= 0");
  if (m->dim == 0 || !m->S0) return fail(ctx, MC_ERR_INVALID_ARG, "S0 missing");
  for (uint32_t a = 0; a < m->dim; ++a)
    if (!finite_pos(m->S0[a])) return fail(ctx, MC_ERR_INVALID_ARG, "S0[%u] must be > 0", a);
  return MC_OK;
}

mc_status validate_gbm(mc_context* ctx, const mc_model* m, const mc_payoff* f,
                       const mc_options& o) {
  if (m->dim != 1) return fail(ctx, MC_ERR_INVALID_ARG, "MC_GBM needs dim == 1");
  if (!m->sigma || !finite_nonneg(m->sigma[0]))
    return fail(ctx, MC_ERR_INVALID_ARG, "sigma must be finite and >= 0");
  if (m->scheme != MC_LOG_EULER && m->scheme != MC_EULER_S)
    return fail(ctx, MC_ERR_INVALID_ARG, "unknown scheme");
  const bool barrier = f->kind == MC_UO_BARRIER_CALL || f->kind == MC_UO_BRIDGE_CALL;
  if (barrier && !(std::isfinite(f->B) && f->B > m->S0[0]))
    return fail(ctx, MC_ERR_INVALID_ARG, "barrier must be finite and above S0");
  if (o.prec != MC_FP32 && o.prec != MC_FP64)
    return fail(ctx, MC_ERR_UNSUPPORTED, "GBM paths run in MC_FP32 or MC_FP64");
  return MC_OK;
}

mc_status validate_heston(mc_context* ctx, const mc_model* m, const mc_options& o) {
  if (m->dim != 1) return fail(ctx, MC_ERR_INVALID_ARG, "MC_HESTON needs dim == 1");
  if (!finite_nonneg(m->v0) || !finite_nonneg(m->kappa) || !finite_nonneg(m->theta) ||
      !finite_nonneg(m->xi))
    return fail(ctx, MC_ERR_INVALID_ARG, "v0, kappa, theta, xi must be finite and >= 0");
  if (!(std::isfinite(m->rho) && std::fabs(m->rho) < 1.0))
    return fail(ctx, MC_ERR_INVALID_ARG, "|rho| must be < 1");
  (void)o;
  return MC_OK;
}

uint32_t gbm_want_mask(const mc_payoff* f, const mc_options& o, mc_status* st);

// Basket checks; on success fills L (d*d, lower Cholesky factor) if given.
mc_status validate_basket(mc_context* ctx, const mc_model* m, const mc_payoff* f,
                          uint32_t n_steps, const mc_options& o, std::vector<double>* L) {
  const uint32_t d = m->dim;
  if (d == 0 || d > 256 || d % 16 != 0)
    return fail(ctx, MC_ERR_UNSUPPORTED, "basket dim must be a multiple of 16 up to 256");
  if (!m->sigma || !m->corr) return fail(ctx, MC_ERR_INVALID_ARG, "basket needs sigma and corr");
  for (uint32_t a = 0; a < d; ++a)
    if (!finite_nonneg(m->sigma[a])) return fail(ctx, MC_ERR_INVALID_ARG, "sigma[%u] invalid", a);
  for (uint32_t i = 0; i < d; ++i)
    for (uint32_t j = 0; j < d; ++j) {
      const double c = m->corr[(size_t)i * d + j];
      if (!std::isfinite(c)) return fail(ctx, MC_ERR_INVALID_ARG, "corr not finite");
      if (c != m->corr[(size_t)j * d + i]) return fail(ctx, MC_ERR_INVALID_ARG, "corr not symmetric");
    }
  if (f->kind != MC_BASKET_CALL) return fail(ctx, MC_ERR_UNSUPPORTED, "basket prices MC_BASKET_CALL");
  if (f->cv != MC_CV_NONE) return fail(ctx, MC_ERR_UNSUPPORTED, "no control variate for the basket");
  if (f->weights)
    for (uint32_t a = 0; a < d; ++a)
      if (!std::isfinite(f->weights[a])) return fail(ctx, MC_ERR_INVALID_ARG, "weights not finite");
  if (o.prec == MC_FP64) return fail(ctx, MC_ERR_UNSUPPORTED, "basket runs in FP32/BF16/FP16");
  if (o.prec != MC_FP32 && o.prec != MC_BF16_GEMM && o.prec != MC_FP16_GEMM &&
      o.prec != MC_BF16X2_GEMM)
    return fail(ctx, MC_ERR_INVALID_ARG, "unknown precision");
  if (o.greeks & MC_GREEK_VEGA) return fail(ctx, MC_ERR_UNSUPPORTED, "basket greeks: delta only");
  if ((uint64_t)n_steps * d / 4 >= (1ull << 32))
    return fail(ctx, MC_ERR_INVALID_ARG, "n_steps * dim above 2^34 normals per path");
  // The factor is cached in the context (validation without a context
  // factorises every time).
  const size_t dd = (size_t)d * d;
  std::vector<double> local;
  const std::vector<double>* Lf = &local;
  bool pd = false;
  if (ctx) {
    if (ctx->chol_corr.size() != dd ||
        std::memcmp(ctx->chol_corr.data(), m->corr, dd * sizeof(double)) != 0) {
      ctx->chol_corr.assign(m->corr, m->corr + dd);
      ctx->chol_L.assign(dd, 0.0);
      ctx->chol_pd = host::cholesky((int)d, m->corr, ctx->chol_L.data());
    }
    Lf = &ctx->chol_L;
    pd = ctx->chol_pd;
  } else {
    local.assign(dd, 0.0);
    pd = host::cholesky((int)d, m->corr, local.data());
  }
  if (!pd) return fail(ctx, MC_ERR_NOT_PD, "correlation matrix is not positive definite");
  if (L) *L = *Lf;
  return MC_OK;
}

mc_status validate_model_payoff(mc_context* ctx, const mc_model* m, const mc_payoff* f,
                                uint64_t n_paths, uint32_t n_steps, const mc_options& o);

// Every check of mc_price, no device access. Finite-difference greeks are
// checked here and the rest as for a run without greeks (the bumped runs
// price the payoff alone).
mc_status validate_all(mc_context* ctx, const mc_model* m, const mc_payoff* f, uint64_t n_paths,
                       uint32_t n_steps, const mc_options& o) {
  if (o.greeks_method != MC_GREEKS_PATHWISE && o.greeks_method != MC_GREEKS_FD_CRN &&
      o.greeks_method != MC_GREEKS_TANGENT)
    return fail(ctx, MC_ERR_INVALID_ARG, "unknown greeks_method");
  if (o.greeks == 0 || o.greeks_method != MC_GREEKS_FD_CRN)
    return validate_model_payoff(ctx, m, f, n_paths, n_steps, o);
  if (!(std::isfinite(o.fd_rel_step) && o.fd_rel_step > 0.0 && o.fd_rel_step < 0.5))
    return fail(ctx, MC_ERR_INVALID_ARG, "fd_rel_step must lie in (0, 0.5)");
  if (o.greeks & ~(MC_GREEK_DELTA | MC_GREEK_VEGA))
    return fail(ctx, MC_ERR_INVALID_ARG, "unknown greek bits");
  mc_options ob = o;
  ob.greeks = 0;
  ob.greeks_method = MC_GREEKS_PATHWISE;
  mc_status st = validate_model_payoff(ctx, m, f, n_paths, n_steps, ob);
  if (st != MC_OK) return st;
  if (f->cv == MC_CV_LEARNED) return fail(ctx, MC_ERR_UNSUPPORTED, "greeks with the learned CV");
  if (m->kind == MC_GBM_BASKET && (o.greeks & MC_GREEK_VEGA))
    return fail(ctx, MC_ERR_UNSUPPORTED, "basket greeks: delta only");
  if ((o.greeks & MC_GREEK_DELTA) && !(m->S0[0] > 0.0))
    return fail(ctx, MC_ERR_INVALID_ARG, "finite differences need S0 > 0");
  if (o.greeks & MC_GREEK_VEGA) {
    const double th = m->kind == MC_HESTON ? m->v0 : m->sigma[0];
    if (!(th > 0.0))
      return fail(ctx, MC_ERR_INVALID_ARG, "relative finite differences need a positive %s",
                  m->kind == MC_HESTON ? "v0" : "sigma");
  }
  return MC_OK;
}

mc_status validate_model_payoff(mc_context* ctx, const mc_model* m, const mc_payoff* f,
                                uint64_t n_paths, uint32_t n_steps, const mc_options& o) {
  mc_status st = validate_common(ctx, m, f, n_paths, n_steps);
  if (st != MC_OK) return st;
  if (o.cv_hedge_every == 0) return fail(ctx, MC_ERR_INVALID_ARG, "cv_hedge_every must be >= 1");
  if (m->kind == MC_GBM) {
    st = validate_gbm(ctx, m, f, o);
    if (st != MC_OK) return st;
    (void)gbm_want_mask(f, o, &st);
    if (st != MC_OK) return fail(ctx, st, "pathwise greeks need a continuous payoff");
    if (f->cv == MC_CV_LEARNED) return fail(ctx, MC_ERR_UNSUPPORTED, "learned CV is Heston-only");
    if (f->cv == MC_CV_GEO_ASIAN && f->kind != MC_ASIAN_ARITH_CALL)
      return fail(ctx, MC_ERR_UNSUPPORTED, "geometric CV applies to the arithmetic Asian");
    if (f->cv == MC_CV_GEO_ASIAN && m->scheme != MC_LOG_EULER)
      return fail(ctx, MC_ERR_UNSUPPORTED, "geometric-Asian CV needs the log-Euler scheme");
    if (f->kind == MC_UO_BRIDGE_CALL && m->scheme != MC_LOG_EULER)
      return fail(ctx, MC_ERR_UNSUPPORTED, "Brownian-bridge barrier needs the log-Euler scheme");
    return MC_OK;
  }
  if (m->kind == MC_HESTON) {
    st = validate_heston(ctx, m, o);
    if (st != MC_OK) return st;
    if (f->kind != MC_EURO_CALL && f->kind != MC_ASIAN_ARITH_CALL)
      return fail(ctx, MC_ERR_UNSUPPORTED, "Heston offers the European and arithmetic-Asian call");
    if (f->cv == MC_CV_GEO_ASIAN)
      return fail(ctx, MC_ERR_UNSUPPORTED, "geometric CV is GBM-only");
    if (f->cv == MC_CV_LEARNED) {
      if (o.greeks) return fail(ctx, MC_ERR_UNSUPPORTED, "greeks with the learned CV");
      if (f->kind != MC_ASIAN_ARITH_CALL)
        return fail(ctx, MC_ERR_UNSUPPORTED, "learned CV covers the arithmetic-Asian call");
      if (!(m->theta > 0.0)) return fail(ctx, MC_ERR_INVALID_ARG, "learned CV needs theta > 0");
      if (o.prec != MC_FP32 && o.prec != MC_BF16_GEMM)
        return fail(ctx, MC_ERR_UNSUPPORTED, "learned CV runs in MC_FP32 or MC_BF16_GEMM");
      if (!o.cv_weights) return fail(ctx, MC_ERR_INVALID_ARG, "MC_CV_LEARNED needs cv_weights");
      if (o.pilot_paths == MC_PILOT_IN_SAMPLE && !std::isfinite(o.cv_beta))
        return fail(ctx, MC_ERR_UNSUPPORTED, "the learned CV's fallback needs a pilot run");
      return MC_OK;
    }
    if (o.prec != MC_FP32 && o.prec != MC_FP64)
      return fail(ctx, MC_ERR_UNSUPPORTED, "Heston paths run in MC_FP32 or MC_FP64");
    if (o.greeks && o.greeks_method != MC_GREEKS_TANGENT && o.prec != MC_FP32)
      return fail(ctx, MC_ERR_UNSUPPORTED, "adjoint greeks run in MC_FP32");
    return MC_OK;
  }
  if (m->kind == MC_GBM_BASKET) return validate_basket(ctx, m, f, n_steps, o, nullptr);
  return fail(ctx, MC_ERR_INVALID_ARG, "unknown model kind");
}

// Device workspace: the caller's, or the context's (grown on demand).
mc_status get_ws(mc_context* ctx, const mc_options& o, size_t bytes, char** base) {
  if (ctx->noalloc) {
    if (bytes > MC_NOALLOC_SCRATCH_BYTES)
      return fail(ctx, MC_ERR_WORKSPACE,
                  "mc_price_noalloc: this run needs %zu bytes of device scratch, the static "
                  "scratch holds %zu", bytes, (size_t)MC_NOALLOC_SCRATCH_BYTES);
    *base = (char*)ctx->scratch;
    return MC_OK;
  }
  if (o.workspace) {
    if (o.workspace_bytes < bytes)
      return fail(ctx, MC_ERR_WORKSPACE, "workspace has %zu bytes, %zu needed", o.workspace_bytes,
                  bytes);
    *base = (char*)o.workspace;
    return MC_OK;
  }
  if (ctx->ws_bytes < bytes) {
    if (ctx->ws) {
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      HIP_TRY(ctx, hipFree(ctx->ws));
      ctx->ws = nullptr;
      ctx->ws_bytes = 0;
    }
    size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
    HIP_TRY(ctx, hipMalloc(&ctx->ws, want));
    ctx->ws_bytes = want;
  }
  *base = (char*)ctx->ws;
  return MC_OK;
}

mc_status get_pinned(mc_context* ctx, size_t count) {
  if (ctx->pinned_count >= count) return MC_OK;
  if (ctx->pinned) HIP_TRY(ctx, hipHostFree(ctx->pinned));
  ctx->pinned = nullptr;
  ctx->pinned_count = 0;
  size_t want = count < 4096 ? 4096 : count;
  HIP_TRY(ctx, hipHostMalloc((void**)&ctx->pinned, want * sizeof(double), hipHostMallocDefault));
  ctx->pinned_count = want;
  return MC_OK;
}

hipStream_t stream_of(mc_context* ctx, const mc_options& o) {
  return o.hip_stream ? (hipStream_t)o.hip_stream : ctx->stream;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Sizes of one moment run.
struct RunLayout {
  uint32_t n_blocks, n_mom, C;
  size_t off_mom, off_path, bytes;
};

// max_blocks: the grid cap of a persistent kernel (its partials are one
// vector per workgroup).
RunLayout layout_for(uint64_t n_paths, int C, bool want_path, uint32_t paths_per_block = kBlock,
                     uint32_t max_blocks = UINT32_MAX) {
  RunLayout L;
  const uint64_t need = (n_paths + paths_per_block - 1) / paths_per_block;
  L.n_blocks = (uint32_t)(need < max_blocks ? need : max_blocks);
  L.C = (uint32_t)C;
  L.n_mom = (uint32_t)n_moments(C);
  L.off_mom = align256((size_t)L.n_mom * L.n_blocks * sizeof(double));
  L.off_path = L.off_mom + align256((size_t)L.n_mom * sizeof(double));
  L.bytes = L.off_path + (want_path ? align256((size_t)n_paths * C * sizeof(double)) : 0);
  return L;
}

// Result of one moment run: n, means and covariances of C channels, from
// the merged (count, means, co-moments) vector the kernels produce.
constexpr int kMaxChannels = kMaxMomentChannels;
struct Moments {
  int C = 0;
  double n = 0, nonfinite = 0;
  double means[kMaxChannels] = {};
  double co[kMaxChannels * (kMaxChannels + 1) / 2] = {};  // upper-triangular row order
  double mean(int c) const { return means[c]; }
  double cov(int a, int b) const {
    if (a > b) std::swap(a, b);
    int idx = 0;
    for (int i = 0; i < a; ++i) idx += C - i;
    idx += b - a;
    return co[idx] / (n - 1.0);
  }
};

// Host form of the kernels' pairwise (Chan) merge of two moment vectors of
// C channels: acc <- acc merged with b. Used to combine chunks.
void merge_moment_vec(double* acc, const double* b, int C) {
  const double nA = acc[0], nB = b[0], nt = nA + nB;
  const double f = nt > 0.0 ? nB / nt : 0.0, g = nA * f;
  acc[1] += b[1];
  double d[kMaxChannels];
  for (int a = 0; a < C; ++a) {
    d[a] = b[2 + a] - acc[2 + a];
    acc[2 + a] += d[a] * f;
  }
  int k = 2 + C;
  for (int a = 0; a < C; ++a)
    for (int c = a; c < C; ++c, ++k) acc[k] += b[k] + d[a] * d[c] * g;
  acc[0] = nt;
}

// Launch wrapper: runs `launch` (which enqueues the path kernel), then the
// final reduction, and brings the moments to the host.
template <typename F>
mc_status run_moments(mc_context* ctx, const mc_options& o, uint64_t n_paths, int C,
                      double* host_path_values, F&& launch, Moments* out, double* kernel_ms,
                      uint32_t paths_per_block = kBlock, uint32_t max_blocks = UINT32_MAX) {
  if (C < 1 || C > kMaxChannels) return fail(ctx, MC_ERR_DEVICE, "channel count %d", C);
  const RunLayout L =
      layout_for(n_paths, C, host_path_values != nullptr, paths_per_block, max_blocks);
  char* base = nullptr;
  mc_status st = get_ws(ctx, o, L.bytes, &base);
  if (st != MC_OK) return st;
  double* hmom = ctx->host_mom;
  if (!ctx->noalloc) {
    st = get_pinned(ctx, L.n_mom);
    if (st != MC_OK) return st;
    hmom = ctx->pinned;
  } else if (host_path_values || ctx->sink) {
    return fail(ctx, MC_ERR_UNSUPPORTED, "mc_price_noalloc writes no per-path values");
  }
  hipStream_t s = stream_of(ctx, o);
  double* partials = (double*)base;
  double* mom = (double*)(base + L.off_mom);
  double* path_out =
      ctx->sink ? ctx->sink : (host_path_values ? (double*)(base + L.off_path) : nullptr);
  HIP_TRY(ctx, hipEventRecord(ctx->ev0, s));
  uint32_t nb = 0;
  HIP_TRY(ctx, launch(partials, path_out, s, &nb));
  HIP_TRY(ctx, hipEventRecord(ctx->ev1, s));
  if (nb == 0 || nb > L.n_blocks) return fail(ctx, MC_ERR_DEVICE, "block count mismatch");
  HIP_TRY(ctx, launch_final_merge(partials, nb, (uint32_t)C, 1, mom, s));
  HIP_TRY(ctx, hipMemcpyAsync(hmom, mom, L.n_mom * sizeof(double), hipMemcpyDeviceToHost, s));
  if (host_path_values && !ctx->sink)
    HIP_TRY(ctx, hipMemcpyAsync(host_path_values, path_out, n_paths * C * sizeof(double),
                                hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  float ms = 0.f;
  HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  if (kernel_ms) *kernel_ms += ms;
  out->C = C;
  out->n = hmom[0];
  out->nonfinite = hmom[1];
  std::copy(hmom + 2, hmom + 2 + C, out->means);
  std::copy(hmom + 2 + C, hmom + L.n_mom, out->co);
  if (out->n < 2) return fail(ctx, MC_ERR_DEVICE, "fewer than two finite paths");
  return MC_OK;
}

void fill_channel(const Moments& m, int c, double* price, double* var, double* se) {
  *price = m.mean(c);
  *var = m.cov(c, c);
  *se = std::sqrt(*var / m.n);
}

// ---------------------------------------------------------------- GBM ----
uint32_t gbm_want_mask(const mc_payoff* f, const mc_options& o, mc_status* st) {
  *st = MC_OK;
  const bool greeks = o.greeks != 0;
  switch (f->kind) {
    case MC_EURO_CALL:
      return G_EURO | (greeks ? G_EURO_G : 0);
    case MC_ASIAN_ARITH_CALL:
      return G_ASIAN | (f->cv == MC_CV_GEO_ASIAN ? G_GEO : 0) | (greeks ? G_ASIAN_G : 0);
    case MC_ASIAN_GEO_CALL:
      if (greeks) *st = MC_ERR_UNSUPPORTED;
      return G_GEO;
    case MC_UO_BARRIER_CALL:
      if (greeks) *st = MC_ERR_UNSUPPORTED;
      return G_UO;
    case MC_UO_BRIDGE_CALL:
      if (greeks) *st = MC_ERR_UNSUPPORTED;
      return G_UOBB;
    default:
      *st = MC_ERR_UNSUPPORTED;
      return 0;
  }
}

// Channel index of functional `bit` (and its second greek) inside `mask`.
int gbm_channel_index(uint32_t mask, uint32_t bit) {
  int c = 0;
  for (uint32_t b = 1; b <= G_ASIAN_G; b <<= 1) {
    if (b == bit) return (mask & b) ? c : -1;
    if (mask & b) c += (b == G_EURO_G || b == G_ASIAN_G) ? 2 : 1;
  }
  return -1;
}

const char* gbm_channel_name(uint32_t mask, uint32_t i) {
  static const char* names[] = {"euro",       "asian",     "geo",         "uo",        "uo_bridge",
                                "euro_delta", "euro_vega", "asian_delta", "asian_vega"};
  int c = 0, slot = 0;
  for (uint32_t b = 1; b <= G_ASIAN_G; b <<= 1) {
    const int w = (b == G_EURO_G || b == G_ASIAN_G) ? 2 : 1;
    if (mask & b) {
      if ((uint32_t)c == i) return names[slot];
      if (w == 2 && (uint32_t)c + 1 == i) return names[slot + 1];
      c += w;
    }
    slot += w;
  }
  return nullptr;
}

GbmParams gbm_params(const mc_model* m, const mc_payoff* f, uint64_t n_paths, uint32_t n_steps,
                     uint64_t seed, const mc_options& o, bool fp64, uint32_t tag) {
  GbmParams p{};
  const double S0 = m->S0[0], sig = m->sigma[0], r = m->r, T = m->T;
  const double dt = T / n_steps;
  const double sc = fp64 ? 1.0 : 1.0 / std::log(2.0);   // log domain of the kernel
  p.n_paths = n_paths;
  p.path_offset = o.path_offset;
  p.n_steps = n_steps;
  p.tag = tag;
  p.k0 = (uint32_t)seed;
  p.k1 = (uint32_t)(seed >> 32);
  p.log_scheme = m->scheme == MC_LOG_EULER;
  p.coarsen = 1;
  p.S0 = S0;
  p.K = f->K;
  p.disc = std::exp(-r * T);
  p.T = T;
  p.dt = dt;
  p.sdt = std::sqrt(dt);
  p.sigma = sig;
  p.drift_dom = (r - 0.5 * sig * sig) * dt * sc;
  p.vol_dom = sig * std::sqrt(dt) * sc;
  const double B = (std::isfinite(f->B) && f->B > 0) ? f->B : 1e300;
  p.barrier_dom = std::log(B / S0) * sc;
  p.bridge_c = 2.0 * dt * sig * sig * (fp64 ? 1.0 : 1.0 / std::log(2.0));
  p.r_dt = r * dt;
  p.vol_sdt = sig * std::sqrt(dt);
  p.barrier_rel = B / S0;
  return p;
}

mc_status gbm_run(mc_context* ctx, const mc_model* m, const mc_payoff* f, uint64_t n_paths,
                  uint32_t n_steps, uint64_t seed, const mc_options& o, uint32_t want,
                  uint32_t tag, double* path_values, Moments* mom, uint32_t* mask_used,
                  double* kernel_ms) {
  const bool fp64 = o.prec == MC_FP64;
  const bool logs = m->scheme == MC_LOG_EULER;
  const uint32_t mask = gbm_pick_mask(want, fp64, logs, ctx->coarsen);
  if (!mask) return fail(ctx, MC_ERR_UNSUPPORTED, "payoff not available for this scheme/precision");
  *mask_used = mask;
  GbmParams p = gbm_params(m, f, n_paths, n_steps, seed, o, fp64, tag);
  p.coarsen = ctx->coarsen;
  return run_moments(ctx, o, n_paths, gbm_channels(mask), path_values,
                     [&](double* partials, double* path_out, hipStream_t s, uint32_t* nb) {
                       p.partials = partials;
                       p.path_out = path_out;
                       return launch_gbm(p, mask, fp64, s, nb);
                     },
                     mom, kernel_ms, kBlock, kGbmMaxBlocks);
}

// Fills `out` for one GBM payoff from the moments of a run.
mc_status gbm_result(mc_context* ctx, const mc_model* m, const mc_payoff* f, uint32_t n_steps,
                     uint64_t seed, const mc_options& o, uint32_t mask, const Moments& mom,
                     double kernel_ms, uint64_t n_paths, mc_result* out) {
  mc_result r{};
  uint32_t bit = 0, gbit = 0;
  switch (f->kind) {
    case MC_EURO_CALL: bit = G_EURO; gbit = G_EURO_G; break;
    case MC_ASIAN_ARITH_CALL: bit = G_ASIAN; gbit = G_ASIAN_G; break;
    case MC_ASIAN_GEO_CALL: bit = G_GEO; break;
    case MC_UO_BARRIER_CALL: bit = G_UO; break;
    case MC_UO_BRIDGE_CALL: bit = G_UOBB; break;
    default: return fail(ctx, MC_ERR_UNSUPPORTED, "payoff not offered for GBM");
  }
  const int c = gbm_channel_index(mask, bit);
  fill_channel(mom, c, &r.price, &r.variance, &r.std_err);
  r.plain_price = r.price;
  r.plain_std_err = r.std_err;
  r.cv_beta = 0.0;
  r.vrf = 1.0;
  if (o.greeks && gbit) {
    const int g = gbm_channel_index(mask, gbit);
    double v;
    if (o.greeks & MC_GREEK_DELTA) fill_channel(mom, g, &r.delta, &v, &r.delta_se);
    if (o.greeks & MC_GREEK_VEGA) fill_channel(mom, g + 1, &r.vega, &v, &r.vega_se);
  }
  if (f->kind == MC_ASIAN_ARITH_CALL && f->cv == MC_CV_GEO_ASIAN) {
    if (m->scheme != MC_LOG_EULER)
      return fail(ctx, MC_ERR_UNSUPPORTED, "geometric-Asian CV needs the log-Euler scheme");
    const int a = c, gi = gbm_channel_index(mask, G_GEO);
    double beta = o.cv_beta;
    if (!std::isfinite(beta) && o.pilot_paths == MC_PILOT_IN_SAMPLE) {
      // In sample: the coefficient from the main paths' own moments.
      beta = mom.cov(a, gi) / mom.cov(gi, gi);
    } else if (!std::isfinite(beta)) {
      // Pilot on stream tag+1 (independent of the main paths).
      Moments pm;
      uint32_t pmask;
      mc_options po = o;
      po.path_offset = 0;
      const uint64_t np = o.pilot_paths ? o.pilot_paths : (1ull << 16);
      mc_status st = gbm_run(ctx, m, f, np, n_steps, seed, po, G_ASIAN | G_GEO, o.stream_tag + 1,
                             nullptr, &pm, &pmask, nullptr);
      if (st != MC_OK) return st;
      const int pa = gbm_channel_index(pmask, G_ASIAN), pg = gbm_channel_index(pmask, G_GEO);
      beta = pm.cov(pa, pg) / pm.cov(pg, pg);
    }
    const double CG = host::geo_asian_call(m->S0[0], f->K, m->r, m->sigma[0], m->T, n_steps);
    r.price = mom.mean(a) - beta * (mom.mean(gi) - CG);
    r.variance = mom.cov(a, a) - 2.0 * beta * mom.cov(a, gi) + beta * beta * mom.cov(gi, gi);
    r.std_err = std::sqrt(r.variance / mom.n);
    r.cv_beta = beta;
    r.vrf = mom.cov(a, a) / r.variance;
  }
  r.n_paths = (uint64_t)mom.n;
  r.n_nonfinite = (uint64_t)mom.nonfinite;
  r.kernel_ms = kernel_ms;
  (void)seed;
  (void)n_paths;
  *out = r;
  return MC_OK;
}

// ------------------------------------------------------------- Heston ----
HestonParams heston_params(const mc_model* m, const mc_payoff* f, uint64_t n_paths,
                           uint32_t n_steps, uint64_t seed, const mc_options& o, uint32_t tag) {
  HestonParams p{};
  p.n_paths = n_paths;
  p.path_offset = o.path_offset;
  p.n_steps = n_steps;
  p.tag = tag;
  p.k0 = (uint32_t)seed;
  p.k1 = (uint32_t)(seed >> 32);
  p.S0 = m->S0[0];
  p.K = f->K;
  p.disc = std::exp(-m->r * m->T);
  p.dt = m->T / n_steps;
  p.sdt = std::sqrt(p.dt);
  p.r = m->r;
  p.v0 = m->v0;
  p.kappa = m->kappa;
  p.theta = m->theta;
  p.xi = m->xi;
  p.rho = m->rho;
  p.rho_c = std::sqrt(1.0 - m->rho * m->rho);
  return p;
}

mc_status heston_cv_price(mc_context* ctx, const mc_model* m, const mc_payoff* f,
                          uint64_t n_paths, uint32_t n_steps, uint64_t seed, const mc_options& o0,
                          mc_result* out);

mc_status heston_price(mc_context* ctx, const mc_model* m, const mc_payoff* f, uint64_t n_paths,
                       uint32_t n_steps, uint64_t seed, const mc_options& o, mc_result* out) {
  if (f->cv == MC_CV_LEARNED) {
    if (o.greeks) return fail(ctx, MC_ERR_UNSUPPORTED, "greeks with the learned CV");
    return heston_cv_price(ctx, m, f, n_paths, n_steps, seed, o, out);
  }
  if (f->cv != MC_CV_NONE) return fail(ctx, MC_ERR_UNSUPPORTED, "control variate not available");
  const bool fp64 = o.prec == MC_FP64;
  if (o.greeks && o.greeks_method == MC_GREEKS_TANGENT) {
    // Forward-mode tangents: channels payoff, delta, d/dv0.
    HestonParams p = heston_params(m, f, n_paths, n_steps, seed, o, o.stream_tag);
    const bool asian = f->kind == MC_ASIAN_ARITH_CALL;
    Moments mom;
    double kms = 0.0;
    mc_status st = run_moments(ctx, o, n_paths, 3, o.path_values,
                               [&](double* partials, double* path_out, hipStream_t s,
                                   uint32_t* nb) {
                                 p.partials = partials;
                                 p.path_out = path_out;
                                 return launch_heston_tangent(p, asian, fp64, s, nb);
                               },
                               &mom, &kms, kBlock, kHestonMaxBlocks);
    if (st != MC_OK) return st;
    mc_result r{};
    double v;
    fill_channel(mom, 0, &r.price, &r.variance, &r.std_err);
    r.plain_price = r.price;
    r.plain_std_err = r.std_err;
    if (o.greeks & MC_GREEK_DELTA) fill_channel(mom, 1, &r.delta, &v, &r.delta_se);
    if (o.greeks & MC_GREEK_VEGA) fill_channel(mom, 2, &r.vega, &v, &r.vega_se);
    r.vrf = 1.0;
    r.n_paths = (uint64_t)mom.n;
    r.n_nonfinite = (uint64_t)mom.nonfinite;
    r.kernel_ms = kms;
    *out = r;
    return MC_OK;
  }
  if (o.greeks) {
    return mc_greeks_adjoint(ctx, m, f, n_paths, n_steps, seed, &o, MC_ADJ_FULL, mcp::kCkpt,
                             nullptr, 0, 1.0, out);
  }
  HestonParams p = heston_params(m, f, n_paths, n_steps, seed, o, o.stream_tag);
  Moments mom;
  double kms = 0.0;
  mc_status st = run_moments(ctx, o, n_paths, 2, o.path_values,
                             [&](double* partials, double* path_out, hipStream_t s, uint32_t* nb) {
                               p.partials = partials;
                               p.path_out = path_out;
                               return launch_heston(p, H_EURO | H_ASIAN, fp64, s, nb);
                             },
                             &mom, &kms, kBlock, kHestonMaxBlocks);
  if (st != MC_OK) return st;
  mc_result r{};
  const int c = f->kind == MC_EURO_CALL ? 0 : 1;
  fill_channel(mom, c, &r.price, &r.variance, &r.std_err);
  r.plain_price = r.price;
  r.plain_std_err = r.std_err;
  r.vrf = 1.0;
  r.n_paths = (uint64_t)mom.n;
  r.n_nonfinite = (uint64_t)mom.nonfinite;
  r.kernel_ms = kms;
  *out = r;
  return MC_OK;
}

// ------------------------------------------------- Learned control variate --
// Device buffers of one learned-CV run: weights, their fragments and the
// undiscounting table, after the moment layout in the workspace.
struct CvBuffers {
  float *theta, *w1f, *w2f, *w2tf, *lanec, *dfac;
};

size_t cv_extra_bytes(uint32_t n_steps) {
  return align256(kMlpNParam * 4) + align256(kW1fFloats * 4) + 2 * align256(kW2fFloats * 4) +
         align256(kLanecFloats * 4) + align256((size_t)(n_steps + 1) * 4);
}

CvBuffers cv_carve(char* p) {
  CvBuffers b;
  b.theta = (float*)p;
  p += align256(kMlpNParam * 4);
  b.w1f = (float*)p;
  p += align256(kW1fFloats * 4);
  b.w2f = (float*)p;
  p += align256(kW2fFloats * 4);
  b.w2tf = (float*)p;
  p += align256(kW2fFloats * 4);
  b.lanec = (float*)p;
  p += align256(kLanecFloats * 4);
  b.dfac = (float*)p;
  return b;
}

std::vector<float> dfac_table(const mc_model* m, uint32_t n_steps) {
  std::vector<float> t(n_steps + 1);
  for (uint32_t i = 0; i <= n_steps; ++i) t[i] = (float)std::exp(m->r * m->T * i / n_steps);
  return t;
}

CvParams cv_params(const mc_model* m, const mc_payoff* f, uint64_t n_paths, uint32_t n_steps,
                   uint64_t seed, const mc_options& o, uint32_t tag, uint32_t hedge_every,
                   bool bf16, const CvBuffers& b) {
  CvParams p{};
  p.h = heston_params(m, f, n_paths, n_steps, seed, o, tag);
  p.hedge_every = hedge_every;
  p.bf16 = bf16 ? 1 : 0;
  p.theta = b.theta;
  p.w1f = b.w1f;
  p.w2f = b.w2f;
  p.w2tf = b.w2tf;
  p.lanec = b.lanec;
  p.dfac = b.dfac;
  return p;
}

// Uploads weights and the discount table, builds the fragments.
mc_status cv_upload(mc_context* ctx, hipStream_t s, const CvBuffers& b, const float* theta_host,
                    const std::vector<float>& dfac) {
  if (theta_host)
    HIP_TRY(ctx, hipMemcpyAsync(b.theta, theta_host, kMlpNParam * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, hipMemcpyAsync(b.dfac, dfac.data(), dfac.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, launch_cv_pack(b.theta, b.w1f, b.w2f, b.w2tf, b.lanec, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return MC_OK;
}

mc_status cv_validate(mc_context* ctx, const mc_model* m, const mc_payoff* f, mc_precision prec,
                      uint32_t hedge_every) {
  if (m->kind != MC_HESTON || f->kind != MC_ASIAN_ARITH_CALL)
    return fail(ctx, MC_ERR_UNSUPPORTED, "learned CV covers the Heston arithmetic-Asian call");
  if (!(m->theta > 0.0)) return fail(ctx, MC_ERR_INVALID_ARG, "learned CV needs theta > 0");
  if (prec != MC_FP32 && prec != MC_BF16_GEMM)
    return fail(ctx, MC_ERR_UNSUPPORTED, "learned CV runs in MC_FP32 or MC_BF16_GEMM");
  if (hedge_every == 0) return fail(ctx, MC_ERR_INVALID_ARG, "hedge_every must be >= 1");
  return MC_OK;
}

// One evaluation pass of the hedged estimator: channels payoff, H, Y.
mc_status cv_eval(mc_context* ctx, const mc_options& o, const CvParams& base, uint64_t n_paths,
                  double* host_path_values, Moments* mom, double* kms) {
  CvParams p = base;
  return run_moments(ctx, o, n_paths, 3, host_path_values,
                     [&](double* partials, double* path_out, hipStream_t s, uint32_t* nb) {
                       p.partials = partials;
                       p.path_out = path_out;
                       return launch_cv_price(p, s, nb);
                     },
                     mom, kms, kCvPathsPerBlock);
}

mc_status heston_cv_price(mc_context* ctx, const mc_model* m, const mc_payoff* f,
                          uint64_t n_paths, uint32_t n_steps, uint64_t seed, const mc_options& o0,
                          mc_result* out) {
  mc_status st = cv_validate(ctx, m, f, o0.prec, o0.cv_hedge_every);
  if (st != MC_OK) return st;
  if (!o0.cv_weights) return fail(ctx, MC_ERR_INVALID_ARG, "MC_CV_LEARNED needs cv_weights");
  for (int i = 0; i < kMlpNParam; ++i)
    if (!std::isfinite(o0.cv_weights[i])) return fail(ctx, MC_ERR_INVALID_ARG, "cv_weights not finite");
  // The pilot runs only when beta is left to it (NaN).
  const bool pilot = !std::isfinite(o0.cv_beta);
  if (pilot && o0.pilot_paths == MC_PILOT_IN_SAMPLE)
    return fail(ctx, MC_ERR_UNSUPPORTED, "the learned CV's fallback needs a pilot run");
  const uint64_t n_pilot = !pilot ? 0 : o0.pilot_paths ? o0.pilot_paths : (1ull << 16);
  const uint64_t n_big = n_paths > n_pilot ? n_paths : n_pilot;
  const RunLayout Lay = layout_for(n_big, 3, o0.path_values != nullptr, kCvPathsPerBlock);
  const size_t off = align256(Lay.bytes);
  char* base = nullptr;
  st = get_ws(ctx, o0, off + cv_extra_bytes(n_steps), &base);
  if (st != MC_OK) return st;
  const CvBuffers b = cv_carve(base + off);
  hipStream_t s = stream_of(ctx, o0);
  st = cv_upload(ctx, s, b, o0.cv_weights, dfac_table(m, n_steps));
  if (st != MC_OK) return st;
  mc_options o = o0;
  o.workspace = base;
  o.workspace_bytes = Lay.bytes;
  const bool bf16 = o0.prec == MC_BF16_GEMM;
  double kms = 0.0;
  // Y = payoff - beta H. A finite cv_beta is the caller's choice; NaN means
  // beta = 1 (the hedge as trained) with a pilot on stream tag+1 deciding
  // between the hedged estimator and plain Monte Carlo.
  const bool fixed = std::isfinite(o0.cv_beta);
  const double beta = fixed ? o0.cv_beta : 1.0;
  if (!fixed) {
    mc_options po = o;
    po.path_offset = 0;
    po.path_values = nullptr;
    Moments pm;
    st = cv_eval(ctx, po, cv_params(m, f, n_pilot, n_steps, seed, po, o0.stream_tag + 1,
                                     o0.cv_hedge_every, bf16, b),
                 n_pilot, nullptr, &pm, &kms);
    if (st != MC_OK) return st;
    const double pilot_vrf = pm.cov(0, 0) / pm.cov(2, 2);
    if (!(pilot_vrf > 1.0)) {
      mc_options plain = o0;
      plain.path_values = nullptr;
      mc_payoff fp = *f;
      fp.cv = MC_CV_NONE;
      st = heston_price(ctx, m, &fp, n_paths, n_steps, seed, plain, out);
      if (st != MC_OK) return st;
      out->cv_fallback = 1;
      out->vrf = pilot_vrf;
      out->kernel_ms += kms;
      return MC_OK;
    }
  }
  Moments mom;
  st = cv_eval(ctx, o, cv_params(m, f, n_paths, n_steps, seed, o, o0.stream_tag, o0.cv_hedge_every,
                                 bf16, b),
               n_paths, o0.path_values, &mom, &kms);
  if (st != MC_OK) return st;
  mc_result r{};
  double v;
  fill_channel(mom, 0, &r.plain_price, &v, &r.plain_std_err);
  r.price = mom.mean(0) - beta * mom.mean(1);
  r.variance = mom.cov(0, 0) - 2.0 * beta * mom.cov(0, 1) + beta * beta * mom.cov(1, 1);
  r.std_err = std::sqrt(r.variance / mom.n);
  r.cv_beta = beta;
  r.vrf = mom.cov(0, 0) / r.variance;
  r.n_paths = (uint64_t)mom.n;
  r.n_nonfinite = (uint64_t)mom.nonfinite;
  r.kernel_ms = kms;
  *out = r;
  return MC_OK;
}

// Training workspace: moments and per-path values of the minibatch, the
// gradient partials, the weights and their fragments, Adam's moments, the
// per-step loss moments and the feature cache of the training paths.
struct CvTrainWs {
  char* eval_base;          // moment layout with per-path values
  size_t eval_bytes;
  float* grad_partials;     // [n_blocks][kGradStride]
  double* grad;             // [kMlpNParam]
  CvBuffers b;
  float *m, *v;             // Adam moments
  double* log;              // [steps][n_mom] forward-pass moments
  float *c_phi, *c_dst;
  double* c_pay;
};

uint32_t cv_segments(uint32_t n_steps, uint32_t hedge_every) {
  return (n_steps + hedge_every - 1) / hedge_every;
}

// Block moments and per-path values of the hedged-value kernel.
RunLayout cv_values_layout(uint64_t batch, uint32_t n_seg) {
  uint32_t split = 1;
  cv_values_blocks(batch, n_seg, &split);
  return layout_for(batch, 3, true, (uint32_t)kCvTrainPathsPerBlock / split);
}

size_t cv_train_bytes(uint64_t batch, uint32_t n_steps, uint32_t steps, uint64_t n_cache,
                      uint32_t n_seg, CvTrainWs* w, char* base) {
  const RunLayout Lay = cv_values_layout(batch, n_seg);
  const uint64_t n_blocks = cv_bwd_blocks(batch, n_seg, nullptr);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += align256(bytes);
    return p;
  };
  char* e = take(Lay.bytes);
  char* gp = take((size_t)kGradStride * n_blocks * 4);
  char* g = take((size_t)kMlpNParam * 8);
  char* cv = take(cv_extra_bytes(n_steps));
  char* mm = take((size_t)kMlpNParam * 4);
  char* vv = take((size_t)kMlpNParam * 4);
  char* lg = take((size_t)(steps ? steps : 1) * Lay.n_mom * 8);
  char* cphi = take((size_t)n_seg * 4 * n_cache * 4);
  char* cdst = take((size_t)n_seg * n_cache * 4);
  char* cpay = take((size_t)n_cache * 8);
  if (w && base) {
    w->eval_base = e;
    w->eval_bytes = Lay.bytes;
    w->grad_partials = (float*)gp;
    w->grad = (double*)g;
    w->b = cv_carve(cv);
    w->m = (float*)mm;
    w->v = (float*)vv;
    w->log = (double*)lg;
    w->c_phi = (float*)cphi;
    w->c_dst = (float*)cdst;
    w->c_pay = (double*)cpay;
  }
  return off;
}

CvParams cv_cache_params(const CvParams& base, const CvTrainWs& w, uint64_t n_cache,
                         uint32_t n_seg) {
  CvParams p = base;
  p.c_phi = w.c_phi;
  p.c_dst = w.c_dst;
  p.c_pay = w.c_pay;
  p.c_stride = n_cache;
  p.n_seg = n_seg;
  return p;
}

// Simulates n_cache training paths (from global path path0 on stream tag
// `tag`) into the feature cache.
mc_status cv_fill_cache(mc_context* ctx, hipStream_t s, const mc_model* m, const mc_payoff* f,
                        uint32_t n_steps, uint64_t seed, uint32_t tag, uint64_t path0,
                        uint64_t n_cache, uint32_t hedge_every, bool bf16, const CvTrainWs& w) {
  mc_options o = defaults();
  o.hip_stream = s;
  o.path_offset = path0;
  const uint32_t n_seg = cv_segments(n_steps, hedge_every);
  CvParams p = cv_cache_params(
      cv_params(m, f, n_cache, n_steps, seed, o, tag, hedge_every, bf16, w.b), w, n_cache, n_seg);
  HIP_TRY(ctx, launch_cv_cache(p, s));
  return MC_OK;
}

// Forward + backward over the minibatch of `batch` cached paths from cache
// path `first`; leaves the FP64 gradient in w.grad and the forward pass's
// moments in log_row.
mc_status cv_loss_grad_device(mc_context* ctx, hipStream_t s, const mc_model* m,
                              const mc_payoff* f, uint32_t n_steps, uint64_t first,
                              uint64_t n_cache, uint64_t batch, uint32_t hedge_every, bool bf16,
                              const CvTrainWs& w, double* log_row,
                              uint32_t* grad_blocks = nullptr, CvValMoments* vm_out = nullptr) {
  mc_options o = defaults();
  o.hip_stream = s;
  const RunLayout Lay = cv_values_layout(batch, cv_segments(n_steps, hedge_every));
  double* partials = (double*)w.eval_base;
  double* mom = log_row ? log_row : (double*)(w.eval_base + Lay.off_mom);
  double* ypath = (double*)(w.eval_base + Lay.off_path);
  CvParams p = cv_cache_params(cv_params(m, f, batch, n_steps, 0, o, 0, hedge_every, bf16, w.b),
                               w, n_cache, cv_segments(n_steps, hedge_every));
  p.c_first = first;
  p.partials = partials;
  p.path_out = ypath;
  uint32_t nb = 0;
  HIP_TRY(ctx, launch_cv_values(p, s, &nb));
  // The backward sums the hedged values' block moments itself (Ybar); the
  // gradient reduction's launch merges them into mom.
  const CvValMoments vm{partials, nb, mom};
  p.path_out = nullptr;
  p.val_blocks = nb;
  p.y_path = ypath;
  p.g_scale = -2.0 / (double)batch;
  p.grad_partials = w.grad_partials;
  HIP_TRY(ctx, launch_cv_backward(p, s, &nb));   // one partial per block
  // With grad_blocks the caller reduces the partials and merges the moments
  // itself (the training loop does it inside its Adam step).
  if (grad_blocks) {
    *grad_blocks = nb;
    if (vm_out) *vm_out = vm;
  } else {
    HIP_TRY(ctx, launch_grad_sum(w.grad_partials, nb, vm, w.grad, s));
  }
  return MC_OK;
}

double loss_from_moments(const double* mom) {
  // Channel 2 (Y) of a 3-channel moment vector: n = mom[0], co-moment
  // sum (Y - Ybar)^2 = mom[10]; the loss is the batch variance (1/B).
  return mom[10] / mom[0];
}

// ------------------------------------------------------------- Basket ----
// L' = diag(sigma_a sqrt(dt) / ln 2) L, packed into the kernel's lower-
// triangular 32x16 blocks (n block nb, k block kb <= 2 nb + 1, block id
// nb (nb + 1) + kb, element [n][k] row-major), in the requested type.
template <typename T, typename F>
void pack_blocks(uint32_t d, uint32_t nd, const std::vector<double>& Ls, F&& conv,
                 std::vector<T>* out) {
  out->assign((size_t)nd * (nd + 1) * 512, conv(0.0));
  for (uint32_t nb = 0; nb < nd; ++nb)
    for (uint32_t kb = 0; kb <= 2 * nb + 1; ++kb) {
      const size_t base = (size_t)(nb * (nb + 1) + kb) * 512;
      for (uint32_t r = 0; r < 32; ++r)
        for (uint32_t j = 0; j < 16; ++j) {
          const uint32_t a = 32 * nb + r, b = 16 * kb + j;
          const double v = (a < d && b < d && b <= a) ? Ls[(size_t)a * d + b] : 0.0;
          (*out)[base + r * 16 + j] = conv(v);
        }
    }
}

uint16_t to_bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}
float from_bf16(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
uint16_t to_f16_rne(float f) {
  _Float16 h = (_Float16)f;   // host conversion rounds to nearest even
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}

// Workspace of a basket run: moment layout, L' blocks (twice for the split
// BF16 form) and the per-asset table.
size_t basket_ws_bytes(size_t layout_bytes, uint32_t d, mc_precision prec) {
  const uint32_t nd = basket_blocks_nd(d);
  const size_t elt = prec == MC_FP32 ? 4 : 2;
  const size_t blk = align256((size_t)nd * (nd + 1) * 512 * elt);
  return align256(layout_bytes) + blk * (prec == MC_BF16X2_GEMM ? 2 : 1) +
         align256(4 * 256 * sizeof(float));
}

// Basket run. With `port` set it prices the call portfolio of the risk
// metrics instead: drifts port->mu (or r) and one per-path channel, the
// horizon P&L (value of the holdings at T minus their Black-Scholes value
// `premium` at 0); out->price / variance / std_err describe that P&L.
// Quasi-Monte Carlo inputs of a basket run (device direction words and
// shifts) and the run's geometric-basket mean, returned to the caller.
struct BasketQmc {
  const uint32_t* V;
  const uint32_t* shift;
  double geo_mean;
};

// Host part of a basket run: checks, Cholesky factor, packed L' and the
// per-asset constants uploaded to the workspace (after the moment area of
// run_moments), and the kernel parameters. *o_run is o0 with the workspace
// narrowed to the moment area.
mc_status basket_setup(mc_context* ctx, const mc_model* m, const mc_payoff* f, uint64_t n_paths,
                       uint32_t n_steps, uint64_t seed, const mc_options& o0,
                       const mc_portfolio* port, double premium, const BasketQmc* qmc,
                       BasketParams* p_out, int* prec_out, mc_options* o_run) {
  std::vector<double> L;
  mc_status st = validate_basket(ctx, m, f, n_steps, o0, &L);
  if (st != MC_OK) return st;
  const uint32_t d = m->dim, nd = basket_blocks_nd(d);
  const double dt = m->T / n_steps, inv_ln2 = 1.0 / std::log(2.0);
  std::vector<double> Ls((size_t)d * d);
  for (uint32_t a = 0; a < d; ++a)
    for (uint32_t b = 0; b < d; ++b)
      Ls[(size_t)a * d + b] = m->sigma[a] * std::sqrt(dt) * inv_ln2 * L[(size_t)a * d + b];
  int prec = BK_FP32;
  std::vector<float> bf32;
  std::vector<uint16_t> b16, b16lo;
  size_t blk_bytes = 0;
  switch (o0.prec) {
    case MC_FP32:
      prec = BK_FP32;
      pack_blocks<float>(d, nd, Ls, [](double v) { return (float)v; }, &bf32);
      blk_bytes = bf32.size() * 4;
      break;
    case MC_BF16_GEMM:
      prec = BK_BF16;
      pack_blocks<uint16_t>(d, nd, Ls, [](double v) { return to_bf16_rne((float)v); }, &b16);
      blk_bytes = b16.size() * 2;
      break;
    case MC_FP16_GEMM:
      prec = BK_FP16;
      pack_blocks<uint16_t>(d, nd, Ls, [](double v) { return to_f16_rne((float)v); }, &b16);
      blk_bytes = b16.size() * 2;
      break;
    default:
      prec = BK_BF16X2;
      pack_blocks<uint16_t>(d, nd, Ls, [](double v) { return to_bf16_rne((float)v); }, &b16);
      pack_blocks<uint16_t>(d, nd, Ls, [](double v) {
        const float hi = from_bf16(to_bf16_rne((float)v));
        return to_bf16_rne((float)(v - (double)hi));
      }, &b16lo);
      blk_bytes = b16.size() * 2;
      break;
  }
  // Per-asset constants: n mu_a in log2 units, w_a S0_a, w_a ln 2, S0_a.
  std::vector<float> asset(4 * 256, 0.f);
  double geo0 = 0.0;
  for (uint32_t a = 0; a < d; ++a) {
    const double w = f->weights ? f->weights[a] : 1.0 / d;
    const double drift = (port && port->mu) ? port->mu[a] : m->r;
    const double mu = (drift - 0.5 * m->sigma[a] * m->sigma[a]) * dt * inv_ln2;
    asset[a] = (float)(n_steps * mu);
    asset[256 + a] = (float)(w * m->S0[a]);
    asset[512 + a] = (float)(w * std::log(2.0));
    asset[768 + a] = (float)m->S0[a];
    geo0 += w * std::log(m->S0[a]);
  }
  const RunLayout Lay = layout_for(n_paths, 3, o0.path_values != nullptr);
  const size_t off_blk = align256(Lay.bytes);
  const size_t off_lo = off_blk + align256(blk_bytes);
  const size_t off_asset = off_lo + (prec == BK_BF16X2 ? align256(blk_bytes) : 0);
  const size_t total = off_asset + align256(asset.size() * 4);
  if (total != basket_ws_bytes(Lay.bytes, d, o0.prec))
    return fail(ctx, MC_ERR_DEVICE, "basket workspace layout mismatch");
  char* base = nullptr;
  st = get_ws(ctx, o0, total, &base);
  if (st != MC_OK) return st;
  hipStream_t s = stream_of(ctx, o0);
  const void* hb = prec == BK_FP32 ? (const void*)bf32.data() : (const void*)b16.data();
  HIP_TRY(ctx, hipMemcpyAsync(base + off_blk, hb, blk_bytes, hipMemcpyHostToDevice, s));
  if (prec == BK_BF16X2)
    HIP_TRY(ctx, hipMemcpyAsync(base + off_lo, b16lo.data(), blk_bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, hipMemcpyAsync(base + off_asset, asset.data(), asset.size() * 4,
                              hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));   // host vectors go out of scope
  mc_options o = o0;
  o.workspace = base;
  o.workspace_bytes = Lay.bytes;
  BasketParams p{};
  p.n_paths = n_paths;
  p.path_offset = o0.path_offset;
  p.n_steps = n_steps;
  p.tag = o0.stream_tag;
  p.k0 = (uint32_t)seed;
  p.k1 = (uint32_t)(seed >> 32);
  p.d = d;
  p.Lblk = base + off_blk;
  p.Lblk_lo = prec == BK_BF16X2 ? base + off_lo : nullptr;
  p.asset = (const float*)(base + off_asset);
  p.disc = std::exp(-m->r * m->T);
  p.K = f->K;
  p.geo0 = geo0;
  p.w0 = f->weights ? f->weights[0] : 1.0 / d;
  p.n_strikes = port ? port->n_strikes : 0u;
  for (uint32_t k = 0; k < p.n_strikes; ++k) {
    p.pm[k] = (float)port->strike_mult[k];
    p.pq[k] = (float)port->quantity[k];
  }
  p.premium = premium;
  p.qV = qmc ? qmc->V : nullptr;
  p.qshift = qmc ? qmc->shift : nullptr;
  *p_out = p;
  *prec_out = prec;
  *o_run = o;
  return MC_OK;
}

mc_status basket_price(mc_context* ctx, const mc_model* m, const mc_payoff* f, uint64_t n_paths,
                       uint32_t n_steps, uint64_t seed, const mc_options& o0, mc_result* out,
                       const mc_portfolio* port = nullptr, double premium = 0.0,
                       BasketQmc* qmc = nullptr) {
  BasketParams p{};
  int prec = BK_FP32;
  mc_options o;
  mc_status st = basket_setup(ctx, m, f, n_paths, n_steps, seed, o0, port, premium, qmc, &p, &prec,
                              &o);
  if (st != MC_OK) return st;
  Moments mom;
  double kms = 0.0;
  st = run_moments(ctx, o, n_paths, port ? 1 : 3, o0.path_values,
                   [&](double* partials, double* path_out, hipStream_t ss, uint32_t* nb) {
                     p.partials = partials;
                     p.path_out = path_out;
                     return launch_basket(p, prec, ss, nb);
                   },
                   &mom, &kms);
  if (st != MC_OK) return st;
  mc_result r{};
  double v;
  fill_channel(mom, 0, &r.price, &r.variance, &r.std_err);
  r.plain_price = r.price;
  r.plain_std_err = r.std_err;
  if (!port && (o0.greeks & MC_GREEK_DELTA)) fill_channel(mom, 2, &r.delta, &v, &r.delta_se);
  if (qmc) qmc->geo_mean = mom.mean(1);
  r.vrf = 1.0;
  r.n_paths = (uint64_t)mom.n;
  r.n_nonfinite = (uint64_t)mom.nonfinite;
  r.kernel_ms = kms;
  *out = r;
  return MC_OK;
}

// ---- multilevel helpers ----

// Per-path channel count of a plain run of (m, f, o) and the payoff's
// channel in it (coarsen: GBM coupling factor of the run).
mc_status payoff_channel(mc_context* ctx, const mc_model* m, const mc_payoff* f,
                         const mc_options& o, uint32_t coarsen, uint32_t* C, uint32_t* ch) {
  if (m->kind == MC_GBM) {
    mc_status st = MC_OK;
    const uint32_t want = gbm_want_mask(f, o, &st);
    if (st != MC_OK) return fail(ctx, st, "payoff not offered for GBM");
    const uint32_t mask =
        gbm_pick_mask(want, o.prec == MC_FP64, m->scheme == MC_LOG_EULER, coarsen);
    if (!mask) return fail(ctx, MC_ERR_UNSUPPORTED, "payoff not available for this coupling");
    uint32_t bit = 0;
    switch (f->kind) {
      case MC_EURO_CALL: bit = G_EURO; break;
      case MC_ASIAN_ARITH_CALL: bit = G_ASIAN; break;
      case MC_ASIAN_GEO_CALL: bit = G_GEO; break;
      case MC_UO_BARRIER_CALL: bit = G_UO; break;
      case MC_UO_BRIDGE_CALL: bit = G_UOBB; break;
      default: return fail(ctx, MC_ERR_UNSUPPORTED, "payoff not offered for GBM");
    }
    const int c = gbm_channel_index(mask, bit);
    if (c < 0) return fail(ctx, MC_ERR_DEVICE, "channel layout mismatch");
    *C = (uint32_t)gbm_channels(mask);
    *ch = (uint32_t)c;
    return MC_OK;
  }
  if (m->kind == MC_HESTON) {
    *C = 2;
    *ch = f->kind == MC_EURO_CALL ? 0u : 1u;
    return MC_OK;
  }
  *C = 3;
  *ch = 0;
  return MC_OK;
}

// Restores the context's plain-run state however a level ends.
struct SinkGuard {
  mc_context* ctx;
  ~SinkGuard() {
    ctx->sink = nullptr;
    ctx->coarsen = 1;
  }
};

// Per-path values of paired runs (multilevel corrections, finite
// differences) are kept on the device in chunks of at most this many paths.
constexpr uint64_t kMlmcChunk = 1ull << 20;

mc_status get_mlmc_buf(mc_context* ctx, size_t bytes, char** base) {
  if (ctx->mlmc_bytes < bytes) {
    if (ctx->mlmc_buf) {
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      HIP_TRY(ctx, hipFree(ctx->mlmc_buf));
      ctx->mlmc_buf = nullptr;
      ctx->mlmc_bytes = 0;
    }
    HIP_TRY(ctx, hipMalloc(&ctx->mlmc_buf, bytes));
    ctx->mlmc_bytes = bytes;
  }
  *base = (char*)ctx->mlmc_buf;
  return MC_OK;
}

mc_status get_lsm_buf(mc_context* ctx, size_t bytes, char** base) {
  if (ctx->lsm_bytes < bytes) {
    if (ctx->lsm_buf) {
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
      HIP_TRY(ctx, hipFree(ctx->lsm_buf));
      ctx->lsm_buf = nullptr;
      ctx->lsm_bytes = 0;
    }
    HIP_TRY(ctx, hipMalloc(&ctx->lsm_buf, bytes));
    ctx->lsm_bytes = bytes;
  }
  *base = (char*)ctx->lsm_buf;
  return MC_OK;
}

mc_status mc_price_impl(mc_context* ctx, const mc_model* m, const mc_payoff* f, uint64_t n_paths,
                        uint32_t n_steps, uint64_t seed, const mc_options& o, mc_result* out);

// Central finite difference on common random numbers (Sec. I-A.3 greeks by
// bumping): the payoff of the models with the parameter theta scaled by
// 1 + h and 1 - h, priced on the same paths (same seed, tag and path
// indices) into device sinks in chunks of at most 2^20 paths; the greek is
// the mean of the per-path differences over 2 h theta, reduced in FP64.
mc_status fd_greek(mc_context* ctx, const mc_model* m, const mc_payoff* f, uint64_t n_paths,
                   uint32_t n_steps, uint64_t seed, const mc_options& o, uint32_t which,
                   double* g, double* se, double* kms) {
  const double h = o.fd_rel_step;
  const uint32_t d = m->dim;
  std::vector<double> s0u(m->S0, m->S0 + d), s0d = s0u, sgu, sgd;
  mc_model mu = *m, md = *m;
  double theta;
  if (which == MC_GREEK_DELTA) {
    theta = m->S0[0];
    s0u[0] = theta * (1.0 + h);
    s0d[0] = theta * (1.0 - h);
    mu.S0 = s0u.data();
    md.S0 = s0d.data();
  } else if (m->kind == MC_HESTON) {
    theta = m->v0;
    mu.v0 = theta * (1.0 + h);
    md.v0 = theta * (1.0 - h);
  } else {
    sgu.assign(m->sigma, m->sigma + d);
    sgd = sgu;
    theta = m->sigma[0];
    sgu[0] = theta * (1.0 + h);
    sgd[0] = theta * (1.0 - h);
    mu.sigma = sgu.data();
    md.sigma = sgd.data();
  }
  mc_payoff fp = *f;
  fp.cv = MC_CV_NONE;
  mc_options ob = o;
  ob.greeks = 0;
  ob.greeks_method = MC_GREEKS_PATHWISE;
  ob.path_values = nullptr;
  ob.cv_beta = std::nan("");
  // A relative bump h leaves about -log10(h) fewer significant digits in the
  // difference: FP32 paths (about 1e-7 relative error per path) would carry
  // errors of order 1e-7 / h into the greek, systematic ones included, so the
  // bumped pairs run in FP64. The basket has no FP64 path; its only bump
  // (S0 of asset 0) scales the terminal values and loses nothing.
  if (m->kind != MC_GBM_BASKET) ob.prec = MC_FP64;
  uint32_t C = 0, ch = 0;
  mc_status st = payoff_channel(ctx, m, &fp, ob, 1, &C, &ch);
  if (st != MC_OK) return st;
  hipStream_t s = stream_of(ctx, o);
  const uint64_t n_chunks = (n_paths + kMlmcChunk - 1) / kMlmcChunk;
  const uint64_t chunk = (n_paths + n_chunks - 1) / n_chunks;
  const size_t bytes_a = align256((size_t)chunk * C * sizeof(double));
  const uint32_t M = (uint32_t)n_moments(3);
  const size_t bytes_p = align256((size_t)kDiffMaxBlocks * M * sizeof(double));
  char* base = nullptr;
  st = get_mlmc_buf(ctx, 2 * bytes_a + bytes_p + align256(M * sizeof(double)), &base);
  if (st != MC_OK) return st;
  st = get_pinned(ctx, M);
  if (st != MC_OK) return st;
  double* A = (double*)base;
  double* B = (double*)(base + bytes_a);
  double* partials = (double*)(base + 2 * bytes_a);
  double* mom = (double*)(base + 2 * bytes_a + bytes_p);
  double acc[n_moments(3)] = {};
  for (uint64_t p0 = 0; p0 < n_paths; p0 += chunk) {
    const uint64_t nc = n_paths - p0 < chunk ? n_paths - p0 : chunk;
    mc_options oc = ob;
    oc.path_offset = o.path_offset + p0;
    mc_result tmp{};
    {
      SinkGuard guard{ctx};
      ctx->sink = A;
      st = mc_price_impl(ctx, &mu, &fp, nc, n_steps, seed, oc, &tmp);
      if (st != MC_OK) return st;
      *kms += tmp.kernel_ms;
      ctx->sink = B;
      st = mc_price_impl(ctx, &md, &fp, nc, n_steps, seed, oc, &tmp);
      if (st != MC_OK) return st;
      *kms += tmp.kernel_ms;
    }
    uint32_t nb = 0;
    HIP_TRY(ctx, launch_diff_moments(A, C, ch, B, C, ch, nc, partials, s, &nb));
    HIP_TRY(ctx, launch_final_merge(partials, nb, 3, 1, mom, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, mom, M * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    merge_moment_vec(acc, ctx->pinned, 3);
  }
  // acc: [n, nonfinite, mean d, mean a, mean b, M_dd, ...]
  const double n = acc[0];
  if (n < 2) return fail(ctx, MC_ERR_DEVICE, "fewer than two finite paths in a bumped run");
  const double var = acc[5] / (n - 1.0);
  *g = acc[2] / (2.0 * h * theta);
  *se = std::sqrt(var / n) / (2.0 * h * theta);
  return MC_OK;
}

// One pricing run of mc_price with the arguments already checked.
mc_status mc_price_impl(mc_context* ctx, const mc_model* m, const mc_payoff* f, uint64_t n_paths,
                        uint32_t n_steps, uint64_t seed, const mc_options& o, mc_result* out) {
  mc_status st = MC_OK;
  if (m->kind == MC_GBM) {
    const uint32_t want = gbm_want_mask(f, o, &st);
    Moments mom;
    uint32_t mask = 0;
    double kms = 0.0;
    st = gbm_run(ctx, m, f, n_paths, n_steps, seed, o, want, o.stream_tag, o.path_values, &mom,
                 &mask, &kms);
    if (st != MC_OK) return st;
    return gbm_result(ctx, m, f, n_steps, seed, o, mask, mom, kms, n_paths, out);
  }
  if (m->kind == MC_GBM_BASKET) return basket_price(ctx, m, f, n_paths, n_steps, seed, o, out);
  return heston_price(ctx, m, f, n_paths, n_steps, seed, o, out);
}

// Mean and standard error from (n, sum, sum of squares).
void moments_mean_se(double n, double s1, double s2, double* mean, double* se) {
  *mean = s1 / n;
  const double v = n > 1 ? std::max(s2 - s1 * s1 / n, 0.0) / (n - 1) : NAN;
  *se = std::sqrt(v / n);
}


}  // namespace

// ================================================================ C ABI ===
extern "C" {

void mc_options_default(mc_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->prec = MC_FP32;
  o->cv_hedge_every = 1;
  o->cv_beta = std::nan("");
  o->greeks_method = MC_GREEKS_PATHWISE;
  o->fd_rel_step = 1e-3;
}

mc_status mc_create(mc_context** out, int device) {
  if (!out) return MC_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return MC_ERR_NO_DEVICE;
  if (device < 0 || device >= n) return MC_ERR_NO_DEVICE;
  mc_context* ctx = new mc_context();
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess || hipStreamCreate(&ctx->stream) != hipSuccess ||
      hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess ||
      hipEventCreate(&ctx->ev2) != hipSuccess || hipEventCreate(&ctx->ev3) != hipSuccess ||
      scratch_address(device, &ctx->scratch) != hipSuccess) {
    mc_destroy(ctx);
    return MC_ERR_DEVICE;
  }
  *out = ctx;
  return MC_OK;
}

mc_status mc_destroy(mc_context* ctx) {
  if (!ctx) return MC_OK;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->mlmc_buf) (void)hipFree(ctx->mlmc_buf);
  if (ctx->qmc_buf) (void)hipFree(ctx->qmc_buf);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->ev2) (void)hipEventDestroy(ctx->ev2);
  if (ctx->ev3) (void)hipEventDestroy(ctx->ev3);
  if (ctx->lsm_buf) (void)hipFree(ctx->lsm_buf);
  for (hipEvent_t e : ctx->lsm_ev) (void)hipEventDestroy(e);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return MC_OK;
}

const char* mc_status_str(mc_status st) {
  switch (st) {
    case MC_OK: return "MC_OK";
    case MC_ERR_INVALID_ARG: return "MC_ERR_INVALID_ARG";
    case MC_ERR_NOT_PD: return "MC_ERR_NOT_PD";
    case MC_ERR_NO_DEVICE: return "MC_ERR_NO_DEVICE";
    case MC_ERR_OOM: return "MC_ERR_OOM";
    case MC_ERR_DEVICE: return "MC_ERR_DEVICE";
    case MC_ERR_UNSUPPORTED: return "MC_ERR_UNSUPPORTED";
    case MC_ERR_WORKSPACE: return "MC_ERR_WORKSPACE";
  }
  return "unknown mc_status";
}

const char* mc_last_error(const mc_context* ctx) { return ctx ? ctx->err.c_str() : ""; }

uint32_t mc_path_channels(const mc_model* m, const mc_payoff* f, const mc_options* opts) {
  if (!m || !f) return 0;
  const mc_options o = opts ? *opts : defaults();
  if (m->kind == MC_GBM) {
    mc_status st;
    const uint32_t want = gbm_want_mask(f, o, &st);
    if (st != MC_OK) return 0;
    const uint32_t mask = gbm_pick_mask(want, o.prec == MC_FP64, m->scheme == MC_LOG_EULER);
    return mask ? (uint32_t)gbm_channels(mask) : 0;
  }
  if (m->kind == MC_HESTON) return (o.greeks || f->cv == MC_CV_LEARNED) ? 3u : 2u;
  if (m->kind == MC_GBM_BASKET) return 3u;
  return 0;
}

const char* mc_path_channel_name(const mc_model* m, const mc_payoff* f, const mc_options* opts,
                                 uint32_t i) {
  if (!m || !f) return nullptr;
  const mc_options o = opts ? *opts : defaults();
  if (m->kind == MC_GBM) {
    mc_status st;
    const uint32_t want = gbm_want_mask(f, o, &st);
    if (st != MC_OK) return nullptr;
    const uint32_t mask = gbm_pick_mask(want, o.prec == MC_FP64, m->scheme == MC_LOG_EULER);
    return mask ? gbm_channel_name(mask, i) : nullptr;
  }
  if (m->kind == MC_HESTON) {
    const bool asian = f->kind == MC_ASIAN_ARITH_CALL;
    if (f->cv == MC_CV_LEARNED) {
      static const char* c[] = {"asian", "hedge_pnl", "asian_minus_hedge"};
      return i < 3 ? c[i] : nullptr;
    }
    if (o.greeks) {
      static const char* e[] = {"euro", "euro_delta", "euro_dv0"};
      static const char* a[] = {"asian", "asian_delta", "asian_dv0"};
      return i < 3 ? (asian ? a[i] : e[i]) : nullptr;
    }
    static const char* n[] = {"euro", "asian"};
    return i < 2 ? n[i] : nullptr;
  }
  if (m->kind == MC_GBM_BASKET) {
    static const char* b[] = {"basket", "geo_basket", "basket_delta0"};
    return i < 3 ? b[i] : nullptr;
  }
  return nullptr;
}

size_t mc_workspace_bytes(const mc_model* m, const mc_payoff* f, uint64_t n_paths,
                          uint32_t n_steps, const mc_options* opts) {
  (void)n_steps;
  if (!m || !f || n_paths < 2) return 0;
  const mc_options o = opts ? *opts : defaults();
  const uint32_t C = mc_path_channels(m, f, &o);
  if (C == 0) return 0;
  // Persistent grids: GBM, and the Heston price and tangent kernels (the
  // adjoint and the learned CV take one path per thread).
  const bool heston_persistent = m->kind == MC_HESTON && f->cv != MC_CV_LEARNED &&
                                 !(o.greeks && o.greeks_method != MC_GREEKS_TANGENT);
  const uint32_t cap = m->kind == MC_GBM ? kGbmMaxBlocks
                       : heston_persistent ? kHestonMaxBlocks
                                           : UINT32_MAX;
  size_t bytes = layout_for(n_paths, (int)C, o.path_values != nullptr, kBlock, cap).bytes;
  if (m->kind == MC_HESTON && o.greeks && o.greeks_method == MC_GREEKS_PATHWISE &&
      (n_steps + mcp::kCkpt - 1) / mcp::kCkpt > (uint32_t)mcp::kLdsCkpt)
    bytes = align256(bytes) + align256(mc_adjoint_ckpt_bytes(n_paths, n_steps, mcp::kCkpt));
  if (m->kind == MC_HESTON && f->cv == MC_CV_LEARNED) {
    const uint64_t n_pilot = std::isfinite(o.cv_beta) || o.pilot_paths == MC_PILOT_IN_SAMPLE ? 0
                             : o.pilot_paths ? o.pilot_paths
                                             : (1ull << 16);
    const uint64_t n_big = n_paths > n_pilot ? n_paths : n_pilot;
    bytes = align256(layout_for(n_big, 3, o.path_values != nullptr, kCvPathsPerBlock).bytes) +
            cv_extra_bytes(n_steps);
  }
  if (m->kind == MC_GBM_BASKET) bytes = basket_ws_bytes(bytes, m->dim, o.prec);
  return bytes;
}

mc_status mc_validate(mc_context* ctx, const mc_model* m, const mc_payoff* f, uint64_t n_paths,
                      uint32_t n_steps, const mc_options* opts) {
  const mc_options o = opts ? *opts : defaults();
  return validate_all(ctx, m, f, n_paths, n_steps, o);
}

mc_status mc_price(mc_context* ctx, const mc_model* m, const mc_payoff* f, uint64_t n_paths,
                   uint32_t n_steps, uint64_t seed, const mc_options* opts, mc_result* out) {
  if (!ctx) return MC_ERR_INVALID_ARG;
  const mc_options o = opts ? *opts : defaults();
  mc_status st = validate_all(ctx, m, f, n_paths, n_steps, o);
  if (st != MC_OK) return st;
  if (!out) return fail(ctx, MC_ERR_INVALID_ARG, "out must not be NULL");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, MC_ERR_DEVICE, "hipSetDevice");
  if (o.greeks == 0 || o.greeks_method != MC_GREEKS_FD_CRN) {
    st = mc_price_impl(ctx, m, f, n_paths, n_steps, seed, o, out);
    if (st == MC_OK && o.greeks) out->greeks_method = (int)o.greeks_method;
    return st;
  }
  // Finite differences on common random numbers: the price run, then one
  // pair of bumped runs per requested greek.
  mc_options ob = o;
  ob.greeks = 0;
  ob.greeks_method = MC_GREEKS_PATHWISE;
  mc_result r{};
  st = mc_price_impl(ctx, m, f, n_paths, n_steps, seed, ob, &r);
  if (st != MC_OK) return st;
  double kms = r.kernel_ms;
  if (o.greeks & MC_GREEK_DELTA) {
    st = fd_greek(ctx, m, f, n_paths, n_steps, seed, o, MC_GREEK_DELTA, &r.delta, &r.delta_se,
                  &kms);
    if (st != MC_OK) return st;
  }
  if (o.greeks & MC_GREEK_VEGA) {
    st = fd_greek(ctx, m, f, n_paths, n_steps, seed, o, MC_GREEK_VEGA, &r.vega, &r.vega_se, &kms);
    if (st != MC_OK) return st;
  }
  r.kernel_ms = kms;
  r.greeks_method = MC_GREEKS_FD_CRN;
  *out = r;
  return MC_OK;
}

size_t mc_noalloc_scratch_bytes(void) { return MC_NOALLOC_SCRATCH_BYTES; }

mc_status mc_price_noalloc(mc_context* ctx, const mc_model* m, const mc_payoff* f,
                           uint64_t n_paths, uint32_t n_steps, uint64_t seed,
                           const mc_options* opts, mc_result* out) {
  if (!ctx) return MC_ERR_INVALID_ARG;
  const mc_options o = opts ? *opts : defaults();
  mc_status st = validate_all(ctx, m, f, n_paths, n_steps, o);
  if (st != MC_OK) return st;
  if (!out) return fail(ctx, MC_ERR_INVALID_ARG, "out must not be NULL");
  if (m->kind != MC_GBM && m->kind != MC_HESTON)
    return fail(ctx, MC_ERR_UNSUPPORTED, "mc_price_noalloc prices MC_GBM and MC_HESTON");
  if (f->cv == MC_CV_LEARNED)
    return fail(ctx, MC_ERR_UNSUPPORTED, "mc_price_noalloc has no learned control variate");
  if (o.path_values)
    return fail(ctx, MC_ERR_UNSUPPORTED, "mc_price_noalloc writes no per-path values");
  if (o.greeks && o.greeks_method == MC_GREEKS_FD_CRN)
    return fail(ctx, MC_ERR_UNSUPPORTED, "mc_price_noalloc offers pathwise greeks only");
  if (m->kind == MC_HESTON && o.greeks && o.greeks_method != MC_GREEKS_TANGENT &&
      (n_steps + mcp::kCkpt - 1) / mcp::kCkpt > (uint32_t)mcp::kLdsCkpt)
    return fail(ctx, MC_ERR_UNSUPPORTED,
                "mc_price_noalloc: the Heston adjoint keeps more than %d checkpoints in device "
                "memory above %d steps; use MC_GREEKS_TANGENT", mcp::kLdsCkpt,
                mcp::kLdsCkpt * mcp::kCkpt);
  if (!ctx->scratch)
    return fail(ctx, MC_ERR_UNSUPPORTED, "no static scratch on device %d", ctx->device);
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, MC_ERR_DEVICE, "hipSetDevice");
  struct NoallocGuard {
    mc_context* c;
    ~NoallocGuard() { c->noalloc = false; }
  } guard{ctx};
  ctx->noalloc = true;
  st = mc_price_impl(ctx, m, f, n_paths, n_steps, seed, o, out);
  if (st == MC_OK && o.greeks) out->greeks_method = (int)o.greeks_method;
  return st;
}

mc_status mc_price_multi(mc_context* ctx, const mc_model* m, const mc_payoff* fs, uint32_t nf,
                         uint64_t n_paths, uint32_t n_steps, uint64_t seed, const mc_options* opts,
                         mc_result* results) {
  if (!ctx) return MC_ERR_INVALID_ARG;
  if (!fs || nf == 0 || !results) return fail(ctx, MC_ERR_INVALID_ARG, "no payoffs");
  mc_status st = validate_common(ctx, m, &fs[0], n_paths, n_steps);
  if (st != MC_OK) return st;
  const mc_options o = opts ? *opts : defaults();
  if (m->kind != MC_GBM) return fail(ctx, MC_ERR_UNSUPPORTED, "mc_price_multi is GBM-only");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, MC_ERR_DEVICE, "hipSetDevice");
  uint32_t want = 0;
  for (uint32_t i = 0; i < nf; ++i) {
    st = validate_gbm(ctx, m, &fs[i], o);
    if (st != MC_OK) return st;
    if (fs[i].cv == MC_CV_LEARNED) return fail(ctx, MC_ERR_UNSUPPORTED, "learned CV is Heston-only");
    want |= gbm_want_mask(&fs[i], o, &st);
    if (st != MC_OK) return fail(ctx, st, "pathwise greeks need a continuous payoff");
  }
  // Barrier levels must agree: one kernel monitors one barrier.
  double B = NAN;
  for (uint32_t i = 0; i < nf; ++i) {
    if (fs[i].kind != MC_UO_BARRIER_CALL && fs[i].kind != MC_UO_BRIDGE_CALL) continue;
    if (std::isnan(B)) B = fs[i].B;
    else if (B != fs[i].B) return fail(ctx, MC_ERR_UNSUPPORTED, "one barrier level per call");
  }
  double Ks = fs[0].K;
  for (uint32_t i = 1; i < nf; ++i)
    if (fs[i].K != Ks) return fail(ctx, MC_ERR_UNSUPPORTED, "one strike per call");
  mc_payoff merged = fs[0];
  merged.B = std::isnan(B) ? fs[0].B : B;
  Moments mom;
  uint32_t mask = 0;
  double kms = 0.0;
  st = gbm_run(ctx, m, &merged, n_paths, n_steps, seed, o, want, o.stream_tag, o.path_values,
               &mom, &mask, &kms);
  if (st != MC_OK) return st;
  std::vector<mc_result> tmp(nf);
  for (uint32_t i = 0; i < nf; ++i) {
    st = gbm_result(ctx, m, &fs[i], n_steps, seed, o, mask, mom, kms, n_paths, &tmp[i]);
    if (st != MC_OK) return st;
  }
  for (uint32_t i = 0; i < nf; ++i) results[i] = tmp[i];
  return MC_OK;
}

// ---------------------------------------------------------- Multilevel ----
mc_status mc_price_mlmc(mc_context* ctx, const mc_model* m, const mc_payoff* f, uint32_t n_levels,
                        const mc_level* levels, uint64_t seed, const mc_options* opts,
                        mc_mlmc_result* out) {
  if (!ctx) return MC_ERR_INVALID_ARG;
  if (!m || !f || !levels || !out) return fail(ctx, MC_ERR_INVALID_ARG, "NULL argument");
  if (n_levels < 1 || n_levels > MC_MLMC_MAX_LEVELS)
    return fail(ctx, MC_ERR_INVALID_ARG, "n_levels must be in 1..%d", MC_MLMC_MAX_LEVELS);
  const mc_options o0 = opts ? *opts : defaults();
  if (f->cv != MC_CV_NONE)
    return fail(ctx, MC_ERR_UNSUPPORTED, "multilevel estimates take payoffs without a control variate");
  if (o0.greeks) return fail(ctx, MC_ERR_UNSUPPORTED, "multilevel estimates carry no greeks");
  if (o0.path_values) return fail(ctx, MC_ERR_UNSUPPORTED, "multilevel estimates return no path values");
  mc_coupling cpl[MC_MLMC_MAX_LEVELS] = {};
  uint32_t cfac[MC_MLMC_MAX_LEVELS] = {};
  for (uint32_t l = 0; l < n_levels; ++l) {
    const mc_level& lv = levels[l];
    if (lv.n_paths < 2 || lv.n_steps == 0)
      return fail(ctx, MC_ERR_INVALID_ARG, "level %u: n_paths >= 2 and n_steps >= 1", l);
    mc_options ol = o0;
    ol.prec = lv.prec;
    mc_status st = validate_all(ctx, m, f, lv.n_paths, lv.n_steps, ol);
    if (st != MC_OK) return st;
    if (l == 0) continue;
    const mc_level& pv = levels[l - 1];
    if (lv.n_steps == pv.n_steps && lv.prec != pv.prec) {
      cpl[l] = MC_COUPLE_PRECISION;
      cfac[l] = 1;
    } else if (lv.prec == pv.prec && (lv.n_steps == 2 * pv.n_steps || lv.n_steps == 4 * pv.n_steps)) {
      if (m->kind != MC_GBM)
        return fail(ctx, MC_ERR_UNSUPPORTED, "time-step coupling is offered for 1-D GBM");
      if (f->kind == MC_UO_BRIDGE_CALL)
        return fail(ctx, MC_ERR_UNSUPPORTED, "time-step coupling of the bridge barrier");
      cpl[l] = MC_COUPLE_TIME;
      cfac[l] = lv.n_steps / pv.n_steps;
    } else {
      return fail(ctx, MC_ERR_UNSUPPORTED,
                  "levels %u and %u: need equal steps with different precision, or equal "
                  "precision with 2x / 4x the steps", l - 1, l);
    }
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, MC_ERR_DEVICE, "hipSetDevice");
  hipStream_t s = stream_of(ctx, o0);
  mc_mlmc_result r{};
  r.n_levels = n_levels;
  double var_over_n = 0.0;
  for (uint32_t l = 0; l < n_levels; ++l) {
    const mc_level& lv = levels[l];
    mc_options ol = o0;
    ol.prec = lv.prec;
    ol.stream_tag = o0.stream_tag + 16u * l;
    r.coupling[l] = cpl[l];
    if (l == 0) {
      mc_result pr{};
      mc_status st = mc_price(ctx, m, f, lv.n_paths, lv.n_steps, seed, &ol, &pr);
      if (st != MC_OK) return st;
      r.mean[0] = r.fine_mean[0] = pr.price;
      r.variance[0] = pr.variance;
      r.n_paths[0] = pr.n_paths;
      r.kernel_ms[0] = pr.kernel_ms;
      var_over_n += pr.variance / (double)pr.n_paths;
      continue;
    }
    // Correction level: fine = this level, coarse = previous level's
    // configuration, on the same paths of this level's stream.
    const mc_level& pv = levels[l - 1];
    mc_options oc = ol;
    oc.prec = pv.prec;
    uint32_t Ca = 0, ca = 0, Cb = 0, cb = 0;
    mc_status st = payoff_channel(ctx, m, f, ol, 1, &Ca, &ca);
    if (st != MC_OK) return st;
    st = payoff_channel(ctx, m, f, oc, cfac[l], &Cb, &cb);
    if (st != MC_OK) return st;
    const uint64_t n_chunks = (lv.n_paths + kMlmcChunk - 1) / kMlmcChunk;
    const uint64_t chunk = (lv.n_paths + n_chunks - 1) / n_chunks;
    const size_t bytes_a = align256((size_t)chunk * Ca * sizeof(double));
    const size_t bytes_b = align256((size_t)chunk * Cb * sizeof(double));
    const uint32_t M = (uint32_t)n_moments(3);
    const size_t bytes_p = align256((size_t)kDiffMaxBlocks * M * sizeof(double));
    char* base = nullptr;
    st = get_mlmc_buf(ctx, bytes_a + bytes_b + bytes_p + align256(M * sizeof(double)), &base);
    if (st != MC_OK) return st;
    st = get_pinned(ctx, M);
    if (st != MC_OK) return st;
    double* A = (double*)base;
    double* B = (double*)(base + bytes_a);
    double* partials = (double*)(base + bytes_a + bytes_b);
    double* mom = (double*)(base + bytes_a + bytes_b + bytes_p);
    double acc[n_moments(3)] = {};
    double kms = 0.0;
    for (uint64_t p0 = 0; p0 < lv.n_paths; p0 += chunk) {
      const uint64_t nc = lv.n_paths - p0 < chunk ? lv.n_paths - p0 : chunk;
      mc_result tmp{};
      {
        SinkGuard guard{ctx};
        mc_options of = ol;
        of.path_offset = o0.path_offset + p0;
        ctx->sink = A;
        ctx->coarsen = 1;
        st = mc_price(ctx, m, f, nc, lv.n_steps, seed, &of, &tmp);
        if (st != MC_OK) return st;
        kms += tmp.kernel_ms;
        mc_options ocp = oc;
        ocp.path_offset = o0.path_offset + p0;
        ctx->sink = B;
        ctx->coarsen = cfac[l];
        st = mc_price(ctx, m, f, nc, pv.n_steps, seed, &ocp, &tmp);
        if (st != MC_OK) return st;
        kms += tmp.kernel_ms;
      }
      uint32_t nb = 0;
      HIP_TRY(ctx, hipEventRecord(ctx->ev0, s));
      HIP_TRY(ctx, launch_diff_moments(A, Ca, ca, B, Cb, cb, nc, partials, s, &nb));
      HIP_TRY(ctx, launch_final_merge(partials, nb, 3, 1, mom, s));
      HIP_TRY(ctx, hipEventRecord(ctx->ev1, s));
      HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, mom, M * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(ctx, hipStreamSynchronize(s));
      float ms = 0.f;
      HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
      kms += ms;
      merge_moment_vec(acc, ctx->pinned, 3);
    }
    // acc: [n, nonfinite, mean d, mean a, mean b, M_dd, M_da, M_db, M_aa, M_ab, M_bb]
    const double n = acc[0];
    if (n < 2) return fail(ctx, MC_ERR_DEVICE, "level %u: fewer than two finite paths", l);
    r.mean[l] = acc[2];
    r.variance[l] = acc[5] / (n - 1.0);
    r.fine_mean[l] = acc[3];
    r.coarse_mean[l] = acc[4];
    r.n_paths[l] = (uint64_t)n;
    r.kernel_ms[l] = kms;
    var_over_n += r.variance[l] / n;
  }
  for (uint32_t l = 0; l < n_levels; ++l) r.price += r.mean[l];
  r.std_err = std::sqrt(var_over_n);
  *out = r;
  return MC_OK;
}

mc_status mc_mlmc_allocate(uint32_t n_levels, const double* var, const double* cost,
                           double target_se, uint64_t* n_paths_out) {
  if (n_levels < 1 || n_levels > MC_MLMC_MAX_LEVELS || !var || !cost || !n_paths_out)
    return MC_ERR_INVALID_ARG;
  if (!(target_se > 0.0) || !std::isfinite(target_se)) return MC_ERR_INVALID_ARG;
  double sum = 0.0;
  for (uint32_t l = 0; l < n_levels; ++l) {
    if (!(var[l] >= 0.0) || !std::isfinite(var[l]) || !(cost[l] > 0.0) || !std::isfinite(cost[l]))
      return MC_ERR_INVALID_ARG;
    sum += std::sqrt(var[l] * cost[l]);
  }
  uint64_t tmp[MC_MLMC_MAX_LEVELS];
  for (uint32_t l = 0; l < n_levels; ++l) {
    const double n = std::ceil(sum * std::sqrt(var[l] / cost[l]) / (target_se * target_se));
    if (!(n < 0x1p62)) return MC_ERR_INVALID_ARG;
    tmp[l] = n < 2.0 ? 2u : (uint64_t)n;
  }
  for (uint32_t l = 0; l < n_levels; ++l) n_paths_out[l] = tmp[l];
  return MC_OK;
}

// ------------------------------------------- Randomised quasi-Monte Carlo ----
mc_status mc_price_qmc(mc_context* ctx, const mc_model* m, const mc_payoff* f, uint64_t n_points,
                       uint32_t n_steps, uint64_t seed, uint32_t n_replicates,
                       const mc_options* opts, mc_qmc_result* out) {
  if (!ctx) return MC_ERR_INVALID_ARG;
  if (!m || !f || !out) return fail(ctx, MC_ERR_INVALID_ARG, "NULL argument");
  const mc_options o0 = opts ? *opts : defaults();
  if (m->kind != MC_GBM_BASKET)
    return fail(ctx, MC_ERR_UNSUPPORTED, "quasi-Monte Carlo runs on the basket model");
  if (n_replicates < 1 || n_replicates > MC_QMC_MAX_REPLICATES)
    return fail(ctx, MC_ERR_INVALID_ARG, "n_replicates must be in 1..%d", MC_QMC_MAX_REPLICATES);
  if (o0.greeks) return fail(ctx, MC_ERR_UNSUPPORTED, "quasi-Monte Carlo carries no greeks");
  // BF16 products are refused: rounding L' to 8 bits biases the price by a
  // few 1e-4 relative when few assets average it out, and the QMC standard
  // error falls below that (16 assets, 16 x 2^16 points: -4 standard errors).
  // FP16 products (11 bits) stay within a small fraction of it.
  if (o0.prec == MC_BF16_GEMM)
    return fail(ctx, MC_ERR_UNSUPPORTED,
                "quasi-Monte Carlo refuses MC_BF16_GEMM (its bias exceeds the QMC standard "
                "error); use MC_FP16_GEMM or MC_FP32");
  if (o0.prec != MC_FP32 && o0.prec != MC_FP16_GEMM)
    return fail(ctx, MC_ERR_UNSUPPORTED, "quasi-Monte Carlo runs in MC_FP32 or MC_FP16_GEMM");
  if (o0.path_values && n_replicates != 1)
    return fail(ctx, MC_ERR_UNSUPPORTED, "path_values need a single replicate");
  mc_status st = validate_all(ctx, m, f, n_points, n_steps, o0);
  if (st != MC_OK) return st;
  if (o0.path_offset + n_points > (1ull << 32))
    return fail(ctx, MC_ERR_INVALID_ARG, "Sobol' point indices must stay below 2^32");
  const uint64_t dims64 = (uint64_t)n_steps * m->dim;
  if (dims64 > (1u << 16))
    return fail(ctx, MC_ERR_INVALID_ARG, "n_steps * dim above 2^16 Sobol' dimensions");
  const uint32_t dims = (uint32_t)dims64;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, MC_ERR_DEVICE, "hipSetDevice");
  hipStream_t s = stream_of(ctx, o0);
  if (ctx->qmc_dims != dims) {
    std::vector<uint32_t> V;
    if (!host::sobol_directions(dims, &V))
      return fail(ctx, MC_ERR_INVALID_ARG, "too many Sobol' dimensions");
    if (ctx->qmc_buf) {
      HIP_TRY(ctx, hipStreamSynchronize(s));
      HIP_TRY(ctx, hipFree(ctx->qmc_buf));
      ctx->qmc_buf = nullptr;
      ctx->qmc_dims = 0;
    }
    HIP_TRY(ctx, hipMalloc((void**)&ctx->qmc_buf, (size_t)dims * 33 * sizeof(uint32_t)));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->qmc_buf, V.data(), V.size() * sizeof(uint32_t),
                                hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));     // V goes out of scope
    ctx->qmc_dims = dims;
  }
  mc_qmc_result r{};
  r.n_replicates = n_replicates;
  r.n_points = n_points;
  if (o0.path_values) {
    // One replicate with per-path values: the plain basket run.
    BasketQmc q{ctx->qmc_buf, ctx->qmc_buf + (size_t)dims * 32, 0.0};
    HIP_TRY(ctx, launch_qmc_shifts((uint32_t)seed, (uint32_t)(seed >> 32), o0.stream_tag + 6u, 0,
                                   1, dims, (uint32_t*)q.shift, s));
    mc_result pr{};
    st = basket_price(ctx, m, f, n_points, n_steps, seed, o0, &pr, nullptr, 0.0, &q);
    if (st != MC_OK) return st;
    r.replicate_price[0] = pr.price;
    r.replicate_geo[0] = q.geo_mean;
    r.kernel_ms = pr.kernel_ms;
  } else {
    // All replicates in one launch each of the shift, path and reduction
    // kernels, one synchronisation at the end.
    const BasketQmc q0{ctx->qmc_buf, ctx->qmc_buf + (size_t)dims * 32, 0.0};
    BasketParams p{};
    int prec = BK_FP32;
    mc_options orun;
    st = basket_setup(ctx, m, f, n_points, n_steps, seed, o0, nullptr, 0.0, &q0, &p, &prec, &orun);
    if (st != MC_OK) return st;
    const RunLayout Lay = layout_for(n_points, 3, false);
    const size_t b_shift = align256((size_t)n_replicates * dims * sizeof(uint32_t));
    const size_t b_part = align256((size_t)n_replicates * Lay.n_mom * Lay.n_blocks * sizeof(double));
    const size_t b_mom = align256((size_t)n_replicates * Lay.n_mom * sizeof(double));
    char* base = nullptr;
    st = get_mlmc_buf(ctx, b_shift + b_part + b_mom, &base);
    if (st != MC_OK) return st;
    st = get_pinned(ctx, (size_t)n_replicates * Lay.n_mom);
    if (st != MC_OK) return st;
    uint32_t* shifts = (uint32_t*)base;
    double* parts = (double*)(base + b_shift);
    double* moms = (double*)(base + b_shift + b_part);
    HIP_TRY(ctx, hipEventRecord(ctx->ev0, s));
    HIP_TRY(ctx, launch_qmc_shifts((uint32_t)seed, (uint32_t)(seed >> 32), o0.stream_tag + 6u, 0,
                                   n_replicates, dims, shifts, s));
    p.qshift = shifts;
    p.q_dims = dims;
    p.partials = parts;
    p.path_out = nullptr;
    uint32_t nb = 0;
    HIP_TRY(ctx, launch_basket_qmc_batch(p, prec, n_replicates, s, &nb));
    if (nb == 0 || nb > Lay.n_blocks) return fail(ctx, MC_ERR_DEVICE, "block count mismatch");
    HIP_TRY(ctx, launch_final_merge(parts, nb, 3, n_replicates, moms, s));
    HIP_TRY(ctx, hipEventRecord(ctx->ev1, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, moms, (size_t)n_replicates * Lay.n_mom * 8,
                                hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    float ms = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    r.kernel_ms = ms;
    for (uint32_t rep = 0; rep < n_replicates; ++rep) {
      // Moments: [n_valid, n_nonfinite, mean basket, mean geometric, ...].
      const double* mr = ctx->pinned + (size_t)rep * Lay.n_mom;
      if (mr[0] < 2) return fail(ctx, MC_ERR_DEVICE, "replicate %u: fewer than two finite paths", rep);
      r.replicate_price[rep] = mr[2];
      r.replicate_geo[rep] = mr[3];
    }
  }
  auto mean_se = [n_replicates](const double* x, double* mean, double* se) {
    double s1 = 0.0;
    for (uint32_t i = 0; i < n_replicates; ++i) s1 += x[i];
    *mean = s1 / n_replicates;
    if (n_replicates < 2) {
      *se = NAN;
      return;
    }
    double s2 = 0.0;
    for (uint32_t i = 0; i < n_replicates; ++i) s2 += (x[i] - *mean) * (x[i] - *mean);
    *se = std::sqrt(s2 / (n_replicates - 1.0) / n_replicates);
  };
  mean_se(r.replicate_price, &r.price, &r.std_err);
  mean_se(r.replicate_geo, &r.geo_price, &r.geo_std_err);
  *out = r;
  return MC_OK;
}

// ------------------------------------------------------- Portfolio risk ----
mc_status mc_risk(mc_context* ctx, const mc_model* m, const mc_portfolio* pf, uint64_t n_paths,
                  uint32_t n_steps, uint64_t seed, const mc_options* opts, mc_risk_result* out) {
  if (!ctx) return MC_ERR_INVALID_ARG;
  if (!m || !pf || !out) return fail(ctx, MC_ERR_INVALID_ARG, "NULL argument");
  const mc_options o0 = opts ? *opts : defaults();
  if (m->kind != MC_GBM_BASKET)
    return fail(ctx, MC_ERR_UNSUPPORTED, "portfolio risk runs on the basket model");
  if (pf->n_strikes < 1 || pf->n_strikes > MC_MAX_STRIKES)
    return fail(ctx, MC_ERR_INVALID_ARG, "n_strikes must be in 1..%d", MC_MAX_STRIKES);
  for (uint32_t k = 0; k < pf->n_strikes; ++k) {
    if (!finite_nonneg(pf->strike_mult[k]))
      return fail(ctx, MC_ERR_INVALID_ARG, "strike_mult[%u] invalid", k);
    if (!std::isfinite(pf->quantity[k]))
      return fail(ctx, MC_ERR_INVALID_ARG, "quantity[%u] not finite", k);
  }
  if (!(pf->alpha > 0.0 && pf->alpha < 1.0))
    return fail(ctx, MC_ERR_INVALID_ARG, "alpha must lie in (0, 1)");
  if (o0.greeks) return fail(ctx, MC_ERR_UNSUPPORTED, "portfolio risk carries no greeks");
  if (o0.prec != MC_FP32 && o0.prec != MC_BF16_GEMM && o0.prec != MC_FP16_GEMM)
    return fail(ctx, MC_ERR_UNSUPPORTED, "portfolio risk runs in MC_FP32, MC_BF16_GEMM, MC_FP16_GEMM");
  mc_payoff f{};
  f.kind = MC_BASKET_CALL;
  f.K = 0.0;
  f.B = NAN;
  f.cv = MC_CV_NONE;
  mc_options ov = o0;
  ov.path_values = nullptr;
  mc_status st = validate_all(ctx, m, &f, n_paths, n_steps, ov);
  if (st != MC_OK) return st;
  if (pf->mu)
    for (uint32_t a = 0; a < m->dim; ++a)
      if (!std::isfinite(pf->mu[a])) return fail(ctx, MC_ERR_INVALID_ARG, "mu[%u] not finite", a);
  const double kr = std::floor((double)n_paths * (1.0 - pf->alpha)) + 1.0;
  const uint64_t k = (uint64_t)kr;
  if (k < 2 || k > n_paths)
    return fail(ctx, MC_ERR_INVALID_ARG, "n_paths (1 - alpha) must be at least 1");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, MC_ERR_DEVICE, "hipSetDevice");
  double V0 = 0.0;
  for (uint32_t a = 0; a < m->dim; ++a)
    for (uint32_t j = 0; j < pf->n_strikes; ++j)
      V0 += pf->quantity[j] *
            host::bs_call(m->S0[a], pf->strike_mult[j] * m->S0[a], m->r, m->sigma[a], m->T);
  // Device scratch: per-path P&L, selection state and histogram, tail partials.
  const size_t bytes_x = align256((size_t)n_paths * sizeof(double));
  const size_t bytes_st = align256(kSelectStateBytes);
  const size_t bytes_h = align256(256 * sizeof(uint32_t));
  const size_t bytes_p = align256((size_t)2 * 1024 * sizeof(double));
  char* base = nullptr;
  st = get_mlmc_buf(ctx, bytes_x + bytes_st + bytes_h + bytes_p + align256(2 * sizeof(double)),
                    &base);
  if (st != MC_OK) return st;
  double* x = (double*)base;
  void* state = base + bytes_x;
  uint32_t* hist = (uint32_t*)(base + bytes_x + bytes_st);
  double* partials = (double*)(base + bytes_x + bytes_st + bytes_h);
  double* tail = (double*)(base + bytes_x + bytes_st + bytes_h + bytes_p);
  mc_result pr{};
  {
    SinkGuard guard{ctx};
    ctx->sink = x;
    st = basket_price(ctx, m, &f, n_paths, n_steps, seed, ov, &pr, pf, V0);
    if (st != MC_OK) return st;
  }
  if (pr.n_nonfinite != 0) return fail(ctx, MC_ERR_DEVICE, "non-finite P&L on %llu paths",
                                       (unsigned long long)pr.n_nonfinite);
  hipStream_t s = stream_of(ctx, o0);
  st = get_pinned(ctx, 4);
  if (st != MC_OK) return st;
  uint32_t nb = 0;
  HIP_TRY(ctx, hipEventRecord(ctx->ev0, s));
  HIP_TRY(ctx, launch_select_kth(x, n_paths, k, state, hist, s));
  HIP_TRY(ctx, launch_tail_sum(x, n_paths, state, partials, s, &nb));
  HIP_TRY(ctx, launch_final_reduce(partials, nb, 2, tail, s));
  HIP_TRY(ctx, hipEventRecord(ctx->ev1, s));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned, state, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned + 1, tail, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  if (o0.path_values)
    HIP_TRY(ctx, hipMemcpyAsync(o0.path_values, x, n_paths * sizeof(double),
                                hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  float ms = 0.f;
  HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  uint64_t key;
  std::memcpy(&key, ctx->pinned, sizeof(key));
  mc_risk_result r{};
  r.quantile_pnl = select_key_to_value(key);
  r.var = -r.quantile_pnl;
  r.n_tail = (uint64_t)ctx->pinned[1];
  r.cvar = r.n_tail ? -ctx->pinned[2] / ctx->pinned[1] : NAN;
  r.pnl_mean = pr.price;
  r.pnl_std_err = pr.std_err;
  r.premium = V0;
  r.k = k;
  r.n_paths = pr.n_paths;
  r.kernel_ms = pr.kernel_ms;
  r.select_ms = ms;
  *out = r;
  return MC_OK;
}

size_t mc_adjoint_ckpt_bytes(uint64_t n_paths, uint32_t n_steps, uint32_t ckpt_every) {
  if (ckpt_every < 2 || ckpt_every > (uint32_t)mcp::kCkptMax || (ckpt_every & 1u) || n_steps == 0)
    return 0;
  const uint64_t n_ckpt = (n_steps + ckpt_every - 1) / ckpt_every;
  return (size_t)(2 * n_ckpt + 1) * n_paths * sizeof(float);
}

mc_status mc_greeks_adjoint(mc_context* ctx, const mc_model* m, const mc_payoff* f,
                            uint64_t n_paths, uint32_t n_steps, uint64_t seed,
                            const mc_options* opts, mc_adjoint_phase phase, uint32_t ckpt_every,
                            void* ckpt, size_t ckpt_bytes, double grad_out, mc_result* out) {
  if (!ctx) return MC_ERR_INVALID_ARG;
  mc_status st = validate_common(ctx, m, f, n_paths, n_steps);
  if (st != MC_OK) return st;
  if (!out) return fail(ctx, MC_ERR_INVALID_ARG, "out must not be NULL");
  mc_options o = opts ? *opts : defaults();
  if (m->kind != MC_HESTON)
    return fail(ctx, MC_ERR_UNSUPPORTED, "the adjoint kernel covers the Heston model");
  st = validate_heston(ctx, m, o);
  if (st != MC_OK) return st;
  if (f->kind != MC_EURO_CALL && f->kind != MC_ASIAN_ARITH_CALL)
    return fail(ctx, MC_ERR_UNSUPPORTED, "adjoint for the European or arithmetic-Asian call");
  if (ckpt_every < 2 || ckpt_every > (uint32_t)mcp::kCkptMax || (ckpt_every & 1u))
    return fail(ctx, MC_ERR_UNSUPPORTED, "checkpoint period must be even, 2..%d", mcp::kCkptMax);
  if (phase != MC_ADJ_FULL && phase != MC_ADJ_FWD && phase != MC_ADJ_REV)
    return fail(ctx, MC_ERR_INVALID_ARG, "unknown phase");
  if (!std::isfinite(grad_out)) return fail(ctx, MC_ERR_INVALID_ARG, "grad_out must be finite");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, MC_ERR_DEVICE, "hipSetDevice");
  const size_t need = mc_adjoint_ckpt_bytes(n_paths, n_steps, ckpt_every);
  const int C = phase == MC_ADJ_FULL ? 3 : phase == MC_ADJ_FWD ? 1 : 2;
  const RunLayout L = layout_for(n_paths, C, o.path_values != nullptr);
  const uint32_t n_ckpt = (n_steps + ckpt_every - 1) / ckpt_every;
  // A one-launch sweep with few checkpoints keeps them in LDS.
  const bool lds = phase == MC_ADJ_FULL && n_ckpt <= (uint32_t)mcp::kLdsCkpt;
  float* ck = lds ? nullptr : (float*)ckpt;
  if (lds) {
  } else if (ck) {
    if (ckpt_bytes < need)
      return fail(ctx, MC_ERR_WORKSPACE, "checkpoint buffer has %zu bytes, %zu needed", ckpt_bytes,
                  need);
  } else {
    if (phase != MC_ADJ_FULL)
      return fail(ctx, MC_ERR_INVALID_ARG, "FWD/REV phases need a checkpoint buffer");
    // Checkpoints after the moment workspace.
    char* base = nullptr;
    st = get_ws(ctx, o, align256(L.bytes) + align256(need), &base);
    if (st != MC_OK) return st;
    ck = (float*)(base + align256(L.bytes));
    o.workspace = base;
    o.workspace_bytes = align256(L.bytes);
  }
  AdjointParams a{};
  a.h = heston_params(m, f, n_paths, n_steps, seed, o, o.stream_tag);
  a.asian = f->kind == MC_ASIAN_ARITH_CALL;
  a.phase = (int)phase;
  a.ckpt = ck;
  a.n_ckpt = n_ckpt;
  a.every = ckpt_every;
  a.grad_out = grad_out;
  Moments mom;
  double kms = 0.0;
  st = run_moments(ctx, o, n_paths, C, o.path_values,
                   [&](double* partials, double* path_out, hipStream_t s, uint32_t* nb) {
                     a.h.partials = partials;
                     a.h.path_out = path_out;
                     return launch_heston_adjoint(a, s, nb);
                   },
                   &mom, &kms);
  if (st != MC_OK) return st;
  mc_result r{};
  double v;
  if (phase != MC_ADJ_REV) {
    fill_channel(mom, 0, &r.price, &r.variance, &r.std_err);
    r.plain_price = r.price;
    r.plain_std_err = r.std_err;
  }
  if (phase != MC_ADJ_FWD) {
    const int g = phase == MC_ADJ_FULL ? 1 : 0;
    fill_channel(mom, g, &r.delta, &v, &r.delta_se);
    fill_channel(mom, g + 1, &r.vega, &v, &r.vega_se);
    r.delta *= grad_out;
    r.delta_se *= std::fabs(grad_out);
    r.vega *= grad_out;
    r.vega_se *= std::fabs(grad_out);
  }
  r.vrf = 1.0;
  r.n_paths = (uint64_t)mom.n;
  r.n_nonfinite = (uint64_t)mom.nonfinite;
  r.kernel_ms = kms;
  *out = r;
  return MC_OK;
}

static mc_status validate_adam(mc_context* ctx, const mc_adam_cfg* cfg, uint64_t n_train) {
  if (!cfg) return fail(ctx, MC_ERR_INVALID_ARG, "cfg must not be NULL");
  if (!(std::isfinite(cfg->lr) && cfg->lr > 0 && cfg->beta1 >= 0 && cfg->beta1 < 1 &&
        cfg->beta2 >= 0 && cfg->beta2 < 1 && cfg->eps > 0))
    return fail(ctx, MC_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  if (cfg->batch < 256 || cfg->batch % 256 != 0)
    return fail(ctx, MC_ERR_INVALID_ARG, "batch must be a positive multiple of 256");
  if (cfg->decay_every > 0 && !(cfg->decay > 0 && cfg->decay <= 1))
    return fail(ctx, MC_ERR_INVALID_ARG, "decay must lie in (0, 1] when decay_every > 0");
  if (n_train && (n_train < cfg->batch || n_train % cfg->batch != 0))
    return fail(ctx, MC_ERR_INVALID_ARG, "n_train must be a multiple of batch");
  return MC_OK;
}

mc_status mc_cv_loss_grad(mc_context* ctx, const mc_model* m, const mc_payoff* f, uint32_t n_steps,
                          uint64_t seed, uint32_t tag, uint64_t path0, uint64_t batch,
                          const mc_adam_cfg* cfg, const float* weights, double* loss_out,
                          float* grad_out) {
  if (!ctx) return MC_ERR_INVALID_ARG;
  mc_status st = validate_common(ctx, m, f, batch, n_steps);
  if (st != MC_OK) return st;
  mc_options o = defaults();
  st = validate_heston(ctx, m, o);
  if (st != MC_OK) return st;
  st = validate_adam(ctx, cfg, 0);
  if (st != MC_OK) return st;
  st = cv_validate(ctx, m, f, cfg->prec, cfg->hedge_every);
  if (st != MC_OK) return st;
  if (!weights || !loss_out || !grad_out) return fail(ctx, MC_ERR_INVALID_ARG, "NULL array");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, MC_ERR_DEVICE, "hipSetDevice");
  const uint32_t n_seg = cv_segments(n_steps, cfg->hedge_every);
  const size_t bytes = cv_train_bytes(batch, n_steps, 1, batch, n_seg, nullptr, nullptr);
  char* base = nullptr;
  st = get_ws(ctx, o, bytes, &base);
  if (st != MC_OK) return st;
  CvTrainWs w;
  cv_train_bytes(batch, n_steps, 1, batch, n_seg, &w, base);
  hipStream_t s = ctx->stream;
  st = cv_upload(ctx, s, w.b, weights, dfac_table(m, n_steps));
  if (st != MC_OK) return st;
  const bool bf16 = cfg->prec == MC_BF16_GEMM;
  st = cv_fill_cache(ctx, s, m, f, n_steps, seed, tag, path0, batch, cfg->hedge_every, bf16, w);
  if (st != MC_OK) return st;
  st = cv_loss_grad_device(ctx, s, m, f, n_steps, 0, batch, batch, cfg->hedge_every, bf16, w,
                           w.log);
  if (st != MC_OK) return st;
  std::vector<double> g(kMlpNParam), mom(n_moments(3));
  HIP_TRY(ctx, hipMemcpyAsync(g.data(), w.grad, kMlpNParam * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(mom.data(), w.log, mom.size() * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  for (int i = 0; i < kMlpNParam; ++i) grad_out[i] = (float)g[i];
  *loss_out = loss_from_moments(mom.data());
  return MC_OK;
}

mc_status mc_cv_train(mc_context* ctx, const mc_model* m, const mc_payoff* f, uint64_t n_train,
                      uint32_t n_steps, uint64_t seed, const mc_adam_cfg* cfg,
                      float* weights_inout, float* loss_log) {
  if (!ctx) return MC_ERR_INVALID_ARG;
  mc_status st = validate_common(ctx, m, f, n_train, n_steps);
  if (st != MC_OK) return st;
  mc_options o = defaults();
  st = validate_heston(ctx, m, o);
  if (st != MC_OK) return st;
  st = validate_adam(ctx, cfg, n_train);
  if (st != MC_OK) return st;
  st = cv_validate(ctx, m, f, cfg->prec, cfg->hedge_every);
  if (st != MC_OK) return st;
  if (!weights_inout) return fail(ctx, MC_ERR_INVALID_ARG, "weights_inout must not be NULL");
  if (cfg->steps == 0) return MC_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, MC_ERR_DEVICE, "hipSetDevice");
  const uint64_t B = cfg->batch;
  const uint32_t n_seg = cv_segments(n_steps, cfg->hedge_every);
  const size_t bytes = cv_train_bytes(B, n_steps, cfg->steps, n_train, n_seg, nullptr, nullptr);
  char* base = nullptr;
  st = get_ws(ctx, o, bytes, &base);
  if (st != MC_OK) return st;
  CvTrainWs w;
  cv_train_bytes(B, n_steps, cfg->steps, n_train, n_seg, &w, base);
  hipStream_t s = ctx->stream;
  st = cv_upload(ctx, s, w.b, weights_inout, dfac_table(m, n_steps));
  if (st != MC_OK) return st;
  HIP_TRY(ctx, hipMemsetAsync(w.m, 0, kMlpNParam * 4, s));
  HIP_TRY(ctx, hipMemsetAsync(w.v, 0, kMlpNParam * 4, s));
  const uint64_t n_batches = n_train / B;
  const uint32_t n_mom = (uint32_t)n_moments(3);
  const bool bf16 = cfg->prec == MC_BF16_GEMM;
  // The fixed training set (stream tag 2), simulated once.
  st = cv_fill_cache(ctx, s, m, f, n_steps, seed, 2, 0, n_train, cfg->hedge_every, bf16, w);
  if (st != MC_OK) return st;
  for (uint32_t t = 0; t < cfg->steps; ++t) {
    // Minibatches cycle through the training set.
    const uint64_t first = (t % n_batches) * B;
    uint32_t nb = 0;
    CvValMoments vm{};
    st = cv_loss_grad_device(ctx, s, m, f, n_steps, first, n_train, B, cfg->hedge_every, bf16, w,
                             w.log + (size_t)t * n_mom, &nb, &vm);
    if (st != MC_OK) return st;
    // Step decay of the learning rate; Adam's moments carry across drops.
    const double lr =
        cfg->decay_every > 0 ? cfg->lr * std::pow(cfg->decay, (double)(t / cfg->decay_every))
                             : cfg->lr;
    HIP_TRY(ctx, launch_adam_pack(w.grad_partials, nb, vm, w.grad, w.b.theta, w.m, w.v,
                                  (int)t + 1, lr, cfg->beta1, cfg->beta2, cfg->eps, w.b.w1f,
                                  w.b.w2f, w.b.w2tf, w.b.lanec, s));
  }
  std::vector<double> log((size_t)cfg->steps * n_mom);
  HIP_TRY(ctx, hipMemcpyAsync(weights_inout, w.b.theta, kMlpNParam * 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(log.data(), w.log, log.size() * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  if (loss_log)
    for (uint32_t t = 0; t < cfg->steps; ++t) loss_log[t] = (float)loss_from_moments(&log[(size_t)t * n_mom]);
  return MC_OK;
}

mc_status mc_price_lsm(mc_context* ctx, const mc_model* m, const mc_lsm_spec* sp,
                       uint64_t n_paths, uint64_t seed, const mc_options* opts,
                       mc_lsm_result* out, const mc_lsm_paths* diag) {
  if (!ctx) return MC_ERR_INVALID_ARG;
  if (!m || !sp || !out) return fail(ctx, MC_ERR_INVALID_ARG, "NULL argument");
  const mc_options o = opts ? *opts : defaults();
  if (m->kind != MC_GBM && m->kind != MC_GBM_BASKET)
    return fail(ctx, MC_ERR_UNSUPPORTED, "Longstaff-Schwartz runs on GBM assets");
  const uint32_t d = m->dim;
  if (d < 1 || d > (uint32_t)kLsmMaxD || (m->kind == MC_GBM && d != 1))
    return fail(ctx, MC_ERR_INVALID_ARG, "dim must be 1..%d (1 for MC_GBM)", kLsmMaxD);
  if (n_paths < 2 || n_paths > (1ull << 32))
    return fail(ctx, MC_ERR_INVALID_ARG, "n_paths must be in 2..2^32");
  if (!finite_pos(m->T)) return fail(ctx, MC_ERR_INVALID_ARG, "T must be finite and > 0");
  if (!std::isfinite(m->r)) return fail(ctx, MC_ERR_INVALID_ARG, "r must be finite");
  if (!m->S0 || !m->sigma) return fail(ctx, MC_ERR_INVALID_ARG, "S0 and sigma are required");
  for (uint32_t a = 0; a < d; ++a) {
    if (!finite_pos(m->S0[a])) return fail(ctx, MC_ERR_INVALID_ARG, "S0[%u] must be > 0", a);
    if (!finite_nonneg(m->sigma[a])) return fail(ctx, MC_ERR_INVALID_ARG, "sigma[%u] invalid", a);
  }
  if (sp->payoff != MC_LSM_MAX_CALL && sp->payoff != MC_LSM_BASKET_PUT &&
      sp->payoff != MC_LSM_BASKET_CALL)
    return fail(ctx, MC_ERR_INVALID_ARG, "unknown payoff");
  if (!finite_pos(sp->K)) return fail(ctx, MC_ERR_INVALID_ARG, "K must be finite and > 0");
  if (!std::isfinite(sp->dividend)) return fail(ctx, MC_ERR_INVALID_ARG, "dividend not finite");
  const uint32_t M = sp->n_dates, spd = sp->steps_per_date;
  if (M < 1 || M > (uint32_t)kLsmMaxDates)
    return fail(ctx, MC_ERR_INVALID_ARG, "n_dates must be in 1..%d", kLsmMaxDates);
  if (spd < 1) return fail(ctx, MC_ERR_INVALID_ARG, "steps_per_date must be >= 1");
  if ((uint64_t)M * spd * d / 4 >= (1ull << 32))
    return fail(ctx, MC_ERR_INVALID_ARG, "more than 2^34 normals per path");
  if (sp->degree < 1 || sp->degree > 3)
    return fail(ctx, MC_ERR_INVALID_ARG, "degree must be in 1..3");
  if (sp->n_paths_oos == 1 || sp->n_paths_oos > (1ull << 36))
    return fail(ctx, MC_ERR_INVALID_ARG, "n_paths_oos must be 0 or in 2..2^36");
  const uint32_t pay_feat = sp->payoff == MC_LSM_MAX_CALL && d >= 2 ? 1u : 0u;
  const uint32_t nf = lsm_n_features(d, sp->degree, pay_feat);
  if (nf == 0 || nf > (uint32_t)kLsmMaxFeat)
    return fail(ctx, MC_ERR_UNSUPPORTED, "%u features; at most %d", nf, kLsmMaxFeat);
  if (o.prec != MC_FP32) return fail(ctx, MC_ERR_UNSUPPORTED, "Longstaff-Schwartz runs in MC_FP32");
  if (o.greeks) return fail(ctx, MC_ERR_UNSUPPORTED, "Longstaff-Schwartz carries no greeks");
  std::vector<double> L((size_t)d * d, 0.0);
  if (d == 1) {
    L[0] = 1.0;
  } else {
    if (!m->corr) return fail(ctx, MC_ERR_INVALID_ARG, "dim > 1 needs corr");
    for (uint32_t i = 0; i < d; ++i)
      for (uint32_t j = 0; j < d; ++j) {
        const double c = m->corr[(size_t)i * d + j];
        if (!std::isfinite(c)) return fail(ctx, MC_ERR_INVALID_ARG, "corr not finite");
        if (c != m->corr[(size_t)j * d + i])
          return fail(ctx, MC_ERR_INVALID_ARG, "corr not symmetric");
      }
    if (!host::cholesky((int)d, m->corr, L.data()))
      return fail(ctx, MC_ERR_NOT_PD, "correlation matrix is not positive definite");
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, MC_ERR_DEVICE, "hipSetDevice");

  LsmParams p{};
  p.n_paths = n_paths;
  p.path_offset = o.path_offset;
  p.tag = o.stream_tag;
  p.k0 = (uint32_t)seed;
  p.k1 = (uint32_t)(seed >> 32);
  p.d = d;
  p.degree = sp->degree;
  p.pay_feat = pay_feat;
  p.kind = (uint32_t)sp->payoff;
  p.n_dates = M;
  p.spd = spd;
  p.nf = nf;
  const double dt = m->T / ((double)M * spd), sdt = std::sqrt(dt), il2 = 1.0 / std::log(2.0);
  for (uint32_t a = 0; a < d; ++a) {
    const double sg = m->sigma[a];
    p.x0[a] = (float)std::log2(m->S0[a] / sp->K);
    p.drift[a] = (float)((m->r - sp->dividend - 0.5 * sg * sg) * dt * il2);
    for (uint32_t b = 0; b <= a; ++b) p.vol[a][b] = (float)(sg * sdt * L[(size_t)a * d + b] * il2);
  }
  for (uint32_t j = 0; j <= M; ++j) p.discK[j] = sp->K * std::exp(-m->r * m->T * j / M);

  // Device memory: states [M-1][d][N] (t_M is used inside the simulation
  // only), cash flows, exercise dates, block
  // partials, one row of reduced moments per stage (simulation, M-1
  // updates, out-of-sample), coefficients and their flags.
  const uint64_t Noos = sp->n_paths_oos;
  const bool want_cf = diag && diag->cash_flow, want_ex = diag && diag->exercise_date;
  const bool want_ov = diag && diag->oos_value, want_oe = diag && diag->oos_exercise_date;
  p.ystride = (n_paths + 63) / 64 * 64;
  const size_t b_y = align256((size_t)(M - 1) * d * p.ystride * sizeof(float));
  const size_t b_c = align256((size_t)p.ystride * sizeof(float));
  const size_t b_e = want_ex ? align256((size_t)n_paths) : 0;
  const size_t b_p = align256((size_t)kLsmMaxMom * kLsmMaxBlocks * sizeof(double));
  const size_t b_s = align256((size_t)(M + 1) * kLsmMaxMom * sizeof(double));
  const size_t b_b = align256((size_t)M * kLsmMaxFeat * sizeof(double));
  const size_t b_v = align256((size_t)M * sizeof(int));
  const size_t b_ov = want_ov ? align256((size_t)Noos * sizeof(double)) : 0;
  const size_t b_oe = want_oe ? align256((size_t)Noos) : 0;
  char* base = nullptr;
  mc_status st = get_lsm_buf(ctx, b_y + b_c + b_e + b_p + b_s + b_b + b_v + b_ov + b_oe, &base);
  if (st != MC_OK) return st;
  char* q = base;
  p.y = (float*)q;                 q += b_y;
  p.C = (float*)q;                 q += b_c;
  p.ex = want_ex ? (uint8_t*)q : nullptr;  q += b_e;
  p.partials = (double*)q;         q += b_p;
  double* sums = (double*)q;       q += b_s;
  double* beta = (double*)q;       q += b_b;
  int* valid = (int*)q;            q += b_v;
  double* oval = want_ov ? (double*)q : nullptr;  q += b_ov;
  uint8_t* oex = want_oe ? (uint8_t*)q : nullptr;
  p.beta = beta;
  p.valid = valid;

  hipStream_t s = stream_of(ctx, o);
  while (ctx->lsm_ev.size() < 2 * (size_t)kLsmMaxDates) {
    hipEvent_t e = nullptr;
    HIP_TRY(ctx, hipEventCreate(&e));
    ctx->lsm_ev.push_back(e);
  }
  const uint32_t nmom = lsm_n_moments(nf);
  uint32_t nb = 0;
  HIP_TRY(ctx, hipEventRecord(ctx->ev0, s));
  HIP_TRY(ctx, launch_lsm_sim(p, s, &nb));
  // Row 0: the simulation's moments; the Gram matrix in them is date M-1's.
  HIP_TRY(ctx, launch_lsm_reduce_solve(p.partials, nb, nmom, sums, nf, M - 1, beta, valid, s));
  HIP_TRY(ctx, hipEventRecord(ctx->ev1, s));
  // Stage t (1..M-1) updates date j = M-t with the coefficients solved at
  // stage t-1; its moments (the Gram matrix of date j-1, solved here, or the
  // price at j = 1) go to row t.
  for (uint32_t t = 1; t < M; ++t) {
    const uint32_t j = M - t;
    HIP_TRY(ctx, hipEventRecord(ctx->lsm_ev[2 * t], s));
    HIP_TRY(ctx, launch_lsm_update(p, j, s, &nb));
    HIP_TRY(ctx, hipEventRecord(ctx->lsm_ev[2 * t + 1], s));
    HIP_TRY(ctx, launch_lsm_reduce_solve(p.partials, nb, nmom, sums + (size_t)t * kLsmMaxMom, nf,
                                         j - 1, beta, valid, s));
  }
  HIP_TRY(ctx, hipEventRecord(ctx->ev2, s));
  if (Noos) {
    LsmParams po = p;
    po.n_paths = Noos;
    po.tag = o.stream_tag + 7;
    po.y = nullptr;
    po.C = nullptr;
    po.ex = oex;
    po.path_value = oval;
    HIP_TRY(ctx, launch_lsm_oos(po, s, &nb));
    HIP_TRY(ctx, launch_final_reduce(p.partials, nb, 2, sums + (size_t)M * kLsmMaxMom, s));
  }
  HIP_TRY(ctx, hipEventRecord(ctx->ev3, s));
  std::vector<double> h_sums((size_t)(M + 1) * kLsmMaxMom), h_beta((size_t)M * kLsmMaxFeat);
  std::vector<int> h_valid(M);
  HIP_TRY(ctx, hipMemcpyAsync(h_sums.data(), sums, h_sums.size() * 8, hipMemcpyDeviceToHost, s));
  if (M > 1) {
    HIP_TRY(ctx, hipMemcpyAsync(h_beta.data(), beta, (size_t)(M - 1) * kLsmMaxFeat * 8,
                                hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(h_valid.data(), valid, (size_t)(M - 1) * sizeof(int),
                                hipMemcpyDeviceToHost, s));
  }
  std::vector<float> h_c(want_cf ? n_paths : 0);
  std::vector<uint8_t> h_e(want_ex ? n_paths : 0), h_oe(want_oe ? Noos : 0);
  if (want_cf)
    HIP_TRY(ctx, hipMemcpyAsync(h_c.data(), p.C, n_paths * 4, hipMemcpyDeviceToHost, s));
  if (want_ex) HIP_TRY(ctx, hipMemcpyAsync(h_e.data(), p.ex, n_paths, hipMemcpyDeviceToHost, s));
  if (want_ov)
    HIP_TRY(ctx, hipMemcpyAsync(diag->oos_value, oval, Noos * 8, hipMemcpyDeviceToHost, s));
  if (want_oe) HIP_TRY(ctx, hipMemcpyAsync(h_oe.data(), oex, Noos, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  float ms_sim = 0.f, ms_reg = 0.f, ms_oos = 0.f;
  HIP_TRY(ctx, hipEventElapsedTime(&ms_sim, ctx->ev0, ctx->ev1));
  HIP_TRY(ctx, hipEventElapsedTime(&ms_reg, ctx->ev1, ctx->ev2));
  HIP_TRY(ctx, hipEventElapsedTime(&ms_oos, ctx->ev2, ctx->ev3));
  double ms_upd = 0.0;
  for (uint32_t t = 1; t < M; ++t) {
    float e = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&e, ctx->lsm_ev[2 * t], ctx->lsm_ev[2 * t + 1]));
    ms_upd += e;
  }

  mc_lsm_result r{};
  const uint32_t ng = (nf + 1) * (nf + 2) / 2;
  const double n = (double)n_paths;
  const double* row0 = h_sums.data();
  moments_mean_se(n, row0[ng], row0[ng + 1], &r.european, &r.european_se);
  const double* last = h_sums.data() + (size_t)(M - 1) * kLsmMaxMom;
  if (M == 1)
    moments_mean_se(n, row0[ng], row0[ng + 1], &r.price, &r.std_err);
  else
    moments_mean_se(n, last[ng], last[ng + 1], &r.price, &r.std_err);
  if (Noos) {
    const double* ro = h_sums.data() + (size_t)M * kLsmMaxMom;
    moments_mean_se((double)Noos, ro[0], ro[1], &r.price_oos, &r.std_err_oos);
  } else {
    r.price_oos = NAN;
    r.std_err_oos = NAN;
  }
  r.n_features = nf;
  for (uint32_t j = 0; j < (uint32_t)MC_LSM_MAX_DATES; ++j)
    for (uint32_t k = 0; k < (uint32_t)MC_LSM_MAX_FEATURES; ++k) r.beta[j][k] = NAN;
  for (uint32_t j = 1; j < M; ++j) {
    r.beta_valid[j - 1] = h_valid[j - 1];
    if (h_valid[j - 1])
      for (uint32_t k = 0; k < nf; ++k) r.beta[j - 1][k] = h_beta[(size_t)(j - 1) * kLsmMaxFeat + k];
    // The Gram matrix of date j was reduced into row M-1-j; entry 0 counts.
    r.n_itm[j - 1] = (uint64_t)h_sums[(size_t)(M - 1 - j) * kLsmMaxMom];
  }
  r.n_itm[M - 1] = (uint64_t)row0[ng + 2];
  r.n_paths = n_paths;
  r.n_paths_oos = Noos;
  r.sim_ms = ms_sim;
  r.regress_ms = ms_reg;
  r.oos_ms = ms_oos;
  r.update_ms = ms_upd;
  if (want_cf)
    for (uint64_t i = 0; i < n_paths; ++i) diag->cash_flow[i] = h_c[i];
  if (want_ex)
    for (uint64_t i = 0; i < n_paths; ++i) diag->exercise_date[i] = h_e[i];
  if (want_oe)
    for (uint64_t i = 0; i < Noos; ++i) diag->oos_exercise_date[i] = h_oe[i];
  *out = r;
  return MC_OK;
}

mc_status mc_philox_words(mc_context* ctx, uint64_t seed, uint32_t tag, uint64_t n,
                          const uint64_t* paths, const uint64_t* blocks, uint32_t* out4) {
  if (!ctx) return MC_ERR_INVALID_ARG;
  if (n == 0) return MC_OK;
  if (!paths || !blocks || !out4) return fail(ctx, MC_ERR_INVALID_ARG, "NULL array");
  for (uint64_t i = 0; i < n; ++i)
    if (blocks[i] > 0xffffffffull) return fail(ctx, MC_ERR_INVALID_ARG, "block index above 2^32");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, MC_ERR_DEVICE, "hipSetDevice");
  mc_options o = defaults();
  const size_t b_in = align256(n * sizeof(uint64_t));
  char* base = nullptr;
  mc_status st = get_ws(ctx, o, 2 * b_in + n * 16, &base);
  if (st != MC_OK) return st;
  uint64_t* dp = (uint64_t*)base;
  uint64_t* db = (uint64_t*)(base + b_in);
  uint32_t* dout = (uint32_t*)(base + 2 * b_in);
  hipStream_t s = ctx->stream;
  HIP_TRY(ctx, hipMemcpyAsync(dp, paths, n * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, hipMemcpyAsync(db, blocks, n * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(ctx, launch_philox_words((uint32_t)seed, (uint32_t)(seed >> 32), tag, n, dp, db, dout, s));
  HIP_TRY(ctx, hipMemcpyAsync(out4, dout, n * 16, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return MC_OK;
}

mc_status mc_normals(mc_context* ctx, uint64_t seed, uint32_t tag, uint64_t path, uint64_t k0,
                     uint64_t count, mc_precision prec, double* out) {
  if (!ctx) return MC_ERR_INVALID_ARG;
  if (count == 0) return MC_OK;
  if (!out) return fail(ctx, MC_ERR_INVALID_ARG, "NULL output");
  if (prec != MC_FP32 && prec != MC_FP64)
    return fail(ctx, MC_ERR_UNSUPPORTED, "normals in MC_FP32 or MC_FP64");
  if ((k0 + count - 1) / 4 > 0xffffffffull)
    return fail(ctx, MC_ERR_INVALID_ARG, "normal index above 2^34");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, MC_ERR_DEVICE, "hipSetDevice");
  mc_options o = defaults();
  char* base = nullptr;
  mc_status st = get_ws(ctx, o, count * sizeof(double), &base);
  if (st != MC_OK) return st;
  hipStream_t s = ctx->stream;
  HIP_TRY(ctx, launch_normals((uint32_t)seed, (uint32_t)(seed >> 32), tag, path, k0, count,
                              prec == MC_FP64, (double*)base, s));
  HIP_TRY(ctx, hipMemcpyAsync(out, base, count * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  return MC_OK;
}

}  // extern "C"
