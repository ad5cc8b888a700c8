// Learned martingale control variate on the Heston Asian call.
//
// A hedge network Delta(t, state), 4 -> 64 -> 64 -> 1 with tanh, is run
// along every path; its discounted hedging P&L
//     H = sum_j Delta(phi_{t_j}) (St_{t_{j+1}} - St_{t_j}),  St = e^{-rt} S,
// has zero mean for any weights (St is a martingale under the log-Euler
// step), so Y = payoff - H is an unbiased estimator of the price (Eq. 3
// applied to Y) whose variance the network is trained to minimise.
//
// Path state: the discounted log-price z~ = log2(St/S0) (the rate cancels
// from its drift) and the variance v; S_i/S0 = 2^{z~_i} * dfac[i] feeds the
// Asian average. Features phi = (t/T, ln(S/K), v/theta, Abar/K - 1).
//
// Network on MFMA, one wave = 32 paths, lanes l and l+32 both follow path
// l mod 32 and each holds half of every hidden layer:
//   layer 1: D1 = [W1 | b1] (64 x 16) . [phi; 1] (16 x 32 paths)
//   layer 2: D2 = W2 (64 x 64) . H1^T (64 x 32 paths)
// An accumulator lane holds units u(mb, r, h) = 32 mb + 8 (r/4) + 4 h +
// (r mod 4). Layer 2's k-slots are ordered so that its B operand is exactly
// the lane's layer-1 output (the host permutes W2 to match), so nothing
// moves between layers. Layer 3 is a per-lane dot product plus one swap of
// halves. tanh(x) = 2 / (1 + e^{-2x}) - 1 on v_exp_f32 / v_rcp_f32. Where
// only Delta is needed, layer 3 runs on r = (1 + tanh) / 2 = 1 / (1 + e^{-2x})
// of layer 2: Delta = sum_u (2 W3_u) r_u + (b3 - sum_u W3_u), one FMA per unit
// fewer (the per-lane constants hold 2 W3).
//
// Training. The network's inputs (the features at each segment's opening
// date) and the segment's price change do not depend on the weights, so
// the training paths are simulated once into a feature cache; an Adam step
// then runs only the network: a forward pass along every 32-path tile of
// the minibatch giving the per-path hedged values and their moments, and
// the backward pass. There, for each hedge segment the upstream
// derivative dL/dDelta = g_b dSt with g_b = -(2/B)(Y_b - Ybar) is pushed
// back through the network; dW2 = delta2^T H1 and dW1 = delta1^T [phi; 1]
// are MFMA products over the wave's 32 paths after a transpose through LDS.
// Each block writes its partial gradient (its waves summed in FP64, stored
// in FP32); a fixed-order FP64 reduction and the Adam step follow in one
// launch.
#include <type_traits>

#include "device/reduce.h"
#include "device/rng.h"
#include "mc_internal.h"

namespace mcp {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(2))) float float2_t;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kCvWaves = 4;
constexpr int kCvThreads = 64 * kCvWaves;
constexpr float kNeg2Log2e = -2.88539008177792681472f;   // -2 / ln 2

// One MFMA operand: 8 k-slots per lane, held as BF16 for the BF16 products
// (converted with round-to-nearest-even once, where the value is made) or as
// FP32 for the FP32 form.
template <bool BF16>
using FragT = std::conditional_t<BF16, __bf16, float>;
template <bool BF16>
struct Op8;
template <>
struct Op8<true> {
  bf16x8 v;
};
template <>
struct Op8<false> {
  float v[8];
};

template <bool BF16>
__device__ __forceinline__ Op8<BF16> op_from(const float (&x)[8]) {
  Op8<BF16> o;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if constexpr (BF16)
      o.v[j] = (__bf16)x[j];
    else
      o.v[j] = x[j];
  }
  return o;
}

template <bool BF16>
__device__ __forceinline__ Op8<BF16> op_zero() {
  Op8<BF16> o;
#pragma unroll
  for (int j = 0; j < 8; ++j) o.v[j] = (FragT<BF16>)0.f;
  return o;
}

// 8 consecutive elements from LDS (16-byte aligned for BF16, 32 for FP32).
template <bool BF16>
__device__ __forceinline__ Op8<BF16> op_lds(const FragT<BF16>* p) {
  Op8<BF16> o;
  if constexpr (BF16) {
    o.v = *(const bf16x8*)p;
  } else {
    const float4 a = *(const float4*)p;
    const float4 b = *(const float4*)(p + 4);
    o.v[0] = a.x; o.v[1] = a.y; o.v[2] = a.z; o.v[3] = a.w;
    o.v[4] = b.x; o.v[5] = b.y; o.v[6] = b.z; o.v[7] = b.w;
  }
  return o;
}

// acc += A x B over one 16-wide k block: one BF16 MFMA, or eight FP32
// MFMAs with the same k-slot order.
template <bool BF16>
__device__ __forceinline__ void mma16(f32x16& acc, const Op8<BF16>& a, const Op8<BF16>& b) {
  if constexpr (BF16) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v, b.v, acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v[j], b.v[j], acc, 0, 0, 0);
  }
}

// 1 / (1 + e^{-2(x + b)}) = (1 + tanh(x + b)) / 2, with cb = -2 b / ln 2
// folded into the exponent.
__device__ __forceinline__ float sigm2_b(float x, float cb) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(__builtin_fmaf(x, kNeg2Log2e, cb)));
}

// tanh(x + b), same folding.
__device__ __forceinline__ float tanh_b(float x, float cb) {
  return __builtin_fmaf(2.0f, sigm2_b(x, cb), -1.0f);
}

// The constant of layer 3 in the sigmoid form, b3 - sum_u W3_u: the 64 W3
// are summed by a fixed butterfly and lane 0's total is broadcast, so every
// lane of every wave and kernel uses the same bits.
__device__ __forceinline__ float out_const(const float* theta) {
  float w = theta[4480 + (threadIdx.x & 63)];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off, 64);
  return theta[4544] - __shfl(w, 0, 64);
}

__device__ __forceinline__ int unit_of(int mb, int r, int h) {
  return 32 * mb + 8 * (r >> 2) + 4 * h + (r & 3);
}

__device__ __forceinline__ void load8(const float* p, float (&x)[8]) {
  const float4 a = *(const float4*)p;
  const float4 b = *(const float4*)(p + 4);
  x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
  x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
}

// Orders one wave's LDS stores before its later loads of the same region
// (a wave runs in lockstep; no other wave shares the region).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kFragFloats = 2 * 4 * 64 * 8;   // one set of layer-2 fragments
constexpr int kLaneFloats = 2 * 64 * 32;      // per-lane b2 (scaled) and 2 W3

// Per-lane constants (b2 scaled, then 2 W3): 32 values per lane, one per unit
// slot q = 16 mb + r, stored as [q / 4][lane][q mod 4] so that the four
// consecutive slots a lane reads at once sit beside those of its neighbours
// (a wave's 16-byte reads cover 1 KB contiguously, free of bank conflicts).
__device__ __forceinline__ int lanec_index(int lane, int q) {
  return (q >> 2) * 256 + lane * 4 + (q & 3);
}

// The layer-2 fragments (optionally also their transposes) and the per-lane
// constants, global -> registers -> LDS: every thread issues all of its
// loads before the first store, so a workgroup waits for one memory
// latency rather than one per element.
constexpr int kFillPer = kFragFloats / kCvThreads;
static_assert(kFragFloats % kCvThreads == 0 && kLaneFloats == kFragFloats, "fragment split");
struct WeightRegs {
  float a[kFillPer], b[kFillPer], c[kFillPer];
};
template <bool WITH_T>
__device__ __forceinline__ void weights_load(const float* w2f, const float* w2tf,
                                             const float* lanec, WeightRegs& r) {
#pragma unroll
  for (int j = 0; j < kFillPer; ++j) {
    const int i = threadIdx.x + j * kCvThreads;
    r.a[j] = w2f[i];
    if constexpr (WITH_T) r.b[j] = w2tf[i];
    r.c[j] = lanec[i];
  }
}
template <bool WITH_T, typename FT>
__device__ __forceinline__ void weights_store(const WeightRegs& r, FT* s_w2f, FT* s_w2tf,
                                              float* s_lanec) {
#pragma unroll
  for (int j = 0; j < kFillPer; ++j) {
    const int i = threadIdx.x + j * kCvThreads;
    s_w2f[i] = (FT)r.a[j];
    if constexpr (WITH_T) s_w2tf[i] = (FT)r.b[j];
    s_lanec[i] = r.c[j];
  }
}

// Forward pass of the hedge network for the wave's 32 paths, keeping the
// activations for the backward pass. phi: the lane's B fragment of layer 1
// (half 0: features and the constant 1; half 1: zeros). Leaves h1, h2.
template <bool BF16>
__device__ __forceinline__ void mlp_forward(const float (&phi)[8], const Op8<BF16> (&w1a)[2],
                                            const FragT<BF16>* w2f, const float* lanec, int lane,
                                            float (&h1)[32], float (&h2)[32]) {
  f32x16 d1[2];
  const Op8<BF16> phio = op_from<BF16>(phi);
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) d1[mb][r] = 0.f;
    mma16<BF16>(d1[mb], w1a[mb], phio);
  }
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int r = 0; r < 16; ++r) h1[mb * 16 + r] = tanh_b(d1[mb][r], 0.f);
  f32x16 d2[2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int r = 0; r < 16; ++r) d2[mb][r] = 0.f;
  // Read the weight fragments from LDS at every use (a compiler barrier
  // keeps them from being hoisted into registers across the time loop,
  // which would halve the occupancy).
  __asm__ volatile("" ::: "memory");
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    float bf[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) bf[j] = h1[(kb >> 1) * 16 + 8 * (kb & 1) + j];
    const Op8<BF16> b = op_from<BF16>(bf);
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
      mma16<BF16>(d2[mb], op_lds<BF16>(&w2f[((mb * 4 + kb) * 64 + lane) * 8]), b);
  }
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int idx = mb * 16 + r;
      h2[idx] = tanh_b(d2[mb][r], lanec[lanec_index(lane, idx)]);
    }
}

// Constants of the Heston step on the discounted log2-price (no rate in
// its drift) and of the features, in FP32.
struct HestonF {
  float dt, kdt, kthdt, xi, rho, rhoc, a1, a2, S0, lnS0K, ln2, rdt2, inv_theta, inv_n, S0K;
  __device__ explicit HestonF(const HestonParams& Hp)
      : dt((float)Hp.dt),
        kdt((float)(Hp.kappa * Hp.dt)),
        kthdt((float)(Hp.kappa * Hp.theta * Hp.dt)),
        xi((float)Hp.xi),
        rho((float)Hp.rho),
        rhoc((float)Hp.rho_c),
        a1((float)(-0.5 * Hp.dt * 1.4426950408889634)),
        a2(1.4426950408889634f),
        S0((float)Hp.S0),
        lnS0K((float)std::log(Hp.S0 / Hp.K)),
        ln2(0.69314718055994531f),
        rdt2((float)(Hp.r * Hp.dt * 1.4426950408889634)),   // log2 e^{r dt}
        inv_theta((float)(1.0 / Hp.theta)),
        inv_n((float)(1.0 / Hp.n_steps)),
        S0K((float)(Hp.S0 / Hp.K)) {}

  // Features at t_i (F_{t_i}-measurable): t/T, ln(S/K), v/theta, Abar/K - 1.
  __device__ __forceinline__ void features(uint32_t i, float z, float v, float sumE,
                                           float (&f)[4]) const {
    const float fi = (float)i;
    const float Abar = (i == 0) ? 1.0f : sumE * __builtin_amdgcn_rcpf(fi);   // running mean of S/S0
    f[0] = fi * inv_n;
    f[1] = (z + rdt2 * fi) * ln2 + lnS0K;          // ln(S_i / K)
    f[2] = v * inv_theta;
    f[3] = Abar * S0K - 1.0f;
  }

  // One full-truncation Euler step of (z~, v).
  __device__ __forceinline__ void step(float& z, float& v, float Z1, float Z2) const {
    const float vp = v > 0.f ? v : 0.f;
    const float sq = __builtin_amdgcn_sqrtf(vp * dt);
    const float Zs = rho * Z1 + rhoc * Z2;
    z = z + a1 * vp + a2 * (sq * Zs);
    v = v + (kthdt - kdt * vp) + xi * (sq * Z1);
  }
};

// The forward pass when only Delta is needed (evaluation and the training
// forward): layer 1's activations go straight into layer 2's B operands, so
// they are held in the operand type (BF16 pairs) rather than as FP32 values,
// and layer 3 takes layer 2's activations in the sigmoid form. c3 =
// out_const(theta). Returns Delta (identical in both halves).
template <bool BF16>
__device__ __forceinline__ float mlp_delta(const float (&phi)[8], const Op8<BF16> (&w1a)[2],
                                           const FragT<BF16>* w2f, const float* lanec, int lane,
                                           float c3) {
  f32x16 d1[2];
  const Op8<BF16> phio = op_from<BF16>(phi);
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) d1[mb][r] = 0.f;
    mma16<BF16>(d1[mb], w1a[mb], phio);
  }
  Op8<BF16> b[4];
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) {
    float bf[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) bf[j] = tanh_b(d1[kb >> 1][8 * (kb & 1) + j], 0.f);
    b[kb] = op_from<BF16>(bf);
  }
  f32x16 d2[2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int r = 0; r < 16; ++r) d2[mb][r] = 0.f;
  __asm__ volatile("" ::: "memory");   // weight fragments are read from LDS at every use
#pragma unroll
  for (int kb = 0; kb < 4; ++kb)
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
      mma16<BF16>(d2[mb], op_lds<BF16>(&w2f[((mb * 4 + kb) * 64 + lane) * 8]), b[kb]);
  float part = 0.f;
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int idx = mb * 16 + r;
      const float v = sigm2_b(d2[mb][r], lanec[lanec_index(lane, idx)]);
      part = __builtin_fmaf(lanec[64 * 32 + lanec_index(lane, idx)], v, part);
    }
  return part + __shfl_xor(part, 32, 64) + c3;
}

// Fills the feature cache: one lane per path (h.n_paths paths from global
// path h.path_offset, stream tag h.tag), the features at every segment's
// opening date, the discounted price change over the segment and the
// discounted Asian payoff.
__global__ __launch_bounds__(kCvThreads) void cv_cache_kernel(const CvParams P) {
  const HestonParams& Hp = P.h;
  const uint64_t pid = (uint64_t)blockIdx.x * kCvThreads + threadIdx.x;
  if (pid >= Hp.n_paths) return;       // no block-level synchronisation follows
  const HestonF c(Hp);
  const uint32_t n = Hp.n_steps, m = P.hedge_every;
  const uint64_t S = P.c_stride;
  const PathCounter pc = make_counter(Hp.path_offset + pid, Hp.tag, Hp.k0, Hp.k1);
  float z = 0.f, v = (float)Hp.v0, sumE = 0.f, st_open = 0.f, Et = 1.f;
  uint32_t k = 0;
  Normals4<float> nz;
  for (uint32_t i = 0; i < n; ++i) {
    if (i % m == 0) {
      float f[4];
      c.features(i, z, v, sumE, f);
#pragma unroll
      for (int q = 0; q < 4; ++q) P.c_phi[((size_t)k * 4 + q) * S + pid] = f[q];
      st_open = Et;
    }
    if ((i & 1) == 0) nz = normals4<float>(philox(i >> 1, pc));
    const float Z1 = (i & 1) ? nz.z[2] : nz.z[0];
    const float Z2 = (i & 1) ? nz.z[3] : nz.z[1];
    c.step(z, v, Z1, Z2);
    Et = __builtin_amdgcn_exp2f(z);
    sumE += Et * P.dfac[i + 1];
    if ((i + 1) % m == 0 || i + 1 == n) {
      P.c_dst[(size_t)k * S + pid] = c.S0 * (Et - st_open);
      ++k;
    }
  }
  const double A = (double)c.S0 * (double)sumE / (double)n;
  P.c_pay[pid] = Hp.disc * (A > Hp.K ? A - Hp.K : 0.0);
}

// Hedged values of the minibatch's paths (h.n_paths paths from cache path
// c_first): a 32-path tile goes through every hedge segment, the network's
// Delta from the cached features, H = sum_k Delta_k dSt_k in segment order
// and Y = payoff - H. The per-path values (channels payoff, H, Y) go to
// path_out when it is set, their block moments to partials. Lane l < 32
// owns path l of the tile (lane l + 32 holds the other half of the hidden
// units), and the next segment's inputs are loaded one segment ahead, so
// that their latency overlaps the network. With seg_split > 1 the tile's
// waves evaluate the network on their own ranges of segments, and its first
// wave forms H from their (Delta, dSt) pairs in segment order: the same
// FMAs in the same order as one wave taking every segment.
template <bool BF16>
__global__ __launch_bounds__(kCvThreads) void cv_values_kernel(const CvParams P) {
  using FT = FragT<BF16>;
  __shared__ __attribute__((aligned(16))) FT s_w2f[kFragFloats];
  __shared__ __attribute__((aligned(16))) float s_lanec[kLaneFloats];
  // (Delta, dSt) of each segment a wave of a split tile takes.
  __shared__ float2 s_dd[kCvWaves][kCvValSlab][32];
  {
    WeightRegs wr;
    weights_load<false>(P.w2f, nullptr, P.lanec, wr);
    weights_store<false>(wr, s_w2f, (FT*)nullptr, s_lanec);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 31, half = lane >> 5;
  Op8<BF16> w1a[2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
    float w[8];
    load8(&P.w1f[(mb * 64 + lane) * 8], w);
    w1a[mb] = op_from<BF16>(w);
  }
  const float c3 = out_const(P.theta);
  const uint64_t n = P.h.n_paths;
  // seg_split waves share a tile, wave `part` taking segments [k0, k1).
  const uint32_t split = P.seg_split, part = (uint32_t)wave % split;
  const uint64_t tile = (uint64_t)blockIdx.x * (kCvWaves / split) + (uint32_t)wave / split;
  const uint32_t k0 = (uint32_t)((uint64_t)P.n_seg * part / split);
  const uint32_t k1 = (uint32_t)((uint64_t)P.n_seg * (part + 1) / split);
  const uint64_t pid = tile * 32 + row;
  const bool active = pid < n;
  const bool lead = active && half == 0;     // lanes holding a path's inputs
  const bool owner = lead && part == 0;      // ... and summing its hedge
  const uint64_t S = P.c_stride, c = P.c_first + pid;
  float nf[4], ndst;
  // Row bases are uniform; the lane adds a 32-bit byte offset (the
  // launcher keeps the minibatch below 2^30 paths).
  const uint32_t ob = (uint32_t)pid * 4u;
  auto at = [&](const float* rowp) { return *(const float*)((const char*)rowp + ob); };
  auto fetch = [&](uint32_t k) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      nf[q] = lead ? at(P.c_phi + ((size_t)k * 4 + q) * S + P.c_first) : 0.f;
    ndst = lead ? at(P.c_dst + (size_t)k * S + P.c_first) : 0.f;
  };
  if (k0 < k1) fetch(k0);
  float H = 0.f;
  for (uint32_t k = k0; k < k1; ++k) {
    float phi[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) phi[q] = nf[q];
    phi[4] = lead ? 1.0f : 0.f;
    phi[5] = phi[6] = phi[7] = 0.f;
    const float dst = ndst;
    if (k + 1 < k1) fetch(k + 1);
    const float d = mlp_delta<BF16>(phi, w1a, s_w2f, s_lanec, lane, c3);
    if (split == 1)
      H = __builtin_fmaf(d, dst, H);
    else if (half == 0)
      s_dd[wave][k - k0][row] = make_float2(d, dst);
  }
  if (split > 1) {
    // The tile's first wave sums the hedge in segment order, as one wave
    // taking every segment does.
    __syncthreads();
    if (part == 0 && half == 0) {
      for (uint32_t p = 0; p < split; ++p) {
        const uint32_t a = (uint32_t)((uint64_t)P.n_seg * p / split);
        const uint32_t b = (uint32_t)((uint64_t)P.n_seg * (p + 1) / split);
        for (uint32_t k = a; k < b; ++k) {
          const float2 e = s_dd[wave + p][k - a][row];
          H = __builtin_fmaf(e.x, e.y, H);
        }
      }
    }
  }
  double y[3] = {0.0, 0.0, 0.0};
  if (owner) {
    const double pay = P.c_pay[c];
    y[0] = pay;
    y[1] = (double)H;
    y[2] = pay - (double)H;
  }
  const bool finite = isfinite(y[0]) && isfinite(y[1]) && isfinite(y[2]);
  if (owner && P.path_out != nullptr) {
#pragma unroll
    for (int q = 0; q < 3; ++q) P.path_out[pid * 3 + q] = y[q];
  }
  block_moments<3, kCvThreads>(y, owner && finite, owner && !finite, P.partials);
}

// Backward pass: a wave takes 32 paths of the minibatch through every hedge
// segment (or, with seg_split > 1, through its range of them), re-running
// the forward pass from the cached features.
//
// Every weight gradient is a product over the wave's 32 paths on the
// matrix cores, accumulated in two register sets:
//   gw2 = delta2^T H1 (64 x 64);
//   gx  = 64 units x 32 columns holding, by column, db2 = delta2^T 1,
//         dW3 = H2^T gD, dW1 = delta1^T phi (4 columns) and db1 = delta1^T 1,
//         each product with a B operand that is zero outside its columns.
// A path-major operand (delta2, H2, H1, delta1) passes through one of the
// wave's two LDS regions to become unit-major, two operands per store ->
// load round trip, with e1 = W2^T delta2 and delta1 computed while the
// stores land; the column operands (gD, phi, 1) are one row each of a small
// part of a region.
template <bool BF16>
__device__ __forceinline__ void cv_bwd_body(const CvParams& P) {
  using FT = FragT<BF16>;
  // One LDS area: the weight fragments and the waves' transpose regions,
  // reused after the segment loop for the block's gradient sum.
  // Rows of kTs elements (32 paths plus padding, so that neither the
  // lanes' 2-byte stores of a unit nor the 16-byte fragment reads of
  // consecutive units fall on one bank group).
  constexpr int kTs = BF16 ? 40 : 36;
  constexpr int kTr = 64 * kTs + 8 * kTs;
  constexpr size_t kLds =
      2 * kFragFloats * sizeof(FT) + kLaneFloats * 4 + kCvWaves * 2 * kTr * sizeof(FT);
  static_assert(kLds >= kCvWaves * kMlpNParam * sizeof(float), "LDS too small for the gradient sum");
  __shared__ __attribute__((aligned(16))) unsigned char lds[kLds];
  FT* s_w2f = (FT*)lds;
  FT* s_w2tf = s_w2f + kFragFloats;
  float* s_lanec = (float*)(lds + 2 * kFragFloats * sizeof(FT));
  FT* tr = (FT*)(lds + 2 * kFragFloats * sizeof(FT) + kLaneFloats * 4);
  // The weight fragments and per-lane constants are loaded into registers
  // first, so that their latency overlaps the sum below.
  WeightRegs wr;
  weights_load<true>(P.w2f, P.w2tf, P.lanec, wr);
  // Ybar = sum n_b mean_b / sum n_b over the hedged-value kernel's block
  // moment vectors, summed in the same fixed order by every block (the full
  // merge of those vectors, the minibatch's loss, runs in the gradient
  // reduction's launch).
  __shared__ double s_ys[kCvWaves][2];
  {
    double sn = 0.0, sy = 0.0;
    for (uint32_t i = threadIdx.x; i < P.val_blocks; i += kCvThreads) {
      const double* v = P.partials + (size_t)i * PartSums<3>::M;
      sn += v[0];
      sy += v[0] * v[2 + 2];             // n and mean of channel 2 (Y)
    }
    // A shuffle-down tree into lane 0 (a butterfly here would share its
    // lane addresses with the epilogue's and keep them live across the
    // segment loop).
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      sn += __shfl_down(sn, off, 64);
      sy += __shfl_down(sy, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      s_ys[threadIdx.x >> 6][0] = sn;
      s_ys[threadIdx.x >> 6][1] = sy;
    }
  }
  weights_store<true>(wr, s_w2f, s_w2tf, s_lanec);
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = lane & 31, half = lane >> 5;
  // seg_split waves share a tile, wave `part` taking segments [k0, k1): the
  // gradient is a sum over (path, segment) items, so any split of the
  // segments gives the same sum up to rounding.
  const uint32_t split = P.seg_split, part = (uint32_t)wave % split;
  const uint64_t tile = (uint64_t)blockIdx.x * (kCvWaves / split) + (uint32_t)wave / split;
  const uint32_t k0 = (uint32_t)((uint64_t)P.n_seg * part / split);
  const uint32_t k1 = (uint32_t)((uint64_t)P.n_seg * (part + 1) / split);
  const uint64_t pid = tile * 32 + row;
  const bool active = pid < P.h.n_paths;
  float g = 0.f;                       // upstream factor of this path
  if (active) {
    double n = 0.0, sy = 0.0;
#pragma unroll
    for (int w = 0; w < kCvWaves; ++w) {
      n += s_ys[w][0];
      sy += s_ys[w][1];
    }
    const double ybar = n > 0.0 ? sy / n : 0.0;
    g = (float)(P.g_scale * (P.y_path[pid * 3 + 2] - ybar));
  }
  Op8<BF16> w1a[2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
    float w[8];
    load8(&P.w1f[(mb * 64 + lane) * 8], w);
    w1a[mb] = op_from<BF16>(w);
  }
  const float col0 = row == 0 ? 1.0f : 0.0f;   // B operand entry: ones in column 0

  f32x16 gw2[2][2], gx[2];
  float gb3 = 0.f;
#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int r = 0; r < 16; ++r) gx[a][r] = 0.f;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) gw2[a][b][r] = 0.f;
  }
  // Two regions per wave, each [64 units][32 paths] plus [8 columns][32
  // paths], row stride kTs: two transposes share one store -> load round trip.
  FT* const T0 = tr + wave * 2 * kTr;
  FT* const T1 = T0 + kTr;
  FT* const TP0 = T0 + 64 * kTs;
  FT* const TP1 = T1 + 64 * kTs;
  // Unit-major A fragments of a region (32 units of block mb x 8 paths).
  auto a_frag = [&](const FT* T, int pk, int mb) {
    return op_lds<BF16>(&T[(32 * mb + row) * kTs + 16 * pk + 8 * half]);
  };
  // Units u(mb, r) and u(mb, r + 1), r even, are consecutive rows: in the
  // BF16 form one packed conversion makes both, stored as its low and high
  // halves.
  auto to_T = [&](FT* T, const float (&x)[32]) {
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int r = 0; r < 16; r += 2) {
        FT* t = &T[unit_of(mb, r, half) * kTs + row];
        if constexpr (BF16) {
          const bf16x2 p = __builtin_convertvector((float2_t){x[mb * 16 + r], x[mb * 16 + r + 1]},
                                                   bf16x2);
          t[0] = p[0];
          t[kTs] = p[1];
        } else {
          t[0] = x[mb * 16 + r];
          t[kTs] = x[mb * 16 + r + 1];
        }
      }
  };

  // A segment's cached features and price change are loaded one segment
  // ahead, so that their latency overlaps the segment before.
  float nf[4], ndst;
  // Row bases are uniform; the lane adds a 32-bit byte offset (the
  // launcher keeps the minibatch below 2^30 paths).
  const uint32_t ob = (uint32_t)pid * 4u;
  auto at = [&](const float* rowp) { return *(const float*)((const char*)rowp + ob); };
  auto fetch = [&](uint32_t k) {
    const uint64_t S = P.c_stride;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      nf[q] = (half == 0 && active) ? at(P.c_phi + ((size_t)k * 4 + q) * S + P.c_first) : 0.f;
    ndst = active ? at(P.c_dst + (size_t)k * S + P.c_first) : 0.f;
  };
  if (k0 < k1) fetch(k0);
  for (uint32_t k = k0; k < k1; ++k) {
    float h1[32], h2[32], phi[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) phi[q] = nf[q];
    phi[4] = (half == 0 && active) ? 1.0f : 0.f;
    phi[5] = phi[6] = phi[7] = 0.f;
    const float dSt = ndst;
    if (k + 1 < k1) fetch(k + 1);
    mlp_forward<BF16>(phi, w1a, s_w2f, s_lanec, lane, h1, h2);
    const float gD = g * dSt;                      // dL/dDelta for this segment
    const float gDh = 0.5f * gD;                   // the constants hold 2 W3
    if (half == 0) gb3 += gD;
    // delta2 = gD W3 (1 - h2^2).
    float d2v[32];
#pragma unroll
    for (int q = 0; q < 32; ++q)
      d2v[q] = gDh * s_lanec[64 * 32 + lanec_index(lane, q)] * (1.0f - h2[q] * h2[q]);
    // Round trip 1: H2 (with gD in column row 1) and delta2 become unit-major.
    to_T(T0, h2);
    if (half == 0) TP0[1 * kTs + row] = (FT)gD;
    to_T(T1, d2v);
    wave_lds_sync();
    // e1 = W2^T delta2 from registers while the stores land.
    f32x16 e1[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int r = 0; r < 16; ++r) e1[mb][r] = 0.f;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      float bf[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) bf[j] = d2v[(kb >> 1) * 16 + 8 * (kb & 1) + j];
      const Op8<BF16> b = op_from<BF16>(bf);
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
        mma16<BF16>(e1[mb], op_lds<BF16>(&s_w2tf[((mb * 4 + kb) * 64 + lane) * 8]), b);
    }
    // dW3 (column 1 of gx) += H2^T gD.
#pragma unroll
    for (int pk = 0; pk < 2; ++pk) {
      const Op8<BF16> b = row == 1 ? op_lds<BF16>(&TP0[1 * kTs + 16 * pk + 8 * half])
                                   : op_zero<BF16>();
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) mma16<BF16>(gx[mb], a_frag(T0, pk, mb), b);
    }
    // db2 (column 0 of gx) += delta2^T 1; delta2's fragments stay for dW2.
    Op8<BF16> A2[2][2];
    {
      float ones[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) ones[j] = col0;
      const Op8<BF16> b = op_from<BF16>(ones);
#pragma unroll
      for (int pk = 0; pk < 2; ++pk)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
          A2[pk][mb] = a_frag(T1, pk, mb);
          mma16<BF16>(gx[mb], A2[pk][mb], b);
        }
    }
    wave_lds_sync();
    // Round trip 2: H1 and delta1 = e1 (1 - h1^2) (with phi and the ones in
    // column rows 2..6) become unit-major.
    to_T(T0, h1);
    {
      float d1v[32];
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int q = mb * 16 + r;
          d1v[q] = e1[mb][r] * (1.0f - h1[q] * h1[q]);
        }
      to_T(T1, d1v);
    }
    if (half == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) TP1[(2 + q) * kTs + row] = (FT)phi[q];
      TP1[6 * kTs + row] = active ? (FT)1.0f : (FT)0.f;
    }
    wave_lds_sync();
    // dW2 += delta2^T H1.
#pragma unroll
    for (int pk = 0; pk < 2; ++pk)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const Op8<BF16> b = op_lds<BF16>(&T0[(32 * nb + row) * kTs + 16 * pk + 8 * half]);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) mma16<BF16>(gw2[mb][nb], A2[pk][mb], b);
      }
    // dW1 and db1 (columns 2..6 of gx) += delta1^T [phi, 1].
#pragma unroll
    for (int pk = 0; pk < 2; ++pk) {
      const Op8<BF16> b = (row >= 2 && row <= 6)
                              ? op_lds<BF16>(&TP1[row * kTs + 16 * pk + 8 * half])
                              : op_zero<BF16>();
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) mma16<BF16>(gx[mb], a_frag(T1, pk, mb), b);
    }
    wave_lds_sync();
  }

  // The block's gradient, in the flat parameter layout W1[64][4], b1[64],
  // W2[64][64], b2[64], W3[64], b3: every wave stores its FP32 accumulators
  // into a row of its own (each slot has one writer per wave; b3's wave sum
  // is FP64 and has a slot of its own), and after one barrier each thread
  // adds the waves' values of its parameters in wave order in FP64 (the
  // conversions are exact), so no wave waits on another's read-modify-write
  // of LDS. The block writes one partial per parameter, rounded to FP32 (the
  // precision of the accumulators it sums; the cross-block sum is FP64).
  float* red = (float*)lds;            // [kCvWaves][kMlpNParam]
  __shared__ double s3w[kCvWaves];
  __syncthreads();                     // every wave has left the segment loop
  {
    float* mine = red + wave * kMlpNParam;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          mine[320 + unit_of(mb, r, half) * 64 + 32 * nb + row] = gw2[mb][nb][r];
    // gx: lane column `row`, unit u(mb, r, half), at slot base + u * step:
    // b2 (column 0), W3 (1), W1 (2..5, one input each), b1 (6).
    if (row <= 6) {
      const int base = row == 0 ? 4416 : row == 1 ? 4480 : row <= 5 ? row - 2 : 256;
      const int step = (row >= 2 && row <= 5) ? 4 : 1;
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int r = 0; r < 16; ++r) mine[base + unit_of(mb, r, half) * step] = gx[mb][r];
    }
    const double s3 = wave_sum((double)gb3);
    if (lane == 0) s3w[wave] = s3;
  }
  __syncthreads();
  // Block-major: the block's 4545 partials are one row (padded to whole
  // 128-byte lines).
  for (int i = threadIdx.x; i < kMlpNParam; i += kCvThreads) {
    double acc = i == kMlpNParam - 1 ? s3w[0] : (double)red[i];
#pragma unroll
    for (int w = 1; w < kCvWaves; ++w)
      acc += i == kMlpNParam - 1 ? s3w[w] : (double)red[w * kMlpNParam + i];
    P.grad_partials[(uint64_t)blockIdx.x * kGradStride + i] = (float)acc;
  }
}

// The BF16 form fits two waves per SIMD (256 VGPRs; 77 KB of LDS, two
// workgroups per CU); the FP32 form's 130 KB allow one workgroup per CU.
__global__ __launch_bounds__(kCvThreads) __attribute__((amdgpu_waves_per_eu(2))) void
cv_bwd_kernel_bf16(const CvParams P) {
  cv_bwd_body<true>(P);
}

__global__ __launch_bounds__(kCvThreads) void cv_bwd_kernel_fp32(const CvParams P) {
  cv_bwd_body<false>(P);
}

// Evaluation kernel, 64 paths per wave: lane l follows its own path, and
// at each rebalancing date the network runs twice, for the sub-tiles of
// paths 0..31 and 32..63 of the wave. Layer 1 takes its features from half 0
// of the lanes, so for the second sub-tile half 0 fetches the features of
// its partner lane (l ^ 32); each lane then keeps Delta of its own sub-tile.
// A path's network output depends only on its own MFMA column, so it is the
// same function the training kernel evaluates.
template <bool BF16>
__global__ __launch_bounds__(kCvThreads) void cv_eval_kernel(const CvParams P) {
  using FT = FragT<BF16>;
  __shared__ __attribute__((aligned(16))) FT s_w2f[kFragFloats];
  __shared__ __attribute__((aligned(16))) float s_lanec[kLaneFloats];
  const HestonParams& Hp = P.h;
  {
    WeightRegs wr;
    weights_load<false>(P.w2f, nullptr, P.lanec, wr);
    weights_store<false>(wr, s_w2f, (FT*)nullptr, s_lanec);
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int half = lane >> 5;
  Op8<BF16> w1a[2];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb) {
    float w[8];
    load8(&P.w1f[(mb * 64 + lane) * 8], w);
    w1a[mb] = op_from<BF16>(w);
  }
  const float c3 = out_const(P.theta);

  const HestonF c(Hp);
  const float S0 = c.S0;
  const uint32_t n = Hp.n_steps, m = P.hedge_every;
  const uint64_t pid = ((uint64_t)blockIdx.x * kCvWaves + wave) * 64 + lane;
  const bool active = pid < Hp.n_paths;
  const PathCounter pc = make_counter(Hp.path_offset + pid, Hp.tag, Hp.k0, Hp.k1);

  float z = 0.f, v = (float)Hp.v0, sumE = 0.f, H = 0.f, delta = 0.f, st_open = 0.f, Et = 1.f;
  Normals4<float> nz;
  for (uint32_t i = 0; i < n; ++i) {
    if (i % m == 0) {
      float own[4];
      c.features(i, z, v, sumE, own);
      float other[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) other[f] = __shfl_xor(own[f], 32, 64);
#pragma unroll 1
      for (int sub = 0; sub < 2; ++sub) {
        float phi[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) phi[j] = 0.f;
        if (half == 0) {
#pragma unroll
          for (int f = 0; f < 4; ++f) phi[f] = sub == 0 ? own[f] : other[f];
          phi[4] = 1.0f;
        }
        const float d = mlp_delta<BF16>(phi, w1a, s_w2f, s_lanec, lane, c3);
        if (sub == half) delta = d;
      }
      st_open = Et;
    }
    if ((i & 1) == 0) nz = normals4<float>(philox(i >> 1, pc));
    const float Z1 = (i & 1) ? nz.z[2] : nz.z[0];
    const float Z2 = (i & 1) ? nz.z[3] : nz.z[1];
    c.step(z, v, Z1, Z2);
    Et = __builtin_amdgcn_exp2f(z);
    sumE += Et * P.dfac[i + 1];
    if ((i + 1) % m == 0 || i + 1 == n) H = __builtin_fmaf(delta, S0 * (Et - st_open), H);
  }
  double y[3] = {0.0, 0.0, 0.0};
  if (active) {
    const double A = (double)S0 * (double)sumE / (double)n;
    const double pay = Hp.disc * (A > Hp.K ? A - Hp.K : 0.0);
    y[0] = pay;
    y[1] = (double)H;
    y[2] = pay - (double)H;
  }
  const bool finite = isfinite(y[0]) && isfinite(y[1]) && isfinite(y[2]);
  if (active && P.path_out != nullptr) {
#pragma unroll
    for (int q = 0; q < 3; ++q) P.path_out[pid * 3 + q] = y[q];
  }
  block_moments<3, kCvThreads>(y, active && finite, active && !finite, P.partials);
}

// Builds the per-lane fragments from the flat weights (one thread per
// output float). Units: u(mb, r, h) as above; layer-2 k-slot (kb, h, j) is
// the layer-1 unit u(kb/2, 8 (kb mod 2) + j, h).
__global__ void cv_pack_kernel(const float* __restrict__ th, float* __restrict__ w1f,
                               float* __restrict__ w2f, float* __restrict__ w2tf,
                               float* __restrict__ lanec) {
  const float* W1 = th;
  const float* b1 = th + 256;
  const float* W2 = th + 320;
  const float* b2 = th + 4416;
  const float* W3 = th + 4480;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < kW1fFloats) {
    const int j = t & 7, lane = (t >> 3) & 63, mb = t >> 9;
    const int row = lane & 31, h = lane >> 5, u = 32 * mb + row;
    w1f[t] = (h == 0 && j < 4) ? W1[u * 4 + j] : (h == 0 && j == 4) ? b1[u] : 0.f;
  }
  if (t < kW2fFloats) {
    const int j = t & 7, lane = (t >> 3) & 63, kb = (t >> 9) & 3, mb = t >> 11;
    const int row = lane & 31, h = lane >> 5;
    const int k_unit = unit_of(kb >> 1, 8 * (kb & 1) + j, h);
    w2f[t] = W2[(32 * mb + row) * 64 + k_unit];
    w2tf[t] = W2[k_unit * 64 + (32 * mb + row)];
  }
  if (t < kLanecFloats / 2) {
    const int q = ((t >> 8) << 2) | (t & 3), lane = (t >> 2) & 63;   // t = lanec_index(lane, q)
    const int h = lane >> 5, mb = q >> 4, r = q & 15;
    const int u = unit_of(mb, r, h);
    lanec[t] = b2[u] * kNeg2Log2e;
    lanec[kLanecFloats / 2 + t] = 2.0f * W3[u];
  }
}

// Inverse of unit_of: the fragment slot (mb, r, h) that holds hidden unit u.
__device__ __forceinline__ void slot_of(int u, int& mb, int& r, int& h) {
  mb = u >> 5;
  const int q = u & 31;
  h = (q >> 2) & 1;
  r = 4 * (q >> 3) + (q & 3);
}

// Gradient reduction of the block-major partials [n_blocks][kGradStride]:
// a block of kGradThreads threads takes kGradCols consecutive parameters
// (32 FP32 partials of a row are one 128-byte line); thread (slice s,
// column p) adds blocks s, s + kGradSlices, ... in order in FP64, then
// slice 0 adds the slices in order. With ADAM, the same thread then takes
// one Adam step on (theta, m, v) with the bias corrections c1 = 1 - b1^t,
// c2 = 1 - b2^t, and the block writes the new values into each fragment
// slot that cv_pack_kernel gives the parameter (W1, b1: one; W2: one in
// each of the two layouts; b2, W3: the 32 lanes of a half-wave). Padding
// slots keep the zeros of the first pack; b3 lives in theta only.
constexpr int kGradThreads = 512, kGradCols = 32, kGradSlices = kGradThreads / kGradCols;
constexpr int kGradBlocks = (kMlpNParam + kGradCols - 1) / kGradCols;

template <bool ADAM>
__global__ __launch_bounds__(kGradThreads) void grad_adam_kernel(
    const float* __restrict__ partials, uint32_t n_blocks, double* __restrict__ grad,
    float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v, float lr, float b1,
    float b2, float eps, float c1, float c2, float* __restrict__ w1f, float* __restrict__ w2f,
    float* __restrict__ w2tf, float* __restrict__ lanec, const double* __restrict__ vpart,
    uint32_t vblocks, double* __restrict__ vmom) {
  if (blockIdx.x == kGradBlocks) {
    // The extra workgroup: the fixed-order merge of the hedged values'
    // block moments (the minibatch's loss), beside the reduction.
    PartSums<3> pm;
    pm.zero();
    for (uint32_t i = threadIdx.x; i < vblocks; i += kGradThreads)
      pm.add_vector(vpart + (size_t)i * PartSums<3>::M);
    block_reduce<3, kGradThreads>(pm, vmom, 0);
    return;
  }
  __shared__ double sh[kGradSlices][kGradCols];
  __shared__ float th_new[kGradCols];
  const int col = threadIdx.x % kGradCols, slice = threadIdx.x / kGradCols;
  const int p0 = blockIdx.x * kGradCols;
  const int i = p0 + col;
  double s = 0.0;
  if (i < kMlpNParam) {
#pragma unroll 8
    for (uint32_t k = slice; k < n_blocks; k += kGradSlices)
      s += partials[(size_t)k * kGradStride + i];
  }
  sh[slice][col] = s;
  __syncthreads();
  if (slice == 0 && i < kMlpNParam) {
    double g = 0.0;
#pragma unroll
    for (int q = 0; q < kGradSlices; ++q) g += sh[q][col];
    grad[i] = g;
    if constexpr (ADAM) {
      const float gr = (float)g;
      const float mi = b1 * m[i] + (1.0f - b1) * gr;
      const float vi = b2 * v[i] + (1.0f - b2) * gr * gr;
      m[i] = mi;
      v[i] = vi;
      const float t = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
      theta[i] = t;
      th_new[col] = t;
    }
  }
  if constexpr (!ADAM) return;
  __syncthreads();
  // Fragment slots: up to 32 per parameter (b2, W3), kGradCols parameters.
  for (int e = threadIdx.x; e < kGradCols * 32; e += kGradThreads) {
    const int c = e >> 5, L = e & 31, ip = p0 + c;
    if (ip >= kMlpNParam) continue;
    const float t = th_new[c];
    if (ip < 320) {                       // W1 [64][4] and b1 [64]: lane = unit row, h = 0
      if (L == 0) {
        const int u = ip < 256 ? ip >> 2 : ip - 256, j = ip < 256 ? (ip & 3) : 4;
        w1f[(u >> 5) * 512 + (u & 31) * 8 + j] = t;
      }
    } else if (ip < 4416) {               // W2 [64 out][64 in]
      if (L < 2) {
        const int q = ip - 320;
        const int a = L == 0 ? q >> 6 : q & 63;   // fragment row
        const int k = L == 0 ? q & 63 : q >> 6;   // k-slot unit
        int mb, r, h;
        slot_of(k, mb, r, h);
        const int dst = (a >> 5) * 2048 + (2 * mb + (r >> 3)) * 512 + ((a & 31) + 32 * h) * 8 + (r & 7);
        (L == 0 ? w2f : w2tf)[dst] = t;
      }
    } else if (ip < 4544) {               // b2 [64] (scaled) and W3 [64]
      const bool is_b2 = ip < 4480;
      const int u = is_b2 ? ip - 4416 : ip - 4480;
      int mb, r, h;
      slot_of(u, mb, r, h);
      const int dst = lanec_index(32 * h + L, 16 * mb + r);
      if (is_b2)
        lanec[dst] = t * kNeg2Log2e;
      else
        lanec[kLanecFloats / 2 + dst] = 2.0f * t;
    }
  }
}

}  // namespace

hipError_t launch_cv_pack(const float* theta, float* w1f, float* w2f, float* w2tf, float* lanec,
                          hipStream_t s) {
  hipLaunchKernelGGL(cv_pack_kernel, dim3(kW2fFloats / 256), dim3(256), 0, s, theta, w1f, w2f,
                     w2tf, lanec);
  return hipGetLastError();
}

hipError_t launch_cv_price(const CvParams& p, hipStream_t s, uint32_t* n_blocks) {
  const uint32_t nb = (uint32_t)((p.h.n_paths + kCvPathsPerBlock - 1) / kCvPathsPerBlock);
  *n_blocks = nb;
  if (p.bf16)
    hipLaunchKernelGGL((cv_eval_kernel<true>), dim3(nb), dim3(kCvThreads), 0, s, p);
  else
    hipLaunchKernelGGL((cv_eval_kernel<false>), dim3(nb), dim3(kCvThreads), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_cv_cache(const CvParams& p, hipStream_t s) {
  const uint32_t nb = (uint32_t)((p.h.n_paths + kCvThreads - 1) / kCvThreads);
  if (nb == 0 || p.n_seg == 0 || p.h.n_paths > p.c_stride) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cv_cache_kernel, dim3(nb), dim3(kCvThreads), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_cv_values(const CvParams& p, hipStream_t s, uint32_t* n_blocks) {
  CvParams q = p;
  const uint32_t nb = cv_values_blocks(p.h.n_paths, p.n_seg, &q.seg_split);
  *n_blocks = nb;
  if (nb == 0 || p.n_seg == 0 || p.c_first + p.h.n_paths > p.c_stride ||
      p.h.n_paths >= (1ull << 30))
    return hipErrorInvalidValue;
  if (p.bf16)
    hipLaunchKernelGGL((cv_values_kernel<true>), dim3(nb), dim3(kCvThreads), 0, s, q);
  else
    hipLaunchKernelGGL((cv_values_kernel<false>), dim3(nb), dim3(kCvThreads), 0, s, q);
  return hipGetLastError();
}

// A small minibatch has too few 32-path tiles to keep every SIMD busy; its
// tiles' segments are then split over two or four waves, which run side by
// side. Each extra workgroup adds its own prologue (weights, Ybar) and
// gradient row, so the backward splits less than the hedged values do
// (measured, 2^14 to 2^16 paths: per Adam step, two waves per tile beat
// four at 512 tiles and one at 1024).
static uint32_t tile_split(uint64_t tiles, uint32_t n_seg, uint64_t four_upto) {
  uint32_t sp = tiles <= four_upto ? 4 : tiles <= 1024 ? 2 : 1;
  while (sp > 1 && sp > n_seg) sp >>= 1;
  return sp;
}

uint32_t cv_bwd_blocks(uint64_t n_paths, uint32_t n_seg, uint32_t* split) {
  const uint64_t tiles = (n_paths + 31) / 32;
  const uint32_t sp = tile_split(tiles, n_seg, 256);
  if (split) *split = sp;
  const uint32_t tiles_per_block = kCvWaves / sp;
  return (uint32_t)((tiles + tiles_per_block - 1) / tiles_per_block);
}

// The hedged values split a tile's segments while each wave's share fits
// its LDS slab (the tile's first wave then sums them in order).
uint32_t cv_values_blocks(uint64_t n_paths, uint32_t n_seg, uint32_t* split) {
  const uint64_t tiles = (n_paths + 31) / 32;
  uint32_t sp = tile_split(tiles, n_seg, 512);
  if (sp > 1 && (n_seg + sp - 1) / sp > (uint32_t)kCvValSlab) sp = 1;
  if (split) *split = sp;
  const uint32_t tiles_per_block = kCvWaves / sp;
  return (uint32_t)((tiles + tiles_per_block - 1) / tiles_per_block);
}

hipError_t launch_cv_backward(const CvParams& p, hipStream_t s, uint32_t* n_blocks) {
  CvParams q = p;
  const uint32_t nb = cv_bwd_blocks(p.h.n_paths, p.n_seg, &q.seg_split);
  *n_blocks = nb;
  if (nb == 0 || p.n_seg == 0 || p.c_first + p.h.n_paths > p.c_stride ||
      p.h.n_paths >= (1ull << 30))
    return hipErrorInvalidValue;
  if (p.bf16)
    hipLaunchKernelGGL(cv_bwd_kernel_bf16, dim3(nb), dim3(kCvThreads), 0, s, q);
  else
    hipLaunchKernelGGL(cv_bwd_kernel_fp32, dim3(nb), dim3(kCvThreads), 0, s, q);
  return hipGetLastError();
}

hipError_t launch_adam_pack(const float* partials, uint32_t n_blocks, const CvValMoments& vm,
                            double* grad, float* theta, float* m, float* v, int t, double lr,
                            double b1, double b2, double eps, float* w1f, float* w2f, float* w2tf,
                            float* lanec, hipStream_t s) {
  if (n_blocks == 0 || vm.n_blocks == 0 || vm.partials == nullptr || vm.out == nullptr)
    return hipErrorInvalidValue;
  const float c1 = (float)(1.0 - std::pow(b1, t)), c2 = (float)(1.0 - std::pow(b2, t));
  hipLaunchKernelGGL(grad_adam_kernel<true>, dim3(kGradBlocks + 1), dim3(kGradThreads), 0, s, partials,
                     n_blocks, grad, theta, m, v, (float)lr, (float)b1, (float)b2, (float)eps, c1,
                     c2, w1f, w2f, w2tf, lanec, vm.partials, vm.n_blocks, vm.out);
  return hipGetLastError();
}

hipError_t launch_grad_sum(const float* partials, uint32_t n_blocks, const CvValMoments& vm,
                           double* grad, hipStream_t s) {
  if (n_blocks == 0 || vm.n_blocks == 0 || vm.partials == nullptr || vm.out == nullptr)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(grad_adam_kernel<false>, dim3(kGradBlocks + 1), dim3(kGradThreads), 0, s, partials,
                     n_blocks, grad, nullptr, nullptr, nullptr, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f,
                     nullptr, nullptr, nullptr, nullptr, vm.partials, vm.n_blocks, vm.out);
  return hipGetLastError();
}

}  // namespace mcp
