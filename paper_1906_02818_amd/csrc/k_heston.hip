// Heston path kernels: full-truncation Euler on (ln S, v), the stochastic-
// volatility form of the Euler-Maruyama scheme (Sec. I-A.1, Sec. II-A.1):
//   v+ = max(v, 0)
//   ln S += (r - v+/2) dt + sqrt(v+ dt) Zs,   Zs = rho Z1 + sqrt(1-rho^2) Z2
//   v    += kappa (theta - v+) dt + xi sqrt(v+ dt) Z1
// Step i uses normals 2i (Z1, the variance driver) and 2i+1 (Z2), so one
// Philox block feeds two steps.
//
// Two kernels:
//  - heston_price_kernel: European and arithmetic-Asian payoffs fused with
//    the block moments (Eq. 3); heston_tangent_kernel: the same with
//    forward-mode delta and d/dv0.
//  - heston_adjoint_kernel: pathwise delta and d/dv0 by reverse-mode
//    differentiation of the simulation (greeks by back-propagation,
//    Sec. I-A.3). The forward sweep stores (ln S, v) every `every` steps
//    (LDS when forward and reverse run in one launch, else a device buffer);
//    the reverse sweep takes the segments from last to first, recomputes
//    each from its checkpoint (regenerating the normals from Philox) with
//    its intermediate states in registers, and back-propagates through it.
#include "device/reduce.h"
#include "device/rng.h"
#include "mc_internal.h"

namespace mcp {
namespace {

template <typename R>
struct HDom;
template <>
struct HDom<float> {
  static constexpr double kLogScale = 1.4426950408889634;  // ln S -> log2 S
  static __device__ __forceinline__ float exp_(float z) { return __builtin_amdgcn_exp2f(z); }
  static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
  static __device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
};
template <>
struct HDom<double> {
  static constexpr double kLogScale = 1.0;
  static __device__ __forceinline__ double exp_(double z) { return exp(z); }
  static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
  static __device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }
};

// z = log(S/S0) in the kernel's domain, v the variance.
template <typename R>
struct HestonStep {
  R a0, a1, a2, kdt, kthdt, xi, rho, rhoc, dt;

  __device__ __forceinline__ void init(const HestonParams& P) {
    const double sc = HDom<R>::kLogScale;
    a0 = (R)(P.r * P.dt * sc);
    a1 = (R)(-0.5 * P.dt * sc);
    a2 = (R)sc;
    kdt = (R)(P.kappa * P.dt);
    kthdt = (R)(P.kappa * P.theta * P.dt);
    xi = (R)P.xi;
    rho = (R)P.rho;
    rhoc = (R)P.rho_c;
    dt = (R)P.dt;
  }

  __device__ __forceinline__ void step(R& z, R& v, R Z1, R Z2, R& Zs) const {
    const R vp = v > R(0) ? v : R(0);
    const R sq = HDom<R>::sqrt_(vp * dt);
    Zs = rho * Z1 + rhoc * Z2;
    z = z + (a0 + a1 * vp) + a2 * (sq * Zs);
    v = v + (kthdt - kdt * vp) + xi * (sq * Z1);
  }
};

template <typename R>
__device__ __forceinline__ R posv(R x) {
  return x > R(0) ? x : R(0);
}

// Persistent grid (at most kHestonMaxBlocks workgroups): each thread prices
// paths pid, pid + stride, ... and keeps their moments in registers.
template <typename R, uint32_t MASK>
__global__ __launch_bounds__(kBlock) void heston_price_kernel(const HestonParams P) {
  constexpr int C = popcount_c(MASK);
  ThreadSums<C> acc;
  acc.zero();
  HestonStep<R> hs;
  hs.init(P);
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t pid = (uint64_t)blockIdx.x * kBlock + threadIdx.x; pid < P.n_paths;
       pid += stride) {
    double y[C];
    const PathCounter pc = make_counter(P.path_offset + pid, P.tag, P.k0, P.k1);
    R z = R(0), v = (R)P.v0, sumE = R(0), Zs;
    const uint32_t n = P.n_steps;
    for (uint32_t j = 0; 2 * j < n; ++j) {
      const Normals4<R> nz = normals4<R>(philox(j, pc));
      hs.step(z, v, nz.z[0], nz.z[1], Zs);
      if constexpr ((MASK & H_ASIAN) != 0) sumE += HDom<R>::exp_(z);
      if (2 * j + 1 < n) {
        hs.step(z, v, nz.z[2], nz.z[3], Zs);
        if constexpr ((MASK & H_ASIAN) != 0) sumE += HDom<R>::exp_(z);
      }
    }
    const R S0 = (R)P.S0, K = (R)P.K, disc = (R)P.disc;
    int c = 0;
    if constexpr ((MASK & H_EURO) != 0) y[c++] = (double)(disc * posv(S0 * HDom<R>::exp_(z) - K));
    if constexpr ((MASK & H_ASIAN) != 0) y[c++] = (double)(disc * posv(S0 * sumE / (R)n - K));
    bool finite = true;
#pragma unroll
    for (int q = 0; q < C; ++q) finite = finite && isfinite(y[q]);
    if (P.path_out != nullptr) {
#pragma unroll
      for (int q = 0; q < C; ++q) P.path_out[pid * C + q] = y[q];
    }
    acc.push(y, finite, !finite);
  }
  PartSums<C> part = acc.part();
  block_reduce<C, kBlock>(part, P.partials, blockIdx.x);
}

// Pathwise delta and d/dv0 in forward mode: the tangents (dz, dv) of the
// state with respect to v0 ride along the step (the derivative of
// sqrt(v+ dt) is taken as 0 where v <= 0), and d/dS0 needs none (z does not
// depend on S0). Two inputs, so this is cheaper than the reverse sweep: no
// checkpoints and no recomputation. Channels: payoff, delta, d/dv0 of the
// European (ASIAN = false) or arithmetic-Asian call.
template <typename R, bool ASIAN>
__global__ __launch_bounds__(kBlock) void heston_tangent_kernel(const HestonParams P) {
  ThreadSums<3> acc;
  acc.zero();
  HestonStep<R> hs;
  hs.init(P);
  const R half_dt = R(0.5) * hs.dt;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t pid = (uint64_t)blockIdx.x * kBlock + threadIdx.x; pid < P.n_paths;
       pid += stride) {
    double y[3];
    const PathCounter pc = make_counter(P.path_offset + pid, P.tag, P.k0, P.k1);
    R z = R(0), v = (R)P.v0, dz = R(0), dv = R(1), sumE = R(0), sumEd = R(0);
    const uint32_t n = P.n_steps;
    auto step = [&](R Z1, R Z2) {
      const R vp = v > R(0) ? v : R(0);
      const R dvp = v > R(0) ? dv : R(0);
      // d sqrt(vp dt) = dt dvp / (2 sqrt(vp dt)); 0 where vp = 0.
      const R dsq = vp > R(0) ? half_dt * dvp * HDom<R>::rsqrt_(vp * hs.dt) : R(0);
      const R Zs = hs.rho * Z1 + hs.rhoc * Z2;
      const R dz_new = dz + hs.a1 * dvp + hs.a2 * (dsq * Zs);
      const R dv_new = dv - hs.kdt * dvp + hs.xi * (dsq * Z1);
      R zs;
      hs.step(z, v, Z1, Z2, zs);
      dz = dz_new;
      dv = dv_new;
      if constexpr (ASIAN) {
        const R E = HDom<R>::exp_(z);
        sumE += E;
        sumEd += E * dz;
      }
    };
    for (uint32_t j = 0; 2 * j < n; ++j) {
      const Normals4<R> nz = normals4<R>(philox(j, pc));
      step(nz.z[0], nz.z[1]);
      if (2 * j + 1 < n) step(nz.z[2], nz.z[3]);
    }
    // z and dz are in the kernel's log domain (log2 for FP32): d exp(x) =
    // exp(x) dz / scale.
    const double S0 = P.S0, K = P.K, disc = P.disc, inv_sc = 1.0 / HDom<R>::kLogScale;
    if constexpr (ASIAN) {
      const double A = S0 * (double)sumE / (double)n;
      y[0] = disc * (A > K ? A - K : 0.0);
      y[1] = A > K ? disc * A / S0 : 0.0;
      y[2] = A > K ? disc * S0 * inv_sc * (double)sumEd / (double)n : 0.0;
    } else {
      const double ST = S0 * (double)HDom<R>::exp_(z);
      y[0] = disc * (ST > K ? ST - K : 0.0);
      y[1] = ST > K ? disc * ST / S0 : 0.0;
      y[2] = ST > K ? disc * ST * inv_sc * (double)dz : 0.0;
    }
    const bool finite = isfinite(y[0]) && isfinite(y[1]) && isfinite(y[2]);
    if (P.path_out != nullptr) {
#pragma unroll
      for (int c = 0; c < 3; ++c) P.path_out[pid * 3 + c] = y[c];
    }
    acc.push(y, finite, !finite);
  }
  PartSums<3> part = acc.part();
  block_reduce<3, kBlock>(part, P.partials, blockIdx.x);
}

// Channel sets of the adjoint phases.
template <int PHASE>
struct AdjC;
template <>
struct AdjC<0> { static constexpr int C = 3; };   // payoff, delta, d/dv0
template <>
struct AdjC<1> { static constexpr int C = 1; };   // payoff
template <>
struct AdjC<2> { static constexpr int C = 2; };   // delta, d/dv0

// Checkpoints (FP32): rows [2c] = z and [2c+1] = v at step c*every, then,
// in the device buffer, one row with the terminal statistic (A/S0 for the
// Asian, S_T/S0 otherwise). FULL mode with at most kLdsCkpt checkpoints
// keeps them in LDS ([row][thread], one thread's column per path, so no
// barrier is needed); otherwise, and for the FWD/REV split behind autograd,
// they live in the device buffer ([row][path]). Only the FP32 kernel is
// built: its state is FP32, so the checkpoints are exact.
template <typename R, int PHASE, bool ASIAN, bool LDS>
__global__ __launch_bounds__(kBlock) void heston_adjoint_kernel(const AdjointParams A) {
  constexpr int C = AdjC<PHASE>::C;
  extern __shared__ float s_ck[];
  const HestonParams& P = A.h;
  const uint64_t pid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = pid < P.n_paths;
  const uint64_t np = P.n_paths;
  auto ck_store = [&](uint32_t row, R x) {
    if constexpr (LDS)
      s_ck[row * kBlock + threadIdx.x] = (float)x;
    else
      A.ckpt[(size_t)row * np + pid] = (float)x;
  };
  auto ck_load = [&](uint32_t row) -> R {
    if constexpr (LDS)
      return (R)s_ck[row * kBlock + threadIdx.x];
    else
      return (R)A.ckpt[(size_t)row * np + pid];
  };
  double y[C];
#pragma unroll
  for (int c = 0; c < C; ++c) y[c] = 0.0;
  if (active) {
    HestonStep<R> hs;
    hs.init(P);
    const PathCounter pc = make_counter(P.path_offset + pid, P.tag, P.k0, P.k1);
    const uint32_t n = P.n_steps, every = A.every;   // every: even, 2..kCkptMax
    const R S0 = (R)P.S0, K = (R)P.K, disc = (R)P.disc, inv_n = R(1) / (R)n;
    R term;  // A/S0 (Asian) or S_T/S0
    if (PHASE != 2) {
      // Forward sweep, storing (z, v) at the start of every segment.
      R z = R(0), v = (R)P.v0, sumE = R(0), Zs;
      for (uint32_t i0 = 0, seg = 0; i0 < n; i0 += every, ++seg) {
        ck_store(2 * seg, z);
        ck_store(2 * seg + 1, v);
        const uint32_t len = min(every, n - i0);
        for (uint32_t q = 0; q < len; q += 2) {
          const Normals4<R> nz = normals4<R>(philox((i0 + q) >> 1, pc));
          hs.step(z, v, nz.z[0], nz.z[1], Zs);
          if (ASIAN) sumE += HDom<R>::exp_(z);
          if (q + 1 < len) {
            hs.step(z, v, nz.z[2], nz.z[3], Zs);
            if (ASIAN) sumE += HDom<R>::exp_(z);
          }
        }
      }
      term = ASIAN ? sumE * inv_n : HDom<R>::exp_(z);
      if (PHASE == 1) A.ckpt[(size_t)(2 * A.n_ckpt) * np + pid] = (float)term;
      const R pay = disc * posv(S0 * term - K);
      if (PHASE == 0) y[0] = (double)pay;
      if (PHASE == 1) y[0] = (double)pay;
    } else {
      term = (R)A.ckpt[(size_t)(2 * A.n_ckpt) * np + pid];
    }
    if (PHASE != 1) {
      // Reverse sweep. xb = dP/d(ln S_i), vb = dP/dv_i, natural-log units,
      // accumulated in FP64: under a violated Feller condition the factor
      // dv_{i+1}/dv_i = 1 - kappa dt + xi Z1 dt / (2 sqrt(v dt)) can reach
      // 10^3 near v = 0, and products of such factors overflow FP32.
      const bool itm = S0 * term > K;
      // Asian: dP/d(ln S_i) = disc 1{A>K} S_i / n = abar * (S_i/S0).
      const double abar = (ASIAN && itm) ? (double)(disc * S0 * inv_n) : 0.0;
      double xb = (!ASIAN && itm) ? (double)(disc * S0 * term) : 0.0;
      double vb = 0.0;
      const R dt = hs.dt, half_dt = R(0.5) * hs.dt, kdt = hs.kdt, xi = hs.xi;
      const uint32_t n_seg = (n + every - 1) / every;
      for (int seg = (int)n_seg - 1; seg >= 0; --seg) {
        const uint32_t i0 = (uint32_t)seg * every;
        const uint32_t len = min(every, n - i0);
        // The checkpoint holds the FP32 state exactly, so the recomputed
        // segment reproduces the forward sweep bit for bit.
        R z = ck_load(2 * seg);
        R v = ck_load(2 * seg + 1);
        R vs[kCkptMax], z1s[kCkptMax], zss[kCkptMax], Es[kCkptMax];
#pragma unroll
        for (int q = 0; q < kCkptMax; q += 2) {
          if ((uint32_t)q < len) {
            const Normals4<R> nz = normals4<R>(philox((i0 + (uint32_t)q) >> 1, pc));
            vs[q] = v;
            z1s[q] = nz.z[0];
            hs.step(z, v, nz.z[0], nz.z[1], zss[q]);
            Es[q] = HDom<R>::exp_(z);
            if ((uint32_t)q + 1 < len) {
              vs[q + 1] = v;
              z1s[q + 1] = nz.z[2];
              hs.step(z, v, nz.z[2], nz.z[3], zss[q + 1]);
              Es[q + 1] = HDom<R>::exp_(z);
            }
          }
        }
#pragma unroll
        for (int q = kCkptMax - 1; q >= 0; --q) {
          if ((uint32_t)q < len) {
            if (ASIAN) xb += abar * (double)Es[q];   // S_{i+1} enters the average
            const R vq = vs[q];
            if (vq > R(0)) {
              const R g = half_dt * HDom<R>::rsqrt_(vq * dt);   // d sqrt(v dt) / dv
              const double dxdv = (double)(-half_dt + zss[q] * g);
              const double dvdv = (double)((R(1) - kdt) + xi * z1s[q] * g);
              vb = xb * dxdv + vb * dvdv;
            }
          }
        }
      }
      const int c0 = PHASE == 0 ? 1 : 0;
      y[c0] = xb / (double)P.S0;   // d/dS0 through ln S0
      y[c0 + 1] = vb;              // d/dv0
    }
  }
  bool finite = true;
#pragma unroll
  for (int c = 0; c < C; ++c) finite = finite && isfinite(y[c]);
  if (active && P.path_out != nullptr) {
#pragma unroll
    for (int c = 0; c < C; ++c) P.path_out[pid * C + c] = y[c];
  }
  block_moments<C, kBlock>(y, active && finite, active && !finite, P.partials);
}

}  // namespace

uint32_t heston_blocks(uint64_t n_paths) {
  const uint64_t need = (n_paths + kBlock - 1) / kBlock;
  return (uint32_t)(need < kHestonMaxBlocks ? need : kHestonMaxBlocks);
}

hipError_t launch_heston(const HestonParams& p, uint32_t mask, bool fp64, hipStream_t s,
                         uint32_t* n_blocks) {
  const uint32_t nb = heston_blocks(p.n_paths);
  *n_blocks = nb;
  constexpr uint32_t EA = H_EURO | H_ASIAN;
  if (mask != EA) return hipErrorInvalidValue;
  if (fp64)
    hipLaunchKernelGGL((heston_price_kernel<double, EA>), dim3(nb), dim3(kBlock), 0, s, p);
  else
    hipLaunchKernelGGL((heston_price_kernel<float, EA>), dim3(nb), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_heston_tangent(const HestonParams& p, bool asian, bool fp64, hipStream_t s,
                                 uint32_t* n_blocks) {
  const uint32_t nb = heston_blocks(p.n_paths);
  *n_blocks = nb;
  if (nb == 0) return hipErrorInvalidValue;
  if (fp64) {
    if (asian)
      hipLaunchKernelGGL((heston_tangent_kernel<double, true>), dim3(nb), dim3(kBlock), 0, s, p);
    else
      hipLaunchKernelGGL((heston_tangent_kernel<double, false>), dim3(nb), dim3(kBlock), 0, s, p);
  } else {
    if (asian)
      hipLaunchKernelGGL((heston_tangent_kernel<float, true>), dim3(nb), dim3(kBlock), 0, s, p);
    else
      hipLaunchKernelGGL((heston_tangent_kernel<float, false>), dim3(nb), dim3(kBlock), 0, s, p);
  }
  return hipGetLastError();
}

template <typename R, int PH, bool AS, bool LDS>
static hipError_t adj_one(const AdjointParams& a, hipStream_t s, uint32_t nb) {
  const size_t lds = LDS ? (size_t)2 * a.n_ckpt * kBlock * sizeof(float) : 0;
  hipLaunchKernelGGL((heston_adjoint_kernel<R, PH, AS, LDS>), dim3(nb), dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

// One path per thread: the sweep's registers leave no room for moment
// accumulators across paths at this occupancy.
hipError_t launch_heston_adjoint(const AdjointParams& a, hipStream_t s, uint32_t* n_blocks) {
  const uint32_t nb = (uint32_t)((a.h.n_paths + kBlock - 1) / kBlock);
  *n_blocks = nb;
  if (a.every < 2 || a.every > (uint32_t)kCkptMax || (a.every & 1u) ||
      a.n_ckpt != (a.h.n_steps + a.every - 1) / a.every)
    return hipErrorInvalidValue;
  const bool as = a.asian != 0;
  const bool lds = a.phase == 0 && a.ckpt == nullptr;
  if (lds && a.n_ckpt > (uint32_t)kLdsCkpt) return hipErrorInvalidValue;
  if (!lds && a.ckpt == nullptr) return hipErrorInvalidValue;
  switch (a.phase) {
    case 0:
      if (lds)
        return as ? adj_one<float, 0, true, true>(a, s, nb) : adj_one<float, 0, false, true>(a, s, nb);
      return as ? adj_one<float, 0, true, false>(a, s, nb) : adj_one<float, 0, false, false>(a, s, nb);
    case 1:
      return as ? adj_one<float, 1, true, false>(a, s, nb) : adj_one<float, 1, false, false>(a, s, nb);
    case 2:
      return as ? adj_one<float, 2, true, false>(a, s, nb) : adj_one<float, 2, false, false>(a, s, nb);
  }
  return hipErrorInvalidValue;
}

}  // namespace mcp
