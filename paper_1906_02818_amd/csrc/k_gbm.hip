// One-dimensional GBM path kernel: Euler-Maruyama (Sec. II-A.1) for
// dS = r S dt + sigma S dW under the risk-neutral measure, fused with the
// path functionals, the payoffs and the first stage of the averaging
// reduction (Eq. 3). A thread prices one path at a time, its state in
// registers, nothing written to memory per step; over a persistent grid it
// prices several paths and keeps their moments in FP64 registers.
//
// Schemes: log-Euler on ln S (exact in law for every step count) and Euler
// on S (first-order weak error, Sec. V-B). In FP32 the log state is kept in
// base 2, z = log2(S/S0), so that S_i/S0 = exp2(z) is one v_exp_f32; in FP64
// it is the natural log.
#include "device/reduce.h"
#include "device/rng.h"
#include "mc_internal.h"

namespace mcp {
namespace {

template <typename R>
struct Dom;
template <>
struct Dom<float> {
  static __device__ __forceinline__ float exp_(float z) { return __builtin_amdgcn_exp2f(z); }
  static __device__ __forceinline__ float neg_log_(float u) { return -__builtin_amdgcn_logf(u); }
  static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
  static __device__ __forceinline__ float uniform(uint32_t w) { return uniform_f32(w); }
};
template <>
struct Dom<double> {
  static __device__ __forceinline__ double exp_(double z) { return exp(z); }
  static __device__ __forceinline__ double neg_log_(double u) { return -log(u); }
  static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
  static __device__ __forceinline__ double uniform(uint32_t w) { return uniform_f64(w); }
};

template <typename R>
__device__ __forceinline__ R pos(R x) {
  return x > R(0) ? x : R(0);
}

// Running state of one path.
template <typename R>
struct GbmState {
  R z;       // log scheme: log(S/S0) in the kernel's domain; Euler-S: S/S0
  R sumE;    // sum of S_i/S0            (Asian)
  R sumz;    // sum of log(S_i/S0)       (geometric Asian)
  R sumZ;    // sum of the normals       (vega)
  R dsig;    // Euler-S: d(S_i/S0)/dsigma
  R accV;    // sum of d(S_i/S0)/dsigma  (Asian vega)
  bool alive, alive_bb;
};

template <typename R, uint32_t MASK, bool LOGS>
struct GbmStepper {
  R dz, vz, zB, cbb, sdt, sig, dt, rdt, vsdt, Brel;

  __device__ __forceinline__ void init(const GbmParams& P) {
    dz = (R)P.drift_dom;
    vz = (R)P.vol_dom;
    zB = (R)P.barrier_dom;
    cbb = (R)P.bridge_c;
    sdt = (R)P.sdt;
    sig = (R)P.sigma;
    dt = (R)P.dt;
    rdt = (R)P.r_dt;
    vsdt = (R)P.vol_sdt;
    Brel = (R)P.barrier_rel;
  }

  // Step i -> i+1 with normal Z (and bridge uniform U when monitored).
  __device__ __forceinline__ void step(GbmState<R>& s, R Z, uint32_t i, R U) const {
    if constexpr (LOGS) {
      const R zp = s.z;
      s.z = s.z + dz + vz * Z;
      R E = R(0);
      if constexpr ((MASK & (G_ASIAN | G_ASIAN_G)) != 0) {
        E = Dom<R>::exp_(s.z);
        s.sumE += E;
      }
      if constexpr ((MASK & G_GEO) != 0) s.sumz += s.z;
      if constexpr ((MASK & G_UO) != 0) s.alive = s.alive && (s.z < zB);
      if constexpr ((MASK & (G_EURO_G | G_ASIAN_G)) != 0) s.sumZ += Z;
      if constexpr ((MASK & G_ASIAN_G) != 0)
        s.accV += E * (sdt * s.sumZ - sig * (dt * (R)(i + 1)));
      if constexpr ((MASK & G_UOBB) != 0) {
        // Maximum of the Brownian bridge between z_i and z_{i+1}.
        const R d = zp - s.z;
        const R twice_max = zp + s.z + Dom<R>::sqrt_(d * d + cbb * Dom<R>::neg_log_(U));
        s.alive_bb = s.alive_bb && (twice_max < R(2) * zB);
      }
    } else {
      const R inc = rdt + vsdt * Z;           // S_{i+1}/S_i - 1
      if constexpr ((MASK & (G_EURO_G | G_ASIAN_G)) != 0) s.dsig = s.dsig * (R(1) + inc) + s.z * sdt * Z;
      s.z = s.z + s.z * inc;
      if constexpr ((MASK & (G_ASIAN | G_ASIAN_G)) != 0) s.sumE += s.z;
      if constexpr ((MASK & G_GEO) != 0) s.sumz += log(s.z);
      if constexpr ((MASK & G_UO) != 0) s.alive = s.alive && (s.z < Brel);
      if constexpr ((MASK & G_ASIAN_G) != 0) s.accV += s.dsig;
    }
  }
};

template <typename R, uint32_t MASK, bool LOGS, uint32_t CO>
__device__ __forceinline__ void simulate(const GbmParams& P, uint64_t path,
                                         double (&y)[gbm_channels(MASK)]) {
  GbmStepper<R, MASK, LOGS> st;
  st.init(P);
  GbmState<R> s;
  s.z = LOGS ? R(0) : R(1);
  s.sumE = s.sumz = s.sumZ = s.dsig = s.accV = R(0);
  s.alive = s.alive_bb = true;
  const PathCounter pc = make_counter(path, P.tag, P.k0, P.k1);
  const PathCounter pcb = make_counter(path, P.tag + 5u, P.k0, P.k1);
  const uint32_t n = P.n_steps;
  if constexpr (CO > 1) {
    // Coupled coarse path: step i takes normals CO i .. CO i + CO - 1 of the
    // fine path, summed and scaled by 1/sqrt(CO) (same Brownian increment
    // over the coarse step). CO divides the 4 normals of a Philox block.
    static_assert(CO == 2 || CO == 4, "coupling factor");
    const R rsc = CO == 2 ? R(0.70710678118654752440) : R(0.5);
    constexpr uint32_t SPB = 4 / CO;              // coarse steps per block
    const uint32_t nb = n / SPB;
    for (uint32_t j = 0; j < nb; ++j) {
      const Normals4<R> nz = normals4<R>(philox(j, pc));
#pragma unroll
      for (uint32_t q = 0; q < SPB; ++q) {
        R Z = nz.z[q * CO];
#pragma unroll
        for (uint32_t t = 1; t < CO; ++t) Z += nz.z[q * CO + t];
        st.step(s, Z * rsc, SPB * j + q, R(0));
      }
    }
    if (n % SPB) {                                 // CO = 2, odd n: one step left
      const Normals4<R> nz = normals4<R>(philox(nb, pc));
      st.step(s, (nz.z[0] + nz.z[1]) * rsc, n - 1, R(0));
    }
  }
  const uint32_t n_full = CO > 1 ? 0u : n >> 2;
  for (uint32_t j = 0; j < n_full; ++j) {
    const Normals4<R> nz = normals4<R>(philox(j, pc));
    Words4 wb{0, 0, 0, 0};
    if constexpr ((MASK & G_UOBB) != 0) wb = philox(j, pcb);
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      R U = R(0);
      if constexpr ((MASK & G_UOBB) != 0) U = Dom<R>::uniform(word_at(wb, q));
      st.step(s, nz.z[q], 4 * j + q, U);
    }
  }
  const uint32_t rem = CO > 1 ? 0u : n & 3u;
  if (rem) {
    const Normals4<R> nz = normals4<R>(philox(n_full, pc));
    Words4 wb{0, 0, 0, 0};
    if constexpr ((MASK & G_UOBB) != 0) wb = philox(n_full, pcb);
    for (uint32_t q = 0; q < rem; ++q) {
      R U = R(0);
      if constexpr ((MASK & G_UOBB) != 0) U = Dom<R>::uniform(word_at(wb, q));
      st.step(s, nz.z[q], 4 * n_full + q, U);
    }
  }

  // Terminal payoffs, discounted (e^{-rT}).
  const R S0 = (R)P.S0, K = (R)P.K, disc = (R)P.disc, inv_n = R(1) / (R)n;
  const R En = LOGS ? Dom<R>::exp_(s.z) : s.z;    // S_n / S0
  const R ST = S0 * En;
  const R call = pos(ST - K);
  const R A = S0 * s.sumE * inv_n;
  int c = 0;
  if constexpr ((MASK & G_EURO) != 0) y[c++] = (double)(disc * call);
  if constexpr ((MASK & G_ASIAN) != 0) y[c++] = (double)(disc * pos(A - K));
  if constexpr ((MASK & G_GEO) != 0) {
    const R G = LOGS ? S0 * Dom<R>::exp_(s.sumz * inv_n)
                     : S0 * (R)exp((double)s.sumz / (double)n);
    y[c++] = (double)(disc * pos(G - K));
  }
  if constexpr ((MASK & G_UO) != 0) y[c++] = s.alive ? (double)(disc * call) : 0.0;
  if constexpr ((MASK & G_UOBB) != 0) y[c++] = s.alive_bb ? (double)(disc * call) : 0.0;
  if constexpr ((MASK & G_EURO_G) != 0) {
    const bool itm = ST > K;
    y[c++] = itm ? (double)(disc * En) : 0.0;     // dS_T/dS0 = S_T/S0
    const R dST = LOGS ? ST * (st.sdt * s.sumZ - st.sig * (R)P.T) : S0 * s.dsig;
    y[c++] = itm ? (double)(disc * dST) : 0.0;
  }
  if constexpr ((MASK & G_ASIAN_G) != 0) {
    const bool itm = A > K;
    y[c++] = itm ? (double)(disc * s.sumE * inv_n) : 0.0;
    y[c++] = itm ? (double)(disc * S0 * s.accV * inv_n) : 0.0;
  }
}

// Persistent grid: at most kGbmMaxBlocks workgroups (one wave of blocks at
// full occupancy); each thread prices paths pid, pid + stride, ... and keeps
// their moments in FP64 registers, so each block writes one moment vector.
template <typename R, uint32_t MASK, bool LOGS, uint32_t CO>
__global__ __launch_bounds__(kBlock) void gbm_path_kernel(const GbmParams P) {
  constexpr int C = gbm_channels(MASK);
  ThreadSums<C> acc;
  acc.zero();
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t pid = (uint64_t)blockIdx.x * kBlock + threadIdx.x; pid < P.n_paths;
       pid += stride) {
    double y[C];
    simulate<R, MASK, LOGS, CO>(P, P.path_offset + pid, y);
    bool finite = true;
#pragma unroll
    for (int c = 0; c < C; ++c) finite = finite && isfinite(y[c]);
    if (P.path_out != nullptr) {
#pragma unroll
      for (int c = 0; c < C; ++c) P.path_out[pid * C + c] = y[c];
    }
    acc.push(y, finite, !finite);
  }
  PartSums<C> part = acc.part();
  block_reduce<C, kBlock>(part, P.partials, blockIdx.x);
}

template <typename R, uint32_t MASK, bool LOGS, uint32_t CO = 1>
hipError_t launch_one(const GbmParams& p, hipStream_t s, uint32_t nb) {
  hipLaunchKernelGGL((gbm_path_kernel<R, MASK, LOGS, CO>), dim3(nb), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

// Coupled coarse paths (multilevel): every channel except the bridge barrier.
constexpr uint32_t kMaskCoupled = G_ALL & ~G_UOBB;

template <typename R, bool LOGS>
hipError_t launch_coupled(const GbmParams& p, hipStream_t s, uint32_t nb) {
  return p.coarsen == 2 ? launch_one<R, kMaskCoupled, LOGS, 2>(p, s, nb)
                        : launch_one<R, kMaskCoupled, LOGS, 4>(p, s, nb);
}

constexpr uint32_t kMaskEuro = G_EURO;
constexpr uint32_t kMaskEuroG = G_EURO | G_EURO_G;
constexpr uint32_t kMaskPath3 = G_ASIAN | G_GEO | G_UO;

}  // namespace

uint32_t gbm_pick_mask(uint32_t want, bool fp64, bool log_scheme, uint32_t coarsen) {
  if (coarsen != 1) {
    if (coarsen != 2 && coarsen != 4) return 0;
    return (want & ~kMaskCoupled) == 0 ? kMaskCoupled : 0;
  }
  const uint32_t f32_log[] = {kMaskEuro, kMaskEuroG, kMaskPath3, G_ALL};
  const uint32_t f64_log[] = {kMaskEuroG, G_ALL};
  const uint32_t any_s[] = {G_ALL & ~G_UOBB};
  const uint32_t* list;
  int n;
  if (!log_scheme) {
    list = any_s;
    n = 1;
  } else if (fp64) {
    list = f64_log;
    n = 2;
  } else {
    list = f32_log;
    n = 4;
  }
  for (int i = 0; i < n; ++i)
    if ((list[i] & want) == want) return list[i];
  return 0;
}

hipError_t launch_gbm(const GbmParams& p, uint32_t mask, bool fp64, hipStream_t s,
                      uint32_t* n_blocks) {
  const uint64_t need = (p.n_paths + kBlock - 1) / kBlock;
  const uint32_t nb = (uint32_t)(need < kGbmMaxBlocks ? need : kGbmMaxBlocks);
  *n_blocks = nb;
  const bool L = p.log_scheme != 0;
  constexpr uint32_t kMaskS = G_ALL & ~G_UOBB;
  if (p.coarsen != 1) {
    if (mask != kMaskCoupled || (p.coarsen != 2 && p.coarsen != 4)) return hipErrorInvalidValue;
    if (L) return fp64 ? launch_coupled<double, true>(p, s, nb) : launch_coupled<float, true>(p, s, nb);
    return fp64 ? launch_coupled<double, false>(p, s, nb) : launch_coupled<float, false>(p, s, nb);
  }
  if (L && !fp64) {
    switch (mask) {
      case kMaskEuro: return launch_one<float, kMaskEuro, true>(p, s, nb);
      case kMaskEuroG: return launch_one<float, kMaskEuroG, true>(p, s, nb);
      case kMaskPath3: return launch_one<float, kMaskPath3, true>(p, s, nb);
      case G_ALL: return launch_one<float, G_ALL, true>(p, s, nb);
    }
  } else if (L && fp64) {
    switch (mask) {
      case kMaskEuroG: return launch_one<double, kMaskEuroG, true>(p, s, nb);
      case G_ALL: return launch_one<double, G_ALL, true>(p, s, nb);
    }
  } else if (mask == kMaskS) {
    return fp64 ? launch_one<double, kMaskS, false>(p, s, nb)
                : launch_one<float, kMaskS, false>(p, s, nb);
  }
  return hipErrorInvalidValue;
}

}  // namespace mcp
