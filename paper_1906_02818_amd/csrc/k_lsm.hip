// Longstaff-Schwartz regression for Bermudan options on d <= 4 correlated
// GBM assets (dynamic programming by chained least-squares regressions,
// Sec. II-A.3; the American max-option experiment of Sec. VI-C).
//
// Data flow, all on one stream with no host round trip:
//  1. lsm_sim_kernel simulates every path once (log-Euler per asset, one
//     lane per path), stores S_a(t_j)/K at each exercise date before t_M in
//     HBM as [date][asset][path] FP32 (coalesced across lanes), sets the cash flow
//     C = K e^{-rT} f(t_M)/K, and accumulates in FP64 the Gram matrix of date
//     M-1: the upper triangle of u u^T, u = (features, C), over the paths in
//     the money there, plus the moments of C (exercise at maturity only).
//  2. For j = M-1 .. 1: the fixed-order reduction of date j's Gram matrix
//     and lsm_solve_kernel (Cholesky, FP64, one thread's registers) give the
//     regression coefficients; then
//     lsm_update_kernel applies date j's exercise rule to every path and, in
//     the same pass, accumulates the Gram matrix of date j-1 with the updated
//     cash flows (or, at j = 1, the moments of the price). One read of the
//     two dates' states and one read-modify-write of C per path and date.
//  3. lsm_oos_kernel applies the fitted rule to fresh paths (no storage).
// Per-block FP64 partials go through the fixed-order final reduction, so
// results do not depend on scheduling.
#include "device/reduce.h"
#include "device/rng.h"
#include "mc_internal.h"

namespace mcp {
namespace {

constexpr int monomials(int D, int DEG) {
  return 1 + (DEG >= 1 ? D : 0) + (DEG >= 2 ? D * (D + 1) / 2 : 0) +
         (DEG >= 3 ? D * (D + 1) * (D + 2) / 6 : 0);
}

// Features of one state: monomials of y by degree, then by the
// nondecreasing index tuple; f/K last when PF.
template <int D, int DEG, int PF>
struct Feat {
  static constexpr int NF = monomials(D, DEG) + PF;
  static constexpr int NU = NF + 1;               // features and the cash flow
  static constexpr int NG = NU * (NU + 1) / 2;    // upper triangle of u u^T
  static constexpr int NMOM = NG + 3;             // + sum C, sum C^2, n in the money at t_M
  static_assert(NF <= kLsmMaxFeat, "feature set too large");

  __device__ static __forceinline__ void eval(const double (&y)[D], double fK, double (&psi)[NF]) {
    int n = 0;
    psi[n++] = 1.0;
    if constexpr (DEG >= 1) {
#pragma unroll
      for (int a = 0; a < D; ++a) psi[n++] = y[a];
    }
    if constexpr (DEG >= 2) {
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b) psi[n++] = y[a] * y[b];
    }
    if constexpr (DEG >= 3) {
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a; b < D; ++b)
#pragma unroll
          for (int c = b; c < D; ++c) psi[n++] = y[a] * y[b] * y[c];
    }
    if constexpr (PF) psi[n++] = fK;
  }

  // acc[0 .. NG) += upper triangle of u u^T with u = (psi, c).
  __device__ static __forceinline__ void gram_add(double (&acc)[NMOM], const double (&psi)[NF],
                                                  double c) {
    double u[NU];
#pragma unroll
    for (int k = 0; k < NF; ++k) u[k] = psi[k];
    u[NF] = c;
    int m = 0;
#pragma unroll
    for (int a = 0; a < NU; ++a)
#pragma unroll
      for (int b = a; b < NU; ++b) {
        acc[m] = fma(u[a], u[b], acc[m]);
        ++m;
      }
  }
};

// f/K of the payoff from y = S/K (equal weights 1/D for the basket payoffs).
template <int D>
__device__ __forceinline__ double payoff_over_K(uint32_t kind, const double (&y)[D]) {
  double m = y[0], s = y[0];
#pragma unroll
  for (int a = 1; a < D; ++a) {
    m = fmax(m, y[a]);
    s += y[a];
  }
  s = s / (double)D;
  const double f = kind == LSM_MAX_CALL ? m - 1.0 : kind == LSM_BASKET_PUT ? 1.0 - s : s - 1.0;
  return f > 0.0 ? f : 0.0;
}

// Normals of one path in index order (normal k is slot k mod 4 of Philox
// block k / 4); the block is refilled every fourth normal.
struct NormalCursor {
  Normals4<float> z;
  uint32_t k = 0;
  __device__ __forceinline__ float next(const PathCounter& pc) {
    const uint32_t s = k & 3u;
    if (s == 0u) z = normals4<float>(philox(k >> 2, pc));
    ++k;
    return s == 0u ? z.z[0] : s == 1u ? z.z[1] : s == 2u ? z.z[2] : z.z[3];
  }
};

// Advances the log2 state over one Euler step: x_a += drift_a + (L' Z)_a.
template <int D>
__device__ __forceinline__ void apply_step(const LsmParams& p, float (&x)[D], const float (&Z)[D]) {
#pragma unroll
  for (int a = 0; a < D; ++a) {
    float dw = p.drift[a];
#pragma unroll
    for (int b = 0; b <= a; ++b) dw = fmaf(p.vol[a][b], Z[b], dw);
    x[a] += dw;
  }
}

template <int D>
__device__ __forceinline__ void euler_step(const LsmParams& p, float (&x)[D], NormalCursor& cur,
                                           const PathCounter& pc) {
  float Z[D];
#pragma unroll
  for (int a = 0; a < D; ++a) Z[a] = cur.next(pc);
  apply_step<D>(p, x, Z);
}

// Dates drawn per group with one Euler step per date: U dates use U D
// normals, a whole number NB of Philox blocks, so every normal's block slot
// is fixed at compile time.
template <int D>
struct DateGroup {
  static constexpr int U = D == 2 ? 2 : D == 4 ? 1 : 4;
  static constexpr int NB = U * D / 4;
};

// Takes the path through exercise dates 1..M (steps_per_date Euler steps
// each), calling at_date(j) after date j. cont() is asked before each group
// of dates (each date when a date has several steps), where control flow is
// uniform over the wave, and ends the walk when it returns false.
template <int D, typename AtDate, typename Cont>
__device__ __forceinline__ void walk_dates(const LsmParams& p, const PathCounter& pc,
                                           float (&x)[D], AtDate&& at_date, Cont&& cont) {
  const uint32_t M = p.n_dates;
  if (p.spd == 1) {
    constexpr int U = DateGroup<D>::U, NB = DateGroup<D>::NB;
    for (uint32_t j0 = 1; j0 <= M; j0 += U) {
      if (!cont()) return;
      const uint32_t blk0 = (j0 - 1) * D / 4;   // (j0 - 1) D is a multiple of 4
      float zz[4 * NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const Normals4<float> q = normals4<float>(philox(blk0 + b, pc));
#pragma unroll
        for (int t = 0; t < 4; ++t) zz[4 * b + t] = q.z[t];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (j0 + u > M) break;
        float Z[D];
#pragma unroll
        for (int a = 0; a < D; ++a) Z[a] = zz[u * D + a];
        apply_step<D>(p, x, Z);
        at_date(j0 + u);
      }
    }
  } else {
    NormalCursor cur;
    for (uint32_t j = 1; j <= M; ++j) {
      if (!cont()) return;
      for (uint32_t s = 0; s < p.spd; ++s) euler_step<D>(p, x, cur, pc);
      at_date(j);
    }
  }
}

template <int D, int DEG, int PF>
__global__ __launch_bounds__(256) void lsm_sim_kernel(LsmParams p) {
  using F = Feat<D, DEG, PF>;
  double acc[F::NMOM];
#pragma unroll
  for (int m = 0; m < F::NMOM; ++m) acc[m] = 0.0;
  const uint32_t M = p.n_dates;
  const uint64_t N = p.n_paths;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += stride) {
    const PathCounter pc = make_counter(p.path_offset + i, p.tag, p.k0, p.k1);
    float x[D], y[D], yprev[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      x[a] = p.x0[a];
      yprev[a] = 0.f;
    }
    walk_dates<D>(
        p, pc, x,
        [&](uint32_t j) {
#pragma unroll
          for (int a = 0; a < D; ++a) {
            y[a] = __builtin_amdgcn_exp2f(x[a]);
            if (j < M) p.y[((size_t)(j - 1) * D + a) * p.ystride + i] = y[a];  // t_M is not read back
          }
          if (j + 1 == M) {
#pragma unroll
            for (int a = 0; a < D; ++a) yprev[a] = y[a];
          }
        },
        [] { return true; });
    double yd[D];
#pragma unroll
    for (int a = 0; a < D; ++a) yd[a] = y[a];
    const double f = payoff_over_K<D>(p.kind, yd);
    const float cf = (float)(p.discK[M] * f);
    p.C[i] = cf;
    if (p.ex) p.ex[i] = f > 0.0 ? (uint8_t)M : (uint8_t)0;
    const double c = cf;
    acc[F::NG] += c;
    acc[F::NG + 1] = fma(c, c, acc[F::NG + 1]);
    acc[F::NG + 2] += f > 0.0 ? 1.0 : 0.0;
    if (M >= 2) {
#pragma unroll
      for (int a = 0; a < D; ++a) yd[a] = yprev[a];
      const double fp = payoff_over_K<D>(p.kind, yd);
      if (fp > 0.0) {
        double psi[F::NF];
        F::eval(yd, fp, psi);
        F::gram_add(acc, psi, c);
      }
    }
  }
  block_sum_wide<F::NMOM, 256>(acc, p.partials, gridDim.x);
}

__device__ __forceinline__ float lane_of(const float4& v, int u) {
  return u == 0 ? v.x : u == 1 ? v.y : u == 2 ? v.z : v.w;
}

// Four consecutive paths per lane: 16-byte loads of each state row and of
// the cash flows (rows are padded to a multiple of 64 floats).
template <int D, int DEG, int PF>
__global__ __launch_bounds__(256) void lsm_update_kernel(LsmParams p, uint32_t j) {
  using F = Feat<D, DEG, PF>;
  double acc[F::NMOM];
#pragma unroll
  for (int m = 0; m < F::NMOM; ++m) acc[m] = 0.0;
  const uint64_t N = p.n_paths, S = p.ystride;
  const bool valid = p.valid[j - 1] != 0;
  double beta[F::NF];
#pragma unroll
  for (int k = 0; k < F::NF; ++k) beta[k] = p.beta[(size_t)(j - 1) * kLsmMaxFeat + k];
  const double dK = p.discK[j];
  const float* yj = p.y + (size_t)(j - 1) * D * S;
  const float* yq = p.y + (size_t)(j >= 2 ? j - 2 : 0) * D * S;
  const uint64_t nq = (N + 3) / 4;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t q = (uint64_t)blockIdx.x * 256 + threadIdx.x; q < nq; q += stride) {
    float4 v[D], vp[D];
#pragma unroll
    for (int a = 0; a < D; ++a) v[a] = *(const float4*)(yj + (size_t)a * S + 4 * q);
    if (j >= 2) {
#pragma unroll
      for (int a = 0; a < D; ++a) vp[a] = *(const float4*)(yq + (size_t)a * S + 4 * q);
    }
    const float4 cv = *(const float4*)(p.C + 4 * q);
    float cq[4] = {cv.x, cv.y, cv.z, cv.w};
    bool changed = false;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint64_t i = 4 * q + u;
      if (i >= N) continue;
      double y[D];
#pragma unroll
      for (int a = 0; a < D; ++a) y[a] = lane_of(v[a], u);
      const double f = payoff_over_K<D>(p.kind, y);
      if (valid && f > 0.0) {
        double psi[F::NF];
        F::eval(y, f, psi);
        double h = 0.0;
#pragma unroll
        for (int k = 0; k < F::NF; ++k) h = fma(psi[k], beta[k], h);
        const double e = dK * f;
        if (e >= h) {
          cq[u] = (float)e;
          changed = true;
          if (p.ex) p.ex[i] = (uint8_t)j;
        }
      }
      const double c = cq[u];
      if (j >= 2) {
        double yp[D];
#pragma unroll
        for (int a = 0; a < D; ++a) yp[a] = lane_of(vp[a], u);
        const double fp = payoff_over_K<D>(p.kind, yp);
        if (fp > 0.0) {
          // FP64 products: the normal equations square the conditioning of
          // the features, so FP32 Gram entries would move the fit far more
          // than the FP32 states do.
          double psi[F::NF];
          F::eval(yp, fp, psi);
          F::gram_add(acc, psi, c);
        }
      } else {
        acc[F::NG] += c;
        acc[F::NG + 1] = fma(c, c, acc[F::NG + 1]);
      }
    }
    // The quad's cash flows go back as one 16-byte store: nearly every
    // 32-byte sector holds an exercising path at some date anyway.
    if (changed) *(float4*)(p.C + 4 * q) = make_float4(cq[0], cq[1], cq[2], cq[3]);
  }
  block_sum_wide<F::NMOM, 256>(acc, p.partials, gridDim.x);
}

// Solves the normal equations of date j from one stage's reduced moments
// (upper triangle of u u^T, u = (psi, C), row-major) in one thread's
// registers: Cholesky factorisation and two triangular solves. No
// regression when fewer paths than features are in the money or a pivot is
// <= 1e-12 times its diagonal entry.
template <int NF>
__global__ __launch_bounds__(64) void lsm_solve_kernel(const double* __restrict__ sh, uint32_t j,
                                                       double* __restrict__ beta,
                                                       int* __restrict__ valid) {
  if (threadIdx.x != 0) return;
  constexpr int NU = NF + 1;
  double G[NF][NF], b[NF], Lc[NF][NF], t[NF], x[NF];
  int m = 0;
#pragma unroll
  for (int a = 0; a < NU; ++a)
#pragma unroll
    for (int c = a; c < NU; ++c, ++m) {
      if (c < NF) G[c][a] = sh[m];
      else if (a < NF) b[a] = sh[m];
    }
  bool ok = G[0][0] >= (double)NF;  // G[0][0] counts the in-the-money paths
#pragma unroll
  for (int c = 0; c < NF; ++c) {
    double s = G[c][c];
#pragma unroll
    for (int k = 0; k < c; ++k) s -= Lc[c][k] * Lc[c][k];
    ok = ok && s > 1e-12 * G[c][c];
    const double l = sqrt(ok ? s : 1.0);
    Lc[c][c] = l;
#pragma unroll
    for (int i = c + 1; i < NF; ++i) {
      double v = G[i][c];
#pragma unroll
      for (int k = 0; k < c; ++k) v -= Lc[i][k] * Lc[c][k];
      Lc[i][c] = v / l;
    }
  }
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    double v = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= Lc[i][k] * t[k];
    t[i] = v / Lc[i][i];
  }
#pragma unroll
  for (int i = NF - 1; i >= 0; --i) {
    double v = t[i];
#pragma unroll
    for (int k = i + 1; k < NF; ++k) v -= Lc[k][i] * x[k];
    x[i] = v / Lc[i][i];
  }
  double* row = beta + (size_t)(j - 1) * kLsmMaxFeat;
#pragma unroll
  for (int k = 0; k < kLsmMaxFeat; ++k) row[k] = (ok && k < NF) ? x[k < NF ? k : 0] : __builtin_nan("");
  valid[j - 1] = ok ? 1 : 0;
}

template <int D, int DEG, int PF>
__global__ __launch_bounds__(256) void lsm_oos_kernel(LsmParams p) {
  using F = Feat<D, DEG, PF>;
  double acc[2] = {0.0, 0.0};
  const uint32_t M = p.n_dates;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < p.n_paths; i += stride) {
    const PathCounter pc = make_counter(p.path_offset + i, p.tag, p.k0, p.k1);
    float x[D];
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = p.x0[a];
    double v = 0.0;
    uint32_t e = 0;
    bool live = true;                    // not exercised yet
    walk_dates<D>(
        p, pc, x,
        [&](uint32_t j) {
          if (!live) return;
          double y[D];
#pragma unroll
          for (int a = 0; a < D; ++a) y[a] = (double)__builtin_amdgcn_exp2f(x[a]);
          const double f = payoff_over_K<D>(p.kind, y);
          if (!(f > 0.0)) return;
          if (j == M) {
            v = p.discK[M] * f;
            e = M;
            live = false;
            return;
          }
          if (!p.valid[j - 1]) return;
          double psi[F::NF];
          F::eval(y, f, psi);
          double h = 0.0;
          const double* bj = p.beta + (size_t)(j - 1) * kLsmMaxFeat;
#pragma unroll
          for (int k = 0; k < F::NF; ++k) h = fma(psi[k], bj[k], h);
          if (p.discK[j] * f >= h) {
            v = p.discK[j] * f;
            e = j;
            live = false;
          }
        },
        [&] { return __any(live); });   // the whole wave has stopped
    acc[0] += v;
    acc[1] = fma(v, v, acc[1]);
    if (p.path_value) p.path_value[i] = v;
    if (p.ex) p.ex[i] = (uint8_t)e;
  }
  block_sum<2, 256>(acc, p.partials, gridDim.x);
}

uint32_t grid_for(uint64_t n, uint32_t cap = kLsmMaxBlocks) {
  const uint64_t need = (n + 255) / 256;
  return (uint32_t)(need < cap ? need : cap);
}

enum class Stage { Sim, Update, Oos };

template <int D, int DEG, int PF>
hipError_t launch_t(const LsmParams& p, Stage stage, uint32_t j, hipStream_t s, uint32_t nb) {
  switch (stage) {
    case Stage::Sim:
      hipLaunchKernelGGL((lsm_sim_kernel<D, DEG, PF>), dim3(nb), dim3(256), 0, s, p);
      break;
    case Stage::Update:
      hipLaunchKernelGGL((lsm_update_kernel<D, DEG, PF>), dim3(nb), dim3(256), 0, s, p, j);
      break;
    case Stage::Oos:
      hipLaunchKernelGGL((lsm_oos_kernel<D, DEG, PF>), dim3(nb), dim3(256), 0, s, p);
      break;
  }
  return hipGetLastError();
}

// Every (d, degree, payoff feature) with at most kLsmMaxFeat features.
hipError_t dispatch(const LsmParams& p, Stage stage, uint32_t j, hipStream_t s, uint32_t nb) {
  const uint32_t key = p.d * 100 + p.degree * 10 + p.pay_feat;
  switch (key) {
    case 110: return launch_t<1, 1, 0>(p, stage, j, s, nb);
    case 120: return launch_t<1, 2, 0>(p, stage, j, s, nb);
    case 130: return launch_t<1, 3, 0>(p, stage, j, s, nb);
    case 210: return launch_t<2, 1, 0>(p, stage, j, s, nb);
    case 211: return launch_t<2, 1, 1>(p, stage, j, s, nb);
    case 220: return launch_t<2, 2, 0>(p, stage, j, s, nb);
    case 221: return launch_t<2, 2, 1>(p, stage, j, s, nb);
    case 230: return launch_t<2, 3, 0>(p, stage, j, s, nb);
    case 231: return launch_t<2, 3, 1>(p, stage, j, s, nb);
    case 310: return launch_t<3, 1, 0>(p, stage, j, s, nb);
    case 311: return launch_t<3, 1, 1>(p, stage, j, s, nb);
    case 320: return launch_t<3, 2, 0>(p, stage, j, s, nb);
    case 321: return launch_t<3, 2, 1>(p, stage, j, s, nb);
    case 410: return launch_t<4, 1, 0>(p, stage, j, s, nb);
    case 411: return launch_t<4, 1, 1>(p, stage, j, s, nb);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

uint32_t lsm_n_features(uint32_t d, uint32_t degree, uint32_t pay_feat) {
  if (d < 1 || d > (uint32_t)kLsmMaxD || degree < 1 || degree > 3) return 0;
  return (uint32_t)monomials((int)d, (int)degree) + (pay_feat ? 1u : 0u);
}

uint32_t lsm_n_moments(uint32_t nf) { return (nf + 1) * (nf + 2) / 2 + 3; }

hipError_t launch_lsm_sim(const LsmParams& p, hipStream_t s, uint32_t* n_blocks) {
  const uint32_t nb = grid_for(p.n_paths);
  *n_blocks = nb;
  if (nb == 0) return hipErrorInvalidValue;
  return dispatch(p, Stage::Sim, 0, s, nb);
}

hipError_t launch_lsm_update(const LsmParams& p, uint32_t j, hipStream_t s, uint32_t* n_blocks) {
  // Four paths per lane; 1024 blocks keep every wave resident at once (four
  // per SIMD). Measured for the 8 launches of a 2^24-path call: 0.62 ms on
  // 1024 or 2048 blocks, 0.72 ms on 512.
  const uint32_t nb = grid_for((p.n_paths + 3) / 4, kLsmMaxBlocks / 2);
  *n_blocks = nb;
  if (nb == 0 || j < 1 || j >= p.n_dates) return hipErrorInvalidValue;
  return dispatch(p, Stage::Update, j, s, nb);
}

hipError_t launch_lsm_reduce_solve(const double* partials, uint32_t nb, uint32_t nmom,
                                  double* out, uint32_t nf, uint32_t j, double* beta, int* valid,
                                  hipStream_t s) {
  if (nmom > (uint32_t)kLsmMaxMom || nb == 0) return hipErrorInvalidValue;
  hipError_t e = launch_final_reduce(partials, nb, nmom, out, s);
  if (e != hipSuccess || j == 0) return e;
#define MCP_LSM_SOLVE(NF)                                                                    \
  case NF:                                                                                   \
    hipLaunchKernelGGL(lsm_solve_kernel<NF>, dim3(1), dim3(64), 0, s, out, j, beta, valid); \
    break;
  switch (nf) {
    MCP_LSM_SOLVE(2) MCP_LSM_SOLVE(3) MCP_LSM_SOLVE(4) MCP_LSM_SOLVE(5) MCP_LSM_SOLVE(6)
    MCP_LSM_SOLVE(7) MCP_LSM_SOLVE(8) MCP_LSM_SOLVE(9) MCP_LSM_SOLVE(10) MCP_LSM_SOLVE(11)
    default: return hipErrorInvalidValue;
  }
#undef MCP_LSM_SOLVE
  return hipGetLastError();
}

hipError_t launch_lsm_oos(const LsmParams& p, hipStream_t s, uint32_t* n_blocks) {
  const uint32_t nb = grid_for(p.n_paths);
  *n_blocks = nb;
  if (nb == 0) return hipErrorInvalidValue;
  return dispatch(p, Stage::Oos, 0, s, nb);
}

}  // namespace mcp
