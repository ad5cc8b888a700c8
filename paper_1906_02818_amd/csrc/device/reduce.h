// Block reduction of per-path values into per-block moments, the first
// stage of the averaging reduction that ends every Monte Carlo estimate
// (Eq. 3) and of its variance term (Sec. V-B).
//
// Moments are kept as (count, means, co-moments about the means) and
// combined by the pairwise update of Chan, Golub and LeVeque: for two parts
// A and B with n = nA + nB and delta = mean_B - mean_A,
//     mean = mean_A + delta nB / n,
//     M_ab = M_ab^A + M_ab^B + delta_a delta_b nA nB / n.
// A thread adds its own paths one at a time (Welford's update, the same
// formula with nB = 1). No sum of squares is formed, so a variance far
// below the square of the mean (a near-perfect control variate) keeps its
// digits.
//
// A moment vector of C channels holds M = 2 + C + C (C+1)/2 doubles:
//   [0] valid paths, [1] non-finite paths, [2 .. 2+C) means,
//   then M_ab for a <= b in row order.
// Block partials are block-major: block b writes partials[b M .. b M + M),
// one contiguous vector. The wave step is a fixed xor butterfly and the
// waves are merged in wave order, so results do not depend on scheduling.
#pragma once

#include <hip/hip_runtime.h>

namespace mcp {

template <int C>
struct Mom {
  static constexpr int NC = C * (C + 1) / 2;
  static constexpr int M = 2 + C + NC;
  double n, bad, mean[C], co[NC];

  __device__ __forceinline__ void zero() {
    n = 0.0;
    bad = 0.0;
#pragma unroll
    for (int a = 0; a < C; ++a) mean[a] = 0.0;
#pragma unroll
    for (int k = 0; k < NC; ++k) co[k] = 0.0;
  }

  // One valid path (Welford).
  __device__ __forceinline__ void add(const double (&y)[C]) {
    n += 1.0;
    const double r = 1.0 / n;
    double d[C];
#pragma unroll
    for (int a = 0; a < C; ++a) {
      d[a] = y[a] - mean[a];
      mean[a] += d[a] * r;
    }
    int k = 0;
#pragma unroll
    for (int a = 0; a < C; ++a)
#pragma unroll
      for (int b = a; b < C; ++b) co[k++] += d[a] * (y[b] - mean[b]);
  }

  // A path: counted as valid (its channels enter the moments) or not, and
  // as non-finite or not.
  __device__ __forceinline__ void push(const double (&y)[C], bool valid, bool nonfinite) {
    if (nonfinite) bad += 1.0;
    if (valid) add(y);
  }

  // Chan's pairwise update; an empty part (n = 0, zero means and
  // co-moments) leaves the other unchanged bit for bit.
  __device__ __forceinline__ void merge(const Mom& o) {
    bad += o.bad;
    const double nt = n + o.n;
    const double f = nt > 0.0 ? o.n / nt : 0.0;
    const double g = n * f;   // nA nB / n
    double d[C];
#pragma unroll
    for (int a = 0; a < C; ++a) {
      d[a] = o.mean[a] - mean[a];
      mean[a] += d[a] * f;
    }
    int k = 0;
#pragma unroll
    for (int a = 0; a < C; ++a)
#pragma unroll
      for (int b = a; b < C; ++b, ++k) co[k] += o.co[k] + d[a] * d[b] * g;
    n = nt;
  }

  __device__ __forceinline__ void store(double* p) const {
    p[0] = n;
    p[1] = bad;
#pragma unroll
    for (int a = 0; a < C; ++a) p[2 + a] = mean[a];
#pragma unroll
    for (int k = 0; k < NC; ++k) p[2 + C + k] = co[k];
  }

  __device__ __forceinline__ void load(const double* p) {
    n = p[0];
    bad = p[1];
#pragma unroll
    for (int a = 0; a < C; ++a) mean[a] = p[2 + a];
#pragma unroll
    for (int k = 0; k < NC; ++k) co[k] = p[2 + C + k];
  }
};

template <int C>
__device__ __forceinline__ void wave_merge(Mom<C>& m) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    Mom<C> o;
    o.n = __shfl_xor(m.n, off, 64);
    o.bad = __shfl_xor(m.bad, off, 64);
#pragma unroll
    for (int a = 0; a < C; ++a) o.mean[a] = __shfl_xor(m.mean[a], off, 64);
#pragma unroll
    for (int k = 0; k < Mom<C>::NC; ++k) o.co[k] = __shfl_xor(m.co[k], off, 64);
    m.merge(o);
  }
}

// Merges the block's per-thread moments and writes the block's vector to
// partials[block * M ...].
template <int C, int BLOCK>
__device__ __forceinline__ void block_reduce_moments(Mom<C>& m, double* __restrict__ partials,
                                                     uint32_t block) {
  constexpr int W = BLOCK / 64, M = Mom<C>::M;
  __shared__ double red[W][M];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  wave_merge(m);
  if (lane == 0) m.store(red[wave]);
  __syncthreads();
  if (threadIdx.x == 0) {
    Mom<C> t;
    t.load(red[0]);
#pragma unroll 1
    for (int w = 1; w < W; ++w) {
      Mom<C> o;
      o.load(red[w]);
      t.merge(o);
    }
    t.store(red[0]);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < M; t += BLOCK) partials[(size_t)block * M + t] = red[0][t];
}

// One path per thread (y[] ignored unless valid).
template <int C, int BLOCK>
__device__ __forceinline__ void block_moments(const double (&y)[C], bool valid, bool nonfinite,
                                              double* __restrict__ partials,
                                              uint32_t block = ~0u) {
  Mom<C> m;
  m.zero();
  m.push(y, valid, nonfinite);
  block_reduce_moments<C, BLOCK>(m, partials, block == ~0u ? blockIdx.x : block);
}

// ---- Plain sums (counts, tail sums, Gram matrices): moment-major ----------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block sum of per-thread vectors, written to partials[m * n_blocks + block]
// (fixed wave butterfly and wave order).
template <int M, int BLOCK>
__device__ __forceinline__ void block_sum(const double (&acc)[M], double* __restrict__ partials,
                                          uint32_t n_blocks) {
  constexpr int W = BLOCK / 64;
  __shared__ double red[M][W];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const double v = wave_sum(acc[m]);
    if (lane == 0) red[m][wave] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < M; t += BLOCK) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) s += red[t][w];
    partials[(size_t)t * n_blocks + blockIdx.x] = s;
  }
}

// Block sum for long vectors (fixed order, like the above): per pass, each
// wave stores 16 entries of its 64 lanes in LDS; lane l adds the 16 values
// of entry l / 4 from lanes 16 (l mod 4) .. 16 (l mod 4) + 15, and two
// butterfly steps combine the four quarters. About a quarter of the
// instructions of a 6-step butterfly per entry.
template <int M, int BLOCK>
__device__ __forceinline__ void block_sum_wide(const double (&acc)[M],
                                               double* __restrict__ partials,
                                               uint32_t n_blocks) {
  constexpr int W = BLOCK / 64, CH = 16;
  __shared__ double buf[W][CH][64 + 1];
  __shared__ double red[M][W];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int c = lane >> 2, q = lane & 3;
  // Orders the wave's own LDS stores before its loads (lockstep wave).
  auto wave_sync = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
#pragma unroll
  for (int m0 = 0; m0 < M; m0 += CH) {
#pragma unroll
    for (int j = 0; j < CH; ++j)
      if (m0 + j < M) buf[wave][j][lane] = acc[m0 + j];
    wave_sync();
    double s = 0.0;
#pragma unroll
    for (int t = 0; t < 16; ++t) s += buf[wave][c][16 * q + t];
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    if (q == 0 && m0 + c < M) red[m0 + c][wave] = s;
    wave_sync();
  }
  __syncthreads();
  for (int t = threadIdx.x; t < M; t += BLOCK) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) s += red[t][w];
    partials[(size_t)t * n_blocks + blockIdx.x] = s;
  }
}

}  // namespace mcp
