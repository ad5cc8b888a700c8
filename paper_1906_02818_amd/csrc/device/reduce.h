// Block reduction of per-path values into per-block moment sums, the first
// stage of the averaging reduction that ends every Monte Carlo estimate
// (Eq. 3; the variance term of Sec. V-B needs the second moments).
//
// Each thread holds the C channel values of its path in double. The block
// writes, for every moment m, one double to partials[m * n_blocks + block]:
//   m = 0: number of valid paths, m = 1: number of non-finite paths,
//   m = 2 .. C+1: sum of y_c, then sum of y_a * y_b for a <= b.
// Wave sums use a fixed xor butterfly and the 4 wave sums are added in
// wave order, so the result does not depend on scheduling.
#pragma once

#include <hip/hip_runtime.h>

namespace mcp {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int C, int BLOCK>
__device__ __forceinline__ void block_moments(const double (&y)[C], bool valid, bool nonfinite,
                                              double* __restrict__ partials,
                                              uint32_t n_blocks, uint32_t block = ~0u) {
  if (block == ~0u) block = blockIdx.x;
  constexpr int M = 2 + C + C * (C + 1) / 2;
  constexpr int W = BLOCK / 64;
  __shared__ double red[M][W];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int m = 0;
  auto push = [&](double v) {
    v = wave_sum(v);
    if (lane == 0) red[m][wave] = v;
    ++m;
  };
  push(valid ? 1.0 : 0.0);
  push(nonfinite ? 1.0 : 0.0);
#pragma unroll
  for (int a = 0; a < C; ++a) push(valid ? y[a] : 0.0);
#pragma unroll
  for (int a = 0; a < C; ++a)
#pragma unroll
    for (int b = a; b < C; ++b) push(valid ? y[a] * y[b] : 0.0);
  __syncthreads();
  for (int t = threadIdx.x; t < M; t += BLOCK) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < W; ++w) s += red[t][w];
    partials[(size_t)t * n_blocks + block] = s;
  }
}

// Per-thread running moments over several paths (same layout as above):
// acc[0] valid count, acc[1] non-finite count, acc[2 + c] sum y_c, then
// sum y_a y_b for a <= b.
template <int C>
__device__ __forceinline__ void accumulate_moments(double (&acc)[2 + C + C * (C + 1) / 2],
                                                   const double (&y)[C], bool valid,
                                                   bool nonfinite) {
  if (nonfinite) acc[1] += 1.0;
  if (!valid) return;
  acc[0] += 1.0;
  int m = 2;
#pragma unroll
  for (int a = 0; a < C; ++a) acc[m++] += y[a];
#pragma unroll
  for (int a = 0; a < C; ++a)
#pragma unroll
    for (int b = a; b < C; ++b) acc[m++] += y[a] * y[b];
}

// Block sum of per-thread moment vectors, written to
// partials[m * n_blocks + block] (fixed wave-butterfly and wave order).
template <int M, int BLOCK>
__device__ __forceinline__ void block_reduce_moments(const double (&acc)[M],
                                                     double* __restrict__ partials,
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

// Block sum for long moment vectors (fixed order, like the above): per
// pass, each wave stores 16 moments of its 64 lanes in LDS; lane l adds the
// 16 values of moment l / 4 from lanes 16 (l mod 4) .. 16 (l mod 4) + 15,
// and two butterfly steps combine the four quarters. About a quarter of the
// instructions of a 6-step butterfly per moment.
template <int M, int BLOCK>
__device__ __forceinline__ void block_reduce_moments_wide(const double (&acc)[M],
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
