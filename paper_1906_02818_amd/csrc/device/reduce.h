// Block reduction of per-path values into per-block moments, the first
// stage of the averaging reduction that ends every Monte Carlo estimate
// (Eq. 3) and of its variance term (Sec. V-B).
//
// A moment vector of C channels holds M = 2 + C + C (C+1)/2 doubles:
//   [0] valid paths, [1] non-finite paths, [2 .. 2+C) means,
//   then the co-moments M_ab = sum (y_a - mean_a)(y_b - mean_b), a <= b, in
//   row order.
// Block partials are block-major: block b writes partials[b M .. b M + M),
// one contiguous vector; the final merge combines them the same way.
//
// Parts are combined by the pairwise update of Chan, Golub and LeVeque,
// written about a shift: a part with n paths, mean m and co-moments M is
// held as (n, c, S1 = n (m - c), S2 = M + n (m - c)(m - c)^T) for a shift c
// that is itself one of the parts' means (a sample of the same spread).
// About a common shift, S1 and S2 add like plain sums, so paths, lanes,
// waves and blocks combine without a division; moving a part to another
// shift c' is exact algebra (S1' = S1 + n e, S2' = S2 + S1 e^T + e S1^T +
// n e e^T with e = c - c'), and the moments come back as m = c + S1 / n,
// M = S2 - S1 S1^T / n. All deviations are of the order of the spread, so a
// variance far below the square of the mean (a near-perfect control
// variate) keeps its digits. A thread of a persistent kernel sums its few
// paths about zero and enters as one part about its own mean (ThreadSums),
// which keeps the path loop's registers and code those of plain sums.
// Sums run in fixed orders (per-thread path order, xor butterfly, wave
// order, block order): results do not depend on scheduling.
#pragma once

#include <hip/hip_runtime.h>

namespace mcp {

template <int C>
struct PartSums {
  static constexpr int NC = C * (C + 1) / 2;
  static constexpr int M = 2 + C + NC;     // doubles in a moment vector
  double n, bad, shift[C], s1[C], s2[NC];

  __device__ __forceinline__ void zero() {
    n = 0.0;
    bad = 0.0;
#pragma unroll
    for (int a = 0; a < C; ++a) shift[a] = s1[a] = 0.0;
#pragma unroll
    for (int k = 0; k < NC; ++k) s2[k] = 0.0;
  }

  // A part (nb paths, means mb, co-moments cb), in this part's shift; the
  // first non-empty part sets the shift.
  __device__ __forceinline__ void add(double nb, const double* mb, const double* cb) {
    if (nb == 0.0) return;
    if (n == 0.0) {
#pragma unroll
      for (int a = 0; a < C; ++a) shift[a] = mb[a];
    }
    double e[C];
#pragma unroll
    for (int a = 0; a < C; ++a) {
      e[a] = mb[a] - shift[a];
      s1[a] += nb * e[a];
    }
    int k = 0;
#pragma unroll
    for (int a = 0; a < C; ++a)
#pragma unroll
      for (int b = a; b < C; ++b, ++k) s2[k] += (cb ? cb[k] : 0.0) + nb * e[a] * e[b];
    n += nb;
  }

  // One path: counted as valid (its channels enter the moments) or not,
  // and as non-finite or not.
  __device__ __forceinline__ void push(const double (&y)[C], bool valid, bool nonfinite) {
    if (nonfinite) bad += 1.0;
    if (valid) add(1.0, y, nullptr);
  }

  // A stored moment vector [n, bad, means, co-moments].
  __device__ __forceinline__ void add_vector(const double* v) {
    bad += v[1];
    add(v[0], v + 2, v + 2 + C);
  }

  // The same part about the shift c.
  __device__ __forceinline__ void rebase(const double (&c)[C]) {
    double e[C];
#pragma unroll
    for (int a = 0; a < C; ++a) e[a] = n > 0.0 ? shift[a] - c[a] : 0.0;
    int k = 0;
#pragma unroll
    for (int a = 0; a < C; ++a)
#pragma unroll
      for (int b = a; b < C; ++b, ++k) s2[k] += s1[a] * e[b] + e[a] * s1[b] + n * e[a] * e[b];
#pragma unroll
    for (int a = 0; a < C; ++a) {
      s1[a] += n * e[a];
      shift[a] = c[a];
    }
  }
};

// Per-thread sums of a persistent kernel's paths, y and y y^T about zero:
// a thread prices at most a few hundred paths, whose rounding errors are
// unbiased and average out across threads; the thread's part enters the
// reduction about its own mean (part()), and everything above the thread
// combines about shifts.
template <int C>
struct ThreadSums {
  static constexpr int NC = C * (C + 1) / 2;
  double n, bad, s[C], ss[NC];

  __device__ __forceinline__ void zero() {
    n = 0.0;
    bad = 0.0;
#pragma unroll
    for (int a = 0; a < C; ++a) s[a] = 0.0;
#pragma unroll
    for (int k = 0; k < NC; ++k) ss[k] = 0.0;
  }

  __device__ __forceinline__ void push(const double (&y)[C], bool valid, bool nonfinite) {
    if (nonfinite) bad += 1.0;
    if (!valid) return;
    n += 1.0;
#pragma unroll
    for (int a = 0; a < C; ++a) s[a] += y[a];
    int k = 0;
#pragma unroll
    for (int a = 0; a < C; ++a)
#pragma unroll
      for (int b = a; b < C; ++b) ss[k++] += y[a] * y[b];
  }

  // (n, shift = mean, S1 = 0, S2 = co-moments).
  __device__ __forceinline__ PartSums<C> part() const {
    PartSums<C> p;
    p.n = n;
    p.bad = bad;
    const double r = n > 0.0 ? 1.0 / n : 0.0;
#pragma unroll
    for (int a = 0; a < C; ++a) {
      p.shift[a] = s[a] * r;
      p.s1[a] = 0.0;
    }
    int k = 0;
#pragma unroll
    for (int a = 0; a < C; ++a)
#pragma unroll
      for (int b = a; b < C; ++b, ++k) p.s2[k] = n > 0.0 ? ss[k] - s[a] * s[b] * r : 0.0;
    return p;
  }
};

// The block's moment vector from its threads' parts, written to
// out[block * M ...]: each wave moves its lanes to the shift of its first
// lane holding a path and sums them (xor butterfly); after one barrier every
// output component is computed by its own thread, moving the waves' sums to
// the shift of the first wave holding a path and adding them in wave order.
template <int C, int BLOCK>
__device__ __forceinline__ void block_reduce(PartSums<C>& t, double* __restrict__ out,
                                             uint32_t block) {
  constexpr int W = BLOCK / 64, NC = PartSums<C>::NC, M = PartSums<C>::M;
  constexpr int R = 2 + 2 * C + NC;        // n, bad, shift, S1, S2 of a wave
  __shared__ double red[W][R];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const unsigned long long holders = __ballot(t.n > 0.0);
  if (holders != 0ull) {                   // wave-uniform
    const int src = __ffsll((long long)holders) - 1;
    double c[C];
#pragma unroll
    for (int a = 0; a < C; ++a) c[a] = __shfl(t.shift[a], src, 64);
    t.rebase(c);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    t.n += __shfl_xor(t.n, off, 64);
    t.bad += __shfl_xor(t.bad, off, 64);
#pragma unroll
    for (int a = 0; a < C; ++a) t.s1[a] += __shfl_xor(t.s1[a], off, 64);
#pragma unroll
    for (int k = 0; k < NC; ++k) t.s2[k] += __shfl_xor(t.s2[k], off, 64);
  }
  if (lane == 0) {
    red[wave][0] = t.n;
    red[wave][1] = t.bad;
#pragma unroll
    for (int a = 0; a < C; ++a) {
      red[wave][2 + a] = t.shift[a];
      red[wave][2 + C + a] = t.s1[a];
    }
#pragma unroll
    for (int k = 0; k < NC; ++k) red[wave][2 + 2 * C + k] = t.s2[k];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < M; q += BLOCK) {
    int w0 = 0;
    while (w0 < W - 1 && red[w0][0] == 0.0) ++w0;   // first wave holding a path
    double n = 0.0, bad = 0.0;
    for (int w = 0; w < W; ++w) {
      n += red[w][0];
      bad += red[w][1];
    }
    // S1 of channel a about the common shift (wave order).
    auto S1 = [&](int a) {
      double s = 0.0;
      for (int w = 0; w < W; ++w)
        s += red[w][2 + C + a] + red[w][0] * (red[w][2 + a] - red[w0][2 + a]);
      return s;
    };
    double v;
    if (q == 0) {
      v = n;
    } else if (q == 1) {
      v = bad;
    } else if (q < 2 + C) {
      const int a = q - 2;
      v = n > 0.0 ? red[w0][2 + a] + S1(a) / n : 0.0;
    } else {
      int k = q - 2 - C, a = 0;
      while (k >= C - a) {
        k -= C - a;
        ++a;
      }
      const int b = a + k, kk = q - 2 - C;
      double s2 = 0.0;
      for (int w = 0; w < W; ++w) {
        const double nw = red[w][0];
        const double ea = red[w][2 + a] - red[w0][2 + a], eb = red[w][2 + b] - red[w0][2 + b];
        const double sa = red[w][2 + C + a], sb = red[w][2 + C + b];
        s2 += red[w][2 + 2 * C + kk] + sa * eb + ea * sb + nw * ea * eb;
      }
      v = n > 0.0 ? s2 - S1(a) * S1(b) / n : 0.0;
    }
    out[(size_t)block * M + q] = v;
  }
}

// One path per thread (y[] ignored unless valid).
template <int C, int BLOCK>
__device__ __forceinline__ void block_moments(const double (&y)[C], bool valid, bool nonfinite,
                                              double* __restrict__ partials,
                                              uint32_t block = ~0u) {
  PartSums<C> m;
  m.zero();
  m.push(y, valid, nonfinite);
  block_reduce<C, BLOCK>(m, partials, block == ~0u ? blockIdx.x : block);
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
