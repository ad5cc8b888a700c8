// Risk metrics of a simulated P&L sample (Sec. VI-B.1): the exact order
// statistic behind Value-at-Risk, and the tail sum behind Conditional
// Value-at-Risk, over per-path values already in device memory.
//
// Selection is a most-significant-digit radix select on 64-bit keys that
// order like the doubles (flip every bit of a negative value, set the sign
// bit of a non-negative one). Eight passes of 8-bit digits: each pass
// histograms, in LDS, the digit of the keys that still match the prefix
// chosen so far; a one-block kernel then scans the 256 counts, fixes the
// digit that holds the k-th key and the rank left inside it, and clears the
// histogram for the next pass. Counts are integer atomics, so the result is
// exact and independent of scheduling; no host round trip between passes.
#include "device/reduce.h"
#include "mc_internal.h"

namespace mcp {
namespace {

struct SelectState {
  unsigned long long prefix;   // digits fixed so far (key bits)
  unsigned long long mask;     // which key bits are fixed
  unsigned long long k;        // 1-based rank still sought within the prefix class
  unsigned long long pad[5];
};
static_assert(sizeof(SelectState) <= kSelectStateBytes, "state size");

__device__ __forceinline__ unsigned long long order_key(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

constexpr uint32_t kSelBlocks = 1024;

__global__ __launch_bounds__(256) void select_init_kernel(SelectState* st, uint32_t* hist,
                                                          unsigned long long k) {
  hist[threadIdx.x] = 0u;
  if (threadIdx.x == 0) {
    st->prefix = 0ull;
    st->mask = 0ull;
    st->k = k;
  }
}

__global__ __launch_bounds__(256) void select_hist_kernel(const double* __restrict__ x,
                                                          uint64_t n,
                                                          const SelectState* __restrict__ st,
                                                          uint32_t shift,
                                                          uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const unsigned long long prefix = st->prefix, mask = st->mask;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const unsigned long long key = order_key(x[i]);
    if ((key & mask) == prefix) atomicAdd(&h[(uint32_t)(key >> shift) & 255u], 1u);
  }
  __syncthreads();
  const uint32_t c = h[threadIdx.x];
  if (c) atomicAdd(&hist[threadIdx.x], c);
}

// One block of 256: inclusive scan of the digit counts, pick the digit whose
// cumulative count first reaches k.
__global__ __launch_bounds__(256) void select_pick_kernel(SelectState* st, uint32_t shift,
                                                          uint32_t* hist) {
  __shared__ unsigned long long c[256];
  __shared__ unsigned long long own[256];
  const int t = threadIdx.x;
  const unsigned long long v = hist[t];
  own[t] = v;
  c[t] = v;
  __syncthreads();
  hist[t] = 0u;                         // ready for the next pass
  for (int off = 1; off < 256; off <<= 1) {
    const unsigned long long add = t >= off ? c[t - off] : 0ull;
    __syncthreads();
    c[t] += add;
    __syncthreads();
  }
  const unsigned long long k = st->k;
  const unsigned long long below = c[t] - own[t];
  __syncthreads();
  if (below < k && k <= c[t]) {
    st->prefix |= (unsigned long long)t << shift;
    st->mask |= 0xFFull << shift;
    st->k = k - below;
  }
}

// Count and sum of the values whose key is strictly below the selected key.
__global__ __launch_bounds__(256) void tail_sum_kernel(const double* __restrict__ x, uint64_t n,
                                                       const SelectState* __restrict__ st,
                                                       double* __restrict__ partials) {
  const unsigned long long thr = st->prefix;
  double acc[2] = {0.0, 0.0};
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
    const double v = x[i];
    if (order_key(v) < thr) {
      acc[0] += 1.0;
      acc[1] += v;
    }
  }
  block_sum<2, 256>(acc, partials, gridDim.x);
}

uint32_t grid_for(uint64_t n) {
  const uint64_t need = (n + 255) / 256;
  return (uint32_t)(need < kSelBlocks ? need : kSelBlocks);
}

}  // namespace

hipError_t launch_select_kth(const double* x, uint64_t n, uint64_t k, void* state, uint32_t* hist,
                             hipStream_t s) {
  if (n == 0 || k == 0 || k > n) return hipErrorInvalidValue;
  SelectState* st = (SelectState*)state;
  hipLaunchKernelGGL(select_init_kernel, dim3(1), dim3(256), 0, s, st, hist,
                     (unsigned long long)k);
  const uint32_t nb = grid_for(n);
  for (int shift = 56; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL(select_hist_kernel, dim3(nb), dim3(256), 0, s, x, n, st, (uint32_t)shift,
                       hist);
    hipLaunchKernelGGL(select_pick_kernel, dim3(1), dim3(256), 0, s, st, (uint32_t)shift, hist);
  }
  return hipGetLastError();
}

hipError_t launch_tail_sum(const double* x, uint64_t n, const void* state, double* partials,
                           hipStream_t s, uint32_t* n_blocks) {
  const uint32_t nb = grid_for(n);
  *n_blocks = nb;
  if (nb == 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(tail_sum_kernel, dim3(nb), dim3(256), 0, s, x, n,
                     (const SelectState*)state, partials);
  return hipGetLastError();
}

double select_key_to_value(uint64_t key) {
  const uint64_t b = (key >> 63) ? (key & 0x7FFFFFFFFFFFFFFFull) : ~key;
  double v;
  static_assert(sizeof(v) == sizeof(b), "double is 64-bit");
  __builtin_memcpy(&v, &b, sizeof(v));
  return v;
}

}  // namespace mcp
