// Second stage of the averaging reduction (Eq. 3) and its variance term
// (Sec. V-B), the reduction of a multilevel correction (difference of two
// runs on the same paths), plain sums, and the
// diagnostic kernels that expose the device random numbers for bit-exact
// checks.
#include "device/reduce.h"
#include "device/rng.h"
#include "mc_internal.h"

namespace mcp {
namespace {

// Plain sums (counts, tail sums, gradients): one workgroup per entry m of
// batch b = blockIdx.y; thread t adds blocks t, t+256, ... in order, then a
// fixed-shape tree adds the 256 partial sums. Deterministic. partials
// [b][m][n_blocks], out [b][n_mom].
__global__ __launch_bounds__(256) void final_reduce_kernel(const double* __restrict__ partials,
                                                           uint32_t n_blocks,
                                                           double* __restrict__ out) {
  __shared__ double sh[256];
  const uint32_t m = blockIdx.x;
  partials += (size_t)blockIdx.y * gridDim.x * n_blocks;
  out += (size_t)blockIdx.y * gridDim.x;
  const double* row = partials + (size_t)m * n_blocks;
  double s = 0.0;
  for (uint32_t i = threadIdx.x; i < n_blocks; i += 256) s += row[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[m] = sh[0];
}

// Moment vectors of C channels (count, means, co-moments): one workgroup of
// NT threads per batch b = blockIdx.x merges the block-major partials
// [b][n_blocks][M], vector i at i * stride * M, into out[b][M]: thread t adds
// vectors t, t + NT, ... in order (about a shift, no division), then the
// block reduction of the path kernels.
template <int C>
constexpr int merge_threads() { return 256; }

template <int C>
__global__ __launch_bounds__(merge_threads<C>()) void final_merge_kernel(
    const double* __restrict__ partials, uint32_t n_blocks, uint32_t stride,
    double* __restrict__ out) {
  constexpr int M = PartSums<C>::M, NT = merge_threads<C>();
  partials += (size_t)blockIdx.x * n_blocks * M;
  PartSums<C> m;
  m.zero();
#pragma unroll 4
  for (uint32_t i = threadIdx.x; i < n_blocks; i += NT)
    m.add_vector(partials + (size_t)i * stride * M);
  block_reduce<C, NT>(m, out, blockIdx.x);
}

// First stage of a long merge (one batch): workgroup g merges the kMergeChunk
// vectors from g * kMergeChunk (fewer in the last chunk) as above and writes
// the result over the chunk's first vector, which no other workgroup reads;
// the block reduction's barrier orders every thread's reads before it.
constexpr uint32_t kMergeChunk = 2048;

template <int C>
__global__ __launch_bounds__(merge_threads<C>()) void chunk_merge_kernel(
    double* __restrict__ partials, uint32_t n_blocks) {
  constexpr int M = PartSums<C>::M, NT = merge_threads<C>();
  const uint32_t first = blockIdx.x * kMergeChunk;
  const uint32_t count = min(kMergeChunk, n_blocks - first);
  double* head = partials + (size_t)first * M;
  PartSums<C> m;
  m.zero();
#pragma unroll 4
  for (uint32_t i = threadIdx.x; i < count; i += NT) m.add_vector(head + (size_t)i * M);
  block_reduce<C, NT>(m, head, 0);
}

__global__ void philox_words_kernel(uint32_t k0, uint32_t k1, uint32_t tag, uint64_t n,
                                    const uint64_t* __restrict__ paths,
                                    const uint64_t* __restrict__ blocks,
                                    uint32_t* __restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const PathCounter pc = make_counter(paths[i], tag, k0, k1);
  const Words4 w = philox((uint32_t)blocks[i], pc);
  out[4 * i + 0] = w.w0;
  out[4 * i + 1] = w.w1;
  out[4 * i + 2] = w.w2;
  out[4 * i + 3] = w.w3;
}

template <typename R>
__global__ void normals_kernel(uint32_t k0, uint32_t k1, uint32_t tag, uint64_t path,
                               uint64_t k_first, uint64_t count, double* __restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t k = k_first + i;
  const PathCounter pc = make_counter(path, tag, k0, k1);
  const Normals4<R> nz = normals4<R>(philox((uint32_t)(k >> 2), pc));
  out[i] = (double)nz.z[k & 3];
}

// Moments of y = (a[ca] - b[cb], a[ca], b[cb]) per path, a and b row-major
// [n][Ca] and [n][Cb] tables of two runs on the same paths. The difference
// is taken in FP64 from the stored values, so its variance carries no
// cancellation from the cross moments.
__global__ __launch_bounds__(kBlock) void diff_moments_kernel(const double* __restrict__ a,
                                                              uint32_t Ca, uint32_t ca,
                                                              const double* __restrict__ b,
                                                              uint32_t Cb, uint32_t cb, uint64_t n,
                                                              double* __restrict__ partials) {
  ThreadSums<3> acc;
  acc.zero();
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const double fa = a[i * Ca + ca], fb = b[i * Cb + cb];
    const double y[3] = {fa - fb, fa, fb};
    const bool finite = isfinite(y[0]) && isfinite(fa) && isfinite(fb);
    acc.push(y, finite, !finite);
  }
  PartSums<3> part = acc.part();
  block_reduce<3, kBlock>(part, partials, blockIdx.x);
}

// Shift row of replicate replicate0 + blockIdx.y: [blockIdx.y][n_dims].
__global__ void qmc_shift_kernel(uint32_t k0, uint32_t k1, uint32_t tag, uint64_t replicate0,
                                 uint32_t n_dims, uint32_t* __restrict__ shift) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;   // block index
  if (4u * j >= n_dims) return;
  shift += (size_t)blockIdx.y * n_dims;
  const PathCounter pc = make_counter(replicate0 + blockIdx.y, tag, k0, k1);
  const Words4 w = philox(j, pc);
  for (uint32_t t = 0; t < 4u && 4u * j + t < n_dims; ++t) shift[4u * j + t] = word_at(w, t);
}

}  // namespace

hipError_t launch_qmc_shifts(uint32_t k0, uint32_t k1, uint32_t tag, uint64_t replicate0,
                             uint32_t n_rep, uint32_t n_dims, uint32_t* shift, hipStream_t s) {
  const uint32_t blocks = (n_dims + 3u) / 4u;
  if (blocks == 0 || n_rep == 0 || n_rep > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(qmc_shift_kernel, dim3((blocks + 255) / 256, n_rep), dim3(256), 0, s, k0, k1,
                     tag, replicate0, n_dims, shift);
  return hipGetLastError();
}

hipError_t launch_diff_moments(const double* a, uint32_t Ca, uint32_t ca, const double* b,
                               uint32_t Cb, uint32_t cb, uint64_t n, double* partials,
                               hipStream_t s, uint32_t* n_blocks) {
  const uint64_t need = (n + kBlock - 1) / kBlock;
  const uint32_t nb = (uint32_t)(need < kDiffMaxBlocks ? need : kDiffMaxBlocks);
  *n_blocks = nb;
  if (nb == 0 || ca >= Ca || cb >= Cb) return hipErrorInvalidValue;
  hipLaunchKernelGGL(diff_moments_kernel, dim3(nb), dim3(kBlock), 0, s, a, Ca, ca, b, Cb, cb, n,
                     partials);
  return hipGetLastError();
}

// One batch of more than two chunks merges in two stages: chunk heads,
// then the heads in chunk order (a fixed order either way); the partials'
// chunk heads are overwritten.
template <int C>
static hipError_t merge_one(double* partials, uint32_t n_blocks, uint32_t n_batch,
                            double* out, hipStream_t s) {
  if (n_batch == 1 && n_blocks > 2 * kMergeChunk) {
    const uint32_t n_chunks = (n_blocks + kMergeChunk - 1) / kMergeChunk;
    hipLaunchKernelGGL(chunk_merge_kernel<C>, dim3(n_chunks), dim3(merge_threads<C>()), 0, s,
                       partials, n_blocks);
    hipLaunchKernelGGL(final_merge_kernel<C>, dim3(1), dim3(merge_threads<C>()), 0, s, partials,
                       n_chunks, kMergeChunk, out);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(final_merge_kernel<C>, dim3(n_batch), dim3(merge_threads<C>()), 0, s,
                     partials, n_blocks, 1u, out);
  return hipGetLastError();
}

hipError_t launch_final_merge(double* partials, uint32_t n_blocks, uint32_t C,
                              uint32_t n_batch, double* out, hipStream_t s) {
  if (n_blocks == 0 || n_batch == 0 || n_batch > 65535) return hipErrorInvalidValue;
  switch (C) {
    case 1: return merge_one<1>(partials, n_blocks, n_batch, out, s);
    case 2: return merge_one<2>(partials, n_blocks, n_batch, out, s);
    case 3: return merge_one<3>(partials, n_blocks, n_batch, out, s);
    case 4: return merge_one<4>(partials, n_blocks, n_batch, out, s);
    case 5: return merge_one<5>(partials, n_blocks, n_batch, out, s);
    case 6: return merge_one<6>(partials, n_blocks, n_batch, out, s);
    case 7: return merge_one<7>(partials, n_blocks, n_batch, out, s);
    case 8: return merge_one<8>(partials, n_blocks, n_batch, out, s);
    case 9: return merge_one<9>(partials, n_blocks, n_batch, out, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_final_reduce(const double* partials, uint32_t n_blocks, uint32_t n_mom,
                               double* out, hipStream_t s) {
  hipLaunchKernelGGL(final_reduce_kernel, dim3(n_mom), dim3(256), 0, s, partials, n_blocks, out);
  return hipGetLastError();
}

hipError_t launch_final_reduce_batch(const double* partials, uint32_t n_blocks, uint32_t n_mom,
                                     uint32_t n_batch, double* out, hipStream_t s) {
  if (n_blocks == 0 || n_mom == 0 || n_batch == 0 || n_batch > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(final_reduce_kernel, dim3(n_mom, n_batch), dim3(256), 0, s, partials,
                     n_blocks, out);
  return hipGetLastError();
}

hipError_t launch_philox_words(uint32_t k0, uint32_t k1, uint32_t tag, uint64_t n,
                               const uint64_t* paths, const uint64_t* blocks, uint32_t* out,
                               hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t nb = (uint32_t)((n + 255) / 256);
  hipLaunchKernelGGL(philox_words_kernel, dim3(nb), dim3(256), 0, s, k0, k1, tag, n, paths,
                     blocks, out);
  return hipGetLastError();
}

hipError_t launch_normals(uint32_t k0, uint32_t k1, uint32_t tag, uint64_t path,
                          uint64_t k_first, uint64_t count, bool fp64, double* out,
                          hipStream_t s) {
  if (count == 0) return hipSuccess;
  const uint32_t nb = (uint32_t)((count + 255) / 256);
  if (fp64)
    hipLaunchKernelGGL(normals_kernel<double>, dim3(nb), dim3(256), 0, s, k0, k1, tag, path,
                       k_first, count, out);
  else
    hipLaunchKernelGGL(normals_kernel<float>, dim3(nb), dim3(256), 0, s, k0, k1, tag, path,
                       k_first, count, out);
  return hipGetLastError();
}

}  // namespace mcp
