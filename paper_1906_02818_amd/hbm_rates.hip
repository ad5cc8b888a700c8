// Streaming HBM bandwidth of simple kernels, the practical ceiling beside the
// 8 TB/s datasheet peak for the memory-bound kernels (the Longstaff-Schwartz
// state stores and per-date reads): 16-byte loads reduced per thread, 4- and
// 16-byte stores, and a 16-byte device copy, each over 1 GiB (well beyond the
// last-level cache), grid-stride loops of 256-thread blocks at three grid
// sizes, three timed launches each (HIP events).
//   hipcc --offload-arch=gfx950 -O3 hbm_rates.hip -o hbm_rates && ./hbm_rates
// Memory: two 1 GiB buffers and a per-thread sink of the largest grid; every
// index stays below its buffer's element count.
#include <hip/hip_runtime.h>

#include <cstdio>

__global__ void read16(const float4* __restrict__ in, size_t n4, float* __restrict__ sink) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  float acc = 0.f;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    const float4 v = in[i];
    acc += v.x + v.y + v.z + v.w;
  }
  sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ void store16(float4* __restrict__ out, size_t n4, float v) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
    out[i] = make_float4(v, v + 1.f, v + 2.f, v + 3.f);
}

__global__ void store4(float* __restrict__ out, size_t n, float v) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = v + (float)(i & 7);
}

__global__ void copy16(const float4* __restrict__ in, float4* __restrict__ out, size_t n4) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
    out[i] = in[i];
}

#define CHECK(x)                                                          \
  do {                                                                    \
    hipError_t e = (x);                                                   \
    if (e != hipSuccess) {                                                \
      std::printf("HIP error %s at line %d\n", hipGetErrorString(e), __LINE__); \
      return 1;                                                           \
    }                                                                     \
  } while (0)

int main() {
  const size_t bytes = (size_t)1 << 30, n = bytes / 4, n4 = bytes / 16;
  const int grids[3] = {2048, 8192, 32768};
  float *a, *b, *sink;
  CHECK(hipMalloc(&a, bytes));
  CHECK(hipMalloc(&b, bytes));
  CHECK(hipMalloc(&sink, (size_t)32768 * 256 * sizeof(float)));
  CHECK(hipMemset(a, 0, bytes));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  std::printf("%-28s %8s %10s %10s\n", "kernel (1 GiB)", "grid", "best ms", "TB/s");
  for (int k = 0; k < 4; ++k) {
    for (int g = 0; g < 3; ++g) {
      float best = 1e30f;
      for (int rep = 0; rep < 4; ++rep) {   // the first launch is a warm-up
        CHECK(hipEventRecord(e0));
        if (k == 0)
          hipLaunchKernelGGL(read16, dim3(grids[g]), dim3(256), 0, 0, (const float4*)a, n4, sink);
        else if (k == 1)
          hipLaunchKernelGGL(store16, dim3(grids[g]), dim3(256), 0, 0, (float4*)b, n4, 1.0f);
        else if (k == 2)
          hipLaunchKernelGGL(store4, dim3(grids[g]), dim3(256), 0, 0, b, n, 1.0f);
        else
          hipLaunchKernelGGL(copy16, dim3(grids[g]), dim3(256), 0, 0, (const float4*)a,
                             (float4*)b, n4);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0 && ms < best) best = ms;
      }
      const char* name[4] = {"read, 16 B per lane", "store, 16 B per lane", "store, 4 B per lane",
                             "copy, 16 B per lane (r+w)"};
      const double moved = k == 3 ? 2.0 * bytes : (double)bytes;
      std::printf("%-28s %8d %10.3f %10.2f\n", name[k], grids[g], best, moved / (best * 1e-3) / 1e12);
    }
  }
  CHECK(hipFree(sink));
  CHECK(hipFree(b));
  CHECK(hipFree(a));
  return 0;
}
