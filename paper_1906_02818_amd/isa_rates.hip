// Issue-rate microbenchmark for the VALU instructions the path kernels are
// made of: the 32x32->64 integer multiply of Philox (v_mad_u64_u32), the
// mul-hi/lo pair, FP32 and FP64 FMA and the transcendental unit
// (v_exp/log/sin/sqrt_f32). Each thread runs 8 independent dependency chains
// so that latency is hidden; the result is wave64 instructions per cycle per
// CU, from which the kernels' ALU roofline is derived. Standalone program:
//   hipcc --offload-arch=gfx950 -O3 isa_rates.hip -o isa_rates && ./isa_rates
// Only one store per thread touches memory (to keep the chains alive); the
// output buffer holds exactly grid*block elements.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                              \
  do {                                                                        \
    hipError_t e = (x);                                                       \
    if (e != hipSuccess) {                                                    \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e));            \
      std::exit(1);                                                           \
    }                                                                         \
  } while (0)

constexpr int kIters = 2048;
constexpr int kChains = 8;

enum Op { MAD_U64, MULHI_LO, FMA_F32, EXP_F32, LOG_F32, SIN_F32, SQRT_F32, FMA_F64 };

template <int OP>
__global__ __launch_bounds__(256) void rate_kernel(unsigned* out, unsigned seed) {
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned a[kChains];
  float f[kChains];
  double d[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    a[c] = t * 2654435761u + seed + c;
    f[c] = 0.5f + 1e-7f * (float)(t & 1023) + 0.01f * c;
    d[c] = (double)f[c];
  }
  for (int it = 0; it < kIters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (OP == MAD_U64) {
        const unsigned long long p = (unsigned long long)a[c] * 0xD2511F53ull;
        a[c] = (unsigned)(p >> 32) ^ (unsigned)p;   // 1 mad + 1 xor
      } else if constexpr (OP == MULHI_LO) {
        a[c] = __umulhi(a[c], 0xCD9E8D57u) ^ (a[c] * 0xCD9E8D57u);
      } else if constexpr (OP == FMA_F32) {
        f[c] = __builtin_fmaf(f[c], 0.999f, 1e-3f);
      } else if constexpr (OP == EXP_F32) {
        f[c] = __builtin_amdgcn_exp2f(f[c]) * -0.5f;
      } else if constexpr (OP == LOG_F32) {
        f[c] = __builtin_amdgcn_logf(f[c]) * -0.5f + 1.5f;
      } else if constexpr (OP == SIN_F32) {
        f[c] = __builtin_amdgcn_sinf(f[c]);
      } else if constexpr (OP == SQRT_F32) {
        f[c] = __builtin_amdgcn_sqrtf(f[c]) + 0.25f;
      } else if constexpr (OP == FMA_F64) {
        d[c] = __builtin_fma(d[c], 0.999, 1e-3);
      }
    }
  }
  unsigned acc = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c)
    acc ^= a[c] ^ __float_as_uint(f[c]) ^ (unsigned)__double_as_longlong(d[c]);
  out[t] = acc;
}

template <int OP>
double run(unsigned* d_out, int blocks, int threads, hipEvent_t e0, hipEvent_t e1) {
  hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(threads), 0, 0, d_out, 1u);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0, 0));
  for (int r = 0; r < 5; ++r)
    hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(threads), 0, 0, d_out, 2u + r);
  CHECK(hipEventRecord(e1, 0));
  CHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  return ms / 5.0;
}

int main() {
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, 0));
  const int cus = prop.multiProcessorCount;
  const double clk_ghz = prop.clockRate / 1e6;
  const int threads = 256;
  const int blocks = cus * 32;              // 8 waves per SIMD
  unsigned* d_out = nullptr;
  CHECK(hipMalloc(&d_out, (size_t)blocks * threads * sizeof(unsigned)));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  std::printf("device %s, %d CUs, clock %.3f GHz\n", prop.name, cus, clk_ghz);
  const double waves = (double)blocks * threads / 64.0;
  const double steps = waves * kIters * kChains;   // wave64 chain steps
  struct Row { const char* name; double ms; double insts_per_step; };
  Row rows[] = {
      {"v_mad_u64_u32 (+1 xor)", run<MAD_U64>(d_out, blocks, threads, e0, e1), 2.0},
      {"v_mul_hi_u32+v_mul_lo_u32 (+1 xor)", run<MULHI_LO>(d_out, blocks, threads, e0, e1), 3.0},
      {"v_fma_f32", run<FMA_F32>(d_out, blocks, threads, e0, e1), 1.0},
      {"v_exp_f32 (+1 mul)", run<EXP_F32>(d_out, blocks, threads, e0, e1), 2.0},
      {"v_log_f32 (+1 fma)", run<LOG_F32>(d_out, blocks, threads, e0, e1), 2.0},
      {"v_sin_f32", run<SIN_F32>(d_out, blocks, threads, e0, e1), 1.0},
      {"v_sqrt_f32 (+1 add)", run<SQRT_F32>(d_out, blocks, threads, e0, e1), 2.0},
      {"v_fma_f64", run<FMA_F64>(d_out, blocks, threads, e0, e1), 1.0},
  };
  std::printf("%-36s %10s %16s %18s\n", "op", "ms", "chain steps/clk/CU", "wave-insts/clk/CU");
  for (const Row& r : rows) {
    const double cycles = r.ms * 1e-3 * clk_ghz * 1e9;
    const double per_cu = steps / cycles / cus;
    std::printf("%-36s %10.4f %16.4f %18.4f\n", r.name, r.ms, per_cu, per_cu * r.insts_per_step);
  }
  CHECK(hipFree(d_out));
  return 0;
}
