// Issue-rate microbenchmark for the VALU instructions the path kernels are
// made of: the 32x32->64 integer product of Philox (v_mad_u64_u32, or the
// v_mul_hi_u32 / v_mul_lo_u32 pair), 32-bit xor, FP32 and FP64 FMA, and the
// transcendental unit (v_exp/log/sin/sqrt/rcp_f32), and the half-precision
// forms a cheaper activation would be built from (v_pk_fma_f16, two FMAs per
// lane; v_exp_f16, v_rcp_f16; v_cvt_pkrtz_f16_f32). Each chain step is ONE
// instruction of the measured kind (sign and absolute value are free source
// modifiers), each thread runs 8 independent chains and every SIMD holds 8
// waves, so latency is hidden. Output: wave64 instructions per clock per CU
// and the issue cost in units of a wave64 FMA at the FP32 vector peak
// ("spec slots"), from which the path kernels' ALU roofline is derived.
// A second table asks whether matrix-core work overlaps vector work on one
// SIMD: the same number of v_mfma_f32_32x32x16_bf16 and of independent
// v_fma_f32 run alone, interleaved in every wave, and split between waves
// (even waves matrix, odd waves vector); overlap shows as a mixed time near
// the larger of the two alone, serialisation as one near their sum.
//   hipcc --offload-arch=gfx950 -O3 isa_rates.hip -o isa_rates && ./isa_rates
// Memory: one store per thread into a buffer of exactly grid x block words.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
extern "C" __device__ _Float16 __ocml_exp2_f16(_Float16);

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

enum Op { FMA_F32, FMAC_F32, FMA_INL, BITOP3, EXP_3FMA, MAD_U64, MUL_HI, MUL_LO, XOR, EXP_F32, LOG_F32, SIN_F32, SQRT_F32, RCP_F32, FMA_F64, PK_FMA_F16, EXP_F16, RCP_F16, CVT_PKRTZ };

template <int OP>
__global__ __launch_bounds__(256) void rate_kernel(unsigned* out, unsigned seed, float kmul) {
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned a[kChains];
  float f[kChains];
  double d[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    a[c] = t * 2654435761u + seed + 977u * c;
    f[c] = 0.5f + 1e-7f * (float)(t & 1023) + 0.01f * c;
    d[c] = (double)f[c];
  }
  unsigned key = seed * 0x9E3779B9u;
  float g[kChains];                     // second FP32 chain of the overlap probe
#pragma unroll
  for (int c = 0; c < kChains; ++c) g[c] = 0.25f + 0.01f * c;
  h2 hv[kChains];                       // half-precision chains
#pragma unroll
  for (int c = 0; c < kChains; ++c) hv[c] = (h2){(_Float16)(0.5f + 0.01f * c), (_Float16)0.25f};
  unsigned f_bits[kChains];             // per-chain third operand (VGPR, loop invariant)
#pragma unroll
  for (int c = 0; c < kChains; ++c) f_bits[c] = t * 0x85EBCA6Bu + 31u * c;
  for (int it = 0; it < kIters; ++it) {
    key += 0xBB67AE85u;                                  // scalar, keeps the xor chain alive
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (OP == FMA_F32) {
        f[c] = __builtin_fmaf(f[c], 0.999f, 1e-3f);      // v_fmamk_f32 (32-bit literal)
      } else if constexpr (OP == FMAC_F32) {
        f[c] = __builtin_fmaf(kmul, f[(c + 1) % kChains], f[c]);   // v_fmac_f32, 4-byte form
      } else if constexpr (OP == FMA_INL) {
        f[c] = __builtin_fmaf(f[c], -0.5f, 2.0f);        // v_fma_f32 with inline constants
      } else if constexpr (OP == MAD_U64) {
        const unsigned long long p = (unsigned long long)a[c] * 0xD2511F53ull;
        a[c] = (unsigned)(p >> 32) ^ (unsigned)p;        // v_mad_u64_u32 + v_xor_b32
      } else if constexpr (OP == MUL_HI) {
        a[c] = __umulhi(a[c], 0xCD9E8D57u);
      } else if constexpr (OP == MUL_LO) {
        a[c] = a[c] * (key | 1u);                        // scalar factor: no folding
      } else if constexpr (OP == XOR) {
        a[c] = a[c] ^ key;
      } else if constexpr (OP == EXP_3FMA) {
        // One transcendental and three independent FMAs per step: issue time
        // tells whether the two kinds overlap (max) or add (sum).
        f[c] = __builtin_amdgcn_exp2f(-f[c]);
        g[c] = __builtin_fmaf(__builtin_fmaf(__builtin_fmaf(g[c], -0.5f, 2.0f), -0.5f, 2.0f),
                              -0.5f, 2.0f);
      } else if constexpr (OP == BITOP3) {
        a[c] = __builtin_amdgcn_bitop3_b32(a[c], key, f_bits[c], 0x96);   // a ^ key ^ const
      } else if constexpr (OP == EXP_F32) {
        f[c] = __builtin_amdgcn_exp2f(-f[c]);            // converges, stays finite
      } else if constexpr (OP == LOG_F32) {
        f[c] = __builtin_amdgcn_logf(__builtin_fabsf(f[c]) + 1.0f);   // log + add
      } else if constexpr (OP == SIN_F32) {
        f[c] = __builtin_amdgcn_sinf(f[c]);
      } else if constexpr (OP == SQRT_F32) {
        f[c] = __builtin_amdgcn_sqrtf(f[c]);
      } else if constexpr (OP == RCP_F32) {
        f[c] = __builtin_amdgcn_rcpf(f[c]);
      } else if constexpr (OP == FMA_F64) {
        d[c] = __builtin_fma(d[c], 0.999, 1e-3);
      } else if constexpr (OP == PK_FMA_F16) {
        hv[c] = __builtin_elementwise_fma(hv[c], (h2){(_Float16)-0.5f, (_Float16)-0.5f},
                                          (h2){(_Float16)2.0f, (_Float16)2.0f});
      } else if constexpr (OP == EXP_F16) {
        hv[c].x = __ocml_exp2_f16(-hv[c].x);                 // v_exp_f16
      } else if constexpr (OP == RCP_F16) {
        hv[c].x = __builtin_amdgcn_rcph(hv[c].x + (_Float16)1.0f);
      } else if constexpr (OP == CVT_PKRTZ) {
        const auto p = __builtin_amdgcn_cvt_pkrtz(f[c], f[c] + 1.0f);
        __builtin_memcpy(&hv[c], &p, 4);
        f[c] = (float)hv[c].x;
      }
    }
  }
  unsigned acc = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c)
    acc ^= a[c] ^ __float_as_uint(f[c]) ^ (unsigned)__double_as_longlong(d[c]) ^
           __float_as_uint(g[c]) ^ __builtin_bit_cast(unsigned, hv[c]);
  out[t] = acc;
}

template <int OP>
double run(unsigned* d_out, int blocks, int threads, hipEvent_t e0, hipEvent_t e1) {
  hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(threads), 0, 0, d_out, 1u, 1e-6f);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0, 0));
  for (int r = 0; r < 5; ++r)
    hipLaunchKernelGGL(rate_kernel<OP>, dim3(blocks), dim3(threads), 0, 0, d_out, 2u + r, 1e-6f);
  CHECK(hipEventRecord(e1, 0));
  CHECK(hipEventSynchronize(e1));
  float ms = 0.f;
  CHECK(hipEventElapsedTime(&ms, e0, e1));
  return ms / 5.0;
}

// Matrix/vector overlap probe. MODE 0: one MFMA per iteration (four
// accumulators in rotation, no back-to-back dependence); MODE 1: kMixFma
// independent FMAs per iteration; MODE 2: both in every wave; MODE 3: even
// waves run MODE 0, odd waves MODE 1 (twice the iterations each, so that
// every SIMD issues the same totals as in MODE 2). MODES 4 and 5 repeat 0
// and 2 with the accumulators in the accumulation registers (AGPRs) rather
// than the vector registers (an empty asm statement that names an AGPR
// makes the compiler choose that MFMA form).
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_t;
typedef __attribute__((ext_vector_type(16))) float f32x16_t;
constexpr int kMixIters = 4096, kMixFma = 16;

template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void mix_kernel(
    unsigned* out, float seed) {
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  const int wave = threadIdx.x >> 6;
  bf16x8_t a, b;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = (__bf16)(1e-3f * (float)((t + j) & 7));
    b[j] = (__bf16)(1e-3f * (float)((t * 3 + j) & 7));
  }
  f32x16_t acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[q][r] = 0.f;
  float f[kMixFma];
#pragma unroll
  for (int c = 0; c < kMixFma; ++c) f[c] = seed + 0.01f * c + 1e-7f * (float)(t & 255);
  if constexpr (MODE >= 4) {
    float zz = seed;
    __asm__ volatile("; accumulation register in use: %0" : "+a"(zz));
    f[0] += zz;
  }
  const bool do_m = MODE == 0 || MODE == 2 || MODE >= 4 || (MODE == 3 && (wave & 1) == 0);
  const bool do_v = MODE == 1 || MODE == 2 || MODE == 5 || (MODE == 3 && (wave & 1) == 1);
  const int iters = MODE == 3 ? 2 * kMixIters : kMixIters;
  for (int it = 0; it < iters; it += 4) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (do_m) acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[q], 0, 0, 0);
      if (do_v) {
#pragma unroll
        for (int c = 0; c < kMixFma; ++c) f[c] = __builtin_fmaf(f[c], -0.5f, 2.0f);
      }
    }
  }
  unsigned x = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) x ^= __float_as_uint(acc[q][r]);
#pragma unroll
  for (int c = 0; c < kMixFma; ++c) x ^= __float_as_uint(f[c]);
  out[t] = x;
}

template <int MODE>
double run_mix(unsigned* d_out, int blocks, int threads, hipEvent_t e0, hipEvent_t e1) {
  hipLaunchKernelGGL(mix_kernel<MODE>, dim3(blocks), dim3(threads), 0, 0, d_out, 0.5f);
  CHECK(hipGetLastError());
  CHECK(hipDeviceSynchronize());
  CHECK(hipEventRecord(e0, 0));
  for (int r = 0; r < 5; ++r)
    hipLaunchKernelGGL(mix_kernel<MODE>, dim3(blocks), dim3(threads), 0, 0, d_out, 0.5f + r);
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
  const double steps = (double)blocks * threads / 64.0 * kIters * kChains;   // wave64 chain steps
  struct Row { const char* name; double ms; double extra; };   // extra: helper insts per step
  Row rows[] = {
      {"v_fmamk_f32 (literal)", run<FMA_F32>(d_out, blocks, threads, e0, e1), 0.0},
      {"v_fmac_f32", run<FMAC_F32>(d_out, blocks, threads, e0, e1), 0.0},
      {"v_fma_f32 (inline consts)", run<FMA_INL>(d_out, blocks, threads, e0, e1), 0.0},
      {"v_mad_u64_u32 (+ v_xor_b32)", run<MAD_U64>(d_out, blocks, threads, e0, e1), 1.0},
      {"v_mul_hi_u32", run<MUL_HI>(d_out, blocks, threads, e0, e1), 0.0},
      {"v_mul_lo_u32", run<MUL_LO>(d_out, blocks, threads, e0, e1), 0.0},
      {"v_xor_b32", run<XOR>(d_out, blocks, threads, e0, e1), 0.0},
      {"v_bitop3_b32 (xor3)", run<BITOP3>(d_out, blocks, threads, e0, e1), 0.0},
      {"v_exp_f32 + 3 v_fma_f32", run<EXP_3FMA>(d_out, blocks, threads, e0, e1), 0.0},
      {"v_exp_f32", run<EXP_F32>(d_out, blocks, threads, e0, e1), 0.0},
      {"v_log_f32 (+ v_add_f32)", run<LOG_F32>(d_out, blocks, threads, e0, e1), 1.0},
      {"v_sin_f32", run<SIN_F32>(d_out, blocks, threads, e0, e1), 0.0},
      {"v_sqrt_f32", run<SQRT_F32>(d_out, blocks, threads, e0, e1), 0.0},
      {"v_rcp_f32", run<RCP_F32>(d_out, blocks, threads, e0, e1), 0.0},
      {"v_fma_f64", run<FMA_F64>(d_out, blocks, threads, e0, e1), 0.0},
      {"v_pk_fma_f16 (2 FMA/lane)", run<PK_FMA_F16>(d_out, blocks, threads, e0, e1), 0.0},
      {"v_exp_f16", run<EXP_F16>(d_out, blocks, threads, e0, e1), 0.0},
      {"v_rcp_f16 (+ v_add_f16)", run<RCP_F16>(d_out, blocks, threads, e0, e1), 1.0},
      {"v_cvt_pkrtz_f16_f32 (+cvt)", run<CVT_PKRTZ>(d_out, blocks, threads, e0, e1), 2.0},
  };
  // "spec slots": issue time in units of one wave64 FMA at the FP32 vector
  // peak (128 FMA lanes per clock per CU = 2 wave64 FMAs per clock per CU).
  // The helper instruction of a two-instruction chain step is not subtracted
  // here; its own row gives its cost.
  std::printf("%-28s %10s %18s %12s\n", "op", "ms", "wave-insts/clk/CU", "spec slots");
  for (const Row& r : rows) {
    const double rate = steps / (r.ms * 1e-3 * clk_ghz * 1e9) / cus;   // chain steps
    std::printf("%-28s %10.4f %18.4f %12.3f\n", r.name, r.ms, rate, 2.0 / rate);
  }
  // Overlap probe: 4 waves per SIMD (16 per CU), each SIMD issuing
  // 4 x kMixIters MFMAs and 4 x kMixIters x kMixFma FMAs in modes 2 and 3.
  {
    const int mblocks = cus * 4;
    const double m_only = run_mix<0>(d_out, mblocks, threads, e0, e1);
    const double v_only = run_mix<1>(d_out, mblocks, threads, e0, e1);
    const double both = run_mix<2>(d_out, mblocks, threads, e0, e1);
    const double split = run_mix<3>(d_out, mblocks, threads, e0, e1);
    const double m_only_a = run_mix<4>(d_out, mblocks, threads, e0, e1);
    const double both_a = run_mix<5>(d_out, mblocks, threads, e0, e1);
    const double cyc = clk_ghz * 1e6;   // cycles per ms
    const double per_simd_mfma = 4.0 * kMixIters, per_simd_fma = 4.0 * kMixIters * kMixFma;
    std::printf("\nmatrix/vector overlap (per SIMD: %.0f v_mfma_f32_32x32x16_bf16, %.0f v_fma_f32)\n",
                per_simd_mfma, per_simd_fma);
    std::printf("%-34s %10s %16s\n", "case", "ms", "cycles per SIMD");
    std::printf("%-34s %10.4f %16.0f  (%.1f cycles per MFMA)\n", "MFMA alone", m_only,
                m_only * cyc, m_only * cyc / per_simd_mfma);
    std::printf("%-34s %10.4f %16.0f  (%.2f cycles per FMA)\n", "FMA alone", v_only, v_only * cyc,
                v_only * cyc / per_simd_fma);
    std::printf("%-34s %10.4f %16.0f\n", "both, interleaved in every wave", both, both * cyc);
    std::printf("%-34s %10.4f %16.0f\n", "split: matrix waves + vector waves", split, split * cyc);
    std::printf("%-34s %10.4f %16.0f  (%.1f cycles per MFMA)\n", "MFMA alone, AGPR accumulators",
                m_only_a, m_only_a * cyc, m_only_a * cyc / per_simd_mfma);
    std::printf("%-34s %10.4f %16.0f\n", "both, AGPR accumulators", both_a, both_a * cyc);
    std::printf("sum of the two alone %.4f ms, larger of the two %.4f ms\n", m_only + v_only,
                m_only > v_only ? m_only : v_only);
  }
  CHECK(hipFree(d_out));
  return 0;
}
