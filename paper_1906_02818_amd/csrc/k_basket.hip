// Basket path kernel: d correlated GBM assets stepped by log-Euler (the
// multivariate Euler-Maruyama scheme of Sec. II-A.2), where each time step
// needs the correlated increment Z L^T, a (paths x d) by (d x d) matrix
// product, on the matrix cores (the MXU product of Sec. VI-A.2 done with
// gfx950 MFMA instead).
//
// Layout. A wave owns a tile of 32 paths x d assets. The log-prices live in
// the MFMA accumulators (d/32 blocks of 32x32 FP32, 16 values per lane per
// block): with L' = diag(sigma_a sqrt(dt)) L the step is
//     X += Z_i L'^T
// and the deterministic drift n (r - sigma_a^2/2) dt is added once after
// the last step (the step is linear in it). Each lane draws the 8 normals
// of its A-operand fragment (path = lane mod 32, assets 16 kb + 8 (lane/32)
// + 0..7) straight from Philox, so Z never touches memory. L' sits in LDS
// as the packed lower-triangular 32x16 blocks (n block nb, k block kb <=
// 2 nb + 1), so the upper triangle costs neither MFMA issue nor LDS.
//
// Precisions: FP32 (v_mfma_f32_32x32x2f32, K permuted inside each 16-wide
// k block so that a lane still consumes its 8 contiguous normals), BF16 and
// FP16 (v_mfma_f32_32x32x16_*), and BF16 with L' split into hi + lo terms.
// Accumulation is FP32 in every case.
#include "device/reduce.h"
#include "device/rng.h"
#include "mc_internal.h"

namespace mcp {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) _Float16 f16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kWaves = 8;                 // 8 tiles of 32 paths per workgroup
constexpr int kThreads = 64 * kWaves;

template <int PREC>
struct BElt;
template <> struct BElt<BK_FP32> { typedef float T; };
template <> struct BElt<BK_BF16> { typedef __bf16 T; };
template <> struct BElt<BK_FP16> { typedef _Float16 T; };
template <> struct BElt<BK_BF16X2> { typedef __bf16 T; };

template <int PREC>
__device__ __forceinline__ void mfma_block(f32x16& acc, const float (&z)[8],
                                           const unsigned char* lds_hi,
                                           const unsigned char* lds_lo, int off_elems) {
  if constexpr (PREC == BK_FP32) {
    const float* b = (const float*)lds_hi + off_elems;
    const float4 b0 = *(const float4*)(b);
    const float4 b1 = *(const float4*)(b + 4);
    const float bb[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
    for (int kk = 0; kk < 8; ++kk)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(z[kk], bb[kk], acc, 0, 0, 0);
  } else if constexpr (PREC == BK_FP16) {
    f16x8 a;
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (_Float16)z[j];
    const f16x8 b = *(const f16x8*)((const _Float16*)lds_hi + off_elems);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc, 0, 0, 0);
  } else {
    bf16x8 a;
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = (__bf16)z[j];
    const bf16x8 b = *(const bf16x8*)((const __bf16*)lds_hi + off_elems);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    if constexpr (PREC == BK_BF16X2) {
      const bf16x8 bl = *(const bf16x8*)((const __bf16*)lds_lo + off_elems);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bl, acc, 0, 0, 0);
    }
  }
}

template <int ND, int PREC, bool PORT, bool QMC>
__global__ __launch_bounds__(kThreads) void basket_kernel(const BasketParams P) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  constexpr int NBLK = ND * (ND + 1);                 // packed triangular blocks
  constexpr int ELT = sizeof(typename BElt<PREC>::T);
  constexpr int BLK_BYTES = NBLK * 512 * ELT;
  // Stage L' (and its lo part) into LDS.
  {
    const uint4* src = (const uint4*)P.Lblk;
    uint4* dst = (uint4*)lds;
    for (int i = threadIdx.x; i < BLK_BYTES / 16; i += kThreads) dst[i] = src[i];
    if constexpr (PREC == BK_BF16X2) {
      const uint4* src2 = (const uint4*)P.Lblk_lo;
      uint4* dst2 = (uint4*)(lds + BLK_BYTES);
      for (int i = threadIdx.x; i < BLK_BYTES / 16; i += kThreads) dst2[i] = src2[i];
    }
  }
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int row = lane & 31;          // A row / B and D column
  const int half = lane >> 5;
  // Block blk of the launch, or of its replicate when replicates share it.
  uint32_t blk = blockIdx.x;
  const uint32_t* qshift = P.qshift;
  double* partials = P.partials;
  if constexpr (QMC) {
    if (P.q_rep_blocks != 0) {
      const uint32_t rep = blockIdx.x / P.q_rep_blocks;
      blk = blockIdx.x - rep * P.q_rep_blocks;
      qshift += (size_t)rep * P.q_dims;
      partials += (size_t)rep * n_moments(PORT ? 1 : 3) * P.q_rep_blocks;
    }
  }
  const uint64_t tile = (uint64_t)blk * kWaves + wave;
  const uint64_t zpath = tile * 32 + row;             // path this lane draws normals for
  const PathCounter pc = make_counter(P.path_offset + zpath, P.tag, P.k0, P.k1);
  const uint32_t d = P.d;
  const int nkb = (int)(d >> 4);

  f32x16 acc[ND];
#pragma unroll
  for (int nb = 0; nb < ND; ++nb)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;

  for (uint32_t i = 0; i < P.n_steps; ++i) {
    const uint64_t kbase = (uint64_t)i * d;          // first normal of step i
#pragma unroll
    for (int kb = 0; kb < 2 * ND; ++kb) {
      if (kb < nkb) {
        const uint32_t j0 = (uint32_t)((kbase + 16u * kb + 8u * half) >> 2);
        Words4 wa, wb;
        if constexpr (QMC) {
          const uint32_t point = (uint32_t)(P.path_offset + zpath);
          wa = sobol_block(P.qV, qshift, j0, point);
          wb = sobol_block(P.qV, qshift, j0 + 1, point);
        } else {
          wa = philox(j0, pc);
          wb = philox(j0 + 1, pc);
        }
        const Normals4<float> za = normals4<float>(wa);
        const Normals4<float> zb = normals4<float>(wb);
        const float z[8] = {za.z[0], za.z[1], za.z[2], za.z[3],
                            zb.z[0], zb.z[1], zb.z[2], zb.z[3]};
#pragma unroll
        for (int nb = kb >> 1; nb < ND; ++nb) {
          const int id = nb * (nb + 1) + kb;
          mfma_block<PREC>(acc[nb], z, lds, lds + BLK_BYTES, (id * 32 + row) * 16 + 8 * half);
        }
      }
    }
  }

  // Terminal values. Lane holds asset a = 32 nb + row for path rows
  // 8 (r/4) + 4 half + (r mod 4), r = 0..15. One row r at a time: the sum
  // over the lane's assets, then over the 32 lanes of its half (few live
  // registers beside the accumulators).
  float B = 0.f, G = 0.f, E0 = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    float bs = 0.f, gs = 0.f, e0 = 0.f;
#pragma unroll
    for (int nb = 0; nb < ND; ++nb) {
      const int a = 32 * nb + row;
      const float x = acc[nb][r] + P.asset[a];          // log2(S_a / S0_a)
      const float E = __builtin_amdgcn_exp2f(x);
      if constexpr (PORT) {
        // Portfolio value of asset a: S0_a sum_k q_k (E - m_k)^+ (zero-padded
        // assets carry S0 = 0).
        float v = 0.f;
        for (uint32_t k = 0; k < P.n_strikes; ++k) {
          const float itm = E - P.pm[k];
          v = __builtin_fmaf(P.pq[k], itm > 0.f ? itm : 0.f, v);
        }
        bs = __builtin_fmaf(P.asset[768 + a], v, bs);
      } else {
        bs += P.asset[256 + a] * E;
        gs += P.asset[512 + a] * x;
        if (nb == 0) e0 = E;
      }
    }
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) {
      bs += __shfl_xor(bs, off, 64);
      if constexpr (!PORT) gs += __shfl_xor(gs, off, 64);
    }
    if constexpr (!PORT) e0 = __shfl(e0, lane & 32, 64);   // asset 0 sits in column 0
    // Lane (half, row < 16) reports path row 8 (row/4) + 4 half + row mod 4.
    if (r == row) {
      B = bs;
      G = gs;
      E0 = e0;
    }
  }
  const int prow = 8 * (row >> 2) + 4 * half + (row & 3);
  const uint64_t pid = tile * 32 + prow;
  const bool active = row < 16 && pid < P.n_paths;
  if constexpr (PORT) {
    double y[1] = {0.0};
    if (active) y[0] = (double)B - P.premium;
    const bool finite = isfinite(y[0]);
    if (active && P.path_out != nullptr) P.path_out[pid] = y[0];
    block_moments<1, kThreads>(y, active && finite, active && !finite, partials, blk);
  } else {
    double y[3] = {0.0, 0.0, 0.0};
    if (active) {
      const double disc = P.disc, K = P.K;
      const double basket = (double)B;
      const double geo = exp(P.geo0 + (double)G);
      y[0] = disc * (basket > K ? basket - K : 0.0);
      y[1] = disc * (geo > K ? geo - K : 0.0);
      y[2] = basket > K ? disc * P.w0 * (double)E0 : 0.0;
    }
    bool finite = isfinite(y[0]) && isfinite(y[1]) && isfinite(y[2]);
    if (active && P.path_out != nullptr) {
#pragma unroll
      for (int c = 0; c < 3; ++c) P.path_out[pid * 3 + c] = y[c];
    }
    block_moments<3, kThreads>(y, active && finite, active && !finite, partials, blk);
  }
}

template <int ND, int PREC, bool PORT, bool QMC>
hipError_t launch_nd_mode(const BasketParams& p, hipStream_t s, uint32_t nb) {
  constexpr int NBLK = ND * (ND + 1);
  constexpr int ELT = sizeof(typename BElt<PREC>::T);
  const size_t lds = (size_t)NBLK * 512 * ELT * (PREC == BK_BF16X2 ? 2 : 1);
  hipError_t e = hipFuncSetAttribute((const void*)basket_kernel<ND, PREC, PORT, QMC>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((basket_kernel<ND, PREC, PORT, QMC>), dim3(nb), dim3(kThreads), lds, s, p);
  return hipGetLastError();
}

template <int ND, int PREC>
hipError_t launch_nd(const BasketParams& p, hipStream_t s, uint32_t nb) {
  if constexpr (PREC == BK_BF16X2) {   // basket call with Philox normals only
    if (p.n_strikes != 0 || p.qV != nullptr) return hipErrorInvalidValue;
    return launch_nd_mode<ND, PREC, false, false>(p, s, nb);
  } else {
    if (p.qV != nullptr) {
      if (p.n_strikes != 0) return hipErrorInvalidValue;
      return launch_nd_mode<ND, PREC, false, true>(p, s, nb);
    }
    if (p.n_strikes == 0) return launch_nd_mode<ND, PREC, false, false>(p, s, nb);
    return launch_nd_mode<ND, PREC, true, false>(p, s, nb);
  }
}

template <int PREC>
hipError_t launch_prec(const BasketParams& p, hipStream_t s, uint32_t nb) {
  const uint32_t nd = (p.d + 31) / 32;
  if (nd <= 1) return launch_nd<1, PREC>(p, s, nb);
  if (nd <= 2) return launch_nd<2, PREC>(p, s, nb);
  if (nd <= 4) return launch_nd<4, PREC>(p, s, nb);
  return launch_nd<8, PREC>(p, s, nb);
}

}  // namespace

uint32_t basket_blocks_nd(uint32_t d) {
  const uint32_t nd = (d + 31) / 32;
  return nd <= 1 ? 1 : nd <= 2 ? 2 : nd <= 4 ? 4 : 8;
}

hipError_t launch_basket_qmc_batch(BasketParams p, int prec, uint32_t n_rep, hipStream_t s,
                                   uint32_t* blocks_per_rep) {
  const uint32_t paths_per_wg = 32 * kWaves;
  const uint64_t nb = (p.n_paths + paths_per_wg - 1) / paths_per_wg;
  *blocks_per_rep = (uint32_t)nb;
  if (p.qV == nullptr || p.n_strikes != 0 || p.path_out != nullptr || n_rep == 0 || nb == 0 ||
      nb * n_rep > 0x7fffffffull || prec == BK_BF16X2)
    return hipErrorInvalidValue;
  p.q_rep_blocks = (uint32_t)nb;
  const uint32_t total = (uint32_t)(nb * n_rep);
  switch (prec) {
    case BK_FP32: return launch_prec<BK_FP32>(p, s, total);
    case BK_BF16: return launch_prec<BK_BF16>(p, s, total);
    case BK_FP16: return launch_prec<BK_FP16>(p, s, total);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_basket(const BasketParams& p, int prec, hipStream_t s, uint32_t* n_blocks) {
  const uint32_t paths_per_wg = 32 * kWaves;
  const uint32_t nb = (uint32_t)((p.n_paths + paths_per_wg - 1) / paths_per_wg);
  *n_blocks = nb;
  switch (prec) {
    case BK_FP32: return launch_prec<BK_FP32>(p, s, nb);
    case BK_BF16: return launch_prec<BK_BF16>(p, s, nb);
    case BK_FP16: return launch_prec<BK_FP16>(p, s, nb);
    case BK_BF16X2: return launch_prec<BK_BF16X2>(p, s, nb);
  }
  return hipErrorInvalidValue;
}

}  // namespace mcp
