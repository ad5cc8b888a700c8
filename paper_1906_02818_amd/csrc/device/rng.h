// Device random numbers for the path kernels: Philox4x32-10, the open-interval
// uniform and Box-Muller (keyed counter-based PRNG of Sec. IV-A; Box-Muller as
// the paper uses it for Sobol points in Sec. VI-D).
//
// Counter layout: normal k of path p in stream `tag` is slot k mod 4 of the
// block with counter (floor(k/4), p mod 2^32, p >> 32, tag) and key
// (seed mod 2^32, seed >> 32). Words (w0, w1) give slots 0, 1 as
// r(w0) cos(2 pi u(w1)), r(w0) sin(2 pi u(w1)); (w2, w3) give slots 2, 3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcp {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

struct Words4 {
  uint32_t w0, w1, w2, w3;
};

// The per-path part of the counter and the key. c1, c2, c3 do not change
// along a path, so the first round's product of c2 is loop invariant.
struct PathCounter {
  uint32_t c1, c2, c3;  // path lo, path hi, tag
  uint32_t k0, k1;      // key (uniform across the launch: scalar registers)
};

__device__ __forceinline__ PathCounter make_counter(uint64_t path, uint32_t tag,
                                                    uint32_t k0, uint32_t k1) {
  PathCounter pc;
  pc.c1 = (uint32_t)path;
  pc.c2 = (uint32_t)(path >> 32);
  pc.c3 = tag;
  pc.k0 = k0;
  pc.k1 = k1;
  return pc;
}

__device__ __forceinline__ void mul_hi_lo(uint32_t a, uint32_t b, uint32_t& hi,
                                          uint32_t& lo) {
  const uint64_t p = (uint64_t)a * (uint64_t)b;
  hi = (uint32_t)(p >> 32);
  lo = (uint32_t)p;
}

// Ten Philox rounds on counter (j, c1, c2, c3).
__device__ __forceinline__ Words4 philox(uint32_t j, const PathCounter& pc) {
  uint32_t c0 = j, c1 = pc.c1, c2 = pc.c2, c3 = pc.c3;
  uint32_t k0 = pc.k0, k1 = pc.k1;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t hi0, lo0, hi1, lo1;
    mul_hi_lo(kPhiloxM0, c0, hi0, lo0);
    mul_hi_lo(kPhiloxM1, c2, hi1, lo1);
    // Three-input xors: one v_bitop3_b32 each (truth table 0x96 = a^b^c).
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32(hi1, c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32(hi0, c3, k1, 0x96);
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return Words4{c0, c1, c2, c3};
}

// u(w) = (2 (w >> 9) + 1) 2^-24, exact in FP32: the top 23 bits fill the
// mantissa of a float in [1, 2), and subtracting 1 - 2^-24 is exact.
__device__ __forceinline__ float uniform_f32(uint32_t w) {
  // (0x7F:w) >> 9 = 0x3F800000 | (w >> 9) in one v_alignbit_b32.
  return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9u)) - 0x1.fffffep-1f;
}

__device__ __forceinline__ double uniform_f64(uint32_t w) {
  return (double)(2u * (w >> 9) + 1u) * 0x1p-24;
}

// Box-Muller in FP32 on the hardware transcendental units:
// v_log_f32 is log2, so -2 ln u = (-2 ln 2) log2 u; v_sin_f32 / v_cos_f32
// take their argument in revolutions, so sin(2 pi u) is sin_rev(u).
__device__ __forceinline__ void box_muller_f32(uint32_t w_rad, uint32_t w_ang, float& z0,
                                               float& z1) {
  const float ur = uniform_f32(w_rad);
  const float ua = uniform_f32(w_ang);
  const float rad = __builtin_amdgcn_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(ur));
  z0 = rad * __builtin_amdgcn_cosf(ua);
  z1 = rad * __builtin_amdgcn_sinf(ua);
}

__device__ __forceinline__ void box_muller_f64(uint32_t w_rad, uint32_t w_ang, double& z0,
                                               double& z1) {
  const double ur = uniform_f64(w_rad);
  const double ua = uniform_f64(w_ang);
  const double rad = sqrt(-2.0 * log(ur));
  const double ang = 6.283185307179586476925286766559 * ua;
  z0 = rad * cos(ang);
  z1 = rad * sin(ang);
}

template <typename R>
struct Normals4 {
  R z[4];
};

template <typename R>
__device__ __forceinline__ Normals4<R> normals4(const Words4& w);

template <>
__device__ __forceinline__ Normals4<float> normals4<float>(const Words4& w) {
  Normals4<float> n;
  box_muller_f32(w.w0, w.w1, n.z[0], n.z[1]);
  box_muller_f32(w.w2, w.w3, n.z[2], n.z[3]);
  return n;
}

template <>
__device__ __forceinline__ Normals4<double> normals4<double>(const Words4& w) {
  Normals4<double> n;
  box_muller_f64(w.w0, w.w1, n.z[0], n.z[1]);
  box_muller_f64(w.w2, w.w3, n.z[2], n.z[3]);
  return n;
}

// Sobol' coordinate of point `point` in dimension `dim`: the xor of the
// direction words V[dim][b] over the set bits b of the point index (point
// indices below 2^32), as a 32-bit fraction. V is [dims][32] in device
// memory.
__device__ __forceinline__ uint32_t sobol_word(const uint32_t* __restrict__ V, uint32_t dim,
                                               uint32_t point) {
  const uint32_t* v = V + (size_t)dim * 32u;
  uint32_t x = 0u;
  while (point) {
    x ^= v[__builtin_ctz(point)];
    point &= point - 1u;
  }
  return x;
}

// Block j of a randomised Sobol' point: dimensions 4j .. 4j+3, each xored
// with its digital shift; these words replace a Philox block and go through
// the same uniform and Box-Muller maps.
__device__ __forceinline__ Words4 sobol_block(const uint32_t* __restrict__ V,
                                              const uint32_t* __restrict__ shift, uint32_t j,
                                              uint32_t point) {
  const uint32_t d = 4u * j;
  return Words4{sobol_word(V, d, point) ^ shift[d], sobol_word(V, d + 1, point) ^ shift[d + 1],
                sobol_word(V, d + 2, point) ^ shift[d + 2],
                sobol_word(V, d + 3, point) ^ shift[d + 3]};
}

__device__ __forceinline__ uint32_t word_at(const Words4& w, uint32_t s) {
  return s == 0 ? w.w0 : s == 1 ? w.w1 : s == 2 ? w.w2 : w.w3;
}

}  // namespace mcp
