// Sobol' direction words for the randomised quasi-Monte Carlo basket
// (quasi-random generator of Sec. IV-B, Sobol' experiment of Sec. VI-D),
// built on the host once per call.
//
// Construction (Sobol'; Bratley and Fox): dimension 0 is the van der Corput
// sequence (direction integers m_i = 1). Dimension j >= 1 takes the j-th
// primitive polynomial over GF(2), ordered by degree s and then by bit
// pattern, p = x^s + a_1 x^(s-1) + ... + a_(s-1) x + 1. Its first s
// direction integers are m_i = 2 (h mod 2^(i-1)) + 1 with h the SplitMix64
// finaliser of 64 j + i (odd and below 2^i); the rest follow
//     m_i = m_(i-s) ^ (m_(i-s) << s) ^ sum_k a_k (m_(i-k) << k).
// The direction word of bit b of a point index is m_(b+1) << (31 - b).
#pragma once

#include <stdint.h>

#include <vector>

namespace mcp {
namespace host {

inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// x^e modulo p in GF(2)[x] (deg p = s), by square and multiply.
inline uint32_t gf2_pow_x(uint64_t e, uint32_t p, int s) {
  auto mul = [p, s](uint32_t a, uint32_t b) {
    uint32_t r = 0;
    for (; b; b >>= 1) {
      if (b & 1u) r ^= a;
      a <<= 1;
      if (a >> s & 1u) a ^= p;
    }
    return r;
  };
  uint32_t base = 2u;
  if (base >> s & 1u) base ^= p;       // degree 1: x reduces modulo p
  uint32_t r = 1u;
  for (; e; e >>= 1) {
    if (e & 1u) r = mul(r, base);
    base = mul(base, base);
  }
  return r;
}

// Primitive: x has multiplicative order exactly 2^s - 1 modulo p.
inline bool gf2_is_primitive(uint32_t p, int s) {
  const uint64_t order = (1ull << s) - 1;
  if (gf2_pow_x(order, p, s) != 1u) return false;
  uint64_t n = order;
  for (uint64_t q = 2; q * q <= n; ++q) {
    if (n % q) continue;
    while (n % q == 0) n /= q;
    if (gf2_pow_x(order / q, p, s) == 1u) return false;
  }
  if (n > 1 && gf2_pow_x(order / n, p, s) == 1u) return false;
  return true;
}

// Direction words [n_dims][32]; false if the polynomial search runs past
// degree 24 (far beyond any supported dimension count).
inline bool sobol_directions(uint32_t n_dims, std::vector<uint32_t>* V) {
  V->assign((size_t)n_dims * 32, 0u);
  uint32_t dim = 0;
  auto emit = [&](const uint64_t (&m)[33]) {
    for (int b = 0; b < 32; ++b) (*V)[(size_t)dim * 32 + b] = (uint32_t)(m[b + 1] << (31 - b));
    ++dim;
  };
  uint64_t m[33];
  for (int i = 1; i <= 32; ++i) m[i] = 1;
  if (n_dims > 0) emit(m);
  for (int s = 1; s <= 24 && dim < n_dims; ++s) {
    for (uint32_t p = (1u << s) | 1u; p < (2u << s) && dim < n_dims; p += 2) {
      if (!gf2_is_primitive(p, s)) continue;
      for (int i = 1; i <= s && i <= 32; ++i)
        m[i] = 2 * (splitmix64(64ull * dim + (uint64_t)i) % (1ull << (i - 1))) + 1;
      for (int i = s + 1; i <= 32; ++i) {
        uint64_t v = m[i - s] ^ (m[i - s] << s);
        for (int k = 1; k < s; ++k)
          if (p >> (s - k) & 1u) v ^= m[i - k] << k;
        m[i] = v;
      }
      emit(m);
    }
  }
  return dim == n_dims;
}

}  // namespace host
}  // namespace mcp
