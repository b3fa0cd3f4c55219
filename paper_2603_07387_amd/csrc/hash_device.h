// Device-side evaluation of the count-sketch hash family of tn_sketch.h.
//
// Def. 11 asks for 2-wise independent buckets and 4-wise independent signs:
// degree-1 and degree-3 polynomials over the Mersenne prime P = 2^31 - 1 whose
// coefficients are SplitMix64 outputs keyed by (network seed, sample, stream).
// Residue products fit in 62 bits and are reduced with 2^31 = 1 (mod P).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tn {

constexpr uint64_t kMersenne31 = 2147483647ull;

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// x < 2^63  ->  x mod P
__device__ __forceinline__ uint32_t mod_p(uint64_t x) {
  uint64_t r = (x & kMersenne31) + (x >> 31);
  r = (r & kMersenne31) + (r >> 31);
  return (uint32_t)(r >= kMersenne31 ? r - kMersenne31 : r);
}

struct HashCoeffs {
  uint32_t a0, a1, c0, c1, c2, c3;
};

__device__ __forceinline__ HashCoeffs hash_coeffs(uint64_t seed, uint64_t sample, uint64_t stream) {
  const uint64_t key = mix64(mix64(mix64(seed) ^ sample) ^ stream);
  uint32_t raw[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) raw[j] = (uint32_t)(mix64(key ^ (uint64_t)j) >> 33);
  const uint32_t P = (uint32_t)kMersenne31;
  HashCoeffs c;
  c.a0 = raw[0] == P ? 0u : raw[0];
  c.a1 = 1u + (raw[1] >= P - 1 ? raw[1] - (P - 1) : raw[1]);
  c.c0 = raw[2] == P ? 0u : raw[2];
  c.c1 = raw[3] == P ? 0u : raw[3];
  c.c2 = raw[4] == P ? 0u : raw[4];
  c.c3 = raw[5] == P ? 0u : raw[5];
  return c;
}

// Packed entry: bucket (m a power of two, mask = m - 1) in bits 0..30, bit 31
// set for sign -1.
__device__ __forceinline__ uint32_t hash_packed(const HashCoeffs &c, uint32_t i, uint32_t mask) {
  const uint32_t h = mod_p((uint64_t)c.a1 * i + c.a0) & mask;
  uint64_t v = c.c3;
  v = mod_p(v * i + c.c2);
  v = mod_p(v * i + c.c1);
  v = mod_p(v * i + c.c0);
  return h | ((v & 1u) ? 0x80000000u : 0u);
}

}  // namespace tn
