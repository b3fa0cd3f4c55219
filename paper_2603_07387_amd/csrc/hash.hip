// Count-sketch hash tables on the device (the hash family of tn_sketch.h).
//
// Def. 11 asks for 2-wise independent buckets h and 4-wise independent signs s.
// Both come from polynomials over the Mersenne prime P = 2^31 - 1 (degree 1 for
// h, degree 3 for s) whose coefficients are SplitMix64 outputs keyed by
// (network seed, sample, stream).  Products of two residues fit in 62 bits and
// are reduced with the Mersenne identity 2^31 = 1 (mod P), so the kernel needs
// no 64-bit division.
#include "tn_internal.h"

namespace tn {
namespace {

constexpr uint64_t kP = 2147483647ull;

__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// x < 2^63  ->  x mod P
__device__ __forceinline__ uint32_t mod_p(uint64_t x) {
  uint64_t r = (x & kP) + (x >> 31);
  r = (r & kP) + (r >> 31);
  return (uint32_t)(r >= kP ? r - kP : r);
}

struct Coeffs {
  uint32_t a0, a1, c0, c1, c2, c3;
};

__device__ __forceinline__ Coeffs coeffs(uint64_t seed, uint64_t sample, uint64_t stream) {
  uint64_t key = mix64(mix64(mix64(seed) ^ sample) ^ stream);
  uint32_t raw[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) raw[j] = (uint32_t)(mix64(key ^ (uint64_t)j) >> 33);
  Coeffs c;
  c.a0 = raw[0] == (uint32_t)kP ? 0u : raw[0];
  c.a1 = 1u + (raw[1] >= (uint32_t)(kP - 1) ? raw[1] - (uint32_t)(kP - 1) : raw[1]);
  c.c0 = raw[2] == (uint32_t)kP ? 0u : raw[2];
  c.c1 = raw[3] == (uint32_t)kP ? 0u : raw[3];
  c.c2 = raw[4] == (uint32_t)kP ? 0u : raw[4];
  c.c3 = raw[5] == (uint32_t)kP ? 0u : raw[5];
  return c;
}

__device__ __forceinline__ uint32_t packed_hash(const Coeffs &c, uint32_t i, uint32_t mask) {
  uint32_t h = mod_p((uint64_t)c.a1 * i + c.a0) & mask;
  uint64_t v = c.c3;
  v = mod_p(v * i + c.c2);
  v = mod_p(v * i + c.c1);
  v = mod_p(v * i + c.c0);
  return h | ((v & 1u) ? kSignBit : 0u);
}

// grid.x: stream, grid.y: sample within the chunk.
__global__ __launch_bounds__(64) void hashgen_kernel(const StreamDesc *__restrict__ streams,
                                                     int64_t W, int64_t sample0, uint32_t mask,
                                                     int32_t *__restrict__ out) {
  const StreamDesc sd = streams[blockIdx.x];
  const int64_t r = blockIdx.y;
  const Coeffs c = coeffs(sd.seed, (uint64_t)(sample0 + r), sd.stream);
  int32_t *dst = out + r * W + sd.offset;
  for (int i = threadIdx.x; i < sd.n; i += 64) dst[i] = (int32_t)packed_hash(c, (uint32_t)i, mask);
}

__global__ void copy_i32_kernel(const int32_t *__restrict__ src, int32_t *__restrict__ dst,
                                int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

int launch_hashgen(const StreamDesc *streams, int64_t n_streams, int64_t W, int64_t sample0,
                   int64_t samples, int64_t m, int32_t *out, hipStream_t st) {
  if (n_streams == 0 || samples == 0) return TN_OK;
  if (samples > 65535 || n_streams > 0x7fffffff)
    return set_error(TN_ERR_UNSUPPORTED, "hashgen: %lld samples x %lld streams per launch",
                     (long long)samples, (long long)n_streams);
  dim3 grid((unsigned)n_streams, (unsigned)samples);
  hipLaunchKernelGGL(hashgen_kernel, grid, dim3(64), 0, st, streams, W, sample0,
                     (uint32_t)(m - 1), out);
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

int launch_copy_i32(const int32_t *src, int32_t *dst, int64_t n, hipStream_t st) {
  if (n == 0) return TN_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(copy_i32_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n);
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

}  // namespace tn
