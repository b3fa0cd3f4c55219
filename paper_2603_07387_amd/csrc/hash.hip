// Count-sketch hash tables on the device (the hash family of tn_sketch.h), one
// packed int32 entry per (sample, stream, index).
#include "hash_device.h"
#include "tn_internal.h"

namespace tn {
namespace {

// grid.x: stream, grid.y: sample within the chunk.
__global__ __launch_bounds__(64) void hashgen_kernel(const StreamDesc *__restrict__ streams,
                                                     int64_t W, int64_t sample0, uint32_t mask,
                                                     int32_t *__restrict__ out) {
  const StreamDesc sd = streams[blockIdx.x];
  const int64_t r = blockIdx.y;
  const HashCoeffs c = hash_coeffs(sd.seed, (uint64_t)(sample0 + r), sd.stream);
  int32_t *dst = out + r * W + sd.offset;
  for (int i = threadIdx.x; i < sd.n; i += 64) dst[i] = (int32_t)hash_packed(c, (uint32_t)i, mask);
}

// Short streams (every stream of at most kShortStream indices): one thread per
// (stream, sample) derives the coefficients once and writes the whole stream,
// instead of a 64-thread block per pair whose lanes all derive the same
// coefficients for a handful of indices.
constexpr int kShortStream = 64;
__global__ __launch_bounds__(256) void hashgen_short_kernel(const StreamDesc *__restrict__ streams,
                                                            int64_t n_streams, int64_t W, int64_t sample0,
                                                            int64_t samples, uint32_t mask,
                                                            int32_t *__restrict__ out) {
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= n_streams * samples) return;
  const int64_t r = gid / n_streams, k = gid - r * n_streams;
  const StreamDesc sd = streams[k];
  const HashCoeffs c = hash_coeffs(sd.seed, (uint64_t)(sample0 + r), sd.stream);
  int32_t *dst = out + r * W + sd.offset;
  for (int i = 0; i < (int)sd.n; ++i) dst[i] = (int32_t)hash_packed(c, (uint32_t)i, mask);
}

__global__ void copy_i32_kernel(const int32_t *__restrict__ src, int32_t *__restrict__ dst,
                                int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

int launch_hashgen(const StreamDesc *streams, int64_t n_streams, int64_t W, int64_t sample0,
                   int64_t samples, int64_t m, int64_t max_n, int32_t *out, hipStream_t st) {
  if (n_streams == 0 || samples == 0) return TN_OK;
  if (!streams || !out) return set_error(TN_ERR_ARG, "hashgen: null stream table or output");
  if (samples > 65535 || n_streams > 0x7fffffff)
    return set_error(TN_ERR_UNSUPPORTED, "hashgen: %lld samples x %lld streams per launch",
                     (long long)samples, (long long)n_streams);
  if (max_n <= kShortStream) {
    const int64_t pairs = n_streams * samples;
    hipLaunchKernelGGL(hashgen_short_kernel, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, st, streams,
                       n_streams, W, sample0, samples, (uint32_t)(m - 1), out);
    TN_HIP_CHECK(hipGetLastError());
    return TN_OK;
  }
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
