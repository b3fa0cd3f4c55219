// Turnstile updates of resident sketches (the streaming setting of the
// cyclic method: Algorithm 1 keeps the sketch x_k of every tensor, and an
// update X_k(i) += delta changes one bucket of it per sample, in O(q_k)).
//
// A resident plan (TN_FLAG_RESIDENT) keeps the time-domain sketches of all S
// samples, [sample][slot][m] (FP64 for FP64 data, FP32 otherwise), and the
// packed hash tables of all samples.  An update adds s(i) delta to bucket
// (sum_u h_u(i_u)) mod m of the tensor's first slot (the combine adds a
// tensor's slots), with the complement bucket on the second mode of each
// contraction (Def. 14), exactly as the scatter would for that entry.
#include <algorithm>

#include "tn_internal.h"

namespace tn {
namespace {

template <typename A>
__global__ __launch_bounds__(256) void stream_update_kernel(
    const ModeDesc *__restrict__ modes, int mode0, int q, int64_t size, const int32_t *__restrict__ tables,
    int64_t W, int64_t S, int log2m, int64_t sample_stride, int64_t slot_off, A *__restrict__ ybuf, int64_t n,
    const int64_t *__restrict__ idx, const double *__restrict__ delta) {
  const uint32_t m = 1u << log2m, mask = m - 1;
  const int64_t total = n * S;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t u = t / S, s = t - u * S;  // consecutive threads: one update, consecutive samples
    int64_t i = idx[u];
    if (i < 0 || i >= size) continue;  // outside the tensor: ignored
    const int32_t *tab = tables + s * W;
    uint32_t b = 0, neg = 0;
    for (int j = q - 1; j >= 0; --j) {  // row-major: the last mode varies fastest
      const ModeDesc md = modes[mode0 + j];
      const int64_t d = i % md.n;
      i /= md.n;
      const uint32_t v = (uint32_t)tab[md.table_off + d];
      uint32_t h = v & ~kSignBit;
      if (md.comp) h = (m - h) & mask;
      b = (b + h) & mask;
      neg ^= v >> 31;
    }
    const double x = neg ? -delta[u] : delta[u];
    atomicAdd(ybuf + s * sample_stride + slot_off + b, (A)x);
  }
}

__global__ __launch_bounds__(256) void fill_zero_kernel(uint32_t *__restrict__ p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

}  // namespace

int launch_stream_update(const ModeDesc *modes, int mode0, int q, int64_t size, const int32_t *tables, int64_t W,
                         int64_t S, int log2m, int64_t n_slots, int32_t slot0, int dtype, void *ybuf, int64_t n,
                         const int64_t *idx, const double *delta, hipStream_t st) {
  if (n == 0) return TN_OK;
  const int64_t total = n * S;
  const unsigned blocks = (unsigned)std::min<int64_t>((total + 255) / 256, 65536);
  const int64_t m = 1ll << log2m;
  if (dtype == TN_F64)
    hipLaunchKernelGGL(stream_update_kernel<double>, dim3(blocks), dim3(256), 0, st, modes, mode0, q, size, tables,
                       W, S, log2m, n_slots * m, (int64_t)slot0 * m, reinterpret_cast<double *>(ybuf), n, idx, delta);
  else
    hipLaunchKernelGGL(stream_update_kernel<float>, dim3(blocks), dim3(256), 0, st, modes, mode0, q, size, tables,
                       W, S, log2m, n_slots * m, (int64_t)slot0 * m, reinterpret_cast<float *>(ybuf), n, idx, delta);
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

// Zero a buffer with a kernel (graph-safe, unlike a memset node).  bytes must
// be a multiple of 4.
int launch_fill_zero(void *buf, size_t bytes, hipStream_t st) {
  const int64_t words = (int64_t)(bytes / 4);
  if (words == 0) return TN_OK;
  const unsigned blocks = (unsigned)std::min<int64_t>((words + 255) / 256, 65536);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, st, reinterpret_cast<uint32_t *>(buf), words);
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

}  // namespace tn
