// Median of means over the per-sample estimates: the amplification step of
// Theorem 1 (the median of O(log 1/delta) averaged estimates reaches success
// probability 1 - delta).  One block per network: the G group means are FP64
// block sums in LDS, then each is ranked against all others (ties broken by
// group index), so the median is the mean of the ranks floor((G-1)/2) and
// floor(G/2) without a sort.
#include "tn_internal.h"

namespace tn {
namespace {

constexpr int kMaxGroups = 1024;

__global__ __launch_bounds__(256) void median_of_means_kernel(const double *__restrict__ est,
                                                              int64_t S, int G,
                                                              double *__restrict__ out) {
  __shared__ double means[kMaxGroups];
  __shared__ double red[4];
  __shared__ double lo, hi;
  __shared__ int bad;
  const double *x = est + (int64_t)blockIdx.x * S;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) bad = 0;
  for (int g = 0; g < G; ++g) {
    const int64_t b0 = (int64_t)g * S / G, b1 = (int64_t)(g + 1) * S / G;
    double v = 0.0;
    for (int64_t i = b0 + tid; i < b1; i += 256) v += x[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wv] = v;
    __syncthreads();
    if (tid == 0) means[g] = (red[0] + red[1] + red[2] + red[3]) / (double)(b1 - b0);
    __syncthreads();
  }
  const int r_lo = (G - 1) / 2, r_hi = G / 2;
  for (int i = tid; i < G; i += 256) {
    const double mi = means[i];
    if (mi != mi) bad = 1;
    int rank = 0;
    for (int j = 0; j < G; ++j) {
      const double mj = means[j];
      rank += (mj < mi || (mj == mi && j < i)) ? 1 : 0;
    }
    if (rank == r_lo) lo = mi;
    if (rank == r_hi) hi = mi;
  }
  __syncthreads();
  if (tid == 0) out[blockIdx.x] = bad ? __longlong_as_double(0x7ff8000000000000ll) : 0.5 * (lo + hi);
}

}  // namespace
}  // namespace tn

using namespace tn;

extern "C" int tn_median_of_means(const double *samples, int64_t n_nets, int64_t S, int32_t groups,
                                  void *stream, double *out) {
  clear_error();
  if (!samples || !out || n_nets < 1 || S < 1) return set_error(TN_ERR_ARG, "bad argument");
  if (groups < 1 || groups > kMaxGroups || groups > S)
    return set_error(TN_ERR_ARG, "groups %d outside [1, min(S, %d)]", groups, kMaxGroups);
  if (n_nets > 0x7fffffff) return set_error(TN_ERR_UNSUPPORTED, "too many networks");
  hipLaunchKernelGGL(median_of_means_kernel, dim3((unsigned)n_nets), dim3(256), 0,
                     (hipStream_t)stream, samples, S, (int)groups, out);
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}
