// Per-tensor statistics for the sketch-size selector's features: sum x, sum x^2,
// sum |x| and the number of entries >= 0, one block per tensor, FP64.
#include <vector>

#include "plan.h"

namespace tn {
namespace {

template <typename T>
__device__ __forceinline__ double fval(const void *p, int64_t i);
template <>
__device__ __forceinline__ double fval<double>(const void *p, int64_t i) {
  return reinterpret_cast<const double *>(p)[i];
}
template <>
__device__ __forceinline__ double fval<float>(const void *p, int64_t i) {
  return (double)reinterpret_cast<const float *>(p)[i];
}
template <>
__device__ __forceinline__ double fval<uint16_t>(const void *p, int64_t i) {
  return (double)__uint_as_float(((uint32_t)reinterpret_cast<const uint16_t *>(p)[i]) << 16);
}

template <typename T>
__global__ __launch_bounds__(256) void tensor_stats_kernel(const void *const *data,
                                                           const int64_t *__restrict__ sizes,
                                                           double *__restrict__ out) {
  __shared__ double red[4][4];
  const void *x = data[blockIdx.x];
  const int64_t n = sizes[blockIdx.x];
  double s = 0.0, s2 = 0.0, sa = 0.0, nn = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = fval<T>(x, i);
    s += v;
    s2 += v * v;
    sa += fabs(v);
    nn += v >= 0.0 ? 1.0 : 0.0;
  }
  double v4[4] = {s, s2, sa, nn};
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v4[k] += __shfl_down(v4[k], off, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
    for (int k = 0; k < 4; ++k) red[w][k] = v4[k];
  __syncthreads();
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    out[(int64_t)blockIdx.x * 4 + k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
  }
}

}  // namespace
}  // namespace tn

using namespace tn;

extern "C" int tn_tensor_stats(const tn_network *nets, int32_t n_nets, void *stream, double *out) {
  clear_error();
  if (!nets || n_nets < 1 || !out) return set_error(TN_ERR_ARG, "null argument");
  std::vector<const void *> ptrs;
  std::vector<int64_t> sizes;
  const int dtype = nets[0].dtype;
  for (int j = 0; j < n_nets; ++j) {
    NetCheck chk;
    const tn_network &n = nets[j];
    if (n.p < 1 || !n.order || !n.dims || !n.data) return set_error(TN_ERR_ARG, "network %d malformed", j);
    if (n.dtype != dtype) return set_error(TN_ERR_ARG, "network %d: dtypes differ", j);
    int64_t u = 0;
    for (int k = 0; k < n.p; ++k) {
      int64_t s = 1;
      for (int i = 0; i < n.order[k]; ++i, ++u) s *= n.dims[u];
      if (!n.data[k]) return set_error(TN_ERR_ARG, "network %d tensor %d: null data", j, k);
      ptrs.push_back(n.data[k]);
      sizes.push_back(s);
    }
  }
  hipStream_t st = (hipStream_t)stream;
  const size_t nt = ptrs.size();
  void *d_ptrs = nullptr, *d_sizes = nullptr, *d_out = nullptr;
  auto cleanup = [&]() {
    if (d_ptrs) (void)hipFree(d_ptrs);
    if (d_sizes) (void)hipFree(d_sizes);
    if (d_out) (void)hipFree(d_out);
  };
  if (hipMalloc(&d_ptrs, nt * sizeof(void *)) != hipSuccess ||
      hipMalloc(&d_sizes, nt * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&d_out, nt * 4 * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    cleanup();
    return set_error(TN_ERR_OOM, "tensor stats: hipMalloc");
  }
  hipError_t e = hipMemcpyAsync(d_ptrs, ptrs.data(), nt * sizeof(void *), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_sizes, sizes.data(), nt * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    if (dtype == TN_F64)
      hipLaunchKernelGGL(tensor_stats_kernel<double>, dim3((unsigned)nt), dim3(256), 0, st,
                         (const void *const *)d_ptrs, (const int64_t *)d_sizes, (double *)d_out);
    else if (dtype == TN_F32)
      hipLaunchKernelGGL(tensor_stats_kernel<float>, dim3((unsigned)nt), dim3(256), 0, st,
                         (const void *const *)d_ptrs, (const int64_t *)d_sizes, (double *)d_out);
    else
      hipLaunchKernelGGL(tensor_stats_kernel<uint16_t>, dim3((unsigned)nt), dim3(256), 0, st,
                         (const void *const *)d_ptrs, (const int64_t *)d_sizes, (double *)d_out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(out, d_out, nt * 4 * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  cleanup();
  if (e != hipSuccess) return set_error(TN_ERR_HIP, "tensor stats: %s", hipGetErrorString(e));
  return TN_OK;
}
