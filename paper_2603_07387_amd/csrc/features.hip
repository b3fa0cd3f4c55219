// Per-tensor statistics for the sketch-size selector's features: sum x, sum x^2,
// sum |x| and the number of entries >= 0, one block per tensor, FP64.
#include <mutex>
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

// Fixed scratch of tn_tensor_stats_noalloc (sized below): each device holds its
// own copy for the life of the process.
static constexpr size_t kScratchBytes = (size_t)32768 * (sizeof(void *) + sizeof(int64_t) + 4 * sizeof(double));
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Host-side validation shared by both entry points: the device pointers and
// entry counts of every tensor, network-major.
int collect_tensors(const tn_network *nets, int32_t n_nets, double *out, std::vector<const void *> *ptrs,
                    std::vector<int64_t> *sizes, int *dtype) {
  if (!nets || n_nets < 1 || !out) return set_error(TN_ERR_ARG, "null argument");
  *dtype = nets[0].dtype;
  for (int j = 0; j < n_nets; ++j) {
    const tn_network &n = nets[j];
    if (n.p < 1 || !n.order || !n.dims || !n.data) return set_error(TN_ERR_ARG, "network %d malformed", j);
    if (n.dtype != *dtype) return set_error(TN_ERR_ARG, "network %d: dtypes differ", j);
    if (n.dtype != TN_F64 && n.dtype != TN_F32 && n.dtype != TN_BF16)
      return set_error(TN_ERR_ARG, "network %d: dtype %d", j, n.dtype);
    int64_t u = 0;
    for (int k = 0; k < n.p; ++k) {
      int64_t s = 1;
      for (int i = 0; i < n.order[k]; ++i, ++u) s *= n.dims[u];
      if (!n.data[k]) return set_error(TN_ERR_ARG, "network %d tensor %d: null data", j, k);
      ptrs->push_back(n.data[k]);
      sizes->push_back(s);
    }
  }
  return TN_OK;
}

// Upload the pointer and size tables to d_ptrs / d_sizes, run one block per
// tensor into d_out, copy the 4 nt doubles to the host and wait.
hipError_t run_stats(const void *const *ptrs, const int64_t *sizes, size_t nt, int dtype, void *d_ptrs,
                     void *d_sizes, void *d_out, hipStream_t st, double *out) {
  hipError_t e = hipMemcpyAsync(d_ptrs, ptrs, nt * sizeof(void *), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(d_sizes, sizes, nt * sizeof(int64_t), hipMemcpyHostToDevice, st);
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
  return e;
}

// ---------------------------------------------------------------------------
// Fixed scratch of the allocation-free entry point: the pointer table, the
// entry counts and the 4 doubles per tensor of kStatsMaxTensors tensors.  The
// array's name is a host-side stand-in: kernels and copies use the device
// address hipGetSymbolAddress returns, fetched once per device.
// ---------------------------------------------------------------------------
constexpr int64_t kStatsMaxTensors = 32768;
constexpr size_t kPtrBytes = (size_t)kStatsMaxTensors * sizeof(void *);
constexpr size_t kSizeBytes = (size_t)kStatsMaxTensors * sizeof(int64_t);
constexpr size_t kOutBytes = (size_t)kStatsMaxTensors * 4 * sizeof(double);
static_assert(kPtrBytes % 256 == 0 && kSizeBytes % 256 == 0, "sub-buffers stay 256-byte aligned");
static_assert(kPtrBytes + kSizeBytes + kOutBytes == kScratchBytes, "scratch layout");
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;                 // held for a whole call: guards the tables below
void *g_scratch_dev[kMaxDevices] = {};   // device address of scratch, per device
// Host staging of the pointer and size tables (the copy from them completes
// before the call returns: it ends with a stream synchronization).
const void *g_host_ptrs[kStatsMaxTensors];
int64_t g_host_sizes[kStatsMaxTensors];

}  // namespace

extern "C" int tn_tensor_stats(const tn_network *nets, int32_t n_nets, void *stream, double *out) {
  clear_error();
  std::vector<const void *> ptrs;
  std::vector<int64_t> sizes;
  int dtype = 0;
  int rc = collect_tensors(nets, n_nets, out, &ptrs, &sizes, &dtype);
  if (rc != TN_OK) return rc;
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
  const hipError_t e = run_stats(ptrs.data(), sizes.data(), nt, dtype, d_ptrs, d_sizes, d_out, st, out);
  cleanup();
  if (e != hipSuccess) return set_error(TN_ERR_HIP, "tensor stats: %s", hipGetErrorString(e));
  return TN_OK;
}

extern "C" int tn_tensor_stats_noalloc(const tn_network *nets, int32_t n_nets, void *stream, double *out) {
  clear_error();
  if (!nets || n_nets < 1 || !out) return set_error(TN_ERR_ARG, "null argument");
  int64_t nt = 0;
  for (int j = 0; j < n_nets; ++j) {
    if (nets[j].p < 1) return set_error(TN_ERR_ARG, "network %d malformed", j);
    nt += nets[j].p;
  }
  if (nt > kStatsMaxTensors)
    return set_error(TN_ERR_UNSUPPORTED, "tensor stats without allocation: %lld tensors exceed %lld",
                     (long long)nt, (long long)kStatsMaxTensors);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  int dev = 0;
  TN_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return set_error(TN_ERR_UNSUPPORTED, "device %d", dev);
  if (!g_scratch_dev[dev]) {
    void *ptr = nullptr;
    TN_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev] = ptr;
  }
  unsigned char *base = static_cast<unsigned char *>(g_scratch_dev[dev]);
  // Validate and stage into the fixed host tables (no host allocation either).
  int dtype = nets[0].dtype;
  int64_t i = 0;
  for (int j = 0; j < n_nets; ++j) {
    const tn_network &n = nets[j];
    if (!n.order || !n.dims || !n.data) return set_error(TN_ERR_ARG, "network %d malformed", j);
    if (n.dtype != dtype) return set_error(TN_ERR_ARG, "network %d: dtypes differ", j);
    if (n.dtype != TN_F64 && n.dtype != TN_F32 && n.dtype != TN_BF16)
      return set_error(TN_ERR_ARG, "network %d: dtype %d", j, n.dtype);
    int64_t u = 0;
    for (int k = 0; k < n.p; ++k, ++i) {
      int64_t s = 1;
      for (int d = 0; d < n.order[k]; ++d, ++u) s *= n.dims[u];
      if (!n.data[k]) return set_error(TN_ERR_ARG, "network %d tensor %d: null data", j, k);
      g_host_ptrs[i] = n.data[k];
      g_host_sizes[i] = s;
    }
  }
  const hipError_t e = run_stats(g_host_ptrs, g_host_sizes, (size_t)nt, dtype, base, base + kPtrBytes,
                                 base + kPtrBytes + kSizeBytes, (hipStream_t)stream, out);
  if (e != hipSuccess) return set_error(TN_ERR_HIP, "tensor stats: %s", hipGetErrorString(e));
  return TN_OK;
}
