// Exact full tensor network contraction in FP64 on the device (Def. 1-3).
//
// Intermediates carry one label per mode (the contraction it belongs to).  A
// tensor whose label appears twice is first traced (a contraction inside one
// tensor, WLOG 2).  Then pairs of tensors sharing labels are contracted in a
// greedy order (smallest result first) until one scalar per connected
// component remains; their product is the result.  Each pairwise step is one
// kernel: a thread owns one output element and sums over the shared labels,
// walking both operands with per-label strides (a label repeated inside an
// operand gets the sum of its strides, i.e. the diagonal).
#include <algorithm>
#include <vector>

#include "plan.h"

namespace tn {
namespace {

constexpr int kMaxLabels = 24;
constexpr int64_t kMaxIntermediate = (int64_t)1 << 31;

struct ContractDesc {
  int n_out, n_sum;
  int64_t out_dims[kMaxLabels];
  int64_t sum_dims[kMaxLabels];
  int64_t a_out[kMaxLabels], b_out[kMaxLabels];
  int64_t a_sum[kMaxLabels], b_sum[kMaxLabels];
};

__global__ void contract_kernel(ContractDesc d, const double *__restrict__ A,
                                const double *__restrict__ B, int64_t out_size,
                                double *__restrict__ C) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < out_size;
       o += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = o, ao = 0, bo = 0;
    for (int i = d.n_out - 1; i >= 0; --i) {
      const int64_t digit = rem % d.out_dims[i];
      rem /= d.out_dims[i];
      ao += digit * d.a_out[i];
      bo += digit * d.b_out[i];
    }
    int64_t idx[kMaxLabels];
    for (int i = 0; i < d.n_sum; ++i) idx[i] = 0;
    double acc = 0.0;
    int64_t as = 0, bs = 0;
    while (true) {
      acc += A[ao + as] * (B ? B[bo + bs] : 1.0);
      int i = d.n_sum - 1;
      for (; i >= 0; --i) {
        if (++idx[i] < d.sum_dims[i]) {
          as += d.a_sum[i];
          bs += d.b_sum[i];
          break;
        }
        as -= (d.sum_dims[i] - 1) * d.a_sum[i];
        bs -= (d.sum_dims[i] - 1) * d.b_sum[i];
        idx[i] = 0;
      }
      if (i < 0) break;
    }
    C[o] = acc;
  }
}

template <typename T>
__global__ void to_f64_kernel(const T *__restrict__ x, int64_t n, double *__restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

__global__ void bf16_to_f64_kernel(const uint16_t *__restrict__ x, int64_t n,
                                   double *__restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (double)__uint_as_float(((uint32_t)x[i]) << 16);
}

struct DTensor {
  double *ptr = nullptr;
  std::vector<int> labels;
  std::vector<int64_t> dims;
  int64_t size = 1;
};

unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 16));
}

// Contract A (and B, if given) over every label that is not kept; `keep`
// lists the output labels in order.
int contract(const DTensor &A, const DTensor *B, const std::vector<int> &keep,
             const std::vector<int64_t> &keep_dims, const std::vector<int> &sum,
             const std::vector<int64_t> &sum_dims, DTensor *C, hipStream_t st) {
  if ((int)keep.size() > kMaxLabels || (int)sum.size() > kMaxLabels)
    return set_error(TN_ERR_UNSUPPORTED, "exact contraction: more than %d labels", kMaxLabels);
  ContractDesc d{};
  d.n_out = (int)keep.size();
  d.n_sum = (int)sum.size();
  auto strides = [](const DTensor &T) {
    std::vector<int64_t> s(T.dims.size());
    int64_t acc = 1;
    for (int i = (int)T.dims.size() - 1; i >= 0; --i) { s[(size_t)i] = acc; acc *= T.dims[(size_t)i]; }
    return s;
  };
  const std::vector<int64_t> sa = strides(A);
  std::vector<int64_t> sb;
  if (B) sb = strides(*B);
  auto stride_of = [](const DTensor &T, const std::vector<int64_t> &s, int label) {
    int64_t v = 0;
    for (size_t i = 0; i < T.labels.size(); ++i)
      if (T.labels[i] == label) v += s[i];
    return v;
  };
  int64_t out_size = 1;
  for (int i = 0; i < d.n_out; ++i) {
    d.out_dims[i] = keep_dims[(size_t)i];
    d.a_out[i] = stride_of(A, sa, keep[(size_t)i]);
    d.b_out[i] = B ? stride_of(*B, sb, keep[(size_t)i]) : 0;
    out_size *= keep_dims[(size_t)i];
  }
  for (int i = 0; i < d.n_sum; ++i) {
    d.sum_dims[i] = sum_dims[(size_t)i];
    d.a_sum[i] = stride_of(A, sa, sum[(size_t)i]);
    d.b_sum[i] = B ? stride_of(*B, sb, sum[(size_t)i]) : 0;
  }
  if (out_size > kMaxIntermediate)
    return set_error(TN_ERR_UNSUPPORTED, "exact contraction: intermediate of %lld entries",
                     (long long)out_size);
  hipError_t e = hipMalloc((void **)&C->ptr, (size_t)out_size * sizeof(double));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(TN_ERR_OOM, "exact contraction: hipMalloc(%lld doubles)", (long long)out_size);
  }
  C->labels = keep;
  C->dims = keep_dims;
  C->size = out_size;
  hipLaunchKernelGGL(contract_kernel, dim3(grid_for(out_size)), dim3(256), 0, st, d, A.ptr,
                     B ? B->ptr : nullptr, out_size, C->ptr);
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

}  // namespace

int contract_exact(const tn_network *net, hipStream_t st, double *out) {
  NetCheck chk;
  int rc = validate_network(net, 0, &chk);
  if (rc != TN_OK) return rc;
  if (!net->data) return set_error(TN_ERR_ARG, "null data array");
  std::vector<DTensor> ts((size_t)net->p);
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    for (DTensor &t : ts)
      if (t.ptr) (void)hipFree(t.ptr);
  };
  for (int k = 0; k < net->p; ++k) {
    DTensor &T = ts[(size_t)k];
    if (!net->data[k]) { cleanup(); return set_error(TN_ERR_ARG, "tensor %d: null data", k); }
    for (int u = chk.offsets[(size_t)k]; u < chk.offsets[(size_t)k + 1]; ++u) {
      T.labels.push_back(chk.edge_of[(size_t)u]);
      T.dims.push_back(net->dims[u]);
    }
    T.size = chk.sizes[(size_t)k];
    hipError_t e = hipMalloc((void **)&T.ptr, (size_t)T.size * sizeof(double));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      cleanup();
      return set_error(TN_ERR_OOM, "exact contraction: hipMalloc");
    }
    const unsigned g = grid_for(T.size);
    if (net->dtype == TN_F64)
      hipLaunchKernelGGL(to_f64_kernel<double>, dim3(g), dim3(256), 0, st,
                         (const double *)net->data[k], T.size, T.ptr);
    else if (net->dtype == TN_F32)
      hipLaunchKernelGGL(to_f64_kernel<float>, dim3(g), dim3(256), 0, st,
                         (const float *)net->data[k], T.size, T.ptr);
    else
      hipLaunchKernelGGL(bf16_to_f64_kernel, dim3(g), dim3(256), 0, st,
                         (const uint16_t *)net->data[k], T.size, T.ptr);
  }
  // Traces inside one tensor.
  for (DTensor &T : ts) {
    std::vector<int> keep, sum;
    std::vector<int64_t> kd, sd;
    for (size_t i = 0; i < T.labels.size(); ++i) {
      const int c = (int)std::count(T.labels.begin(), T.labels.end(), T.labels[i]);
      if (c == 1) { keep.push_back(T.labels[i]); kd.push_back(T.dims[i]); }
      else if (std::find(sum.begin(), sum.end(), T.labels[i]) == sum.end()) {
        sum.push_back(T.labels[i]);
        sd.push_back(T.dims[i]);
      }
    }
    if (sum.empty()) continue;
    DTensor C;
    if ((rc = contract(T, nullptr, keep, kd, sum, sd, &C, st)) != TN_OK) { cleanup(); return rc; }
    (void)hipStreamSynchronize(st);
    (void)hipFree(T.ptr);
    T = C;
  }
  // Greedy pairwise contractions.
  while (true) {
    int best_a = -1, best_b = -1;
    int64_t best_size = 0;
    double best_flops = 0.0;
    for (size_t a = 0; a < ts.size(); ++a) {
      for (size_t b = a + 1; b < ts.size(); ++b) {
        bool share = false;
        int64_t osize = 1;
        double shared = 1.0;
        for (size_t i = 0; i < ts[a].labels.size(); ++i) {
          if (std::find(ts[b].labels.begin(), ts[b].labels.end(), ts[a].labels[i]) != ts[b].labels.end()) {
            share = true;
            shared *= (double)ts[a].dims[i];
          } else {
            osize *= ts[a].dims[i];
          }
        }
        if (!share) continue;
        for (size_t i = 0; i < ts[b].labels.size(); ++i)
          if (std::find(ts[a].labels.begin(), ts[a].labels.end(), ts[b].labels[i]) == ts[a].labels.end())
            osize *= ts[b].dims[i];
        const double flops = (double)osize * shared;
        if (best_a < 0 || osize < best_size || (osize == best_size && flops < best_flops)) {
          best_a = (int)a;
          best_b = (int)b;
          best_size = osize;
          best_flops = flops;
        }
      }
    }
    if (best_a < 0) break;
    DTensor &A = ts[(size_t)best_a];
    DTensor &B = ts[(size_t)best_b];
    std::vector<int> keep, sum;
    std::vector<int64_t> kd, sd;
    for (size_t i = 0; i < A.labels.size(); ++i) {
      if (std::find(B.labels.begin(), B.labels.end(), A.labels[i]) != B.labels.end()) {
        sum.push_back(A.labels[i]);
        sd.push_back(A.dims[i]);
      } else {
        keep.push_back(A.labels[i]);
        kd.push_back(A.dims[i]);
      }
    }
    for (size_t i = 0; i < B.labels.size(); ++i)
      if (std::find(A.labels.begin(), A.labels.end(), B.labels[i]) == A.labels.end()) {
        keep.push_back(B.labels[i]);
        kd.push_back(B.dims[i]);
      }
    DTensor C;
    if ((rc = contract(A, &B, keep, kd, sum, sd, &C, st)) != TN_OK) { cleanup(); return rc; }
    (void)hipStreamSynchronize(st);
    (void)hipFree(A.ptr);
    (void)hipFree(B.ptr);
    A = C;
    ts.erase(ts.begin() + best_b);
  }
  double result = 1.0;
  for (DTensor &T : ts) {
    if (T.size != 1) { cleanup(); return set_error(TN_ERR_HIP, "exact contraction left an open tensor"); }
    double v = 0.0;
    hipError_t e = hipMemcpyAsync(&v, T.ptr, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) { cleanup(); return set_error(TN_ERR_HIP, "exact contraction: %s", hipGetErrorString(e)); }
    result *= v;
  }
  cleanup();
  *out = result;
  return TN_OK;
}

}  // namespace tn
