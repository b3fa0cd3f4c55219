// Regressor of the learned sketch-size selector (tn_mlp.h): a 3-layer tanh
// perceptron in FP32 with hand-written forward, backward and Adam kernels.
//
//   mlp_fwd_bwd_kernel : a block takes 64 rows; the parameters and the rows'
//                        activations live in LDS; it writes predictions and/or
//                        the block's partial gradient (sums over its rows) and
//                        partial loss, FP64.
//   mlp_reduce_kernel  : one thread per parameter sums the blocks' partials in
//                        a fixed order (deterministic) and either exports the
//                        gradient or applies a bias-corrected Adam step.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/tn_mlp.h"
#include "tn_internal.h"

struct tn_mlp {
  int device = 0;
  int D = 0, H = 0;
  int64_t P = 0;
  float *d_params = nullptr;
  float *d_m = nullptr, *d_v = nullptr;
  double *d_partial = nullptr;  // [blocks][P + 1]
  int64_t partial_blocks = 0;
  double *d_scalar = nullptr;   // [0] loss of the last reduction, [1] running epoch loss
  int64_t t = 0;                // Adam steps taken
  size_t lds = 0;
};

namespace tn {
namespace {

constexpr int kRows = 64;  // rows per block

__global__ __launch_bounds__(256) void mlp_fwd_bwd_kernel(
    const float *__restrict__ params, int D, int H, const float *__restrict__ X,
    const float *__restrict__ y, int64_t row0, int64_t n, float scale, float *__restrict__ pred,
    double *__restrict__ partial, int64_t P) {
  extern __shared__ __align__(16) float sm[];
  float *W1 = sm;                 // [H][D]
  float *b1 = W1 + H * D;         // [H]
  float *W2 = b1 + H;             // [H][H]
  float *b2 = W2 + H * H;         // [H]
  float *W3 = b2 + H;             // [H]
  float *b3 = W3 + H;             // [1] (+1 pad)
  float *xs = b3 + 2;             // [64][D]
  float *h1 = xs + kRows * D;     // [64][H]
  float *h2 = h1 + kRows * H;     // [64][H]
  float *d2 = h2 + kRows * H;     // [64][H]  dL/da2
  float *d1 = d2 + kRows * H;     // [64][H]  dL/da1
  float *dy = d1 + kRows * H;     // [64]
  __shared__ double lpart[kRows];

  const int tid = threadIdx.x;
  const int64_t base = row0 + (int64_t)blockIdx.x * kRows;
  for (int64_t i = tid; i < P; i += 256) sm[i] = params[i];
  for (int i = tid; i < kRows * D; i += 256) {
    const int s = i / D, d = i - s * D;
    xs[i] = (base + s < n) ? X[(base + s) * D + d] : 0.f;
  }
  __syncthreads();
  for (int i = tid; i < kRows * H; i += 256) {
    const int s = i / H, j = i - s * H;
    float a = b1[j];
    for (int d = 0; d < D; ++d) a = fmaf(W1[j * D + d], xs[s * D + d], a);
    h1[i] = tanhf(a);
  }
  __syncthreads();
  for (int i = tid; i < kRows * H; i += 256) {
    const int s = i / H, j = i - s * H;
    float a = b2[j];
    for (int k = 0; k < H; ++k) a = fmaf(W2[j * H + k], h1[s * H + k], a);
    h2[i] = tanhf(a);
  }
  __syncthreads();
  if (tid < kRows) {
    const int s = tid;
    float o = b3[0];
    for (int j = 0; j < H; ++j) o = fmaf(W3[j], h2[s * H + j], o);
    const bool valid = base + s < n;
    if (pred && valid) pred[base + s] = o;
    if (partial) {
      const float r = valid ? o - y[base + s] : 0.f;
      dy[s] = r * scale;
      lpart[s] = 0.5 * (double)r * (double)r;
    }
  }
  if (!partial) return;
  __syncthreads();
  for (int i = tid; i < kRows * H; i += 256) {
    const int s = i / H, j = i - s * H;
    const float t = h2[i];
    d2[i] = dy[s] * W3[j] * (1.f - t * t);
  }
  __syncthreads();
  for (int i = tid; i < kRows * H; i += 256) {
    const int s = i / H, k = i - s * H;
    float a = 0.f;
    for (int j = 0; j < H; ++j) a = fmaf(W2[j * H + k], d2[s * H + j], a);
    const float t = h1[i];
    d1[i] = a * (1.f - t * t);
  }
  __syncthreads();
  double *out = partial + (int64_t)blockIdx.x * (P + 1);
  for (int64_t p = tid; p < P; p += 256) {
    double g = 0.0;
    if (p < (int64_t)H * D) {                                   // W1[j][d]
      const int j = (int)(p / D), d = (int)(p - (int64_t)j * D);
      for (int s = 0; s < kRows; ++s) g += (double)d1[s * H + j] * xs[s * D + d];
    } else if (p < (int64_t)H * D + H) {                        // b1[j]
      const int j = (int)(p - (int64_t)H * D);
      for (int s = 0; s < kRows; ++s) g += d1[s * H + j];
    } else if (p < (int64_t)H * D + H + H * H) {                // W2[j][k]
      const int q = (int)(p - (int64_t)H * D - H), j = q / H, k = q - j * H;
      for (int s = 0; s < kRows; ++s) g += (double)d2[s * H + j] * h1[s * H + k];
    } else if (p < (int64_t)H * D + 2 * H + H * H) {            // b2[j]
      const int j = (int)(p - (int64_t)H * D - H - H * H);
      for (int s = 0; s < kRows; ++s) g += d2[s * H + j];
    } else if (p < P - 1) {                                     // W3[j]
      const int j = (int)(p - (int64_t)H * D - 2 * H - H * H);
      for (int s = 0; s < kRows; ++s) g += (double)dy[s] * h2[s * H + j];
    } else {                                                    // b3
      for (int s = 0; s < kRows; ++s) g += dy[s];
    }
    out[p] = g;
  }
  if (tid == 0) {
    double l = 0.0;
    for (int s = 0; s < kRows; ++s) l += lpart[s];
    out[P] = l;
  }
}

// mode 0: grad[p] = sum; mode 1: Adam.  scalar[0] = summed loss * loss_scale and
// scalar[1] += summed loss * epoch_scale (the epoch's mean loss, batch by batch).
__global__ void mlp_reduce_kernel(const double *__restrict__ partial, int64_t blocks, int64_t P,
                                  int mode, float *__restrict__ grad, float *__restrict__ params,
                                  float *__restrict__ m, float *__restrict__ v, float lr, float c1,
                                  float c2, double loss_scale, double epoch_scale,
                                  double *__restrict__ scalar) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p > P) return;
  double g = 0.0;
  for (int64_t b = 0; b < blocks; ++b) g += partial[b * (P + 1) + p];
  if (p == P) {
    scalar[0] = g * loss_scale;
    scalar[1] += g * epoch_scale;
    return;
  }
  if (mode == 0) {
    grad[p] = (float)g;
    return;
  }
  const float gf = (float)g;
  const float mm = 0.9f * m[p] + 0.1f * gf;
  const float vv = 0.999f * v[p] + 0.001f * gf * gf;
  m[p] = mm;
  v[p] = vv;
  params[p] -= lr * (mm * c1) / (sqrtf(vv * c2) + 1e-8f);
}

uint64_t splitmix(uint64_t &state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

int ensure_partial(tn_mlp *net, int64_t blocks) {
  if (blocks <= net->partial_blocks) return TN_OK;
  if (net->d_partial) (void)hipFree(net->d_partial);
  net->d_partial = nullptr;
  net->partial_blocks = 0;
  hipError_t e = hipMalloc((void **)&net->d_partial, (size_t)blocks * (size_t)(net->P + 1) * 8);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(TN_ERR_OOM, "mlp: hipMalloc of the gradient partials");
  }
  net->partial_blocks = blocks;
  return TN_OK;
}

int fwd_bwd(tn_mlp *net, const float *X, const float *y, int64_t row0, int64_t rows, int64_t n,
            hipStream_t st, float *pred, bool grad) {
  const int64_t blocks = (rows + kRows - 1) / kRows;
  if (blocks == 0) return TN_OK;
  if (blocks > 0x7fffffff) return set_error(TN_ERR_UNSUPPORTED, "mlp: too many rows");
  if (grad) {
    int rc = ensure_partial(net, blocks);
    if (rc != TN_OK) return rc;
  }
  hipLaunchKernelGGL(mlp_fwd_bwd_kernel, dim3((unsigned)blocks), dim3(256), net->lds, st,
                     net->d_params, net->D, net->H, X, y, row0, row0 + rows < n ? row0 + rows : n,
                     (float)(1.0 / (double)rows), pred, grad ? net->d_partial : nullptr, net->P);
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

int reduce(tn_mlp *net, int64_t rows, int mode, float *grad, float lr, hipStream_t st,
           double epoch_scale = 0.0) {
  const int64_t blocks = (rows + kRows - 1) / kRows;
  float c1 = 1.f, c2 = 1.f;
  if (mode == 1) {
    net->t += 1;
    c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)net->t)));
    c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)net->t)));
  }
  const unsigned g = (unsigned)((net->P + 1 + 255) / 256);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3(g), dim3(256), 0, st, net->d_partial, blocks, net->P,
                     mode, grad, net->d_params, net->d_m, net->d_v, lr, c1, c2,
                     1.0 / (double)rows, epoch_scale, net->d_scalar);
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

}  // namespace
}  // namespace tn

using namespace tn;

extern "C" {

int tn_mlp_create(int32_t d_in, int32_t hidden, uint64_t seed, tn_mlp **out) {
  clear_error();
  if (!out) return set_error(TN_ERR_ARG, "out is null");
  *out = nullptr;
  if (d_in < 1 || d_in > 256 || hidden < 1 || hidden > 128)
    return set_error(TN_ERR_ARG, "mlp: d_in %d or hidden %d out of range", d_in, hidden);
  tn_mlp *net = new (std::nothrow) tn_mlp();
  if (!net) return set_error(TN_ERR_OOM, "host allocation");
  net->D = d_in;
  net->H = hidden;
  net->P = (int64_t)hidden * d_in + hidden + (int64_t)hidden * hidden + hidden + hidden + 1;
  const int64_t floats = net->P + 2 + (int64_t)kRows * d_in + 4 * (int64_t)kRows * hidden + kRows;
  net->lds = (size_t)floats * 4;
  int dev = 0, maxlds = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
    delete net;
    return set_error(TN_ERR_HIP, "mlp: no device");
  }
  net->device = dev;
  if (net->lds + 1024 > (size_t)maxlds) {
    delete net;
    return set_error(TN_ERR_UNSUPPORTED, "mlp: %zu bytes of LDS needed", net->lds);
  }
  if (net->lds > 65536 &&
      hipFuncSetAttribute((const void *)mlp_fwd_bwd_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)net->lds) != hipSuccess) {
    delete net;
    return set_error(TN_ERR_HIP, "mlp: LDS attribute");
  }
  std::vector<float> h((size_t)net->P, 0.f);
  uint64_t state = seed;
  auto fill = [&](int64_t off, int fan_out, int fan_in) {
    const double a = std::sqrt(6.0 / (double)(fan_in + fan_out));
    for (int64_t i = 0; i < (int64_t)fan_out * fan_in; ++i) {
      const double u = (double)(splitmix(state) >> 11) * (1.0 / 9007199254740992.0);
      h[(size_t)(off + i)] = (float)((2.0 * u - 1.0) * a);
    }
  };
  const int64_t o1 = 0, o2 = (int64_t)hidden * d_in + hidden, o3 = o2 + (int64_t)hidden * hidden + hidden;
  fill(o1, hidden, d_in);
  fill(o2, hidden, hidden);
  fill(o3, 1, hidden);
  bool ok = hipMalloc((void **)&net->d_params, (size_t)net->P * 4) == hipSuccess &&
            hipMalloc((void **)&net->d_m, (size_t)net->P * 4) == hipSuccess &&
            hipMalloc((void **)&net->d_v, (size_t)net->P * 4) == hipSuccess &&
            hipMalloc((void **)&net->d_scalar, 16) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    tn_mlp_destroy(net);
    return set_error(TN_ERR_OOM, "mlp: hipMalloc");
  }
  if (hipMemcpy(net->d_params, h.data(), (size_t)net->P * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(net->d_m, 0, (size_t)net->P * 4) != hipSuccess ||
      hipMemset(net->d_v, 0, (size_t)net->P * 4) != hipSuccess ||
      hipMemset(net->d_scalar, 0, 16) != hipSuccess) {
    tn_mlp_destroy(net);
    return set_error(TN_ERR_HIP, "mlp: initial upload");
  }
  *out = net;
  return TN_OK;
}

int64_t tn_mlp_num_params(const tn_mlp *net) {
  if (!net) return set_error(TN_ERR_ARG, "null net");
  return net->P;
}

int tn_mlp_shape(const tn_mlp *net, int32_t *d_in, int32_t *hidden) {
  clear_error();
  if (!net || !d_in || !hidden) return set_error(TN_ERR_ARG, "null argument");
  *d_in = net->D;
  *hidden = net->H;
  return TN_OK;
}

int tn_mlp_get_params(const tn_mlp *net, float *host_out) {
  clear_error();
  if (!net || !host_out) return set_error(TN_ERR_ARG, "null argument");
  TN_HIP_CHECK(hipDeviceSynchronize());
  TN_HIP_CHECK(hipMemcpy(host_out, net->d_params, (size_t)net->P * 4, hipMemcpyDeviceToHost));
  return TN_OK;
}

int tn_mlp_set_params(tn_mlp *net, const float *host_in) {
  clear_error();
  if (!net || !host_in) return set_error(TN_ERR_ARG, "null argument");
  TN_HIP_CHECK(hipDeviceSynchronize());
  TN_HIP_CHECK(hipMemcpy(net->d_params, host_in, (size_t)net->P * 4, hipMemcpyHostToDevice));
  TN_HIP_CHECK(hipMemset(net->d_m, 0, (size_t)net->P * 4));
  TN_HIP_CHECK(hipMemset(net->d_v, 0, (size_t)net->P * 4));
  TN_HIP_CHECK(hipDeviceSynchronize());
  net->t = 0;
  return TN_OK;
}

int tn_mlp_predict(tn_mlp *net, const float *X, int64_t n, void *stream, float *out) {
  clear_error();
  if (!net || n < 0) return set_error(TN_ERR_ARG, "bad argument");
  if (n == 0) return TN_OK;
  if (!X || !out) return set_error(TN_ERR_ARG, "null X or out");
  return fwd_bwd(net, X, nullptr, 0, n, n, (hipStream_t)stream, out, false);
}

int tn_mlp_grad(tn_mlp *net, const float *X, const float *y, int64_t n, void *stream, float *grad,
                double *loss) {
  clear_error();
  if (!net || !X || !y || !grad || n < 1) return set_error(TN_ERR_ARG, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  int rc = fwd_bwd(net, X, y, 0, n, n, st, nullptr, true);
  if (rc == TN_OK) rc = reduce(net, n, 0, grad, 0.f, st);
  if (rc == TN_OK && loss) {
    TN_HIP_CHECK(hipMemcpyAsync(loss, net->d_scalar, 8, hipMemcpyDeviceToHost, st));
    TN_HIP_CHECK(hipStreamSynchronize(st));
  }
  return rc;
}

int tn_mlp_step(tn_mlp *net, const float *X, const float *y, int64_t n, float lr, void *stream) {
  clear_error();
  if (!net || !X || !y || n < 1) return set_error(TN_ERR_ARG, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  int rc = fwd_bwd(net, X, y, 0, n, n, st, nullptr, true);
  if (rc == TN_OK) rc = reduce(net, n, 1, nullptr, lr, st);
  return rc;
}

int tn_mlp_train(tn_mlp *net, const float *X, const float *y, int64_t n, int32_t batch,
                 int32_t epochs, float lr, void *stream, double *losses) {
  clear_error();
  if (!net || !X || !y || n < 1 || batch < 1 || epochs < 0) return set_error(TN_ERR_ARG, "bad argument");
  hipStream_t st = (hipStream_t)stream;
  for (int ep = 0; ep < epochs; ++ep) {
    if (losses) TN_HIP_CHECK(hipMemsetAsync(net->d_scalar + 1, 0, 8, st));
    for (int64_t r0 = 0; r0 < n; r0 += batch) {
      const int64_t rows = std::min<int64_t>(batch, n - r0);
      int rc = fwd_bwd(net, X, y, r0, rows, n, st, nullptr, true);
      if (rc == TN_OK) rc = reduce(net, rows, 1, nullptr, lr, st, 1.0 / (double)n);
      if (rc != TN_OK) return rc;
    }
    if (losses) {
      TN_HIP_CHECK(hipMemcpyAsync(&losses[ep], net->d_scalar + 1, 8, hipMemcpyDeviceToHost, st));
      TN_HIP_CHECK(hipStreamSynchronize(st));
    }
  }
  return TN_OK;
}

void tn_mlp_destroy(tn_mlp *net) {
  if (!net) return;
  (void)hipDeviceSynchronize();
  if (net->d_params) (void)hipFree(net->d_params);
  if (net->d_m) (void)hipFree(net->d_m);
  if (net->d_v) (void)hipFree(net->d_v);
  if (net->d_partial) (void)hipFree(net->d_partial);
  if (net->d_scalar) (void)hipFree(net->d_scalar);
  delete net;
}

}  // extern "C"
