// The cyclic method's combine (Eq. (1): y = e_1^T F^{-1}(prod_k F y_k)) with the
// m-point DFTs taken as small dense products on the BF16 matrix cores, for
// m = 1024 (TN_FLAG_DFT_BF16).
//
// Four-step form, m = 32 x 32: with b = 32 b1 + b2 and j = j1 + 32 j2,
//   Y[j1 + 32 j2] = sum_b2 w32^(b2 j2) [ w1024^(b2 j1) sum_b1 w32^(b1 j1) y[32 b1 + b2] ],
// w_n = exp(-2 pi i / n).  With Ymat[b1][b2] = y[32 b1 + b2] (the row-major
// 32 x 32 view of the sketch) and F the 32-point DFT matrix:
//   A = F Ymat          (a real operand: two real 32 x 32 x 32 products),
//   B = A o T,  T[j1][b2] = w1024^(b2 j1)          (twiddles, FP32),
//   Z = B F             (four real products),
// and Z[j1][j2] = Y[j1 + 32 j2].  Every tensor's spectrum comes out in the same
// (j1, j2) arrangement, and the estimate only needs the sum over all
// frequencies of the product over tensors, so no reordering is needed.
//
// Block: one (network, sample), four waves; wave w owns the 16 x 16 tile
// (rows 16 (w / 2), columns 16 (w % 2)) of A, of B's twiddled copy and of Z.
// Products on v_mfma_f32_16x16x32_bf16 (A[i][k] in lane i + 16 (k / 8) element
// k % 8, B[k][j] in lane j + 16 (k / 8) element k % 8, D[i][j] in lane
// j + 16 (i / 4) item i % 4), operands rounded to BF16 (nearest even), FP32
// accumulation; the running product over tensors and the final sum in FP64.
#include <hip/hip_bf16.h>

#include "m1_device.h"

namespace tn {
namespace {

using namespace m1dev;

typedef __bf16 dbf16x8 __attribute__((ext_vector_type(8)));
typedef float df32x4 __attribute__((ext_vector_type(4)));

constexpr int kYStr = 40;  // bf16 per LDS row of the staged matrices (80 bytes: rows start 16-byte aligned)

__global__ __launch_bounds__(256) void m1_combine_dft32_kernel(const NetDesc *__restrict__ nets,
                                                               const int32_t *__restrict__ tbeg,
                                                               const int32_t *__restrict__ tend,
                                                               const float *__restrict__ ybuf, int64_t n_slots,
                                                               int64_t sample0, int64_t S, double *__restrict__ est) {
  constexpr int M = 1024;
  __shared__ __align__(16) __bf16 yT[32 * kYStr];      // yT[b2][b1] = y[32 b1 + b2]
  __shared__ __align__(16) __bf16 bR[32 * kYStr];      // B[j1][b2], real part
  __shared__ __align__(16) __bf16 bI[32 * kYStr];      // imaginary part
  __shared__ double red[4];
  const NetDesc nd = nets[blockIdx.x];
  const int64_t s = blockIdx.y;
  const float *y = ybuf + s * n_slots * (int64_t)M;
  auto load4 = [&](int64_t off) { return *reinterpret_cast<const float4 *>(y + off); };
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int ti = w >> 1, tj = w & 1;
  const int l16 = lane & 15, g = lane >> 4;  // operand lane (row or column, k group)

  // Constant operands.  Step 1's A operand: F[16 ti + l16][8 g + e]; step 3's
  // B operand: F[8 g + e][16 tj + l16].  F is symmetric.
  dbf16x8 fr1, fi1, fr3, fi3;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    float sv, cv;
    sincospif(-2.0f * (float)(((16 * ti + l16) * (8 * g + e)) & 31) / 32.0f, &sv, &cv);
    fr1[e] = (__bf16)cv;
    fi1[e] = (__bf16)sv;
    sincospif(-2.0f * (float)(((8 * g + e) * (16 * tj + l16)) & 31) / 32.0f, &sv, &cv);
    fr3[e] = (__bf16)cv;
    fi3[e] = (__bf16)sv;
  }
  // This lane's D items r: row i = 4 g + r (j1 = 16 ti + i), column l16 (b2 or
  // j2 = 16 tj + l16).  Twiddles w1024^(b2 j1) for step 2.
  float twr[4], twi[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int j1 = 16 * ti + 4 * g + r, b2 = 16 * tj + l16;
    sincospif(-2.0f * (float)((j1 * b2) & (M - 1)) / (float)M, &twi[r], &twr[r]);
  }
  double pr[4] = {1.0, 1.0, 1.0, 1.0}, pi[4] = {0.0, 0.0, 0.0, 0.0};

  // The first slot of the next tensor is loaded while the current one is
  // transformed: its load latency hides behind the barriers and products.
  float4 vn = make_float4(0.f, 0.f, 0.f, 0.f);
  if (nd.t0 < nd.t1) vn = load4((int64_t)tbeg[nd.t0] * M + 4 * tid);
  for (int k = nd.t0; k < nd.t1; ++k) {
    // stage the sketch (sum of its slots), transposed, as BF16: thread tid holds
    // points 4 tid .. 4 tid + 3 (row b1 = tid / 8, columns b2 = 4 (tid % 8) + c)
    const int a0 = tbeg[k], a1 = tend[k];
    float4 v = vn;
    if (k + 1 < nd.t1) vn = load4((int64_t)tbeg[k + 1] * M + 4 * tid);
    for (int sl = a0 + 1; sl < a1; ++sl) {
      const float4 u = load4((int64_t)sl * M + 4 * tid);
      v.x += u.x;
      v.y += u.y;
      v.z += u.z;
      v.w += u.w;
    }
    {
      const int b1 = tid >> 3, c0 = 4 * (tid & 7);
      yT[(c0 + 0) * kYStr + b1] = (__bf16)v.x;
      yT[(c0 + 1) * kYStr + b1] = (__bf16)v.y;
      yT[(c0 + 2) * kYStr + b1] = (__bf16)v.z;
      yT[(c0 + 3) * kYStr + b1] = (__bf16)v.w;
    }
    __syncthreads();
    // step 1: A tile = F[16 ti .. +16][0..32) Ymat[0..32)[16 tj .. +16); the B
    // operand Ymat[8 g + e][16 tj + l16] = yT[16 tj + l16][8 g + e]
    const dbf16x8 yb = *reinterpret_cast<const dbf16x8 *>(yT + (16 * tj + l16) * kYStr + 8 * g);
    const df32x4 zero = {0.f, 0.f, 0.f, 0.f};
    const df32x4 ar = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr1, yb, zero, 0, 0, 0);
    const df32x4 ai = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fi1, yb, zero, 0, 0, 0);
    // step 2: B = A o T, stored row-major B[j1][b2] for step 3's A operand
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j1 = 16 * ti + 4 * g + r, b2 = 16 * tj + l16;
      const float br = ar[r] * twr[r] - ai[r] * twi[r];
      const float bi = ar[r] * twi[r] + ai[r] * twr[r];
      bR[j1 * kYStr + b2] = (__bf16)br;
      bI[j1 * kYStr + b2] = (__bf16)bi;
    }
    __syncthreads();
    // step 3: Z tile = B[16 ti .. +16][0..32) F[0..32)[16 tj .. +16)
    const dbf16x8 xr = *reinterpret_cast<const dbf16x8 *>(bR + (16 * ti + l16) * kYStr + 8 * g);
    const dbf16x8 xi = *reinterpret_cast<const dbf16x8 *>(bI + (16 * ti + l16) * kYStr + 8 * g);
    dbf16x8 nxi;
#pragma unroll
    for (int e = 0; e < 8; ++e) nxi[e] = -xi[e];
    df32x4 zr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xr, fr3, zero, 0, 0, 0);
    zr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nxi, fi3, zr, 0, 0, 0);
    df32x4 zi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xr, fi3, zero, 0, 0, 0);
    zi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xi, fr3, zi, 0, 0, 0);
    // running product over the tensors, in FP64
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double a = zr[r], b = zi[r];
      const double nr = pr[r] * a - pi[r] * b, ni = pr[r] * b + pi[r] * a;
      pr[r] = nr;
      pi[r] = ni;
    }
  }
  // (1/m) Re sum over all m frequencies (each lane holds 4; the block 1024)
  double part = pr[0] + pr[1] + pr[2] + pr[3];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
  if (lane == 0) red[w] = part;
  __syncthreads();
  if (tid == 0) est[(int64_t)blockIdx.x * S + sample0 + s] = (red[0] + red[1] + red[2] + red[3]) / (double)M;
}

}  // namespace

int launch_m1_combine_dft32(const NetDesc *nets, int64_t n_nets, const int32_t *tbeg, const int32_t *tend,
                            const void *ybuf, int64_t n_slots, int64_t samples, int64_t sample0, int64_t S,
                            double *est, hipStream_t st) {
  if (n_nets == 0 || samples == 0) return TN_OK;
  if (samples > 65535) return set_error(TN_ERR_UNSUPPORTED, "combine: samples per launch");
  hipLaunchKernelGGL(m1_combine_dft32_kernel, dim3((unsigned)n_nets, (unsigned)samples), dim3(256), 0, st, nets,
                     tbeg, tend, reinterpret_cast<const float *>(ybuf), n_slots, sample0, S, est);
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

}  // namespace tn
