// The cyclic method's combine (Eq. (1): y = e_1^T F^{-1}(prod_k F y_k)) with the
// m-point DFTs taken as small dense products on the BF16 matrix cores, for
// m = 1024 (TN_FLAG_DFT_BF16), or on the FP8 ones (TN_FLAG_DFT_FP8, below).
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
// Block: one network and spb of its samples in turn (see the launcher), four
// waves; wave w owns the 16 x 16 tile
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
// Samples one BF16 block transforms in turn when the launch has enough
// (network, sample) pairs to fill the GPU anyway (measured on the batch, 1, 2,
// 4, 8: combine 0.66, 0.57, 0.55, 0.57 ms per step); one otherwise, so that a
// plan of few networks keeps its blocks.
constexpr int kDftSamplesPerBlock = 4;
constexpr int64_t kDftSplitPairs = 16384;  // (network, sample) pairs from which blocks take kDftSamplesPerBlock

__global__ __launch_bounds__(256) void m1_combine_dft32_kernel(const NetDesc *__restrict__ nets,
                                                               const int32_t *__restrict__ tbeg,
                                                               const int32_t *__restrict__ tend,
                                                               const float *__restrict__ ybuf, int64_t n_slots,
                                                               int64_t n_samp, int spb, int64_t sample0, int64_t S,
                                                               const float2 *__restrict__ tw,
                                                               double *__restrict__ est) {
  constexpr int M = 1024;
  __shared__ __align__(16) __bf16 yT[32 * kYStr];      // yT[b2][b1] = y[32 b1 + b2]
  __shared__ __align__(16) __bf16 bR[32 * kYStr];      // B[j1][b2], real part
  __shared__ __align__(16) __bf16 bI[32 * kYStr];      // imaginary part
  __shared__ double red[4];
  const NetDesc nd = nets[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int ti = w >> 1, tj = w & 1;
  const int l16 = lane & 15, g = lane >> 4;  // operand lane (row or column, k group)
  // The block's samples sA .. sA + ns - 1 (of this launch), one after the
  // other: the constants below are set up once, and the tensor loop runs on
  // across the samples, so the loads of the next sample's first tensors are
  // in flight during the last ones of the current sample.
  const int64_t sA = (int64_t)blockIdx.y * spb;
  const int ns = (int)min((int64_t)spb, n_samp - sA);
  const int p = nd.t1 - nd.t0, nsteps = ns * p;  // step g: sample g / p, tensor t0 + g % p
  auto load4 = [&](int64_t si, int64_t off) {
    return *reinterpret_cast<const float4 *>(ybuf + (sA + si) * n_slots * (int64_t)M + off);
  };
  auto load_first = [&](int gi) {  // the first slot of step gi's sketch
    const int si = gi / p;
    return load4(si, (int64_t)tbeg[nd.t0 + gi - si * p] * M + 4 * tid);
  };

  // Constant operands, read from the plan's half table of 1024-point twiddles
  // (tw[j] = w1024^j for j < 512; w1024^(j + 512) = -tw[j]): w32^k = w1024^(32 k).
  // Step 1's A operand: F[16 ti + l16][8 g + e]; step 3's B operand:
  // F[8 g + e][16 tj + l16].  F is symmetric.
  auto w1024 = [&](int j) {
    j &= M - 1;
    const float2 t = tw[j & (M / 2 - 1)];
    return j < M / 2 ? t : make_float2(-t.x, -t.y);
  };
  dbf16x8 fr1, fi1, fr3, fi3, nfi3;  // nfi3 = -fi3 (for the real part of step 3)
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float2 a = w1024(32 * ((16 * ti + l16) * (8 * g + e))), b = w1024(32 * ((8 * g + e) * (16 * tj + l16)));
    fr1[e] = (__bf16)a.x;
    fi1[e] = (__bf16)a.y;
    fr3[e] = (__bf16)b.x;
    fi3[e] = (__bf16)b.y;
    nfi3[e] = (__bf16)(-b.y);
  }
  // This lane's D items r: row i = 4 g + r (j1 = 16 ti + i), column l16 (b2 or
  // j2 = 16 tj + l16).  Twiddles w1024^(b2 j1) for step 2.
  float twr[4], twi[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float2 t = w1024((16 * ti + 4 * g + r) * (16 * tj + l16));
    twr[r] = t.x;
    twi[r] = t.y;
  }
  double pr[4] = {1.0, 1.0, 1.0, 1.0}, pi[4] = {0.0, 0.0, 0.0, 0.0};

  constexpr int kAhead = 2;  // measured: 1, 2, 3, 4 ahead: combine 0.705, 0.658, 0.737, 0.723 ms per batched step (3 and 4 cost a wave per SIMD)
  // Step gi's transform (sample si = gi / p, tensor k).  vr holds the first
  // slot of its sketch; once that is staged, vr is reloaded with the first
  // slot of step gi + kAhead, so with kAhead such registers (the loop below,
  // unrolled) the loads of the next kAhead steps are in flight during the
  // barriers and products.  A register is reloaded only after its use, so no
  // load is waited for early.  After a sample's last tensor its estimate is
  // written and the running product restarts.
  auto step = [&](float4 &vr, int gi) {
    const int si = gi / p, k = nd.t0 + gi - si * p;
    // stage the sketch (sum of its slots), transposed, as BF16: thread tid holds
    // points 4 tid .. 4 tid + 3 (row b1 = tid / 8, columns b2 = 4 (tid % 8) + c)
    const int a0 = tbeg[k], a1 = tend[k];
    float4 v = vr;
    for (int sl = a0 + 1; sl < a1; ++sl) {
      const float4 u = load4(si, (int64_t)sl * M + 4 * tid);
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
    if (gi + kAhead < nsteps) vr = load_first(gi + kAhead);
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
    df32x4 zr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xr, fr3, zero, 0, 0, 0);
    zr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xi, nfi3, zr, 0, 0, 0);
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
    if (k == nd.t1 - 1) {  // the sample's last tensor (uniform over the block)
      // (1/m) Re sum over all m frequencies (each lane holds 4; the block 1024).
      // red is rewritten only after the next tensor's two barriers.
      double part = pr[0] + pr[1] + pr[2] + pr[3];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
      if (lane == 0) red[w] = part;
      __syncthreads();
      if (tid == 0)
        est[(int64_t)blockIdx.x * S + sample0 + sA + si] = (red[0] + red[1] + red[2] + red[3]) / (double)M;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        pr[r] = 1.0;
        pi[r] = 0.0;
      }
    }
  };
  float4 vq[kAhead];
#pragma unroll
  for (int a = 0; a < kAhead; ++a) vq[a] = a < nsteps ? load_first(a) : make_float4(0.f, 0.f, 0.f, 0.f);
  for (int gb = 0; gb < nsteps; gb += kAhead) {
#pragma unroll
    for (int a = 0; a < kAhead; ++a)
      if (gb + a < nsteps) step(vq[a], gb + a);
  }
}

// ---------------------------------------------------------------------------
// The same four-step transform on the FP8 matrix cores (TN_FLAG_DFT_FP8):
// v_mfma_f32_16x16x32_fp8_fp8 with OCP E4M3 operands (3 mantissa bits, largest
// finite 448, rounded to nearest even; A[i][k] in lane i + 16 (k / 8) byte k % 8,
// B[k][j] in lane j + 16 (k / 8) byte k % 8, D as for BF16), FP32 accumulation.
// FP8 has no exponent range to spare, so each operand block is scaled by a
// power of two before rounding: the sketch by 2^s1 and the twiddled
// intermediate by 2^s2, each chosen from its block-wide maximum so that the
// largest magnitude lands in [128, 256); the product is scaled back by
// 2^-(s1 + s2) in FP64, exactly.  Both staged matrices stay FP32 in LDS until
// their operands are loaded.
// Keeping the estimator unbiased: rounding the DFT constants to nearest is the
// same error in every sample (one E4M3 copy of F shrank the estimates by 0.7 %
// on a positive triangle), so F is carried as two E4M3 terms, F = F_hi + F_lo
// with F_lo the rounded residual (error about 2^-8 relative), and every product
// with F takes two matrix instructions.  Rounding the data to nearest is a
// fixed function of each bucket's value, which depends on the hashes the
// tensors share, so those errors correlate across tensors and the product over
// tensors picked up a bias (+0.5 % on the same triangle).  The data operands
// are therefore rounded stochastically (v_cvt_sr_fp8_f32: E[round(x)] = x), with
// random bits from a counter-based hash of (network, sample, tensor, stage,
// element), independent of the sketch hashes: each stage is then an unbiased
// linear map of its input, and the product over tensors of independent
// unbiased spectra is unbiased.  The price is rounding noise below one ulp
// (2^-3 relative) instead of half of one.
typedef long dfp8x8;  // 8 E4M3 values, byte e holds element e

__device__ __forceinline__ dfp8x8 pack_fp8(const float *v, int sc) {
  int w0 = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(v[0], sc), ldexpf(v[1], sc), 0, false);
  w0 = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(v[2], sc), ldexpf(v[3], sc), w0, true);
  int w1 = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(v[4], sc), ldexpf(v[5], sc), 0, false);
  w1 = __builtin_amdgcn_cvt_pk_fp8_f32(ldexpf(v[6], sc), ldexpf(v[7], sc), w1, true);
  return (dfp8x8)((unsigned long)(unsigned)w0 | ((unsigned long)(unsigned)w1 << 32));
}

// Two E4M3 terms of 8 values (unscaled, |v| <= 1): hi = fp8(v), lo = fp8(v - hi).
typedef float dfv2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void pack_fp8_split(const float *v, dfp8x8 *hi, dfp8x8 *lo) {
  *hi = pack_fp8(v, 0);
  float r[8];
  const int w0 = (int)(unsigned)(unsigned long)*hi, w1 = (int)(unsigned)((unsigned long)*hi >> 32);
  const dfv2 a = __builtin_amdgcn_cvt_pk_f32_fp8(w0, false), b = __builtin_amdgcn_cvt_pk_f32_fp8(w0, true);
  const dfv2 c = __builtin_amdgcn_cvt_pk_f32_fp8(w1, false), d = __builtin_amdgcn_cvt_pk_f32_fp8(w1, true);
  r[0] = v[0] - a.x;
  r[1] = v[1] - a.y;
  r[2] = v[2] - b.x;
  r[3] = v[3] - b.y;
  r[4] = v[4] - c.x;
  r[5] = v[5] - c.y;
  r[6] = v[6] - d.x;
  r[7] = v[7] - d.y;
  *lo = pack_fp8(r, 0);
}

// 32-bit integer hash (the "lowbias32" finalizer published by C. Wellons).
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// 8 values scaled by 2^sc, rounded stochastically to E4M3; value e of the
// operand is element elem0 + e of the stage whose key is `key`.  One hash per 8
// values: value e takes it times a distinct odd constant (a bijection of 32-bit
// words, so each value's bits stay uniform; the 8 roundings of a lane are then
// not independent of each other, which leaves each one unbiased).
__device__ __forceinline__ dfp8x8 pack_fp8_sr(const float *v, int sc, uint32_t key, uint32_t elem0) {
  const uint32_t h = hash32(key ^ elem0 * 0x9e3779b9u);
  auto rnd = [&](int e) { return (int)(h * (0x9e3779b9u + 2u * 0x85ebca6bu * (uint32_t)e)); };
  int w0 = __builtin_amdgcn_cvt_sr_fp8_f32(ldexpf(v[0], sc), rnd(0), 0, 0);
  w0 = __builtin_amdgcn_cvt_sr_fp8_f32(ldexpf(v[1], sc), rnd(1), w0, 1);
  w0 = __builtin_amdgcn_cvt_sr_fp8_f32(ldexpf(v[2], sc), rnd(2), w0, 2);
  w0 = __builtin_amdgcn_cvt_sr_fp8_f32(ldexpf(v[3], sc), rnd(3), w0, 3);
  int w1 = __builtin_amdgcn_cvt_sr_fp8_f32(ldexpf(v[4], sc), rnd(4), 0, 0);
  w1 = __builtin_amdgcn_cvt_sr_fp8_f32(ldexpf(v[5], sc), rnd(5), w1, 1);
  w1 = __builtin_amdgcn_cvt_sr_fp8_f32(ldexpf(v[6], sc), rnd(6), w1, 2);
  w1 = __builtin_amdgcn_cvt_sr_fp8_f32(ldexpf(v[7], sc), rnd(7), w1, 3);
  return (dfp8x8)((unsigned long)(unsigned)w0 | ((unsigned long)(unsigned)w1 << 32));
}

// Exponent s with bm 2^s in [128, 256) (0 for an all-zero block).
__device__ __forceinline__ int fp8_scale(float bm) {
  if (!(bm > 0.f)) return 0;
  int e;
  (void)frexpf(bm, &e);  // bm = f 2^e, f in [0.5, 1)
  return 8 - e;
}

constexpr int kFStr = 36;  // floats per LDS row of the staged matrices (rows 16-byte aligned)

__global__ __launch_bounds__(256) void m1_combine_dft32_fp8_kernel(const NetDesc *__restrict__ nets,
                                                                   const int32_t *__restrict__ tbeg,
                                                                   const int32_t *__restrict__ tend,
                                                                   const float *__restrict__ ybuf, int64_t n_slots,
                                                                   int64_t n_samp, int spb, int64_t sample0, int64_t S,
                                                                   const float2 *__restrict__ tw,
                                                                   double *__restrict__ est) {
  constexpr int M = 1024;
  __shared__ __align__(16) float yT[32 * kFStr];  // yT[b2][b1] = y[32 b1 + b2]
  __shared__ __align__(16) float bR[32 * kFStr];  // B[j1][b2], real part
  __shared__ __align__(16) float bI[32 * kFStr];  // imaginary part
  __shared__ float rmax[2][4];
  __shared__ double red[4];
  const NetDesc nd = nets[blockIdx.x];
  const int64_t s = blockIdx.y;
  const float *y = ybuf + s * n_slots * (int64_t)M;
  auto load4 = [&](int64_t off) { return *reinterpret_cast<const float4 *>(y + off); };
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int ti = w >> 1, tj = w & 1;
  const int l16 = lane & 15, g = lane >> 4;
  auto wave_max = [](float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
  };

  // constant operands, as in the BF16 kernel (from the twiddle table), each as
  // two E4M3 terms
  auto w1024 = [&](int j) {
    j &= M - 1;
    const float2 t = tw[j & (M / 2 - 1)];
    return j < M / 2 ? t : make_float2(-t.x, -t.y);
  };
  dfp8x8 fr1, fi1, fr3, fi3, fr1l, fi1l, fr3l, fi3l;
  {
    float c1[8], s1[8], c3[8], s3[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float2 a = w1024(32 * ((16 * ti + l16) * (8 * g + e))), b = w1024(32 * ((8 * g + e) * (16 * tj + l16)));
      c1[e] = a.x;
      s1[e] = a.y;
      c3[e] = b.x;
      s3[e] = b.y;
    }
    pack_fp8_split(c1, &fr1, &fr1l);
    pack_fp8_split(s1, &fi1, &fi1l);
    pack_fp8_split(c3, &fr3, &fr3l);
    pack_fp8_split(s3, &fi3, &fi3l);
  }
  float twr[4], twi[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float2 t = w1024((16 * ti + 4 * g + r) * (16 * tj + l16));
    twr[r] = t.x;
    twi[r] = t.y;
  }
  double pr[4] = {1.0, 1.0, 1.0, 1.0}, pi[4] = {0.0, 0.0, 0.0, 0.0};

  // Tensor k's transform; the loads of the next tensors' first slots rotate
  // through kAhead registers as in the BF16 kernel.
  auto step = [&](float4 &vr, int k, int knext) {
    const int a0 = tbeg[k], a1 = tend[k];
    float4 v = vr;
    for (int sl = a0 + 1; sl < a1; ++sl) {
      const float4 u = load4((int64_t)sl * M + 4 * tid);
      v.x += u.x;
      v.y += u.y;
      v.z += u.z;
      v.w += u.w;
    }
    {
      const int b1 = tid >> 3, c0 = 4 * (tid & 7);
      yT[(c0 + 0) * kFStr + b1] = v.x;
      yT[(c0 + 1) * kFStr + b1] = v.y;
      yT[(c0 + 2) * kFStr + b1] = v.z;
      yT[(c0 + 3) * kFStr + b1] = v.w;
      const float mx = wave_max(fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
      if (lane == 0) rmax[0][w] = mx;
    }
    if (knext < nd.t1) vr = load4((int64_t)tbeg[knext] * M + 4 * tid);  // kAhead tensors ahead
    __syncthreads();
    const int s1 = fp8_scale(fmaxf(fmaxf(rmax[0][0], rmax[0][1]), fmaxf(rmax[0][2], rmax[0][3])));
    // rounding keys of this (network, sample, tensor): stage 0 the sketch, 1 and 2 B
    const uint32_t key = hash32(hash32((uint32_t)blockIdx.x * 0x85ebca6bu ^ hash32((uint32_t)(sample0 + s))) ^
                                (uint32_t)k * 0xc2b2ae35u);
    // step 1: A tile = F[16 ti .. +16][0..32) (Ymat 2^s1)[0..32)[16 tj .. +16); both waves
    // that load an element round it alike (its key is the element's)
    const dfp8x8 yb = pack_fp8_sr(yT + (16 * tj + l16) * kFStr + 8 * g, s1, hash32(key),
                                  (uint32_t)((16 * tj + l16) * 32 + 8 * g));
    const df32x4 zero = {0.f, 0.f, 0.f, 0.f};
    df32x4 ar = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(fr1l, yb, zero, 0, 0, 0);
    ar = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(fr1, yb, ar, 0, 0, 0);
    df32x4 ai = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(fi1l, yb, zero, 0, 0, 0);
    ai = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(fi1, yb, ai, 0, 0, 0);
    // step 2: B = A o T (FP32), stored row-major B[j1][b2], and its block maximum
    float bmx = 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j1 = 16 * ti + 4 * g + r, b2 = 16 * tj + l16;
      const float br = ar[r] * twr[r] - ai[r] * twi[r];
      const float bi = ar[r] * twi[r] + ai[r] * twr[r];
      bR[j1 * kFStr + b2] = br;
      bI[j1 * kFStr + b2] = bi;
      bmx = fmaxf(bmx, fmaxf(fabsf(br), fabsf(bi)));
    }
    bmx = wave_max(bmx);
    if (lane == 0) rmax[1][w] = bmx;
    __syncthreads();
    const int s2 = fp8_scale(fmaxf(fmaxf(rmax[1][0], rmax[1][1]), fmaxf(rmax[1][2], rmax[1][3])));
    // step 3: Z tile = (B 2^s2)[16 ti .. +16][0..32) F[0..32)[16 tj .. +16)
    const uint32_t eb = (uint32_t)((16 * ti + l16) * 32 + 8 * g);
    const dfp8x8 xr = pack_fp8_sr(bR + (16 * ti + l16) * kFStr + 8 * g, s2, hash32(key ^ 1u), eb);
    const dfp8x8 xi = pack_fp8_sr(bI + (16 * ti + l16) * kFStr + 8 * g, s2, hash32(key ^ 2u), eb);
    const dfp8x8 nxi = xi ^ (dfp8x8)0x8080808080808080ull;  // E4M3 negation: the sign bit of each byte
    df32x4 zr = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(xr, fr3l, zero, 0, 0, 0);
    zr = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(nxi, fi3l, zr, 0, 0, 0);
    zr = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(xr, fr3, zr, 0, 0, 0);
    zr = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(nxi, fi3, zr, 0, 0, 0);
    df32x4 zi = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(xr, fi3l, zero, 0, 0, 0);
    zi = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(xi, fr3l, zi, 0, 0, 0);
    zi = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(xr, fi3, zi, 0, 0, 0);
    zi = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(xi, fr3, zi, 0, 0, 0);
    // the spectrum carries 2^(s1 + s2): undone in FP64, then the running product
    const double us = ldexp(1.0, -(s1 + s2));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double a = (double)zr[r] * us, b = (double)zi[r] * us;
      const double nr = pr[r] * a - pi[r] * b, ni = pr[r] * b + pi[r] * a;
      pr[r] = nr;
      pi[r] = ni;
    }
  };
  constexpr int kAhead = 2;
  float4 vq[kAhead];
#pragma unroll
  for (int a = 0; a < kAhead; ++a)
    vq[a] = nd.t0 + a < nd.t1 ? load4((int64_t)tbeg[nd.t0 + a] * M + 4 * tid) : make_float4(0.f, 0.f, 0.f, 0.f);
  for (int k = nd.t0; k < nd.t1; k += kAhead) {
#pragma unroll
    for (int a = 0; a < kAhead; ++a)
      if (k + a < nd.t1) step(vq[a], k + a, k + a + kAhead);
  }
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
                            const void *twiddles, double *est, bool fp8, hipStream_t st) {
  if (n_nets == 0 || samples == 0) return TN_OK;
  if (samples > 65535) return set_error(TN_ERR_UNSUPPORTED, "combine: samples per launch");
  const int spb = !fp8 && n_nets * samples >= kDftSplitPairs ? kDftSamplesPerBlock : 1;
  const unsigned gy = (unsigned)((samples + spb - 1) / spb);
  hipLaunchKernelGGL(fp8 ? m1_combine_dft32_fp8_kernel : m1_combine_dft32_kernel, dim3((unsigned)n_nets, gy),
                     dim3(256), 0, st, nets, tbeg, tend, reinterpret_cast<const float *>(ybuf), n_slots, samples,
                     spb, sample0, S, reinterpret_cast<const float2 *>(twiddles), est);
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

}  // namespace tn
