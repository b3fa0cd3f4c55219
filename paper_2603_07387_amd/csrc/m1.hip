// Cyclic-network estimator (Eq. (1), Algorithm 1) on gfx950.
//
// Per sample r and tensor k the time-domain tensor sketch is
//     y_{k,r}[(sum_u h_u(i_u)) mod m] += (prod_u s_u(i_u)) X_k(i)
// (Def. 12 in the column form of Algorithm 3; the second mode of every
// contraction uses the complement bucket (m - h) mod m, Def. 14).  The
// estimate is e_1^T F^{-1}(F y_1 o ... o F y_p) = (1/m) sum_j prod_k Y_k[j].
//
// Kernels:
//   m1_scatter  : one block streams one slot (a run of rows of one tensor)
//                 once from HBM, coalesced, and accumulates the sketches of SB
//                 samples in LDS in 64-bit fixed point (packed bucket/sign
//                 tables in LDS too).
//   m1_combine  : one block per (network, sample): two real sketches share one
//                 complex FFT in LDS (z = y_a + i y_b), the pair's product
//                 spectrum Y_a Y_b = (Z[j]^2 - conj(Z[-j])^2) / 4i is folded into
//                 per-thread FP64 accumulators over the half spectrum, and the
//                 Hermitian sum (1/m)(P_0 + P_{m/2} + 2 Re sum_{0<j<m/2} P_j)
//                 gives the estimate.
//   sample_stats: FP64 mean and unbiased variance over samples per network.
#include "m1_device.h"

#include <hip/hip_bf16.h>

namespace tn {
namespace {

using namespace m1dev;


// One block streams one slot and accumulates the sketches of SB samples (see
// scatter_slot), then writes them out as floating point.
// Blocks of 256 threads with one bank, 512 with two (twice the accumulator LDS
// per block, the same waves per CU).
template <typename T, typename A, int SB, int BANKS>
__global__ __launch_bounds__(256 * BANKS) void m1_scatter_kernel(
    const ScatterSlot *__restrict__ slots, const ModeDesc *__restrict__ modes,
    const void *const *__restrict__ data, const int32_t *__restrict__ tables, int64_t W,
    int64_t samples, int log2m, int64_t n_slots, A *__restrict__ ybuf) {
  // No static LDS: the accumulators start at LDS address 0, so their offsets
  // need no base add per term.
  extern __shared__ __align__(16) unsigned char smem[];
  const ScatterSlot sl = slots[blockIdx.x];
  const int tid = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.y * SB;
  const int nsb = (int)min((int64_t)SB, samples - s0);
  const uint32_t m = 1u << log2m, mask = m - 1;
  // BANKS banks of m words per sample (see scatter_slot), then the tables
  const uint32_t signbit = BANKS == 2 ? sign_bank_offset(SB, m) : 0u;
  const size_t acc_bytes = BANKS == 2 ? sign_bank_bytes(SB, m) : (size_t)SB * 8 * m;
  const size_t acc_end = (acc_bytes + 15) & ~(size_t)15;
  unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem);
  unsigned long long *s_max = reinterpret_cast<unsigned long long *>(smem + acc_end);  // [2]
  uint32_t *colt = reinterpret_cast<uint32_t *>(smem + acc_end + 16);                  // [SB][L]
  uint32_t *rowt = colt + SB * sl.L;                                                   // [SB][rows]
  constexpr int NT = 256 * BANKS;
  for (int i = tid; i < (int)(acc_bytes / 8); i += NT) acc[i] = 0ull;
  if (tid < 2) s_max[tid] = 0ull;
  const uint32_t N = (uint32_t)sl.rows * (uint32_t)sl.L;
  FixedScale fs;
  fs.lgN = max(N > 1 ? 32 - __clz(N - 1) : 0, 11);
  scatter_slot<T, SB, BANKS, NT>(sl, modes, data, tables + s0 * W, W, nsb, log2m, acc, 8u * m, signbit, colt,
                             rowt, s_max, fs);
  const unsigned long long *neg = acc + signbit / 8;
  for (int i = tid; i < nsb * (int)m; i += NT) {
    const int s = i >> log2m;
    const int b = i & mask;
    // positive bank minus negative bank
    const long long v = BANKS == 2 ? (long long)(acc[i] - neg[i]) : (long long)acc[i];
    ybuf[((s0 + s) * n_slots + blockIdx.x) * (int64_t)m + b] = (A)ldexp((double)v, -fs.scale);
  }
}

template <typename A, int LOG2M>
__global__ __launch_bounds__(256) void m1_combine_kernel(
    const NetDesc *__restrict__ nets, const int32_t *__restrict__ tslot,
    const A *__restrict__ ybuf, int64_t n_slots, int64_t sample0, int64_t S,
    const typename Cplx<A>::type *__restrict__ tw, double *__restrict__ est) {
  using A2 = typename Cplx<A>::type;
  constexpr int M = 1 << LOG2M;
  constexpr int H = M / 2 + 1;
  constexpr int NC = (H + 255) / 256;
  extern __shared__ __align__(16) unsigned char smem[];
  A2 *z = reinterpret_cast<A2 *>(smem);
  __shared__ double red[4];

  const NetDesc nd = nets[blockIdx.x];
  const int64_t s = blockIdx.y;
  const A *y = ybuf + s * n_slots * (int64_t)M;
  const int tid = threadIdx.x;

  double pr[NC], pi[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) { pr[c] = 1.0; pi[c] = 0.0; }

  for (int k = nd.t0; k < nd.t1; k += 2) {
    const bool pair = (k + 1) < nd.t1;
    const int a0 = tslot[k], a1 = tslot[k + 1];
    const int b1 = pair ? tslot[k + 2] : a1;
    for (int b = tid; b < M; b += 256) {
      A v1 = 0, v2 = 0;
      for (int sl = a0; sl < a1; ++sl) v1 += y[(int64_t)sl * M + b];
      for (int sl = a1; sl < b1; ++sl) v2 += y[(int64_t)sl * M + b];
      z[bitrev<LOG2M>(b)] = A2{v1, v2};
    }
    __syncthreads();
    fft_lds<A, LOG2M>(z, tw);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = tid + 256 * c;
      if (j < H) {
        const A2 za = z[j], zb = z[(M - j) & (M - 1)];
        const double ar = za.x, ai = za.y, br = zb.x, bi = -(double)zb.y;  // B = conj(Z[-j])
        double qr, qi;
        if (pair) {
          const double dr = (ar * ar - ai * ai) - (br * br - bi * bi);
          const double di = 2.0 * (ar * ai - br * bi);
          qr = 0.25 * di;     // -i (A^2 - B^2) / 4
          qi = -0.25 * dr;
        } else {
          qr = 0.5 * (ar + br);  // (A + B) / 2
          qi = 0.5 * (ai + bi);
        }
        const double nr = pr[c] * qr - pi[c] * qi;
        const double ni = pr[c] * qi + pi[c] * qr;
        pr[c] = nr;
        pi[c] = ni;
      }
    }
    __syncthreads();
  }

  double part = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int j = tid + 256 * c;
    if (j < H) part += ((j == 0 || 2 * j == M) ? 1.0 : 2.0) * pr[c];
  }
  const double tot = block_sum_256(part, red);
  if (tid == 0) est[(int64_t)blockIdx.x * S + sample0 + s] = tot / (double)M;
}

__global__ __launch_bounds__(256) void sample_stats_kernel(const double *__restrict__ est,
                                                           int64_t S, double *__restrict__ stats) {
  __shared__ double red[4];
  __shared__ double mean_sh;
  const double *x = est + (int64_t)blockIdx.x * S;
  double sum = 0.0;
  for (int64_t i = threadIdx.x; i < S; i += 256) sum += x[i];
  const double tot = block_sum_256(sum, red);
  if (threadIdx.x == 0) mean_sh = tot / (double)S;
  __syncthreads();
  const double mu = mean_sh;
  double sq = 0.0;
  for (int64_t i = threadIdx.x; i < S; i += 256) {
    const double d = x[i] - mu;
    sq += d * d;
  }
  const double ss = block_sum_256(sq, red);
  if (threadIdx.x == 0) {
    stats[2 * blockIdx.x] = mu;
    stats[2 * blockIdx.x + 1] = S > 1 ? ss / (double)(S - 1) : 0.0;
  }
}

template <typename A>
__global__ void slots_to_tensors_kernel(const int32_t *__restrict__ tslot, int64_t n_tensors,
                                        const A *__restrict__ ybuf, int64_t n_slots, int log2m,
                                        double *__restrict__ out) {
  const int64_t m = 1ll << log2m;
  const int64_t k = blockIdx.x, s = blockIdx.y;
  for (int64_t b = threadIdx.x; b < m; b += blockDim.x) {
    double v = 0.0;
    for (int sl = tslot[k]; sl < tslot[k + 1]; ++sl) v += (double)ybuf[(s * n_slots + sl) * m + b];
    out[(s * n_tensors + k) * m + b] = v;
  }
}

template <typename A>
__global__ void twiddle_kernel(int64_t m, typename Cplx<A>::type *out) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m / 2;
       j += (int64_t)gridDim.x * blockDim.x) {
    double sv, cv;
    sincospi(-2.0 * (double)j / (double)m, &sv, &cv);
    out[j] = typename Cplx<A>::type{(A)cv, (A)sv};
  }
}

template <typename T, typename A, int SB>
int scatter_sb(const M1Launch &L, hipStream_t st) {
  auto kern = L.banks == 2 ? m1_scatter_kernel<T, A, SB, 2> : m1_scatter_kernel<T, A, SB, 1>;
  if (L.lds_bytes > 65536)
    TN_HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)L.lds_bytes));
  dim3 grid((unsigned)L.n_slots, (unsigned)((L.samples + SB - 1) / SB));
  hipLaunchKernelGGL(kern, grid, dim3(256 * L.banks), L.lds_bytes, st, L.slots, L.modes, L.data, L.tables,
                     L.W, L.samples, L.log2m, L.n_slots, reinterpret_cast<A *>(L.ybuf));
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

template <typename T, typename A>
int scatter_t(const M1Launch &L, hipStream_t st) {
  switch (L.sb) {
    case 1: return scatter_sb<T, A, 1>(L, st);
    case 2: return scatter_sb<T, A, 2>(L, st);
    case 4: return scatter_sb<T, A, 4>(L, st);
    case 8: return scatter_sb<T, A, 8>(L, st);
    case 16: return scatter_sb<T, A, 16>(L, st);
    default: return set_error(TN_ERR_ARG, "scatter: unsupported sample batch %d", L.sb);
  }
}

template <typename A, int LOG2M>
int combine_m(const NetDesc *nets, int64_t n_nets, const int32_t *tslot, const void *ybuf,
              int64_t n_slots, int64_t samples, int64_t sample0, int64_t S, const void *tw,
              double *est, hipStream_t st) {
  using A2 = typename Cplx<A>::type;
  auto kern = m1_combine_kernel<A, LOG2M>;
  const size_t lds = sizeof(A2) << LOG2M;
  if (lds > 65536)
    TN_HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds));
  dim3 grid((unsigned)n_nets, (unsigned)samples);
  hipLaunchKernelGGL(kern, grid, dim3(256), lds, st, nets, tslot,
                     reinterpret_cast<const A *>(ybuf), n_slots, sample0, S,
                     reinterpret_cast<const A2 *>(tw), est);
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

template <typename A>
int combine_t(const NetDesc *nets, int64_t n_nets, const int32_t *tslot, const void *ybuf,
              int64_t n_slots, int64_t samples, int64_t sample0, int64_t S, int log2m,
              const void *tw, double *est, hipStream_t st) {
#define TN_COMBINE_CASE(LG) \
  case LG: return combine_m<A, LG>(nets, n_nets, tslot, ybuf, n_slots, samples, sample0, S, tw, est, st);
  switch (log2m) {
    TN_COMBINE_CASE(0) TN_COMBINE_CASE(1) TN_COMBINE_CASE(2) TN_COMBINE_CASE(3)
    TN_COMBINE_CASE(4) TN_COMBINE_CASE(5) TN_COMBINE_CASE(6) TN_COMBINE_CASE(7)
    TN_COMBINE_CASE(8) TN_COMBINE_CASE(9) TN_COMBINE_CASE(10) TN_COMBINE_CASE(11)
    TN_COMBINE_CASE(12) TN_COMBINE_CASE(13) TN_COMBINE_CASE(14)
    default: return set_error(TN_ERR_UNSUPPORTED, "combine: log2(m) = %d", log2m);
  }
#undef TN_COMBINE_CASE
}

}  // namespace

int launch_m1_scatter(const M1Launch &L, hipStream_t st) {
  if (L.n_slots == 0 || L.samples == 0) return TN_OK;
  if ((L.samples + L.sb - 1) / L.sb > 65535)
    return set_error(TN_ERR_UNSUPPORTED, "scatter: too many sample batches in one launch");
  switch (L.dtype) {
    case TN_F64: return scatter_t<double, double>(L, st);
    case TN_F32: return scatter_t<float, float>(L, st);
    case TN_BF16: return scatter_t<uint16_t, float>(L, st);
    default: return set_error(TN_ERR_ARG, "scatter: dtype %d", L.dtype);
  }
}

int launch_m1_combine(const NetDesc *nets, int64_t n_nets, const int32_t *tslot, int dtype,
                      const void *ybuf, int64_t n_slots, int64_t samples, int64_t sample0,
                      int64_t S, int log2m, const void *tw, double *est, hipStream_t st) {
  if (n_nets == 0 || samples == 0) return TN_OK;
  if (samples > 65535) return set_error(TN_ERR_UNSUPPORTED, "combine: samples per launch");
  if (dtype == TN_F64)
    return combine_t<double>(nets, n_nets, tslot, ybuf, n_slots, samples, sample0, S, log2m, tw,
                             est, st);
  return combine_t<float>(nets, n_nets, tslot, ybuf, n_slots, samples, sample0, S, log2m, tw, est,
                          st);
}

int launch_m1_slots_to_tensors(const int32_t *tslot, int64_t n_tensors, int dtype,
                               const void *ybuf, int64_t n_slots, int64_t samples, int log2m,
                               double *out, hipStream_t st) {
  if (n_tensors == 0 || samples == 0) return TN_OK;
  dim3 grid((unsigned)n_tensors, (unsigned)samples);
  if (dtype == TN_F64)
    hipLaunchKernelGGL(slots_to_tensors_kernel<double>, grid, dim3(256), 0, st, tslot, n_tensors,
                       reinterpret_cast<const double *>(ybuf), n_slots, log2m, out);
  else
    hipLaunchKernelGGL(slots_to_tensors_kernel<float>, grid, dim3(256), 0, st, tslot, n_tensors,
                       reinterpret_cast<const float *>(ybuf), n_slots, log2m, out);
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

int launch_twiddles(int64_t m, int dtype, void *out, hipStream_t st) {
  if (m < 2) return TN_OK;
  const unsigned blocks = (unsigned)((m / 2 + 255) / 256);
  if (dtype == TN_F64)
    hipLaunchKernelGGL(twiddle_kernel<double>, dim3(blocks), dim3(256), 0, st, m,
                       reinterpret_cast<double2 *>(out));
  else
    hipLaunchKernelGGL(twiddle_kernel<float>, dim3(blocks), dim3(256), 0, st, m,
                       reinterpret_cast<float2 *>(out));
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

int launch_sample_stats(const double *est, int64_t n_nets, int64_t S, double *stats,
                        hipStream_t st) {
  if (n_nets == 0) return TN_OK;
  hipLaunchKernelGGL(sample_stats_kernel, dim3((unsigned)n_nets), dim3(256), 0, st, est, S, stats);
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

}  // namespace tn
