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


constexpr int kStageMaxLog2M = 12;  // largest log2 m that stages the column hash words

// Waves per SIMD the register allocation must allow: four (two blocks per CU)
// for the 512-thread FP32 blocks whose loop keeps 8 loads in flight (their
// LDS leaves room for two blocks at m = 1024); no constraint otherwise.
template <typename T, int SB, int NT>
constexpr int kScatterWavesPerEU = (NT == 512 && sizeof(T) == 4 && SB * 4 <= 16) ? 4 : 1;

// One block streams one slot and accumulates the sketches of SB samples (see
// scatter_slot), then writes them out as floating point.
// Blocks of 256 threads with one bank, 512 with two (twice the accumulator LDS
// per block, the same waves per CU); NT = 1024 when one block fills a CU's LDS
// (large m or many samples per pass), so that the CU still runs 16 waves.
// RANGED (m above kMaxLog2Acc buckets): blockIdx.z selects the range of
// 2^log2acc buckets the block accumulates (one bank, one sample per pass).
// Fixed-point scale: with bound_in, slot b's entries are all below
// bound_in[b] (a power of two, or 0 for an all-zero slot) and the scale is set
// once; otherwise the block keeps a running maximum (a barrier per load round)
// and, with bound_out, records the power-of-two bound it ends with.
// Sample batch blockIdx.y + y0 of the launch's samples.
template <typename T, typename A, int SB, int BANKS, bool RANGED = false, int NT = 256 * BANKS>
__global__ __launch_bounds__(NT, (kScatterWavesPerEU<T, SB, NT>)) void m1_scatter_kernel(
    const ScatterSlot *__restrict__ slots, const ModeDesc *__restrict__ modes,
    const void *const *__restrict__ data, const int32_t *__restrict__ tables, int64_t W,
    int64_t samples, int log2m, int log2acc, int64_t n_slots, A *__restrict__ ybuf,
    const double *__restrict__ bound_in, double *__restrict__ bound_out, int y0) {
  // No static LDS: the accumulators start at LDS address 0, so their offsets
  // need no base add per term.
  extern __shared__ __align__(16) unsigned char smem[];
  const ScatterSlot sl = slots[blockIdx.x];
  const int tid = threadIdx.x;
  const int64_t s0 = ((int64_t)blockIdx.y + y0) * SB;
  const int nsb = (int)min((int64_t)SB, samples - s0);
  const uint32_t m = 1u << log2m;
  const uint32_t ma = RANGED ? 1u << log2acc : m, amask = ma - 1;  // accumulator words per sample
  const uint32_t r0 = RANGED ? blockIdx.z * ma : 0u;              // first bucket of the range
  // BANKS banks of m words per sample (see scatter_slot), then the tables
  const uint32_t signbit = BANKS == 2 ? sign_bank_offset(SB, m) : 0u;
  const size_t acc_bytes = BANKS == 2 ? sign_bank_bytes(SB, m) : (size_t)SB * 8 * ma;
  const size_t acc_end = (acc_bytes + 15) & ~(size_t)15;
  unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem);
  unsigned long long *s_max = reinterpret_cast<unsigned long long *>(smem + acc_end);  // [2]
  uint32_t *tabs = reinterpret_cast<uint32_t *>(smem + acc_end + 16);  // column and row tables
  // Up to m = 4096 the column tables are built from hash words staged in the
  // not yet cleared accumulators (scatter_slot clears them afterwards); above
  // it the clear of the large accumulators is better done first (measured).
  const bool stage = log2m <= kStageMaxLog2M;
  if (!stage) lds_zero(acc, (uint32_t)acc_bytes, tid, NT);
  if (tid < 2) s_max[tid] = 0ull;
  const uint32_t N = (uint32_t)sl.rows * (uint32_t)sl.L;
  FixedScale fs;
  fs.lgN = max(N > 1 ? 32 - __clz(N - 1) : 0, 11);
  if (bound_in != nullptr) {
    const double b = bound_in[blockIdx.x];
    if (b > 0.0) {
      int e;
      (void)frexp(b, &e);  // b = 2^(e - 1)
      fs.scale = 62 - fs.lgN - (e - 1);
      fs.sc = ldexp(1.0, fs.scale);
      fs.bound = b;
    }
    fs.known = true;
  }
  scatter_slot<T, SB, BANKS, NT, RANGED>(sl, modes, data, tables + s0 * W, W, nsb, log2m, acc, 8u * ma, signbit,
                                         tabs, s_max, fs, blockIdx.z, RANGED ? log2acc : -1,
                                         stage ? reinterpret_cast<uint32_t *>(acc) : nullptr,
                                         stage ? (uint32_t)(acc_bytes / 4) : 0u);
  if (bound_out != nullptr && tid == 0 && blockIdx.y == 0 && blockIdx.z == 0) bound_out[blockIdx.x] = fs.bound;
  const unsigned long long *neg = acc + signbit / 8;
  const int lga = RANGED ? log2acc : log2m;
  // (positive bank minus negative bank) 2^-scale, four buckets per thread and
  // 16-byte accesses when a sketch has at least four
  auto value = [&](int i) {
    const long long v = BANKS == 2 ? (long long)(acc[i] - neg[i]) : (long long)acc[i];
    return (A)ldexp((double)v, -fs.scale);
  };
  if (lga >= 2) {
    for (int i4 = tid; i4 < (nsb << (lga - 2)); i4 += NT) {
      const int i = 4 * i4, s = i >> lga, b = i & (int)amask;
      const A v0 = value(i), v1 = value(i + 1), v2 = value(i + 2), v3 = value(i + 3);
      A *dst = ybuf + ((s0 + s) * n_slots + blockIdx.x) * (int64_t)m + r0 + b;
      if constexpr (sizeof(A) == 4) {
        *reinterpret_cast<float4 *>(dst) = make_float4(v0, v1, v2, v3);
      } else {
        reinterpret_cast<double2 *>(dst)[0] = make_double2(v0, v1);
        reinterpret_cast<double2 *>(dst)[1] = make_double2(v2, v3);
      }
    }
  } else {
    for (int i = tid; i < (nsb << lga); i += NT)
      ybuf[((s0 + (i >> lga)) * n_slots + blockIdx.x) * (int64_t)m + r0 + (i & (int)amask)] = value(i);
  }
}

// NTH threads: 256, or 1024 for m >= 8192 (a block then fills most of a
// CU's LDS, and the per-thread share of the half spectrum stays small).
// The transform is held padded in LDS (pad32).  TWL: the half table of
// twiddles is staged beside it (padded too); otherwise (no room for it) the
// two-level table (Tw2) is.
// Network j's tensors are the entries [nets[j].t0, nets[j].t1) of the slot
// ranges: entry k's sketch is the sum of the slots [tbeg[k], tend[k]) (a
// plan's tensors in order: tbeg = first slot of each tensor, tend = tbeg + 1;
// a partial plan lists each entry's sub-tensors).
template <typename A, int LOG2M, bool TWL, int NTH = 256>
__global__ __launch_bounds__(NTH) void m1_combine_kernel(
    const NetDesc *__restrict__ nets, const int32_t *__restrict__ tbeg, const int32_t *__restrict__ tend,
    const A *__restrict__ ybuf, int64_t n_slots, int64_t sample0, int64_t S,
    const typename Cplx<A>::type *__restrict__ tw, double *__restrict__ est, double2 *__restrict__ part) {
  using A2 = typename Cplx<A>::type;
  constexpr int M = 1 << LOG2M;
  constexpr int H = M / 2 + 1;
  constexpr int NC = (H + NTH - 1) / NTH;
  // sketch points per thread and load round: all of a round's loads are in
  // flight together
  constexpr int G = M >= 8 * NTH ? 8 : (M >= NTH ? M / NTH : 1);
  extern __shared__ __align__(16) unsigned char smem[];
  A2 *z = reinterpret_cast<A2 *>(smem);
  __shared__ double red[NTH / 64];

  const NetDesc nd = nets[blockIdx.x];
  const int64_t s = blockIdx.y;
  const A *y = ybuf + s * n_slots * (int64_t)M;
  const int tid = threadIdx.x;
  // Tensors [kb, ke): the network's, or with part (gridDim.z blocks per
  // network and sample) share blockIdx.z of its pairs, pairs taken from t0 on
  // (an empty share leaves the product at 1).
  int kb = nd.t0, ke = nd.t1;
  if (part != nullptr) {
    const int np = (nd.t1 - nd.t0 + 1) / 2, per = (np + (int)gridDim.z - 1) / (int)gridDim.z;
    kb = min(nd.t1, nd.t0 + 2 * per * (int)blockIdx.z);
    ke = min(nd.t1, kb + 2 * per);
  }
  // Twiddles: staged in LDS after z (every butterfly pass reads them; from the
  // global table each pass would wait on a cache round trip).  The first
  // barrier below publishes them.
  A2 *t = z + pad32(M);
  if constexpr (TWL) {
    for (int j = tid; j < M / 2; j += NTH) t[pad32(j)] = tw[j];
  } else {
    static_assert(M >= 128, "two-level twiddles");
    for (int j = tid; j < M / 128 + 64; j += NTH) t[j] = tw[j < M / 128 ? 64 * j : j - M / 128];
  }

  double pr[NC], pi[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) { pr[c] = 1.0; pi[c] = 0.0; }

  // With one load round per pair (M <= NTH G), the first slot of each tensor
  // of the next pair is loaded before this pair's transform: the loads stay
  // in flight through the transform's LDS passes and barriers.
  constexpr bool ONE_ROUND = M <= NTH * G;
  A f1[G], f2[G];
  auto first_slots = [&](int k) {
    const bool pk = (k + 1) < ke;
    const int s1 = tbeg[k], s2 = pk ? tbeg[k + 1] : s1;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int b = g * NTH + tid;
      f1[g] = y[(int64_t)s1 * M + (b < M ? b : 0)];
      f2[g] = pk ? y[(int64_t)s2 * M + (b < M ? b : 0)] : (A)0;
    }
  };
  if constexpr (ONE_ROUND)
    if (kb < ke) first_slots(kb);

  for (int k = kb; k < ke; k += 2) {
    const bool pair = (k + 1) < ke;
    // slots [a0, a1) of the first tensor of the pair, [b0, b1) of the second
    const int a0 = tbeg[k], a1 = tend[k];
    const int b0 = pair ? tbeg[k + 1] : 0, b1 = pair ? tend[k + 1] : 0;
    if constexpr (ONE_ROUND) {
      A v1[G], v2[G];
#pragma unroll
      for (int g = 0; g < G; ++g) { v1[g] = f1[g]; v2[g] = f2[g]; }
      for (int sl = a0 + 1; sl < a1; ++sl) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int b = g * NTH + tid;
          v1[g] += y[(int64_t)sl * M + (b < M ? b : 0)];
        }
      }
      for (int sl = b0 + 1; sl < b1; ++sl) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int b = g * NTH + tid;
          v2[g] += y[(int64_t)sl * M + (b < M ? b : 0)];
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int b = g * NTH + tid;
        if (b < M) z[pad32(bitrev<LOG2M>(b))] = A2{v1[g], v2[g]};
      }
    }
    for (int p0 = 0; !ONE_ROUND && p0 < M; p0 += NTH * G) {
      A v1[G], v2[G];
#pragma unroll
      for (int g = 0; g < G; ++g) v1[g] = v2[g] = 0;
      // (b < M only fails when M < NTH: those threads read point 0 and store nothing)
      for (int sl = a0; sl < a1; ++sl) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int b = p0 + g * NTH + tid;
          v1[g] += y[(int64_t)sl * M + (b < M ? b : 0)];
        }
      }
      for (int sl = b0; sl < b1; ++sl) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int b = p0 + g * NTH + tid;
          v2[g] += y[(int64_t)sl * M + (b < M ? b : 0)];
        }
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int b = p0 + g * NTH + tid;
        if (b < M) z[pad32(bitrev<LOG2M>(b))] = A2{v1[g], v2[g]};
      }
    }
    __syncthreads();
    if constexpr (ONE_ROUND)
      if (k + 2 < ke) first_slots(k + 2);
    if constexpr (TWL)
      fft_lds<A, LOG2M, true, NTH>(z, t);
    else
      fft_lds_tw<A, LOG2M, true, NTH>(z, Tw2<A>{t, t + M / 128});
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = tid + NTH * c;
      if (j < H) {
        const A2 za = z[pad32(j)], zb = z[pad32((M - j) & (M - 1))];
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

  if (part != nullptr) {  // this share's product spectrum, for m1_combine_join_kernel
    double2 *o = part + (((int64_t)blockIdx.x * gridDim.y + s) * gridDim.z + blockIdx.z) * H;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = tid + NTH * c;
      if (j < H) o[j] = make_double2(pr[c], pi[c]);
    }
    return;
  }
  double sum = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int j = tid + NTH * c;
    if (j < H) sum += ((j == 0 || 2 * j == M) ? 1.0 : 2.0) * pr[c];
  }
  const double tot = block_sum<NTH>(sum, red);
  if (tid == 0) est[(int64_t)blockIdx.x * S + sample0 + s] = tot / (double)M;
}

// The split combine's join: per (network, sample) the product over its
// gsplit shares' spectra, in share order, then the Hermitian sum as in
// m1_combine_kernel.
__global__ __launch_bounds__(256) void m1_combine_join_kernel(const double2 *__restrict__ part, int gsplit,
                                                              int64_t m, int64_t sample0, int64_t S,
                                                              double *__restrict__ est) {
  __shared__ double red[4];
  const int64_t H = m / 2 + 1;
  const double2 *q = part + ((int64_t)blockIdx.x * gridDim.y + blockIdx.y) * gsplit * H;
  double sum = 0.0;
  for (int64_t j = threadIdx.x; j < H; j += 256) {
    double pr = 1.0, pi = 0.0;
    for (int g = 0; g < gsplit; ++g) {
      const double2 v = q[(int64_t)g * H + j];
      const double nr = pr * v.x - pi * v.y, ni = pr * v.y + pi * v.x;
      pr = nr;
      pi = ni;
    }
    sum += ((j == 0 || 2 * j == m) ? 1.0 : 2.0) * pr;
  }
  const double tot = block_sum<256>(sum, red);
  if (threadIdx.x == 0) est[(int64_t)blockIdx.x * S + sample0 + blockIdx.y] = tot / (double)m;
}

// ---------------------------------------------------------------------------
// Combine when the m-point FFT does not fit in LDS (m = 2^14 with FP64 data,
// m >= 2^15):
// the same estimate (1/m) Re sum_j prod_k Y_k[j], with the spectra taken in two
// passes through HBM.  As in the in-LDS combine, the tensors of a network go
// in pairs, z = y_a + i y_b (an odd one out with y_b = 0), and the pair's
// product spectrum is Y_a Y_b = (Z[j]^2 - conj(Z[-j])^2) / 4i.  With
// m = n1 n2 (n2 = 256), b = b1 + n1 b2 and j = j2 + n2 j1,
//   Z[j2 + n2 j1] = sum_b1 w_n1^(b1 j1) w_m^(b1 j2) sum_b2 z[b1 + n1 b2] w_n2^(b2 j2),
// w_n = exp(-2 pi i / n).
// Pass 1 (per pair, sample and run of columns b1): the n2-point DFTs over b2
// of the columns, all in one batched LDS transform, times w_m^(b1 j2), stored
// transposed as C[j2][b1].
// Pass 2 (per network, sample and mirror pair of rows): -(j2 + n2 j1) mod m is
// (n2 - j2) + n2 (n1 - 1 - j1) for j2 > 0, so row j2 holds the negated
// frequencies of row n2 - j2.  A block takes rows j2 and n2 - j2 (j2 in
// 1..127), or the self-mirrored rows 0 and 128, of every pair of the network,
// takes their n1-point DFTs in one batched LDS transform, and sums
// prod_pairs (Y_a Y_b)[j] over its frequencies in FP64: 2 Re over row j2 (row
// n2 - j2 holds the conjugates), Re over both self-mirrored rows.  Every
// frequency is visited once and the blocks' sums are added in a fixed order,
// so the result matches the in-LDS combine up to FFT rounding.
constexpr int kBigN2 = 256, kBigRowPairs = kBigN2 / 2;
static_assert(kBigRowPairs == kBigPartials, "one partial sum per row block");
// LDS stride between the transforms of a batch: pad32(256) and one more
// element, so that reading the same point of consecutive transforms (the
// transposed store) falls into distinct banks.
constexpr int kBigStr = kBigN2 + kBigN2 / 32 + 1;

// w_m^e from the half table tw[j] = w_m^j, j < m/2.
template <typename A2>
__device__ __forceinline__ A2 twiddle_at(const A2 *__restrict__ tw, uint32_t e, uint32_t m) {
  e &= m - 1;
  if (e < m / 2) return tw[e];
  const A2 t = tw[e - m / 2];
  return A2{-t.x, -t.y};
}

// Columns per pass-1 block: one 128-byte line of each input row per block
// for FP32 sketches, 256 bytes for FP64 (the transforms then fill 68 KB of LDS).
template <typename A>
constexpr int big_cols() { return sizeof(A) == 4 ? 32 : 16; }
// LDS: the batch of transforms, the padded 256-point half table, and the
// two-level table of the transposed store's twiddles w_m^e = hi[e / 256]
// lo[e % 256] (m / 256 <= 256 and 256 entries).
template <typename A>
constexpr size_t big_cols_lds() {
  return sizeof(typename Cplx<A>::type) * (size_t)(big_cols<A>() * kBigStr + kBigN2 / 2 + kBigN2 / 64 + 2 * kBigN2);
}

template <typename A>
__global__ __launch_bounds__(256) void m1_big_cols_kernel(const int32_t *__restrict__ tslot,
                                                          const int32_t *__restrict__ pairs, int64_t n_pairs,
                                                          const A *__restrict__ ybuf, int64_t n_slots, int log2m,
                                                          const typename Cplx<A>::type *__restrict__ tw,
                                                          typename Cplx<A>::type *__restrict__ cbuf) {
  using A2 = typename Cplx<A>::type;
  constexpr int CB = big_cols<A>();    // columns b1 of this block
  constexpr int RS = 256 / CB;         // b2 = r0 + RS i: the thread's points of its column
  constexpr int RPT = kBigN2 / RS;     // points per thread
  constexpr int G = 8;                 // loads in flight per tensor and round
  static_assert(RPT % G == 0, "load rounds");
  extern __shared__ __align__(16) unsigned char smem[];
  A2 *z = reinterpret_cast<A2 *>(smem);
  A2 *tw2 = z + CB * kBigStr;
  A2 *thi = tw2 + kBigN2 / 2 + kBigN2 / 64, *tlo = thi + kBigN2;
  const uint32_t m = 1u << log2m, n1 = m / kBigN2;
  const int64_t pr = blockIdx.x, s = blockIdx.y;
  const uint32_t b1_0 = blockIdx.z * CB;
  const int tid = threadIdx.x, c = tid % CB, r0 = tid / CB;
  if (tid < kBigN2 / 2) tw2[pad32(tid)] = tw[(uint32_t)tid * n1];  // w_n2^t = w_m^(t n1)
  if ((uint32_t)tid < n1) thi[tid] = twiddle_at(tw, (uint32_t)tid * kBigN2, m);  // (published by the
  tlo[tid] = twiddle_at(tw, (uint32_t)tid, m);                                  //  barrier below)
  const int ta = pairs[2 * pr], tb = pairs[2 * pr + 1];
  const int a0 = tslot[ta], a1 = tslot[ta + 1];
  const int bb0 = tb >= 0 ? tslot[tb] : 0, bb1 = tb >= 0 ? tslot[tb + 1] : 0;
  const A *y = ybuf + s * n_slots * (int64_t)m + b1_0 + c;
  // z[b1 + n1 b2] = y_a + i y_b (each summed over its tensor's slots), stored
  // bit-reversed for the transform of column c
  for (int i0 = 0; i0 < RPT; i0 += G) {
    A va[G], vb[G];
#pragma unroll
    for (int g = 0; g < G; ++g) va[g] = vb[g] = 0;
    for (int sl = a0; sl < a1; ++sl) {
#pragma unroll
      for (int g = 0; g < G; ++g) va[g] += y[(int64_t)sl * m + (int64_t)n1 * (r0 + RS * (i0 + g))];
    }
    for (int sl = bb0; sl < bb1; ++sl) {
#pragma unroll
      for (int g = 0; g < G; ++g) vb[g] += y[(int64_t)sl * m + (int64_t)n1 * (r0 + RS * (i0 + g))];
    }
#pragma unroll
    for (int g = 0; g < G; ++g) z[c * kBigStr + pad32(bitrev<8>(r0 + RS * (i0 + g)))] = A2{va[g], vb[g]};
  }
  __syncthreads();
  fft_lds_batch<A, 8, kBigStr, 256>(z, tw2, CB);  // ends with a barrier
  // C[j2][b1] = Z_b1[j2] w_m^(b1 j2): lanes of consecutive b1 write one
  // contiguous run per j2
  A2 *out = cbuf + (s * n_pairs + pr) * (int64_t)m + b1_0 + c;
  const uint32_t b1 = b1_0 + c;
#pragma unroll 4
  for (int i = 0; i < RPT; ++i) {
    const int j2 = r0 + RS * i;
    const uint32_t e = (b1 * (uint32_t)j2) & (m - 1);
    const A2 v = z[c * kBigStr + pad32(j2)], wh = thi[e / kBigN2], wl = tlo[e % kBigN2];
    const A2 w = A2{wh.x * wl.x - wh.y * wl.y, wh.x * wl.y + wh.y * wl.x};
    out[(int64_t)j2 * n1] = A2{v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x};
  }
}

// Pairs per pass-2 round: 2 rows each, KP * 2 transforms in LDS (34 KB).
template <typename A>
constexpr int big_rows_pairs() { return sizeof(A) == 4 ? 8 : 4; }

template <typename A, int LOG2N1>
__global__ __launch_bounds__(256) void m1_big_rows_kernel(const int32_t *__restrict__ pair0,
                                                          const int32_t *__restrict__ pairs, int64_t n_pairs,
                                                          const typename Cplx<A>::type *__restrict__ cbuf,
                                                          const typename Cplx<A>::type *__restrict__ tw,
                                                          double *__restrict__ partial) {
  using A2 = typename Cplx<A>::type;
  constexpr int N1 = 1 << LOG2N1;
  constexpr uint32_t M = (uint32_t)N1 * kBigN2;
  constexpr int KP = big_rows_pairs<A>();
  constexpr int STR = N1 + N1 / 32 + 1;
  constexpr int NL = 2 * KP * N1 / 256;  // loads per thread and round
  static_assert(NL >= 1 && (2 * KP * N1) % 256 == 0, "load rounds");
  __shared__ A2 z[2 * KP * STR];
  __shared__ A2 tw1[N1 / 2 + N1 / 64];
  __shared__ double red[4];
  const int net = blockIdx.x;
  const int64_t s = blockIdx.y;
  const int rp = blockIdx.z, tid = threadIdx.x;
  const int rowA = rp == 0 ? 0 : rp, rowB = rp == 0 ? kBigN2 / 2 : kBigN2 - rp;
  if (tid < N1 / 2) tw1[pad32(tid)] = tw[(uint32_t)tid * kBigN2];  // w_n1^t = w_m^(t n2)
  const int p0 = pair0[net], p1 = pair0[net + 1];
  double pr1 = 1.0, pi1 = 0.0, pr2 = 1.0, pi2 = 0.0;  // rows A and (rp = 0) B
  // pair product at frequency (row t, point j1), mirror at (row u, point j1m)
  auto pair_q = [&](int t, int j1, int u, int j1m, bool pair, double &qr, double &qi) {
    const A2 za = z[t * STR + pad32(j1)], zb = z[u * STR + pad32(j1m)];
    const double ar = za.x, ai = za.y, br = zb.x, bi = -(double)zb.y;  // B = conj(Z[-j])
    if (pair) {
      const double dr = (ar * ar - ai * ai) - (br * br - bi * bi);
      const double di = 2.0 * (ar * ai - br * bi);
      qr = 0.25 * di;  // -i (A^2 - B^2) / 4
      qi = -0.25 * dr;
    } else {
      qr = 0.5 * (ar + br);  // (A + B) / 2
      qi = 0.5 * (ai + bi);
    }
  };
  for (int q0 = p0; q0 < p1; q0 += KP) {
    const int nk = min(KP, p1 - q0);
    __syncthreads();  // the previous round's readers are done (and tw1 is written)
    A2 v[NL];
#pragma unroll
    for (int g = 0; g < NL; ++g) {
      const int i = min(tid + 256 * g, 2 * nk * N1 - 1);
      const int t = i / N1, e = i % N1;  // transform t: pair q0 + t/2, row A or B
      v[g] = cbuf[(s * n_pairs + q0 + t / 2) * (int64_t)M + (int64_t)((t & 1) ? rowB : rowA) * N1 + e];
    }
#pragma unroll
    for (int g = 0; g < NL; ++g) {
      const int i = tid + 256 * g;
      if (i < 2 * nk * N1) z[(i / N1) * STR + pad32(bitrev<LOG2N1>(i % N1))] = v[g];
    }
    __syncthreads();
    fft_lds_batch<A, LOG2N1, STR, 256>(z, tw1, 2 * nk);  // ends with a barrier
    if (tid < N1) {
      for (int k = 0; k < nk; ++k) {
        const bool pair = pairs[2 * (q0 + k) + 1] >= 0;
        double qr, qi, nr;
        if (rp == 0) {
          pair_q(2 * k, tid, 2 * k, (N1 - tid) & (N1 - 1), pair, qr, qi);  // row 0
          nr = pr1 * qr - pi1 * qi;
          pi1 = pr1 * qi + pi1 * qr;
          pr1 = nr;
          pair_q(2 * k + 1, tid, 2 * k + 1, N1 - 1 - tid, pair, qr, qi);  // row n2 / 2
          nr = pr2 * qr - pi2 * qi;
          pi2 = pr2 * qi + pi2 * qr;
          pr2 = nr;
        } else {
          pair_q(2 * k, tid, 2 * k + 1, N1 - 1 - tid, pair, qr, qi);  // row j2, mirror in row n2 - j2
          nr = pr1 * qr - pi1 * qi;
          pi1 = pr1 * qi + pi1 * qr;
          pr1 = nr;
        }
      }
    }
  }
  const double part = tid < N1 ? (rp == 0 ? pr1 + pr2 : 2.0 * pr1) : 0.0;
  const double tot = block_sum_256(part, red);
  if (tid == 0) partial[((int64_t)net * gridDim.y + s) * kBigRowPairs + rp] = tot;
}

__global__ __launch_bounds__(256) void m1_big_sum_kernel(const double *__restrict__ partial, int64_t n_nets,
                                                         int64_t samples, int parts, int64_t sample0, int64_t S,
                                                         double inv_m, double *__restrict__ est) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;  // (network, sample)
  if (i >= n_nets * samples) return;
  const int64_t net = i / samples, s = i - net * samples;
  double v = 0.0;
  for (int q = 0; q < parts; ++q) v += partial[i * parts + q];
  est[net * S + sample0 + s] = v * inv_m;
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

constexpr size_t kWideLds = 81920;

template <typename T, typename A, int SB>
int scatter_sb(const M1Launch &L, hipStream_t st) {
  const bool ranged = L.log2m > kMaxLog2Acc;
  if (ranged && (SB != 1 || L.banks != 1))
    return set_error(TN_ERR_ARG, "scatter: m = 2^%d takes one bank and one sample per pass", L.log2m);
  if constexpr (SB * (16 / (int)sizeof(T)) > kMaxScatterWords) {
    return set_error(TN_ERR_UNSUPPORTED, "scatter: %d samples per pass of %d-byte data", SB, (int)sizeof(T));
  } else {
    // One block per CU when its LDS exceeds half a CU's: then 1024 threads, or
    // 512 where a thread's SB x (entries per 16-byte load) table words would
    // not fit the 128 registers of a 1024-thread block.
    constexpr int kWideNT = SB * (16 / (int)sizeof(T)) <= 16 ? 1024 : 512;
    const bool wide = ranged || L.lds_bytes > kWideLds;
    auto kern = wide ? (L.banks == 2 ? m1_scatter_kernel<T, A, SB, 2, false, kWideNT>
                                     : m1_scatter_kernel<T, A, SB, 1, false, kWideNT>)
                     : (L.banks == 2 ? m1_scatter_kernel<T, A, SB, 2> : m1_scatter_kernel<T, A, SB, 1>);
    if constexpr (SB == 1)
      if (ranged) kern = m1_scatter_kernel<T, A, 1, 1, true, 1024>;
    if (L.lds_bytes > 65536)
      TN_HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)L.lds_bytes));
    // Slot bounds: without a bound array every block keeps a running
    // maximum.  Else the first sample batch keeps one and records each slot's
    // bound (when this launch is the first to see the data), and the other
    // batches, in a second launch on the same stream, start from it.
    const unsigned batches = (unsigned)((L.samples + SB - 1) / SB);
    const unsigned z = ranged ? 1u << (L.log2m - kMaxLog2Acc) : 1u;
    const dim3 block(ranged ? 1024 : wide ? kWideNT : 256 * L.banks);
    A *y = reinterpret_cast<A *>(L.ybuf);
    if (L.slot_bound == nullptr) {
      hipLaunchKernelGGL(kern, dim3((unsigned)L.n_slots, batches, z), block, L.lds_bytes, st, L.slots, L.modes,
                         L.data, L.tables, L.W, L.samples, L.log2m, kMaxLog2Acc, L.n_slots, y, nullptr, nullptr, 0);
      TN_HIP_CHECK(hipGetLastError());
      return TN_OK;
    }
    int y0 = 0;
    if (L.record_bound) {
      hipLaunchKernelGGL(kern, dim3((unsigned)L.n_slots, 1u, z), block, L.lds_bytes, st, L.slots, L.modes, L.data,
                         L.tables, L.W, L.samples, L.log2m, kMaxLog2Acc, L.n_slots, y, nullptr, L.slot_bound, 0);
      TN_HIP_CHECK(hipGetLastError());
      y0 = 1;
    }
    if (batches > (unsigned)y0) {
      hipLaunchKernelGGL(kern, dim3((unsigned)L.n_slots, batches - (unsigned)y0, z), block, L.lds_bytes, st,
                         L.slots, L.modes, L.data, L.tables, L.W, L.samples, L.log2m, kMaxLog2Acc, L.n_slots, y,
                         L.slot_bound, nullptr, y0);
      TN_HIP_CHECK(hipGetLastError());
    }
    return TN_OK;
  }
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
int combine_m(const NetDesc *nets, int64_t n_nets, const int32_t *tbeg, const int32_t *tend, const void *ybuf,
              int64_t n_slots, int64_t samples, int64_t sample0, int64_t S, const void *tw,
              double *est, int32_t csplit, double *cpart, hipStream_t st) {
  using A2 = typename Cplx<A>::type;
  // z (m points, one spare element per 32: bank spread) and, when the total
  // stays within 64 KB, the m/2 twiddles (padded), else the two-level table
  constexpr int M = 1 << LOG2M;
  constexpr size_t zt = sizeof(A2) * (size_t)(M + M / 32 + M / 2 + M / 64 + 2);
  constexpr bool TWL = zt <= 65536 || M < 128;
  constexpr size_t lds = TWL ? zt : sizeof(A2) * (size_t)(M + M / 32 + M / 128 + 64);
  if constexpr (lds > kMaxLdsBytes) {
    return set_error(TN_ERR_UNSUPPORTED, "combine: the %d-point transform does not fit in LDS", M);
  } else {
    constexpr int NTH = LOG2M >= 13 ? 1024 : 256;
    auto kern = m1_combine_kernel<A, LOG2M, TWL, NTH>;
    if (lds > 65536)
      TN_HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds));
    const bool split = csplit > 1 && cpart != nullptr;
    dim3 grid((unsigned)n_nets, (unsigned)samples, split ? (unsigned)csplit : 1u);
    double2 *part = split ? reinterpret_cast<double2 *>(cpart) : nullptr;
    hipLaunchKernelGGL(kern, grid, dim3(NTH), lds, st, nets, tbeg, tend,
                       reinterpret_cast<const A *>(ybuf), n_slots, sample0, S,
                       reinterpret_cast<const A2 *>(tw), est, part);
    TN_HIP_CHECK(hipGetLastError());
    if (split) {
      hipLaunchKernelGGL(m1_combine_join_kernel, dim3((unsigned)n_nets, (unsigned)samples), dim3(256), 0, st,
                         part, (int)csplit, (int64_t)M, sample0, S, est);
      TN_HIP_CHECK(hipGetLastError());
    }
    return TN_OK;
  }
}

template <typename A>
int combine_big(int64_t n_nets, const int32_t *tslot, const int32_t *pairs, const int32_t *pair0,
                int64_t n_pairs, const void *ybuf, int64_t n_slots, int64_t samples, int64_t sample0, int64_t S,
                int log2m, const void *tw, void *cbuf, double *partial, double *est, hipStream_t st) {
  using A2 = typename Cplx<A>::type;
  const uint32_t m = 1u << log2m, n1 = m / kBigN2;
  constexpr size_t lds = big_cols_lds<A>();
  TN_HIP_CHECK(hipFuncSetAttribute((const void *)m1_big_cols_kernel<A>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(m1_big_cols_kernel<A>, dim3((unsigned)n_pairs, (unsigned)samples, n1 / big_cols<A>()),
                     dim3(256), lds, st, tslot, pairs, n_pairs, reinterpret_cast<const A *>(ybuf), n_slots, log2m,
                     reinterpret_cast<const A2 *>(tw), reinterpret_cast<A2 *>(cbuf));
  TN_HIP_CHECK(hipGetLastError());
  dim3 g2((unsigned)n_nets, (unsigned)samples, kBigRowPairs);
  const A2 *cb = reinterpret_cast<const A2 *>(cbuf), *t2 = reinterpret_cast<const A2 *>(tw);
  if (log2m == 14)
    hipLaunchKernelGGL((m1_big_rows_kernel<A, 6>), g2, dim3(256), 0, st, pair0, pairs, n_pairs, cb, t2, partial);
  else if (log2m == 15)
    hipLaunchKernelGGL((m1_big_rows_kernel<A, 7>), g2, dim3(256), 0, st, pair0, pairs, n_pairs, cb, t2, partial);
  else
    hipLaunchKernelGGL((m1_big_rows_kernel<A, 8>), g2, dim3(256), 0, st, pair0, pairs, n_pairs, cb, t2, partial);
  TN_HIP_CHECK(hipGetLastError());
  const int64_t np = n_nets * samples;
  hipLaunchKernelGGL(m1_big_sum_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, partial, n_nets,
                     samples, kBigRowPairs, sample0, S, 1.0 / (double)m, est);
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

template <typename A>
int combine_t(const NetDesc *nets, int64_t n_nets, const int32_t *tbeg, const int32_t *tend, const void *ybuf,
              int64_t n_slots, int64_t samples, int64_t sample0, int64_t S, int log2m,
              const void *tw, double *est, int32_t csplit, double *cpart, hipStream_t st) {
#define TN_COMBINE_CASE(LG)                                                                            \
  case LG:                                                                                             \
    return combine_m<A, LG>(nets, n_nets, tbeg, tend, ybuf, n_slots, samples, sample0, S, tw, est, csplit, \
                            cpart, st);
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

int launch_m1_combine(const NetDesc *nets, int64_t n_nets, const int32_t *tbeg, const int32_t *tend, int dtype,
                      const void *ybuf, int64_t n_slots, int64_t samples, int64_t sample0,
                      int64_t S, int log2m, const void *tw, double *est, int32_t csplit, double *cpart,
                      hipStream_t st) {
  if (n_nets == 0 || samples == 0) return TN_OK;
  if (samples > 65535) return set_error(TN_ERR_UNSUPPORTED, "combine: samples per launch");
  if (dtype == TN_F64)
    return combine_t<double>(nets, n_nets, tbeg, tend, ybuf, n_slots, samples, sample0, S, log2m, tw, est, csplit,
                             cpart, st);
  return combine_t<float>(nets, n_nets, tbeg, tend, ybuf, n_slots, samples, sample0, S, log2m, tw, est, csplit,
                          cpart, st);
}

int launch_m1_combine_big(int64_t n_nets, const int32_t *tslot, const int32_t *pairs, const int32_t *pair0,
                          int64_t n_pairs, int dtype, const void *ybuf, int64_t n_slots, int64_t samples,
                          int64_t sample0, int64_t S, int log2m, const void *tw, void *cbuf, double *partial,
                          double *est, hipStream_t st) {
  if (n_nets == 0 || samples == 0) return TN_OK;
  if (samples > 65535) return set_error(TN_ERR_UNSUPPORTED, "combine: samples per launch");
  if (log2m < kMaxLog2Acc || log2m > kMaxLog2M1)
    return set_error(TN_ERR_ARG, "two-pass combine: m = 2^%d", log2m);
  if (n_pairs > 0x7fffffff) return set_error(TN_ERR_UNSUPPORTED, "two-pass combine: %lld tensor pairs",
                                             (long long)n_pairs);
  if (dtype == TN_F64)
    return combine_big<double>(n_nets, tslot, pairs, pair0, n_pairs, ybuf, n_slots, samples, sample0, S, log2m,
                               tw, cbuf, partial, est, st);
  return combine_big<float>(n_nets, tslot, pairs, pair0, n_pairs, ybuf, n_slots, samples, sample0, S, log2m, tw,
                            cbuf, partial, est, st);
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
