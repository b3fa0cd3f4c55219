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
#include "tn_internal.h"

#include <hip/hip_bf16.h>

namespace tn {
namespace {

template <typename T>
__device__ __forceinline__ float to_acc(T v);
template <>
__device__ __forceinline__ float to_acc<float>(float v) { return v; }
template <>
__device__ __forceinline__ float to_acc<uint16_t>(uint16_t v) {
  return __uint_as_float(((uint32_t)v) << 16);
}

__device__ __forceinline__ double to_acc_any(double v) { return v; }
__device__ __forceinline__ float to_acc_any(float v) { return v; }
__device__ __forceinline__ float to_acc_any(uint16_t v) { return to_acc<uint16_t>(v); }

// 16-byte vector of tensor entries (clang vector types, so they can be read
// through a global-address-space pointer: global_load_dwordx4, not flat).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = f32x4;
};
template <>
struct Vec16<double> {
  using type = f64x2;
};
template <>
struct Vec16<uint16_t> {
  using type = u16x8;
};

// N consecutive packed column hashes from LDS (16-byte aligned for N >= 4,
// 8-byte aligned for N = 2).
template <int N>
__device__ __forceinline__ void load_cols(const uint32_t *p, uint32_t *out);
template <>
__device__ __forceinline__ void load_cols<2>(const uint32_t *p, uint32_t *out) {
  const uint2 t = *reinterpret_cast<const uint2 *>(p);
  out[0] = t.x; out[1] = t.y;
}
template <>
__device__ __forceinline__ void load_cols<4>(const uint32_t *p, uint32_t *out) {
  const uint4 t = *reinterpret_cast<const uint4 *>(p);
  out[0] = t.x; out[1] = t.y; out[2] = t.z; out[3] = t.w;
}
template <>
__device__ __forceinline__ void load_cols<8>(const uint32_t *p, uint32_t *out) {
  load_cols<4>(p, out);
  load_cols<4>(p + 4, out + 4);
}

// Packed bucket/sign of a contiguous run of modes for one index: the sum of
// the modes' buckets mod m and the product of their signs.
__device__ __forceinline__ uint32_t combine_modes(const int32_t *__restrict__ tab,
                                                  const ModeDesc *__restrict__ modes,
                                                  int u_first, int u_last, uint32_t idx,
                                                  uint32_t m, uint32_t mask) {
  uint32_t acc = 0;
  for (int u = u_last; u >= u_first; --u) {
    const ModeDesc md = modes[u];
    const uint32_t d = idx % (uint32_t)md.n;
    idx /= (uint32_t)md.n;
    const uint32_t v = (uint32_t)tab[md.table_off + d];
    uint32_t h = v & ~kSignBit;
    if (md.comp) h = (m - h) & mask;
    acc = (((acc & ~kSignBit) + h) & mask) | ((acc ^ v) & kSignBit);
  }
  return acc;
}

// The sketches of one block are accumulated in 64-bit fixed point in LDS:
// x -> round(x 2^scale) with ds_add_u64, which on gfx950 sustains about 16x the
// rate of LDS float atomics, and makes every sketch independent of the order
// of the atomic adds.  The block scale follows a running maximum of |x|:
// scale = 62 - ceil(log2 N) - e with max|x| < 2^e, so N terms of the slot
// cannot overflow; when a larger |x| appears the accumulators are shifted
// right to the new scale before any further add.
template <typename T, typename A, int SB>
__global__ __launch_bounds__(256) void m1_scatter_kernel(
    const ScatterSlot *__restrict__ slots, const ModeDesc *__restrict__ modes,
    const void *const *__restrict__ data, const int32_t *__restrict__ tables, int64_t W,
    int64_t samples, int log2m, int64_t n_slots, A *__restrict__ ybuf) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ unsigned long long s_max[2];
  const ScatterSlot sl = slots[blockIdx.x];
  const int tid = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.y * SB;
  const int nsb = (int)min((int64_t)SB, samples - s0);
  const uint32_t m = 1u << log2m, mask = m - 1;
  const int L = sl.L, rows = sl.rows;

  unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem);  // [SB][m]
  uint32_t *colt = reinterpret_cast<uint32_t *>(smem + ((SB * m * 8 + 15) & ~15u));  // [SB][L]
  uint32_t *rowt = colt + SB * L;                                         // [SB][rows]

  for (int i = tid; i < SB * (int)m; i += 256) acc[i] = 0ull;
  if (tid < 2) s_max[tid] = 0ull;
  // Packed tables hold the byte offset of the bucket (bucket * 8) and the sign
  // bit, so a sum of a row and a column entry masked with 8(m - 1) is the LDS
  // offset of the target accumulator.
  auto to_offset = [](uint32_t v) { return ((v & ~kSignBit) << 3) | (v & kSignBit); };
  for (int i = tid; i < nsb * L; i += 256) {
    const int s = i / L, c = i - s * L;
    colt[s * L + c] = to_offset(combine_modes(tables + (s0 + s) * W, modes, sl.mode0 + sl.split,
                                              sl.mode0 + sl.q - 1, c, m, mask));
  }
  for (int i = tid; i < nsb * rows; i += 256) {
    const int s = i / rows, r = i - s * rows;
    rowt[s * rows + r] = to_offset(combine_modes(tables + (s0 + s) * W, modes, sl.mode0,
                                                 sl.mode0 + sl.split - 1,
                                                 (uint32_t)(sl.row0 + r), m, mask));
  }
  __syncthreads();
  const uint32_t mask8 = mask << 3;
  char *acc8 = reinterpret_cast<char *>(smem);

  const T *X = reinterpret_cast<const T *>(data[sl.tensor]) + sl.row0 * (int64_t)L;
  const uint32_t N = (uint32_t)rows * (uint32_t)L;
  // Headroom: N terms below 2^(62 - lgN) each cannot overflow, and every
  // scaled term stays below 2^51 so the magic-number conversion is exact.
  const int lgN = max(N > 1 ? 32 - __clz(N - 1) : 0, 11);
  int scale = 0;       // accumulators hold x 2^scale
  double sc = 1.0;     // 2^scale
  double bound = 0.0;  // every |x| seen is < bound (0: none seen yet)
  int par = 0;

  // Block-wide running max of |x| (double-buffered so the read of one
  // iteration cannot race with the next iteration's update), then a rescale
  // when it reaches the bound.  Called by every thread once per iteration.
  auto update_scale = [&](double lmax) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, off, 64));
    if ((tid & 63) == 0) atomicMax(&s_max[par], (unsigned long long)__double_as_longlong(lmax));
    __syncthreads();
    const double bm = __longlong_as_double((long long)s_max[par]);
    par ^= 1;
    if (bm >= bound && bm > 0.0) {
      int e;
      (void)frexp(bm, &e);  // bm < 2^e
      const int ns = 62 - lgN - e;
      if (bound > 0.0 && scale > ns) {
        const int d = scale - ns;
        for (int i = tid; i < SB * (int)m; i += 256)
          acc[i] = (unsigned long long)((long long)acc[i] >> d);
        __syncthreads();
      }
      scale = ns;
      sc = ldexp(1.0, ns);
      bound = ldexp(1.0, e);
    }
  };
  // round(x 2^scale) for |x 2^scale| < 2^51: adding 1.5 2^52 leaves the
  // rounded integer in the low mantissa bits.
  auto to_fixed = [&](double x) -> long long {
    const double kMagic = 6755399441055744.0;
    return __double_as_longlong(fma(x, sc, kMagic)) - __double_as_longlong(kMagic);
  };
  // One fixed-point add: the sample's accumulator block starts at s * 8m bytes
  // and the masked offset sum stays inside it.
  auto add_fixed = [&](int s, uint32_t hv, uint32_t lv, long long v) {
    const uint32_t a = ((hv + lv) & mask8) | ((uint32_t)s * (m << 3));
    atomicAdd(reinterpret_cast<unsigned long long *>(acc8 + a),
              (unsigned long long)(((hv ^ lv) & kSignBit) ? -v : v));
  };
  // Add entry x (row r, column c) to the sketch of every sample of the batch.
  auto scatter_one = [&](double x, uint32_t r, uint32_t c) {
    const long long v = to_fixed(x);
    uint32_t hv[SB], lv[SB];
#pragma unroll
    for (int s = 0; s < SB; ++s) { hv[s] = rowt[s * rows + r]; lv[s] = colt[s * L + c]; }
#pragma unroll
    for (int s = 0; s < SB; ++s)
      if (s < nsb) add_fixed(s, hv[s], lv[s], v);
  };
  constexpr int VEC = 16 / (int)sizeof(T);   // entries per 16-byte load
  // Row and column entries of every sample for VEC consecutive entries of one
  // row (all reads issued before any add, so one LDS wait covers them).
  auto read_tabs = [&](uint32_t r, uint32_t c, uint32_t *hv, uint32_t (*lv)[VEC]) {
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      hv[s] = rowt[s * rows + r];
      load_cols<VEC>(colt + s * L + c, lv[s]);
    }
  };
  constexpr int UNROLL = 4;                  // 16-byte loads in flight per thread
  const bool vec = (L % VEC == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  if (vec) {
    // Rows are multiples of VEC long and the slot starts 16-byte aligned, so
    // the VEC entries of one load share a row.
    using V = typename Vec16<T>::type;
    const V __attribute__((address_space(1))) *Xv =
        (const V __attribute__((address_space(1))) *)reinterpret_cast<const V *>(X);
    const uint32_t NV = N / VEC;
    for (uint32_t v0 = 0; v0 < NV; v0 += 256 * UNROLL) {
      // Unconditional loads (index clamped into the slot) keep all UNROLL loads
      // in flight; out-of-range lanes are masked when the values are used.
      V buf[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) buf[u] = Xv[min(v0 + u * 256 + tid, NV - 1)];
      double lmax = 0.0;
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const T *xs = reinterpret_cast<const T *>(&buf[u]);
#pragma unroll
        for (int i = 0; i < VEC; ++i) lmax = fmax(lmax, fabs((double)to_acc_any(xs[i])));
      }
      update_scale(lmax);
      uint32_t rr[UNROLL], cc[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const uint32_t e = min(v0 + u * 256 + tid, NV - 1) * VEC;  // clamped: valid table reads
        rr[u] = (L == 1) ? e : __umulhi(e, sl.magic);
        cc[u] = e - rr[u] * (uint32_t)L;
      }
      // Software pipeline: the table reads of vector u + 1 are issued before the
      // adds of vector u.
      uint32_t hv[2][SB], lv[2][SB][VEC];
      read_tabs(rr[0], cc[0], hv[0], lv[0]);
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        if (u + 1 < UNROLL) read_tabs(rr[u + 1], cc[u + 1], hv[(u + 1) & 1], lv[(u + 1) & 1]);
        if (v0 + u * 256 + tid < NV) {
          const T *xs = reinterpret_cast<const T *>(&buf[u]);
          long long q[VEC];
#pragma unroll
          for (int i = 0; i < VEC; ++i) q[i] = to_fixed((double)to_acc_any(xs[i]));
#pragma unroll
          for (int s = 0; s < SB; ++s)
            if (s < nsb) {
#pragma unroll
              for (int i = 0; i < VEC; ++i) add_fixed(s, hv[u & 1][s], lv[u & 1][s][i], q[i]);
            }
        }
      }
    }
  } else {
    const T __attribute__((address_space(1))) *Xg =
        (const T __attribute__((address_space(1))) *)X;
    for (uint32_t e0 = 0; e0 < N; e0 += 256 * UNROLL) {
      T buf[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) buf[u] = Xg[min(e0 + u * 256 + tid, N - 1)];
      double lmax = 0.0;
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) lmax = fmax(lmax, fabs((double)to_acc_any(buf[u])));
      update_scale(lmax);
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const uint32_t e = e0 + u * 256 + tid;
        if (e < N) {
          const uint32_t r = (L == 1) ? e : __umulhi(e, sl.magic);
          scatter_one((double)to_acc_any(buf[u]), r, e - r * (uint32_t)L);
        }
      }
    }
  }
  __syncthreads();

  for (int i = tid; i < nsb * (int)m; i += 256) {
    const int s = i >> log2m;
    const int b = i & mask;
    ybuf[((s0 + s) * n_slots + blockIdx.x) * (int64_t)m + b] =
        (A)ldexp((double)(long long)acc[i], -scale);
  }
}

template <typename A>
struct Cplx;
template <>
struct Cplx<float> {
  using type = float2;
};
template <>
struct Cplx<double> {
  using type = double2;
};

// In-place radix-2 decimation-in-time FFT of M points held in LDS in
// bit-reversed order; natural-order output.  F[j][b] = exp(-2 pi i j b / M).
template <typename A, int LOG2M>
__device__ __forceinline__ void fft_lds(typename Cplx<A>::type *z,
                                        const typename Cplx<A>::type *__restrict__ tw) {
  constexpr int M = 1 << LOG2M;
  using A2 = typename Cplx<A>::type;
#pragma unroll 1
  for (int lg = 1; lg <= LOG2M; ++lg) {
    const int half = 1 << (lg - 1);
    for (int q = threadIdx.x; q < M / 2; q += 256) {
      const int k = q & (half - 1);
      const int a = ((q >> (lg - 1)) << lg) + k;
      const int b = a + half;
      const A2 w = tw[k << (LOG2M - lg)];
      const A2 za = z[a], zb = z[b];
      const A tr = w.x * zb.x - w.y * zb.y;
      const A ti = w.x * zb.y + w.y * zb.x;
      z[a] = A2{za.x + tr, za.y + ti};
      z[b] = A2{za.x - tr, za.y - ti};
    }
    __syncthreads();
  }
}

template <int LOG2M>
__device__ __forceinline__ int bitrev(int b) {
  if constexpr (LOG2M == 0) {
    return 0;
  } else {
    return (int)(__brev((unsigned)b) >> (32 - LOG2M));
  }
}

__device__ __forceinline__ double block_sum_256(double v, double *red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return t;
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
  auto kern = m1_scatter_kernel<T, A, SB>;
  if (L.lds_bytes > 65536)
    TN_HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)L.lds_bytes));
  dim3 grid((unsigned)L.n_slots, (unsigned)((L.samples + SB - 1) / SB));
  hipLaunchKernelGGL(kern, grid, dim3(256), L.lds_bytes, st, L.slots, L.modes, L.data, L.tables,
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
