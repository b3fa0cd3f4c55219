// Persistent, fused form of the cyclic estimator (Eq. (1)) for batches of
// uneven networks.
//
// Work item = (network, batch of up to SB samples).  Items are sorted by
// decreasing work on the host and handed out through one device counter: each
// block of a grid sized to the machine takes the next item until the queue is
// empty (every block reaches that exit).  For its item a block walks the
// network's tensors two at a time:
//   1. both tensors' slots are scattered into 64-bit fixed-point sketches in
//      LDS (the same scatter as the slot kernel, one scale per tensor);
//   2. per sample, the two real sketches share one complex FFT in LDS
//      (z = y_a + i y_b), and the pair's product spectrum
//      Y_a Y_b = (Z[j]^2 - conj(Z[-j])^2) / 4i is multiplied into per-thread
//      FP64 accumulators over the half spectrum;
// and finally writes (1/m)(P_0 + P_{m/2} + 2 Re sum_{0<j<m/2} P_j) per sample.
// The sketches never leave LDS: no HBM round trip between scatter and DFT, no
// second launch, and small networks cost no per-slot block start-up.
#include "m1_device.h"

namespace tn {
namespace {

using namespace m1dev;

__global__ void reset_counter_kernel(int32_t *counter) {
  if (threadIdx.x == 0) counter[0] = 0;
}

template <typename T, typename A, int SB, int LOG2M, int BANKS>
__global__ __launch_bounds__(256) void m1_fused_kernel(
    const FusedItem *__restrict__ items, int32_t n_items, int32_t *__restrict__ counter,
    const NetDesc *__restrict__ nets, const int32_t *__restrict__ tslot,
    const ScatterSlot *__restrict__ slots, const int32_t *__restrict__ tensor_lgn,
    const ModeDesc *__restrict__ modes, const void *const *__restrict__ data,
    const int32_t *__restrict__ tables, int64_t W, int64_t chunk, int64_t sample0, int64_t S,
    int32_t worst, const typename Cplx<A>::type *__restrict__ tw, double *__restrict__ est) {
  using A2 = typename Cplx<A>::type;
  constexpr int M = 1 << LOG2M;
  constexpr int H = M / 2 + 1;
  constexpr int NC = (H + 255) / 256;
  extern __shared__ __align__(16) unsigned char smem[];
  // The pair's two tensors are the "virtual samples" 2s and 2s + 1 of one
  // layout of 2 SB sketches (see scatter_slot): (positive) banks at
  // 8M (2s + side) bytes, with BANKS = 2 negative banks kSignbit bytes
  // further.  Sample s's FFT input later overwrites its two first banks (16M
  // bytes).
  constexpr uint32_t kSignbit = BANKS == 2 ? sign_bank_offset(2 * SB, M) : 0u;
  constexpr size_t kAcc = BANKS == 2 ? sign_bank_bytes(2 * SB, M) : (size_t)16 * SB * M;
  constexpr int PER = (M + 255) / 256;  // sketch entries per thread
  static_assert(sizeof(A2) * M <= 16 * (size_t)M, "FFT input fits two positive banks");
  unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem);
  uint32_t *tabs = reinterpret_cast<uint32_t *>(smem + kAcc);  // [SB * worst]
  __shared__ unsigned long long s_max[2];
  __shared__ double red[4];
  __shared__ int32_t item_sh;
  const int tid = threadIdx.x;

  for (;;) {
    if (tid == 0) item_sh = atomicAdd(counter, 1);
    __syncthreads();
    const int32_t it = item_sh;
    if (it >= n_items) break;  // the same value in every thread
    const FusedItem fi = items[it];
    if ((int64_t)fi.s0 >= chunk) {  // batch beyond this launch's samples
      __syncthreads();
      continue;
    }
    const int nsb = (int)min((int64_t)SB, chunk - fi.s0);
    const NetDesc nd = nets[fi.net];
    const int32_t *tab0 = tables + (int64_t)fi.s0 * W;

    double pr[SB][NC], pi[SB][NC];
#pragma unroll
    for (int s = 0; s < SB; ++s)
#pragma unroll
      for (int c = 0; c < NC; ++c) { pr[s][c] = 1.0; pi[s][c] = 0.0; }

    for (int k = nd.t0; k < nd.t1; k += 2) {
      const bool pair = (k + 1) < nd.t1;
      for (int i = tid; i < (int)(kAcc / 8); i += 256) acc[i] = 0ull;
      FixedScale fs[2];
#pragma unroll
      for (int side = 0; side < 2; ++side) {  // unrolled: fs[] indexed by constants
        if (side == 1 && !pair) break;
        const int t = k + side;
        if (tid < 2) s_max[tid] = 0ull;
        fs[side].lgN = tensor_lgn[t];
        for (int si = tslot[t]; si < tslot[t + 1]; ++si) {
          const ScatterSlot sl = slots[si];
          scatter_slot<T, SB, BANKS, 256>(sl, modes, data, tab0, W, nsb, LOG2M, acc + side * M, 16u * M, kSignbit,
                              tabs, s_max, fs[side]);
        }
      }
      const double ia = ldexp(1.0, -fs[0].scale);
      const double ib = pair ? ldexp(1.0, -fs[1].scale) : 0.0;
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        if (s < nsb) {
          A va[PER], vb[PER];
#pragma unroll
          for (int i = 0; i < PER; ++i) {
            const int b = tid + 256 * i;
            va[i] = vb[i] = (A)0;
            if (b < M) {
              const unsigned long long *pa = acc + (size_t)(2 * s) * M + b;  // side 0, positive bank
              const unsigned long long *pb = pa + M;                          // side 1
              const long long xa = BANKS == 2 ? (long long)(pa[0] - pa[kSignbit / 8]) : (long long)pa[0];
              const long long xb = BANKS == 2 ? (long long)(pb[0] - pb[kSignbit / 8]) : (long long)pb[0];
              va[i] = (A)((double)xa * ia);
              if (pair) vb[i] = (A)((double)xb * ib);
            }
          }
          __syncthreads();
          A2 *z = reinterpret_cast<A2 *>(acc + (size_t)(2 * s) * M);
#pragma unroll
          for (int i = 0; i < PER; ++i) {
            const int b = tid + 256 * i;
            if (b < M) z[bitrev<LOG2M>(b)] = A2{va[i], vb[i]};
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
              const double nr = pr[s][c] * qr - pi[s][c] * qi;
              const double ni = pr[s][c] * qi + pi[s][c] * qr;
              pr[s][c] = nr;
              pi[s][c] = ni;
            }
          }
          __syncthreads();
        }
      }
    }
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      if (s < nsb) {
        double part = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int j = tid + 256 * c;
          if (j < H) part += ((j == 0 || 2 * j == M) ? 1.0 : 2.0) * pr[s][c];
        }
        const double tot = block_sum_256(part, red);
        if (tid == 0) est[(int64_t)fi.net * S + sample0 + fi.s0 + s] = tot / (double)M;
      }
    }
    __syncthreads();
  }
}

template <typename T, typename A, int SB, int LOG2M>
int fused_launch(const M1FusedLaunch &L, hipStream_t st) {
  auto k = L.banks == 2 ? m1_fused_kernel<T, A, SB, LOG2M, 2> : m1_fused_kernel<T, A, SB, LOG2M, 1>;
  if (L.lds_bytes > 65536)
    TN_HIP_CHECK(hipFuncSetAttribute((const void *)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)L.lds_bytes));
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, L.counter);
  hipLaunchKernelGGL(k, dim3((unsigned)L.blocks), dim3(256), L.lds_bytes, st, L.items, L.n_items, L.counter,
                     L.nets, L.tslot, L.slots, L.tensor_lgn, L.modes, L.data, L.tables, L.W, L.chunk,
                     L.sample0, L.S, L.worst, reinterpret_cast<const typename Cplx<A>::type *>(L.twiddles),
                     L.est);
  TN_HIP_CHECK(hipGetLastError());
  return TN_OK;
}

template <typename T, typename A, int SB>
int fused_m(const M1FusedLaunch &L, hipStream_t st) {
  switch (L.log2m) {
    case 6: return fused_launch<T, A, SB, 6>(L, st);
    case 7: return fused_launch<T, A, SB, 7>(L, st);
    case 8: return fused_launch<T, A, SB, 8>(L, st);
    case 9: return fused_launch<T, A, SB, 9>(L, st);
    case 10: return fused_launch<T, A, SB, 10>(L, st);
    case 11: return fused_launch<T, A, SB, 11>(L, st);
    case 12: return fused_launch<T, A, SB, 12>(L, st);
    default: return set_error(TN_ERR_UNSUPPORTED, "persistent kernel: m = 2^%d outside 2^6..2^12", L.log2m);
  }
}

template <typename T, typename A>
int fused_t(const M1FusedLaunch &L, hipStream_t st) {
  switch (L.sb) {
    case 1: return fused_m<T, A, 1>(L, st);
    case 2: return fused_m<T, A, 2>(L, st);
    case 4: return fused_m<T, A, 4>(L, st);
    default: return set_error(TN_ERR_ARG, "persistent kernel: samples per item %d", L.sb);
  }
}

}  // namespace

size_t m1_fused_lds(int sb, int banks, int64_t m, int32_t worst) {
  const size_t acc = banks == 2 ? sign_bank_bytes(2 * sb, (uint32_t)m) : (size_t)16 * sb * m;
  return acc + (size_t)sb * worst * 4;
}

int launch_m1_fused(const M1FusedLaunch &L, hipStream_t st) {
  switch (L.dtype) {
    case TN_F64: return fused_t<double, double>(L, st);
    case TN_F32: return fused_t<float, float>(L, st);
    default: return fused_t<uint16_t, float>(L, st);
  }
}

}  // namespace tn
