// Device code shared by the cyclic method's kernels (m1.hip, fused.hip):
// element conversions, vector types, the packed mode hashes, the fixed-point
// slot scatter and the LDS FFT.
#pragma once

#include <type_traits>

#include "tn_internal.h"

namespace tn {
namespace m1dev {

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

// Clear `bytes` (a multiple of 8) of 16-byte-aligned LDS with the threads of
// a block (tid of nt): 16-byte stores, then the last 8 bytes if any.
__device__ __forceinline__ void lds_zero(void *p, uint32_t bytes, int tid, int nt) {
  uint4 *q = reinterpret_cast<uint4 *>(p);
  for (uint32_t i = tid; i < bytes / 16; i += nt) q[i] = make_uint4(0u, 0u, 0u, 0u);
  if ((bytes & 15u) && tid == 0) reinterpret_cast<unsigned long long *>(p)[bytes / 8 - 1] = 0ull;
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

// Fixed-point state of one set of sketch accumulators.  The sketches are
// accumulated in 64-bit fixed point in LDS: x -> round(x 2^scale) with
// ds_add_u64, which on gfx950 sustains about 16x the rate of LDS float atomics
// and makes every sketch independent of the order of the atomic adds.  The
// scale follows a running maximum of |x|: scale = 62 - lgN - e with
// max|x| < 2^e, where 2^lgN bounds the number of terms the set receives, so
// they cannot overflow; when a larger |x| appears the accumulators are shifted
// right to the new scale before any further add.
struct FixedScale {
  int scale = 0;       // accumulators hold x 2^scale
  double sc = 1.0;     // 2^scale
  double bound = 0.0;  // every |x| seen is < bound (0: none seen yet)
  int lgN = 11;        // >= ceil(log2(terms)) and >= 11
  int par = 0;         // parity of the double-buffered running maximum
  bool known = false;  // bound given up front: no running maximum
};

// Layout of SB two-bank sketches of m words: positive banks of the SB samples
// back to back, the negative banks `signbit` bytes after them.
__host__ __device__ constexpr uint32_t sign_bank_offset(int sb, uint32_t m) {
  return 8u * m * (sb <= 2 ? 2u : sb <= 4 ? 4u : sb <= 8 ? 8u : 16u);
}
__host__ __device__ constexpr size_t sign_bank_bytes(int sb, uint32_t m) {
  return (size_t)sign_bank_offset(sb, m) + (size_t)sb * 8u * m;
}

// Scatter one slot (a run of rows of one tensor) into the fixed-point
// sketches of nsb samples.  With BANKS = 1 a sketch is one bank of m words
// and a term of sign -1 is negated before its add (sample s's bank at byte
// s * sbytes; signbit unused).  With BANKS = 2 each sketch is a pair of banks of m words: terms
// of sign +1 go to the positive bank, terms of sign -1 to the negative one,
// and the sketch is their difference.  Sample s's positive bank starts at byte
// s * sbytes from acc, its negative bank `signbit` bytes further; signbit is a
// power of two of at least 16 m.  The packed tables hold bucket * 8 plus
// signbit for sign -1, so the sum of a row and a column entry has the product
// of the two signs in the signbit position (the bucket sum stays below 16 m),
// and masking it with 8(m - 1) | signbit leaves the byte offset of the target
// word: no sign test and no negation per term.
// Builds the slot's packed column and row tables in `tabs` (LDS, SB (L +
// kColPad + rows) + 1 words), then streams the slot once from HBM with 16-byte
// loads.  s_max (2 words of LDS) holds the running maximum; both it and fs
// carry over between calls that feed the same sketches.  All NT threads of
// the block call it; it starts and ends with a barrier.
// fresh (optional): the accumulators, fresh_words 4-byte words, not yet
// cleared; the column tables are then built from the modes' hash words staged
// there, and the accumulators are cleared before the scatter.  Without it the
// caller clears them.
// RANGED (one bank): the LDS holds only the 2^log2acc buckets starting at
// bucket rsel * 2^log2acc of each sketch; terms outside that range are
// dropped.  Every range sees the same terms in the same order, so all ranges
// of a slot reach the same fixed-point scale.
template <typename T, int SB, int BANKS, int NT, bool RANGED = false>
__device__ __forceinline__ void scatter_slot(const ScatterSlot &sl, const ModeDesc *__restrict__ modes,
                                             const void *const *__restrict__ data,
                                             const int32_t *__restrict__ tables, int64_t W, int nsb,
                                             int log2m, unsigned long long *acc, uint32_t sbytes,
                                             uint32_t signbit, uint32_t *tabs,
                                             unsigned long long *s_max, FixedScale &fs, uint32_t rsel = 0,
                                             int log2acc = -1, uint32_t *fresh = nullptr,
                                             uint32_t fresh_words = 0) {
  static_assert(!RANGED || BANKS == 1, "bucket ranges use one bank");
  if (log2acc < 0) log2acc = log2m;
  const uint32_t rshift = 3u + (uint32_t)log2acc;  // byte offset >> rshift = range index
  const int tid = threadIdx.x;
  const uint32_t m = 1u << log2m, mask = m - 1;
  const int L = sl.L, rows = sl.rows;
  constexpr int VEC = 16 / (int)sizeof(T);  // entries per 16-byte load
  // Column tables first, sample s's at colt + s Lp: its L words, then the
  // first VEC - 1 columns again (word L + j holds column j mod L), so a
  // vector that runs on into the next row reads its VEC column words without
  // a wrap test.  Row tables after them, sample s's at rowt + s rows, and one
  // more word (a vector in the last row reads the word after that row).
  const int Lp = L + kColPad, Lb = L + VEC - 1;
  static_assert(VEC - 1 <= kColPad, "column table padding");
  uint32_t *colt = tabs;
  uint32_t *rowt = tabs + SB * Lp;
  auto to_offset = [signbit](uint32_t v) {
    (void)signbit;  // unused with one bank
    if constexpr (BANKS == 2) return ((v & ~kSignBit) << 3) + ((v & kSignBit) ? signbit : 0u);
    else return ((v & ~kSignBit) << 3) | (v & kSignBit);  // sign stays in bit 31
  };
  __syncthreads();  // earlier readers of the tables are done
  const int uc0 = sl.mode0 + sl.split, uc1 = sl.mode0 + sl.q - 1;  // column modes
  int qc = 0;  // their hash words per sample
  for (int u = uc0; u <= uc1; ++u) qc += modes[u].n;
  if (fresh != nullptr && (uint32_t)(nsb * qc) <= fresh_words) {
    // The column modes' hash words of the nsb samples, complement applied,
    // staged in the (not yet cleared) accumulator LDS: sample s, mode u,
    // index d at fresh[s qc + off_u + d], modes in order.  One global read
    // per word instead of one per (column, mode).
    for (int i = tid; i < nsb * qc; i += NT) {
      const int s = i / qc;
      int d = i - s * qc, u = uc0;
      while (d >= modes[u].n) d -= modes[u++].n;
      const ModeDesc md = modes[u];
      const uint32_t v = (uint32_t)tables[s * W + md.table_off + d];
      uint32_t h = v & ~kSignBit;
      if (md.comp) h = (m - h) & mask;
      fresh[i] = h | (v & kSignBit);
    }
    __syncthreads();
    // Column c's word per sample: the digits of c mod L, last mode fastest,
    // found once for all samples.
    for (int c = tid; c < Lb; c += NT) {
      uint32_t idx = (uint32_t)(c < L ? c : c % L), w[SB];
#pragma unroll
      for (int s = 0; s < SB; ++s) w[s] = 0;
      int off = qc;
      for (int u = uc1; u >= uc0; --u) {
        const uint32_t n = (uint32_t)modes[u].n;
        off -= (int)n;
        const uint32_t d = idx % n;
        idx /= n;
#pragma unroll
        for (int s = 0; s < SB; ++s)
          if (s < nsb) {
            const uint32_t v = fresh[s * qc + off + d];
            w[s] = (((w[s] & ~kSignBit) + (v & ~kSignBit)) & mask) | ((w[s] ^ v) & kSignBit);
          }
      }
#pragma unroll
      for (int s = 0; s < SB; ++s)
        if (s < nsb) colt[s * Lp + c] = to_offset(w[s]);
    }
  } else {
    for (int i = tid; i < nsb * Lb; i += NT) {
      const int s = i / Lb, c = i - s * Lb;
      colt[s * Lp + c] = to_offset(combine_modes(tables + s * W, modes, uc0, uc1, c < L ? c : c % L, m, mask));
    }
  }
  for (int i = tid; i < nsb * rows; i += NT) {
    const int s = i / rows, r = i - s * rows;
    rowt[s * rows + r] = to_offset(combine_modes(tables + s * W, modes, sl.mode0, sl.mode0 + sl.split - 1,
                                                 (uint32_t)(sl.row0 + r), m, mask));
  }
  __syncthreads();
  if (fresh != nullptr) {  // clear the accumulators (they held the staged words)
    lds_zero(fresh, fresh_words * 4u, tid, NT);
    __syncthreads();
  }
  const uint32_t amask = (mask << 3) | (BANKS == 2 ? signbit : 0u);
  char *acc8 = reinterpret_cast<char *>(acc);
  // The slot's entries as 16-byte vectors: from the start when every row is a
  // whole number of vectors and the slot starts 16-byte aligned (vec), else
  // from the first aligned vector (the entries before it and after the last
  // whole vector are read singly).
  using V = typename Vec16<T>::type;
  // 16-byte loads in flight per thread: 8 in the 512-thread blocks (two per CU,
  // registers to spare; half the barriers per entry), else 4; 4 in the
  // unaligned loop (its tables take the registers)
  constexpr int UNROLL = NT == 512 && SB * VEC <= 16 ? 8 : 4;
  constexpr int UNW = 4;
  const T *X = reinterpret_cast<const T *>(data[sl.tensor]) + sl.row0 * (int64_t)L;
  const uint32_t N = (uint32_t)rows * (uint32_t)L;
  const bool vec = (L % VEC == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  const uint32_t head =
      vec ? 0u : min(N, ((16u - ((uint32_t)reinterpret_cast<uintptr_t>(X) & 15u)) & 15u) / (uint32_t)sizeof(T));
  const uint32_t NV = (N - head) / VEC;
  const V __attribute__((address_space(1))) *Xv =
      (const V __attribute__((address_space(1))) *)reinterpret_cast<const V *>(X + head);

  // Block-wide running max of |x| (double-buffered so the read of one
  // iteration cannot race with the next iteration's update), then a rescale
  // when it reaches the bound.  Called by every thread once per iteration,
  // unless the block starts from a known bound.
  auto update_scale = [&](double lmax) {
    if (fs.known) return;  // uniform over the block
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lmax = fmax(lmax, __shfl_xor(lmax, off, 64));
    if ((tid & 63) == 0) atomicMax(&s_max[fs.par], (unsigned long long)__double_as_longlong(lmax));
    __syncthreads();
    const double bm = __longlong_as_double((long long)s_max[fs.par]);
    fs.par ^= 1;
    if (bm >= fs.bound && bm > 0.0) {
      int e;
      (void)frexp(bm, &e);  // bm < 2^e
      const int ns = 62 - fs.lgN - e;
      if (fs.bound > 0.0 && fs.scale > ns) {
        const int d = fs.scale - ns;
        for (int i = tid; i < (BANKS * nsb) << log2acc; i += NT) {
          const int si = BANKS == 2 ? i >> (log2acc + 1) : i >> log2acc;
          const int bank = BANKS == 2 ? (i >> log2acc) & 1 : 0, b = i & ((1 << log2acc) - 1);
          unsigned long long *w = reinterpret_cast<unsigned long long *>(
              reinterpret_cast<char *>(acc) + (size_t)si * sbytes + (bank ? signbit : 0u)) + b;
          *w = (unsigned long long)((long long)*w >> d);
        }
        __syncthreads();
      }
      fs.scale = ns;
      fs.sc = ldexp(1.0, ns);
      fs.bound = ldexp(1.0, e);
    }
  };
  // round(x 2^scale) for |x 2^scale| < 2^51: adding 1.5 2^52 leaves the
  // rounded integer in the low mantissa bits.
  auto to_fixed = [&](double x) -> long long {
    const double kMagic = 6755399441055744.0;
    return __double_as_longlong(fma(x, fs.sc, kMagic)) - __double_as_longlong(kMagic);
  };
  // One fixed-point add into sample s's sketch (its sign selects the bank).
  // (nv = -v, formed once per entry for all samples of the batch.)
  auto add_fixed = [&](int s, uint32_t hv, uint32_t lv, long long v, long long nv) {
    if constexpr (RANGED) {
      const uint32_t o = (hv + lv) & amask;
      if ((o >> rshift) != rsel) return;
      atomicAdd(reinterpret_cast<unsigned long long *>(acc8 + (o & ((1u << rshift) - 1u)) + (uint32_t)s * sbytes),
                (unsigned long long)(((hv ^ lv) & kSignBit) ? nv : v));
      return;
    }
    const uint32_t a = ((hv + lv) & amask) + (uint32_t)s * sbytes;
    if constexpr (BANKS == 2)
      atomicAdd(reinterpret_cast<unsigned long long *>(acc8 + a), (unsigned long long)v);
    else
      atomicAdd(reinterpret_cast<unsigned long long *>(acc8 + a),
                (unsigned long long)(((hv ^ lv) & kSignBit) ? nv : v));
  };
  // Add entry x (row r, column c) to the sketch of every sample of the batch.
  auto scatter_one = [&](double x, uint32_t r, uint32_t c) {
    const long long v = to_fixed(x), nv = -v;
    uint32_t hv[SB], lv[SB];
#pragma unroll
    for (int s = 0; s < SB; ++s) { hv[s] = rowt[s * rows + r]; lv[s] = colt[s * Lp + c]; }
#pragma unroll
    for (int s = 0; s < SB; ++s)
      if (s < nsb) add_fixed(s, hv[s], lv[s], v, nv);
  };
  // Row and column entries of every sample for VEC consecutive entries of one
  // row (all reads issued before any add, so one LDS wait covers them).
  auto read_tabs = [&](uint32_t r, uint32_t c, uint32_t *hv, uint32_t (*lv)[VEC]) {
#pragma unroll
    for (int s = 0; s < SB; ++s) {
      hv[s] = rowt[s * rows + r];
      load_cols<VEC>(colt + s * Lp + c, lv[s]);
    }
  };
  if (vec) {
    // Rows are multiples of VEC long and the slot starts 16-byte aligned, so
    // the VEC entries of one load share a row.
    // Unconditional loads (index clamped into the slot) keep all UNROLL loads
    // in flight; out-of-range lanes are masked when the values are used.
    // Blocks of 512 or more threads (few blocks per CU: their LDS is large)
    // issue the next iteration's loads before this iteration's adds, so the
    // load latency hides behind the LDS atomics; small blocks overlap with
    // other blocks instead and keep the registers.
    constexpr bool PREFETCH = NT >= 512;
    if constexpr (NT == 512) {
      // 512-thread blocks: when NT * VEC is a multiple of the row length, every
      // vector a thread loads starts at the same column (tid * VEC) mod L, so
      // its column-table entries are read once, not once per vector (a third
      // of the loop's LDS bytes otherwise).  The loop is instantiated for both
      // cases; blocks of other sizes keep the general loop below (they have no
      // registers to spare for a second instantiation).
      auto vec_loop = [&](auto FIXED_) {
        constexpr bool FIXED = decltype(FIXED_)::value;
        uint32_t lvf[SB][VEC];
        if constexpr (FIXED) {
#pragma unroll
          for (int s = 0; s < SB; ++s) load_cols<VEC>(colt + s * Lp + ((uint32_t)tid * VEC) % (uint32_t)L, lvf[s]);
        }
        V buf[UNROLL], nxt[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) nxt[u] = Xv[min((uint32_t)(u * NT + tid), NV - 1)];
        for (uint32_t v0 = 0; v0 < NV; v0 += NT * UNROLL) {
#pragma unroll
          for (int u = 0; u < UNROLL; ++u) buf[u] = nxt[u];
          if (!fs.known) {  // running maximum of this load round (uniform over the block)
            double lmax = 0.0;
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
              const T *xs = reinterpret_cast<const T *>(&buf[u]);
#pragma unroll
              for (int i = 0; i < VEC; ++i) lmax = fmax(lmax, fabs((double)to_acc_any(xs[i])));
            }
            update_scale(lmax);
          }
          if (v0 + NT * UNROLL < NV) {  // uniform over the block
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) nxt[u] = Xv[min(v0 + (u + UNROLL) * NT + tid, NV - 1)];
          }
          uint32_t rr[UNROLL], cc[UNROLL];
#pragma unroll
          for (int u = 0; u < UNROLL; ++u) {
            const uint32_t e = min(v0 + u * NT + tid, NV - 1) * VEC;  // clamped: valid table reads
            rr[u] = (L == 1) ? e : __umulhi(e, sl.magic);
            cc[u] = e - rr[u] * (uint32_t)L;
          }
          // the table reads of vector u + 1 are issued before the adds of vector u
          uint32_t hv[2][SB], lv[2][SB][VEC];
          auto tabs = [&](int u, int k) {
            if constexpr (FIXED) {
#pragma unroll
              for (int s = 0; s < SB; ++s) hv[k][s] = rowt[s * rows + rr[u]];
            } else {
              read_tabs(rr[u], cc[u], hv[k], lv[k]);
            }
          };
          tabs(0, 0);
#pragma unroll
          for (int u = 0; u < UNROLL; ++u) {
            if (u + 1 < UNROLL) tabs(u + 1, (u + 1) & 1);
            if (v0 + u * NT + tid < NV) {
              const T *xs = reinterpret_cast<const T *>(&buf[u]);
              long long q[VEC], nq[VEC];
#pragma unroll
              for (int i = 0; i < VEC; ++i) {
                q[i] = to_fixed((double)to_acc_any(xs[i]));
                nq[i] = BANKS == 2 ? 0 : -q[i];
              }
#pragma unroll
              for (int s = 0; s < SB; ++s)
                if (s < nsb) {
#pragma unroll
                  for (int i = 0; i < VEC; ++i)
                    add_fixed(s, hv[u & 1][s], FIXED ? lvf[s][i] : lv[u & 1][s][i], q[i], nq[i]);
                }
            }
          }
        }
      };
      if (((uint32_t)(NT * VEC)) % (uint32_t)L == 0)
        vec_loop(std::true_type{});
      else
        vec_loop(std::false_type{});
    } else {
      V buf[UNROLL], nxt[UNROLL];
      if constexpr (PREFETCH) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) nxt[u] = Xv[min((uint32_t)(u * NT + tid), NV - 1)];
      }
      for (uint32_t v0 = 0; v0 < NV; v0 += NT * UNROLL) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) buf[u] = PREFETCH ? nxt[u] : Xv[min(v0 + u * NT + tid, NV - 1)];
        if (!fs.known) {  // running maximum of this load round (uniform over the block)
          double lmax = 0.0;
#pragma unroll
          for (int u = 0; u < UNROLL; ++u) {
            const T *xs = reinterpret_cast<const T *>(&buf[u]);
#pragma unroll
            for (int i = 0; i < VEC; ++i) lmax = fmax(lmax, fabs((double)to_acc_any(xs[i])));
          }
          update_scale(lmax);
        }
        if (PREFETCH && v0 + NT * UNROLL < NV) {  // uniform over the block
#pragma unroll
          for (int u = 0; u < UNROLL; ++u) nxt[u] = Xv[min(v0 + (u + UNROLL) * NT + tid, NV - 1)];
        }
        uint32_t rr[UNROLL], cc[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const uint32_t e = min(v0 + u * NT + tid, NV - 1) * VEC;  // clamped: valid table reads
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
          if (v0 + u * NT + tid < NV) {
            const T *xs = reinterpret_cast<const T *>(&buf[u]);
            long long q[VEC], nq[VEC];
#pragma unroll
            for (int i = 0; i < VEC; ++i) {
              q[i] = to_fixed((double)to_acc_any(xs[i]));
              nq[i] = BANKS == 2 ? 0 : -q[i];
            }
#pragma unroll
            for (int s = 0; s < SB; ++s)
              if (s < nsb) {
#pragma unroll
                for (int i = 0; i < VEC; ++i) add_fixed(s, hv[u & 1][s], lv[u & 1][s][i], q[i], nq[i]);
              }
          }
        }
      }
    }
  } else {
    // Rows whose length is not a multiple of VEC, or a slot that starts
    // inside a 16-byte vector: the slot's flat entry range is read as aligned
    // 16-byte vectors, each entry finding its own row and column.  The fewer
    // than VEC entries before the first aligned vector and after the last one
    // are read singly, one per thread, first.
    const T __attribute__((address_space(1))) *Xg =
        (const T __attribute__((address_space(1))) *)X;
    const uint32_t body = head + NV * VEC;
    {
      const uint32_t singles = head + (N - body);  // < 2 VEC <= NT
      const uint32_t e = (uint32_t)tid < head ? (uint32_t)tid : body + ((uint32_t)tid - head);
      const bool act = (uint32_t)tid < singles;
      const double x = act ? (double)to_acc_any(Xg[e]) : 0.0;
      update_scale(fabs(x));
      if (act) {
        const uint32_t r = (L == 1) ? e : __umulhi(e, sl.magic);
        scatter_one(x, r, e - r * (uint32_t)L);
      }
    }
    if (NV > 0) {  // uniform over the block
      constexpr bool PREFETCH = NT >= 512;
      V buf[UNW], nxt[UNW];
      if constexpr (PREFETCH) {
#pragma unroll
        for (int u = 0; u < UNW; ++u) nxt[u] = Xv[min((uint32_t)(u * NT + tid), NV - 1)];
      }
      for (uint32_t v0 = 0; v0 < NV; v0 += NT * UNW) {
#pragma unroll
        for (int u = 0; u < UNW; ++u) buf[u] = PREFETCH ? nxt[u] : Xv[min(v0 + u * NT + tid, NV - 1)];
        if (!fs.known) {  // running maximum of this load round (uniform over the block)
          double lmax = 0.0;
#pragma unroll
          for (int u = 0; u < UNW; ++u) {
            const T *xs = reinterpret_cast<const T *>(&buf[u]);
#pragma unroll
            for (int i = 0; i < VEC; ++i) lmax = fmax(lmax, fabs((double)to_acc_any(xs[i])));
          }
          update_scale(lmax);
        }
        if (PREFETCH && v0 + NT * UNW < NV) {  // uniform over the block
#pragma unroll
          for (int u = 0; u < UNW; ++u) nxt[u] = Xv[min(v0 + (u + UNW) * NT + tid, NV - 1)];
        }
        if (L >= VEC) {  // uniform over the block: a vector spans at most two rows
          // Per sample the row words of the vector's row and of the next one
          // and its VEC column words from the wrapped table, all read before
          // the vector's adds; entry i takes the next row's word when column
          // c + i passes the row's end.
#pragma unroll
          for (int u = 0; u < UNW; ++u) {
            if (v0 + u * NT + tid < NV) {
              const uint32_t e = head + (v0 + u * NT + tid) * VEC;
              const uint32_t r = __umulhi(e, sl.magic), c = e - r * (uint32_t)L;
              uint32_t h0[SB], h1[SB], lw[SB][VEC];
#pragma unroll
              for (int s = 0; s < SB; ++s) {
                h0[s] = rowt[s * rows + r];
                h1[s] = rowt[s * rows + r + 1];
#pragma unroll
                for (int i = 0; i < VEC; ++i) lw[s][i] = colt[s * Lp + c + i];
              }
              const T *xs = reinterpret_cast<const T *>(&buf[u]);
#pragma unroll
              for (int i = 0; i < VEC; ++i) {
                const long long q = to_fixed((double)to_acc_any(xs[i]));
                const bool same = c + i < (uint32_t)L;
#pragma unroll
                for (int s = 0; s < SB; ++s)
                  if (s < nsb) add_fixed(s, same ? h0[s] : h1[s], lw[s][i], q, -q);
              }
            }
          }
        } else {  // rows shorter than a vector
#pragma unroll
          for (int u = 0; u < UNW; ++u) {
            if (v0 + u * NT + tid < NV) {
              const uint32_t e = head + (v0 + u * NT + tid) * VEC;
              uint32_t r = (L == 1) ? e : __umulhi(e, sl.magic);
              uint32_t c = e - r * (uint32_t)L;
              const T *xs = reinterpret_cast<const T *>(&buf[u]);
#pragma unroll
              for (int i = 0; i < VEC; ++i) {
                scatter_one((double)to_acc_any(xs[i]), r, c);
                if (++c == (uint32_t)L) {  // the vector runs on into the next row
                  c = 0;
                  ++r;
                }
              }
            }
          }
        }
      }
    }
  }
  __syncthreads();
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
// Stages are taken two at a time: a thread carries the four points of a
// radix-2^2 group through both stages in registers (the same butterflies and
// twiddles as two radix-2 passes), which halves the barriers and LDS passes; an
// odd stage count starts with one single stage.
// PAD: z and tw are held with one spare element after every 32 (element e at
// pad32(e)), which spreads the strided accesses of the first passes, the
// bit-reversed loads and the twiddle reads over the LDS banks.
__device__ __forceinline__ constexpr int pad32(int e) { return e + (e >> 5); }

// twf(e) returns w_M^e for e < M/2.
template <typename A, int LOG2M, bool PAD, int NTH, typename TwF>
__device__ __forceinline__ void fft_lds_tw(typename Cplx<A>::type *z, TwF twf) {
  constexpr int M = 1 << LOG2M;
  using A2 = typename Cplx<A>::type;
  auto P = [](int e) { return PAD ? pad32(e) : e; };
  auto bfly = [](A2 &za, A2 &zb, const A2 w) {
    const A tr = w.x * zb.x - w.y * zb.y;
    const A ti = w.x * zb.y + w.y * zb.x;
    zb = A2{za.x - tr, za.y - ti};
    za = A2{za.x + tr, za.y + ti};
  };
  int lg = 1;
  if constexpr ((LOG2M & 1) != 0) {
    const A2 w0 = twf(0);
    for (int q = threadIdx.x; q < M / 2; q += NTH) {
      A2 za = z[P(2 * q)], zb = z[P(2 * q + 1)];
      bfly(za, zb, w0);
      z[P(2 * q)] = za;
      z[P(2 * q + 1)] = zb;
    }
    __syncthreads();
    lg = 2;
  }
#pragma unroll 1
  for (; lg < LOG2M; lg += 2) {
    const int h = 1 << (lg - 1);
    for (int q = threadIdx.x; q < M / 4; q += NTH) {
      const int k = q & (h - 1);
      const int base = ((q >> (lg - 1)) << (lg + 1)) + k;
      A2 z0 = z[P(base)], z1 = z[P(base + h)], z2 = z[P(base + 2 * h)], z3 = z[P(base + 3 * h)];
      const A2 w1 = twf(k << (LOG2M - lg));
      bfly(z0, z1, w1);  // stage lg: (base, base + h), (base + 2h, base + 3h)
      bfly(z2, z3, w1);
      bfly(z0, z2, twf(k << (LOG2M - lg - 1)));  // stage lg + 1: (base, base + 2h), (base + h, base + 3h)
      bfly(z1, z3, twf((k + h) << (LOG2M - lg - 1)));
      z[P(base)] = z0;
      z[P(base + h)] = z1;
      z[P(base + 2 * h)] = z2;
      z[P(base + 3 * h)] = z3;
    }
    __syncthreads();
  }
}

// The twiddles from the half table tw[j] = w_M^j; TWPAD: the table is padded
// the same way (it is, when staged in LDS).
template <typename A, int LOG2M, bool PAD = false, int NTH = 256, bool TWPAD = PAD>
__device__ __forceinline__ void fft_lds(typename Cplx<A>::type *z,
                                        const typename Cplx<A>::type *__restrict__ tw) {
  fft_lds_tw<A, LOG2M, PAD, NTH>(z, [tw](int e) { return tw[TWPAD ? pad32(e) : e]; });
}

// Two-level twiddles for transforms whose half table does not fit in LDS
// beside them: w_M^e = hi[e / 64] lo[e % 64], hi[i] = w_M^(64 i) (M/128
// entries), lo[j] = w_M^j (64 entries), one complex product per twiddle.
template <typename A>
struct Tw2 {
  using A2 = typename Cplx<A>::type;
  const A2 *hi, *lo;
  __device__ __forceinline__ A2 operator()(int e) const {
    const A2 a = hi[e >> 6], b = lo[e & 63];
    return A2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
  }
};

// nb transforms of M points each, transform t at z + t * STR (STR >= pad32(M)),
// element e of a transform at pad32(e); the same radix-2^2 passes as fft_lds,
// with the groups of all transforms spread over the block (NTH threads) in
// every pass.  tw is the padded half table of w_M.
template <typename A, int LOG2M, int STR, int NTH>
__device__ __forceinline__ void fft_lds_batch(typename Cplx<A>::type *z,
                                              const typename Cplx<A>::type *__restrict__ tw, int nb) {
  static_assert(LOG2M >= 2, "batched transforms of at least 4 points");
  constexpr int M = 1 << LOG2M;
  using A2 = typename Cplx<A>::type;
  auto bfly = [](A2 &za, A2 &zb, const A2 w) {
    const A tr = w.x * zb.x - w.y * zb.y;
    const A ti = w.x * zb.y + w.y * zb.x;
    zb = A2{za.x - tr, za.y - ti};
    za = A2{za.x + tr, za.y + ti};
  };
  int lg = 1;
  if constexpr ((LOG2M & 1) != 0) {
    for (int q = threadIdx.x; q < nb * (M / 2); q += NTH) {
      A2 *zt = z + (q >> (LOG2M - 1)) * STR;
      const int qq = q & (M / 2 - 1);
      A2 za = zt[pad32(2 * qq)], zb = zt[pad32(2 * qq + 1)];
      bfly(za, zb, tw[0]);
      zt[pad32(2 * qq)] = za;
      zt[pad32(2 * qq + 1)] = zb;
    }
    __syncthreads();
    lg = 2;
  }
#pragma unroll 1
  for (; lg < LOG2M; lg += 2) {
    const int h = 1 << (lg - 1);
    for (int q = threadIdx.x; q < nb * (M / 4); q += NTH) {
      A2 *zt = z + (q >> (LOG2M - 2)) * STR;
      const int qq = q & (M / 4 - 1);
      const int k = qq & (h - 1);
      const int base = ((qq >> (lg - 1)) << (lg + 1)) + k;
      A2 z0 = zt[pad32(base)], z1 = zt[pad32(base + h)], z2 = zt[pad32(base + 2 * h)], z3 = zt[pad32(base + 3 * h)];
      const A2 w1 = tw[pad32(k << (LOG2M - lg))];
      bfly(z0, z1, w1);
      bfly(z2, z3, w1);
      bfly(z0, z2, tw[pad32(k << (LOG2M - lg - 1))]);
      bfly(z1, z3, tw[pad32((k + h) << (LOG2M - lg - 1))]);
      zt[pad32(base)] = z0;
      zt[pad32(base + h)] = z1;
      zt[pad32(base + 2 * h)] = z2;
      zt[pad32(base + 3 * h)] = z3;
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

// Block sum of one double per thread (NTH threads, red holds NTH / 64);
// the total is returned to thread 0.
template <int NTH = 256>
__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NTH / 64; ++w) t += red[w];
  }
  __syncthreads();
  return t;
}
__device__ __forceinline__ double block_sum_256(double v, double *red) { return block_sum<256>(v, red); }

}  // namespace m1dev
}  // namespace tn
