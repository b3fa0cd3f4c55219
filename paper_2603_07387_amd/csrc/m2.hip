// Acyclic-network estimator (Eq. (2), Algorithms 2-5) on gfx950.
//
// The tree is rooted at tensor o; for a non-root tensor the mode on its parent
// contraction plays the role of the first mode and its other modes (in mode
// order) lead to its children Gamma(k) (footnote of the rooted-tree notation).
// Each tensor k with children carries a recursive sketch R_k = Q_k S_k of order
// |Gamma(k)|, padded to the next power of two with index 0 of extra count
// sketches (footnote of Def. 13), whose S_k part is the children's count
// sketches C_{k,l}.  Sketches are built leaves to root (Algorithm 2).
//
// GPU formulation.  Write x_l = C_{k,l} w_l, where w_l = mat(X_l) R_l^T r_l is
// the child's n-vector (w_l = X_l for a leaf).  Then
//     r_k = Q_k (kron_l x_l) = R_k (kron_l w_l),
// so r_k is a scatter of the Kronecker product of the children's w over the
// child index space with the recursive-sketch hash (sign, row) of Algorithm 4,
// and the SMVP of Algorithm 5 is
//     w_k[i_1] = sum_{i_c} X_k(i_1, i_c) g[i_c],   g[i_c] = sigma(i_c) r_k[b(i_c)],
// a dense matrix product with the same (b, sigma).  For many samples the second
// step is one GEMM per tensor: mat(X_k) [rows x cols] times G [cols x samples].
// The root is the same product with one row: y = sum_i X_o(i) sigma(i) r_o[b(i)]
// = (R_o vec X_o)^T r_o.
//
// Kernels, one pair per tree depth (deepest first), every tensor of that depth
// of every network in the plan in one launch:
//   m2_gather : block per (tensor, sample): hash tables of its children in LDS,
//               scatter of the children's Kronecker products into an LDS
//               fixed-point sketch r_k, then the gather g over the child index
//               space, written to HBM.
//   m2_gemm16 : w_k = mat(X_k) G over all samples of the chunk on the FP64
//               matrix cores (operands widened exactly, FP64 accumulation),
//               blocks of 64 rows x 64 samples staged through LDS; on levels
//               with few tiles the columns are split over blocks and the FP64
//               partials summed in a fixed order by m2_reduce.
#include <algorithm>
#include <mutex>
#include <new>
#include <queue>
#include <type_traits>
#include <vector>

#include "hash_device.h"
#include "plan.h"

namespace tn {

constexpr int kM2MaxChildren = 8;       // children per tensor (padded order <= 8)
constexpr int kM2MaxTableSum = 4096;    // sum of child mode sizes per tensor
constexpr int kM2MaxLog2M = 13;         // m <= 8192 (LDS sketch of 64 KB)

struct M2Node {
  int32_t tensor;   // global tensor index (data pointer)
  int32_t net;
  int32_t local;    // tensor index within its network (stream ids)
  int32_t root;
  int32_t rows;     // size of the parent contraction (1 for the root)
  int32_t nchild;
  int32_t qt;       // padded order: next power of two >= nchild
  int32_t depth;
  int64_t ncols;    // product of the child mode sizes
  int64_t after;    // X viewed as [ncols / after][rows][after]
  int64_t g_off;    // offset of g within a sample's row of the level buffer
  int64_t w_off;    // offset of w within a sample's w row (non-root with children)
  uint64_t seed;
  int64_t parent_edge;  // non-root: stream id of the parent contraction
  int64_t parent_tab;   // its table offset
  int64_t t_tab;        // table offset of the tensor-sketch streams (level-major)
  int32_t child_dim[kM2MaxChildren];
  int32_t child_tensor[kM2MaxChildren];  // leaf child: its global tensor; else -1
  int64_t child_w_off[kM2MaxChildren];   // non-leaf child: offset of its w
  int64_t child_edge[kM2MaxChildren];    // stream id of the child contraction
  int64_t child_tab[kM2MaxChildren];     // its table offset
  int64_t pad_tab[kM2MaxChildren];       // table offset of padding slot j (j >= nchild)
  int32_t child_tile0[kM2MaxChildren];   // non-leaf child: its first row tile within its depth
};

struct M2Tile {
  int32_t node;  // index into the node array
  int32_t row0;
};

struct M2Plan {
  std::vector<M2Node> h_nodes;
  M2Node *d_nodes = nullptr;
  std::vector<std::vector<int32_t>> level_nodes;  // per depth: nodes with children
  std::vector<std::vector<M2Tile>> level_tiles;
  std::vector<int64_t> level_maxcols;             // per depth: widest node
  std::vector<int32_t> level_splits;              // per depth: column ranges of the FP64 product
  std::vector<int32_t> level_kcols;               // per depth: columns per range
  double *d_part = nullptr;                       // column-split partials (largest level)
  std::vector<char> level_fuse;                   // per depth: the parents' gathers sum its partials
  uint32_t *d_ltab = nullptr;                     // slot tables: [tensor of all_nodes][sample][tcap]
  std::vector<int32_t> all_nodes;                 // tensors with children, depth by depth
  std::vector<int64_t> level_off;                 // per depth: its first position in all_nodes
  int32_t *d_all_nodes = nullptr;
  std::vector<int32_t *> d_level_nodes;
  std::vector<M2Tile *> d_level_tiles;
  int64_t g_row = 0;    // entries of g per sample (max over depths)
  int64_t w_row = 0;    // entries of w per sample
  void *d_g = nullptr;  // [chunk][g_row]
  void *d_w = nullptr;  // [chunk][w_row]
  double *d_r = nullptr;  // root sketches for export: [chunk][n_nets][m]
  int64_t chunk = 0;
  int32_t tcap = 4;     // slot-table entries per tensor (max over tensors, multiple of 2)
  std::vector<int32_t> node_of_tensor;  // global tensor -> node index
  int32_t split_target = 512;   // blocks a product level aims for with its column split
  int32_t gather_target = 0;    // blocks a gather level aims for (0: the kernel's default)
};

namespace {


template <typename T>
__device__ __forceinline__ double load_val(const void *p, int64_t i);
template <>
__device__ __forceinline__ double load_val<double>(const void *p, int64_t i) {
  return reinterpret_cast<const double *>(p)[i];
}
template <>
__device__ __forceinline__ double load_val<float>(const void *p, int64_t i) {
  return (double)reinterpret_cast<const float *>(p)[i];
}
template <>
__device__ __forceinline__ double load_val<uint16_t>(const void *p, int64_t i) {
  return (double)__uint_as_float(((uint32_t)reinterpret_cast<const uint16_t *>(p)[i]) << 16);
}

__device__ __forceinline__ uint32_t sum_packed(uint32_t a, uint32_t b, uint32_t mask) {
  return (((a & 0x7fffffffu) + (b & 0x7fffffffu)) & mask) | ((a ^ b) & 0x80000000u);
}

// Packed value of tensor sketch T_{tix}, side d, at an m-valued index: from the
// injected tables or evaluated from the hash coefficients.
__device__ __forceinline__ uint32_t tsketch(const M2Node &nd, const int32_t *tab,
                                            const HashCoeffs *coef, int c, uint32_t m,
                                            uint32_t mask, int tix, int d, uint32_t idx) {
  if (tab) return (uint32_t)tab[nd.t_tab + (int64_t)(2 * tix + d) * m + idx];
  return hash_packed(coef[c + 2 * tix + d], idx, mask);
}

// Both passes over the child index space of one (tensor, sample) for padded
// order QT: the scatter r_k = R_k (kron_l w_l) into the fixed-point LDS sketch,
// then the gather g[col] = sigma(col) r_k[b(col)].  A thread walks columns
// col = tid + 256 i; the child index tuple (row-major over the children, the
// last child fastest) advances by the mixed-radix digits of 256, so the loop
// divides nothing and every array stays in registers.
// One value of g in its storage type G: A itself, or (G = uint16_t, BF16
// products) the BF16 bits of the value rounded to nearest even via FP32, which
// is the rounding the BF16 product applies to an A-typed g.
template <typename G, typename A>
__device__ __forceinline__ void store_g(G *g, size_t i, A v) {
  if constexpr (sizeof(G) == 2) {
    const __bf16 b = (__bf16)(float)v;
    g[i] = *reinterpret_cast<const uint16_t *>(&b);
  } else {
    g[i] = v;
  }
}

// AW: the fixed-point accumulator word (64-bit; 32-bit for BF16 g, see
// m2_gather_kernel).
template <typename A, typename G, int QT, typename AW>
__device__ __forceinline__ void gather_columns(const M2Node &nd, int c, const int32_t *tab_base,
                                               const uint32_t *dtab, const double *wv,
                                               AW *acc, const int32_t *tab,
                                               const HashCoeffs *coef, uint32_t mask, uint32_t m,
                                               double sc, double inv_sc, G *g) {
  const int tid = threadIdx.x;
  const uint32_t ncols = (uint32_t)nd.ncols;
  uint32_t dim[QT], step[QT], idx0[QT];
  int32_t tb[QT];
  {
    uint32_t col = (uint32_t)tid, st = 256u;
#pragma unroll
    for (int j = QT - 1; j >= 0; --j) {
      tb[j] = tab_base[j];
      if (j < c) {
        dim[j] = (uint32_t)nd.child_dim[j];
        idx0[j] = col % dim[j];
        col /= dim[j];
        step[j] = st % dim[j];
        st /= dim[j];
      } else {
        dim[j] = 1u;
        idx0[j] = 0u;
        step[j] = 0u;
      }
    }
    // the most significant digit absorbs what is left (it can exceed its
    // radix only once the column is past the end)
    if (c > 0) {
      idx0[0] += col * dim[0];
      step[0] += st * dim[0];
    }
  }
  // Recursive-sketch hash (Algorithm 4) of a child index tuple.
  auto rs_hash = [&](const uint32_t *idx) -> uint32_t {
    uint32_t v[QT];
#pragma unroll
    for (int j = 0; j < QT; ++j) v[j] = dtab[tb[j] + (j < c ? (int32_t)idx[j] : 0)];
    if constexpr (QT == 1) {
      return v[0];
    } else {
      uint32_t b[QT / 2];
#pragma unroll
      for (int t = 0; t < QT / 2; ++t) b[t] = sum_packed(v[2 * t], v[2 * t + 1], mask);
#pragma unroll
      for (int l = QT / 2; l >= 2; l /= 2) {
#pragma unroll
        for (int t = 0; t < l / 2; ++t) {
          const int tix = QT - l + t;
          const uint32_t t0 = tsketch(nd, tab, coef, c, m, mask, tix, 0, b[2 * t] & 0x7fffffffu);
          const uint32_t t1 = tsketch(nd, tab, coef, c, m, mask, tix, 1, b[2 * t + 1] & 0x7fffffffu);
          const uint32_t sg = (b[2 * t] ^ b[2 * t + 1] ^ t0 ^ t1) & 0x80000000u;
          b[t] = (((t0 & 0x7fffffffu) + (t1 & 0x7fffffffu)) & mask) | sg;
        }
      }
      return b[0];
    }
  };
  auto advance = [&](uint32_t *idx) {
    uint32_t carry = 0u;
#pragma unroll
    for (int j = QT - 1; j >= 0; --j) {
      if (j < c) {
        const uint32_t v = idx[j] + step[j] + carry;
        carry = v >= dim[j] && j > 0 ? 1u : 0u;
        idx[j] = v - carry * dim[j];
      }
    }
  };
  const double kMagic = 6755399441055744.0;
  uint32_t idx[QT];
#pragma unroll
  for (int j = 0; j < QT; ++j) idx[j] = idx0[j];
  for (uint32_t col = (uint32_t)tid; col < ncols; col += 256u) {
    const uint32_t h = rs_hash(idx);
    double p = 1.0;
#pragma unroll
    for (int j = 0; j < QT; ++j)
      if (j < c) p *= wv[tb[j] + (int32_t)idx[j]];
    const long long v = __double_as_longlong(fma(p, sc, kMagic)) - __double_as_longlong(kMagic);
    atomicAdd(&acc[h & mask], (AW)((h & 0x80000000u) ? -v : v));
    advance(idx);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < QT; ++j) idx[j] = idx0[j];
  for (uint32_t col = (uint32_t)tid; col < ncols; col += 256u) {
    const uint32_t h = rs_hash(idx);
    const double r = (double)(std::make_signed_t<AW>)acc[h & mask] * inv_sc;
    store_g(g, col, (A)((h & 0x80000000u) ? -r : r));
    advance(idx);
  }
}

// Two children with the faster one of at most 256 values (the usual shape: a
// bond and a physical leg).  Thread t keeps i1 = t mod d1 for the whole pass and
// walks i0 = t / d1 + R k, R = floor(256 / d1), so the second child's table
// entry and w value stay in registers and a wave reads the first child's by
// broadcast; columns are i0 d1 + i1 as in gather_columns.  The sign of a column
// is folded into the product before the fixed-point conversion: fma rounds
// +x and -x symmetrically, so every sketch entry and every g value is bitwise
// that of gather_columns<A, G, 2>.
template <typename A, typename G, typename AW>
__device__ __forceinline__ void gather_pair(const M2Node &nd, const int32_t *tab_base, const uint32_t *dtab,
                                            const double *wv, AW *acc, uint32_t mask, double sc,
                                            double inv_sc, G *g) {
  const uint32_t tid = threadIdx.x;
  const uint32_t d0 = (uint32_t)nd.child_dim[0], d1 = (uint32_t)nd.child_dim[1];
  const uint32_t R = 256u / d1;
  const bool active = tid < R * d1;
  const uint32_t i1 = tid % d1, i0s = tid / d1;
  const uint32_t *t0 = dtab + tab_base[0];
  const double *w0 = wv + tab_base[0];
  const uint32_t v1 = active ? dtab[tab_base[1] + (int32_t)i1] : 0u;
  const uint32_t v1m = v1 & 0x7fffffffu;
  const double w1 = active ? wv[tab_base[1] + (int32_t)i1] : 0.0;
  const double kMagic = 6755399441055744.0;
  const long long kMagicBits = __double_as_longlong(kMagic);
  // U rows per step, their table and w reads issued before the dependent LDS
  // operations (the compiler cannot reorder them across the atomics itself:
  // both arrays live in the same LDS allocation).  Rows past d0 read row d0 - 1
  // and are dropped.
  constexpr int U = 4;
  if (active) {
    for (uint32_t i0 = i0s; i0 < d0; i0 += U * R) {
      uint32_t v0[U];
      double x0[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t ii = min(i0 + u * R, d0 - 1);
        v0[u] = t0[ii];
        x0[u] = w0[ii];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (i0 + u * R < d0) {
          const uint32_t b = ((v0[u] & 0x7fffffffu) + v1m) & mask;
          const long long sg = (long long)((v0[u] ^ v1) & 0x80000000u) << 32;
          const double p = __longlong_as_double(__double_as_longlong(x0[u] * w1) ^ sg);
          atomicAdd(&acc[b], (AW)(__double_as_longlong(fma(p, sc, kMagic)) - kMagicBits));
        }
      }
    }
  }
  __syncthreads();
  if (active) {
    for (uint32_t i0 = i0s; i0 < d0; i0 += U * R) {
      uint32_t v0[U];
      AW a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v0[u] = t0[min(i0 + u * R, d0 - 1)];
#pragma unroll
      for (int u = 0; u < U; ++u) a[u] = acc[((v0[u] & 0x7fffffffu) + v1m) & mask];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t ii = i0 + u * R;
        if (ii < d0) {
          const A r = (A)((double)(std::make_signed_t<AW>)a[u] * inv_sc);
          store_g(g, (size_t)ii * d1 + i1, ((v0[u] ^ v1) & 0x80000000u) ? -r : r);
        }
      }
    }
  }
}

// Hash coefficients of tensor nd for one sample: child contractions [0, c),
// tensor sketches [c, c + 2(qt-1)), padding slots after that; thread tid < c +
// 2(qt-1) + (qt-c) writes coef[tid].
// Stream id of coefficient slot j of tensor nd (layout as in node_coeffs).
__device__ __forceinline__ uint64_t node_stream(const M2Node &nd, int j) {
  const int c = nd.nchild, qt = nd.qt, n_t = 2 * (qt - 1);
  if (j < c) return (uint64_t)nd.child_edge[j];
  if (j < c + n_t) {
    const int k = j - c, tix = k >> 1, d = k & 1;
    // tix enumerates (level l, index j) level-major from l = qt: tix = qt - l + j
    int l = qt, base = 0;
    while (tix - base >= l / 2) { base += l / 2; l /= 2; }
    return (1ull << 62) + ((uint64_t)nd.local << 32) + ((uint64_t)l << 16) + (uint64_t)(2 * (tix - base) + d);
  }
  return (1ull << 63) + ((uint64_t)nd.local << 32) + (uint64_t)(c + j - c - n_t);
}

__device__ __forceinline__ void node_coeffs(const M2Node &nd, uint64_t sample, HashCoeffs *coef) {
  const int tid = threadIdx.x, c = nd.nchild, qt = nd.qt, n_t = 2 * (qt - 1);
  if (tid >= c + n_t + (qt - c)) return;
  coef[tid] = hash_coeffs(nd.seed, sample, node_stream(nd, tid));
}

// Level-one slot tables of every (tensor with children, sample): the child
// (or padding) count sketch of each slot, combined with the
// first tensor sketch of its pair when qt >= 2 (Algorithm 4's first level),
// packed as bucket | sign << 31.  out: [tensor of `list`][sample][tcap], `list`
// holding the tensors of every depth (the gather of depth d reads from its
// offset).  Computed apart from the gathers, in one launch per estimate, so
// that the serial hash arithmetic of one sample does not hold up the LDS work
// of another.
constexpr int kTabThreads = 256, kTabSamples = 32;  // samples per block

// One block per (tensor, run of kTabSamples samples): first the hash
// coefficients of every (sample, stream) pair, one per thread (a sample's pairs
// are few, so a block per sample left most lanes idle), then every slot-table
// entry of the run's samples.
__global__ __launch_bounds__(kTabThreads) void m2_tables_kernel(const M2Node *__restrict__ nodes,
                                                                const int32_t *__restrict__ list,
                                                                const int32_t *__restrict__ tables, int64_t W,
                                                                int64_t sample0, int64_t n_samples, int log2m,
                                                                uint32_t *__restrict__ out, int tcap) {
  constexpr int NCO = 3 * kM2MaxChildren;
  __shared__ HashCoeffs coef[kTabSamples][NCO];
  __shared__ int32_t base_of[kM2MaxChildren + 1];
  const M2Node &nd = nodes[list[blockIdx.x]];
  const int64_t s0 = (int64_t)blockIdx.y * kTabSamples;
  const int ns = (int)min((int64_t)kTabSamples, n_samples - s0);
  const int tid = threadIdx.x, c = nd.nchild, qt = nd.qt, n_t = 2 * (qt - 1);
  const int nco = c + n_t + (qt - c);
  const uint32_t m = 1u << log2m, mask = m - 1;
  if (!tables) {
    for (int i = tid; i < ns * nco; i += kTabThreads) {
      const int sl = i / nco, j = i - sl * nco;
      coef[sl][j] = hash_coeffs(nd.seed, (uint64_t)(sample0 + s0 + sl), node_stream(nd, j));
    }
  }
  if (tid == 0) {
    int b = 0;
    for (int j = 0; j < qt; ++j) {
      base_of[j] = b;
      b += j < c ? nd.child_dim[j] : 1;
    }
    base_of[qt] = b;
  }
  __syncthreads();
  const int n_ent = base_of[qt];
  for (int i = tid; i < ns * n_ent; i += kTabThreads) {
    const int sl = i / n_ent, e = i - sl * n_ent;
    int j = 0;
    while (e >= base_of[j + 1]) ++j;
    const int ii = e - base_of[j];
    const int64_t s = s0 + sl;
    const int32_t *tab = tables ? tables + s * W : nullptr;
    const HashCoeffs *cf = coef[sl];
    uint32_t v;
    if (j < c)
      v = tab ? (uint32_t)tab[nd.child_tab[j] + ii] : hash_packed(cf[j], (uint32_t)ii, mask);
    else
      v = tab ? (uint32_t)tab[nd.pad_tab[j]] : hash_packed(cf[c + n_t + (j - c)], 0u, mask);
    if (qt >= 2) {
      const uint32_t t = tsketch(nd, tab, cf, c, m, mask, j >> 1, j & 1, v & 0x7fffffffu);
      v = (t & 0x7fffffffu) | ((v ^ t) & 0x80000000u);
    }
    out[((int64_t)blockIdx.x * n_samples + s) * tcap + e] = v;
  }
}

// Sketches r_k and gathers g of tensor k for the samples blockIdx.y + i gridDim.y
// (see the file comment).  Per block, once: the slot-table bases and the leaf
// children's w (data vectors, the same for every sample) with their max |w|.
// Per sample: the slot tables (from m2_tables_kernel) and the non-leaf
// children's w, both loaded into registers during the previous sample's columns
// when they fit (at most kTPre table entries per thread; each non-leaf child at
// most 256 values and at most kWPre of them); the hash coefficients only when
// qt >= 4 (the column hash then evaluates the higher tensor-sketch levels); the
// fixed-point scale, the scatter and the gather.  With csplits > 0 the
// non-leaf child's w is the fixed-order sum of its product's csplits column
// partials (cpart: [split][tile of the child depth][sample][64], ctiles tiles),
// rounded to A as the partials' sum kernel would store it.
// A: storage type of w and g (float for FP32/BF16 data, double for FP64).
constexpr int kWPre = 4, kTPre = 2;
constexpr int kMaxSplit = 8;  // column ranges per product tile (products below)

// Byte offset of the gather's w values in its LDS (after the m accumulator
// words and the tcap slot-table words, 8-byte aligned), and its LDS size.
template <typename G>
__host__ __device__ constexpr size_t gather_wv_offset(uint32_t m, int tcap) {
  return ((size_t)m * (sizeof(G) == 2 ? 4 : 8) + (size_t)tcap * 4 + 7) & ~(size_t)7;
}
template <typename G>
constexpr size_t gather_lds(uint32_t m, int tcap) {
  return gather_wv_offset<G>(m, tcap) + (size_t)tcap * 8;
}

// PAIR: every node of the launch has two children, the second of at most 256
// values (the two-child loop only: fewer registers, more blocks per CU).
template <typename T, typename A, typename G, bool PAIR = false>
__global__ __launch_bounds__(256) void m2_gather_kernel(
    const M2Node *__restrict__ nodes, const int32_t *__restrict__ level, const void *const *data,
    const int32_t *__restrict__ tables, int64_t W, int64_t sample0, int64_t n_samples, int log2m,
    const uint32_t *__restrict__ ltab, int64_t ltab_off, const A *__restrict__ wbuf, int64_t w_row, G *__restrict__ gbuf,
    int64_t g_row, double *__restrict__ r_out, int64_t r_stride, int tcap, const double *__restrict__ cpart,
    int32_t csplits, int32_t ctiles) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ HashCoeffs coef[3 * kM2MaxChildren];
  __shared__ unsigned long long wmax[kM2MaxChildren], wmax_leaf[kM2MaxChildren];
  __shared__ int32_t tab_base[kM2MaxChildren + 1];

  const M2Node &nd = nodes[level[blockIdx.x]];
  const int tid = threadIdx.x;
  const uint32_t m = 1u << log2m, mask = m - 1;
  const int c = nd.nchild, qt = nd.qt;

  // Fixed-point accumulators: 64-bit words, or 32-bit ones when g is stored
  // as BF16 (the products' own rounding, 2^-9 relative, dwarfs the 32-bit
  // resolution of 2^-(30 - lgN) of the largest product): the faster 32-bit
  // atomic and half the LDS (gather 1.18 -> 1.11 ms per caterpillar step).
  using AW = std::conditional_t<sizeof(G) == 2, uint32_t, unsigned long long>;
  constexpr int kAccBits = sizeof(G) == 2 ? 30 : 62;
  AW *acc = reinterpret_cast<AW *>(smem);                                  // [m]
  uint32_t *dtab = reinterpret_cast<uint32_t *>(acc + m);                  // [tcap] slot tables
  double *wv = reinterpret_cast<double *>(smem + gather_wv_offset<G>(m, tcap));  // [tcap] children's w

  if (tid == 0) {
    int b = 0;
    for (int j = 0; j < qt; ++j) {
      tab_base[j] = b;
      b += j < c ? nd.child_dim[j] : 1;
    }
    tab_base[qt] = b;
  }
  if (tid < kM2MaxChildren) wmax_leaf[tid] = 0ull;
  __syncthreads();
  // leaf children: w is the data vector itself
  for (int j = 0; j < c; ++j) {
    if (nd.child_tensor[j] < 0) continue;
    const void *xd = data[nd.child_tensor[j]];
    double lm = 0.0;
    for (int i = tid; i < nd.child_dim[j]; i += 256) {
      const double x = load_val<T>(xd, i);
      wv[tab_base[j] + i] = x;
      lm = fmax(lm, fabs(x));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lm = fmax(lm, __shfl_xor(lm, off, 64));
    if ((tid & 63) == 0) atomicMax(&wmax_leaf[j], (unsigned long long)__double_as_longlong(lm));
  }
  __syncthreads();  // wmax_leaf complete before any thread copies it
  // non-leaf children eligible for the register prefetch
  int pre_j[kWPre];
  int n_pre = 0;
  bool pre_ok = true;
  for (int j = 0; j < c; ++j) {
    if (nd.child_tensor[j] >= 0) continue;
    if (n_pre == kWPre || nd.child_dim[j] > 256) {
      pre_ok = false;
      break;
    }
    pre_j[n_pre++] = j;
  }
  A pre[kWPre];
  double praw[kMaxSplit];
  uint32_t tpre[kTPre];
  const int n_ent = tab_base[qt];  // slot-table entries of this tensor
  const bool tpre_ok = n_ent <= 256 * kTPre;
  const uint32_t *ltab_node = ltab + (ltab_off + blockIdx.x) * n_samples * tcap;
  auto prefetch = [&](int64_t sp) {
    if (csplits > 0) {  // at most one non-leaf child (planner): its column partials
      if (n_pre > 0 && tid < nd.child_dim[pre_j[0]]) {
        const int64_t tile = nd.child_tile0[pre_j[0]] + (tid >> 6);
#pragma unroll
        for (int zz = 0; zz < kMaxSplit; ++zz)
          if (zz < csplits) praw[zz] = cpart[(((int64_t)zz * ctiles + tile) * n_samples + sp) * 64 + (tid & 63)];
      }
    } else {
#pragma unroll
      for (int q = 0; q < kWPre; ++q)
        if (pre_ok && q < n_pre && tid < nd.child_dim[pre_j[q]])
          pre[q] = wbuf[sp * w_row + nd.child_w_off[pre_j[q]] + tid];
    }
#pragma unroll
    for (int q = 0; q < kTPre; ++q)
      if (tpre_ok && tid + 256 * q < n_ent) tpre[q] = ltab_node[sp * tcap + tid + 256 * q];
  };

  const int64_t s_first = blockIdx.y, s_step = gridDim.y;
  if (s_first < n_samples) prefetch(s_first);
  // wmax holds the leaf maxima at the start of every sample (reset again at the
  // end of each sample, when nothing reads it, so no barrier is added).
  if (tid < kM2MaxChildren) wmax[tid] = wmax_leaf[tid];
  __syncthreads();
  for (int64_t s = s_first; s < n_samples; s += s_step) {
    const int32_t *tab = tables ? tables + s * W : nullptr;
    if (qt >= 4 && !tab) node_coeffs(nd, (uint64_t)(sample0 + s), coef);
    if constexpr (sizeof(AW) == 8) {  // clear the m words: 16-byte stores (and a last 8-byte word at m = 1)
      uint4 *a16 = reinterpret_cast<uint4 *>(acc);
      for (uint32_t i = tid; i < m / 2; i += 256) a16[i] = make_uint4(0u, 0u, 0u, 0u);
      if ((m & 1u) && tid == 0) acc[m - 1] = 0;
    } else {  // 32-bit words (BF16 g): 16-byte stores measured slower here
      for (uint32_t i = tid; i < m; i += 256) acc[i] = 0;
    }
    // Level-one slot tables.
    if (tpre_ok) {
#pragma unroll
      for (int q = 0; q < kTPre; ++q)
        if (tid + 256 * q < n_ent) dtab[tid + 256 * q] = tpre[q];
    } else {
      for (int i = tid; i < n_ent; i += 256) dtab[i] = ltab_node[s * tcap + i];
    }
    // Non-leaf children's w and their max |w|.
    if (pre_ok) {
#pragma unroll
      for (int q = 0; q < kWPre; ++q) {
        if (q >= n_pre) break;
        const int j = pre_j[q];
        double lm = 0.0;
        if (tid < nd.child_dim[j]) {
          double x;
          if (csplits > 0) {
            double v = 0.0;  // the partials' sum kernel's order
#pragma unroll
            for (int zz = 0; zz < kMaxSplit; ++zz)
              if (zz < csplits) v += praw[zz];
            x = (double)(A)v;
          } else {
            x = (double)pre[q];
          }
          wv[tab_base[j] + tid] = x;
          lm = fabs(x);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) lm = fmax(lm, __shfl_xor(lm, off, 64));
        if ((tid & 63) == 0) atomicMax(&wmax[j], (unsigned long long)__double_as_longlong(lm));
      }
    } else {
      for (int j = 0; j < c; ++j) {
        if (nd.child_tensor[j] >= 0) continue;
        double lm = 0.0;
        for (int i = tid; i < nd.child_dim[j]; i += 256) {
          const double x = (double)wbuf[s * w_row + nd.child_w_off[j] + i];
          wv[tab_base[j] + i] = x;
          lm = fmax(lm, fabs(x));
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) lm = fmax(lm, __shfl_xor(lm, off, 64));
        if ((tid & 63) == 0) atomicMax(&wmax[j], (unsigned long long)__double_as_longlong(lm));
      }
    }
    __syncthreads();
    if (s + s_step < n_samples) prefetch(s + s_step);  // in flight during the columns

    // Fixed-point scale: every product is below prod_j max|w_j| < 2^e; ncols terms.
    double pmax = 1.0;
    for (int j = 0; j < c; ++j) pmax *= __longlong_as_double((long long)wmax[j]);
    const int lgN = max(nd.ncols > 1 ? 64 - __clzll((unsigned long long)(nd.ncols - 1)) : 0, 11);
    int e = 0;
    if (pmax > 0.0) (void)frexp(pmax, &e);
    const double sc = ldexp(1.0, kAccBits - lgN - e);
    const double inv_sc = ldexp(1.0, -(kAccBits - lgN - e));

    G *g = gbuf + s * g_row + nd.g_off;
    if constexpr (PAIR) {
      gather_pair<A, G, AW>(nd, tab_base, dtab, wv, acc, mask, sc, inv_sc, g);
    } else {
    switch (qt) {
      case 1: gather_columns<A, G, 1, AW>(nd, c, tab_base, dtab, wv, acc, tab, coef, mask, m, sc, inv_sc, g); break;
      case 2:
        if (nd.child_dim[1] <= 256)
          gather_pair<A, G, AW>(nd, tab_base, dtab, wv, acc, mask, sc, inv_sc, g);
        else
          gather_columns<A, G, 2, AW>(nd, c, tab_base, dtab, wv, acc, tab, coef, mask, m, sc, inv_sc, g);
        break;
      case 4: gather_columns<A, G, 4, AW>(nd, c, tab_base, dtab, wv, acc, tab, coef, mask, m, sc, inv_sc, g); break;
      default: gather_columns<A, G, 8, AW>(nd, c, tab_base, dtab, wv, acc, tab, coef, mask, m, sc, inv_sc, g); break;
    }
    }
    if (r_out && nd.root) {
      for (uint32_t b = tid; b < m; b += 256)
        r_out[s * r_stride + (int64_t)nd.net * m + b] = (double)(std::make_signed_t<AW>)acc[b] * inv_sc;
    }
    if (tid < kM2MaxChildren) wmax[tid] = wmax_leaf[tid];
    __syncthreads();  // acc, coef, the tables and wmax are rewritten for the next sample
  }
}

// ---------------------------------------------------------------------------
// w_k = mat(X_k) G: operand loads shared by the matrix-core products below.
typedef float gf32x4 __attribute__((ext_vector_type(4)));
typedef double gf64x2 __attribute__((ext_vector_type(2)));
typedef unsigned short gu16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 gbf16x8 __attribute__((ext_vector_type(8)));
typedef float gf32x4acc __attribute__((ext_vector_type(4)));
#define TN_GLOBAL __attribute__((address_space(1)))

// W consecutive values as loaded (16 B of FP32, 8 B of BF16, 16 B of FP64),
// widened to FP64 only when used.
template <typename T>
struct RawW;
template <>
struct RawW<float> {
  static constexpr int W = 4;
  gf32x4 v;
  __device__ __forceinline__ void load(const void *base, int64_t off) {
    v = *((const TN_GLOBAL gf32x4 *)(reinterpret_cast<const float *>(base) + off));
  }
  __device__ __forceinline__ void set(int i, const void *base, int64_t off) {
    v[i] = reinterpret_cast<const float *>(base)[off];
  }
  __device__ __forceinline__ double get(int i) const { return (double)v[i]; }
};
template <>
struct RawW<double> {
  static constexpr int W = 2;
  gf64x2 v;
  __device__ __forceinline__ void load(const void *base, int64_t off) {
    v = *((const TN_GLOBAL gf64x2 *)(reinterpret_cast<const double *>(base) + off));
  }
  __device__ __forceinline__ void set(int i, const void *base, int64_t off) {
    v[i] = reinterpret_cast<const double *>(base)[off];
  }
  __device__ __forceinline__ double get(int i) const { return v[i]; }
};
template <>
struct RawW<uint16_t> {
  static constexpr int W = 4;
  gu16x4 v;
  __device__ __forceinline__ void load(const void *base, int64_t off) {
    v = *((const TN_GLOBAL gu16x4 *)(reinterpret_cast<const uint16_t *>(base) + off));
  }
  __device__ __forceinline__ void set(int i, const void *base, int64_t off) {
    v[i] = reinterpret_cast<const uint16_t *>(base)[off];
  }
  __device__ __forceinline__ double get(int i) const { return (double)__uint_as_float((uint32_t)v[i] << 16); }
};


// ---------------------------------------------------------------------------
// The product on v_mfma_f64_16x16x4f64 (A[i][k] in lane i + 16k, B[k][j] in
// lane j + 16k, D[i][j] as element i / 4 of lane j + 16 (i % 4)); with
// kProdBF16 (TN_FLAG_MFMA_BF16) on v_mfma_f32_16x16x32_bf16 (A[i][k] in lane
// i + 16 (k / 8) element k % 8, B[k][j] in lane j + 16 (k / 8) element k % 8,
// D[i][j] in lane j + 16 (i / 4) item i % 4), operands rounded to BF16, FP32
// accumulation; with kProdF32 (TN_FLAG_MFMA_F32) on v_mfma_f32_16x16x4f32
// (A and B as for FP64, D as for BF16), FP32 operands (exact for FP32 and BF16
// data and for g, which is stored in FP32), FP32 accumulation.  The same
// staging, partials and reduction in FP64 for all three.  A block of four
// waves owns 64 rows x 64 samples and a column range; each wave a 32 x 32 corner
// (2 x 2 accumulators of 16 x 16).  Per chunk of 16 W columns the block stages the
// X rows and the G rows in double-buffered LDS, one 16-byte vector (W columns) per
// (row, slot), with the next chunk's global loads in flight during the matrix
// instructions.  Lane (i, kk) takes slots kk + 4q: column W (kk + 4q) + e of the
// chunk enters instruction (q, e) at contraction index kk, so every column of
// the chunk is summed once.  The 64 x 64 result goes through LDS to coalesced
// stores: FP64 partials [split][tile][sample][64] when the columns are split,
// else w or the estimates.
constexpr int kG16Rows = 64, kG16Samples = 64, kG16Threads = 256, kG16Pad = 17;
constexpr int kProdF64 = 0, kProdBF16 = 1, kProdF32 = 2;  // matrix-core product precision

template <typename T, typename A>
constexpr size_t g16_lds_bytes() {  // T: X data, A: g storage
  constexpr size_t tiles = (size_t)2 * kG16Pad * (kG16Rows * sizeof(RawW<T>) + kG16Samples * sizeof(RawW<A>));
  constexpr size_t outb = (size_t)kG16Samples * (kG16Rows + 1) * sizeof(double);
  return tiles > outb ? tiles : outb;
}

// G: storage type of g (A, or BF16 bits with kProdBF16).
template <typename T, typename A, typename G, int PM>
__global__ __launch_bounds__(kG16Threads) void m2_gemm16_kernel(
    const M2Node *__restrict__ nodes, const M2Tile *__restrict__ tiles, int32_t n_tiles,
    const void *const *data, const G *__restrict__ gbuf, int64_t g_row, int64_t samples,
    A *__restrict__ wbuf, int64_t w_row, double *__restrict__ est, int64_t S, int64_t sample0,
    int32_t kcols, double *__restrict__ part) {
  constexpr int W = RawW<T>::W;
  static_assert(RawW<G>::W == W, "operand widths differ");
  static_assert(PM == kProdBF16 || sizeof(G) == sizeof(A), "BF16 g only with BF16 products");
  constexpr bool BF = PM == kProdBF16;
  constexpr int32_t CC = 16 * W;  // columns per chunk
  constexpr int ROWV = kG16Pad;   // vectors per LDS row (16 + 1 pad)
  using V = RawW<T>;
  using VA = RawW<G>;
  extern __shared__ __align__(16) unsigned char g16_smem[];
  V *Xs = reinterpret_cast<V *>(g16_smem);                                     // [2][64][ROWV]
  VA *Gs = reinterpret_cast<VA *>(g16_smem + (size_t)2 * kG16Rows * ROWV * sizeof(V));  // [2][64][ROWV]
  const M2Tile tl = tiles[blockIdx.x];
  const M2Node &nd = nodes[tl.node];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, ws = wave >> 1;
  const int li = lane & 15, kk = lane >> 4;
  const int64_t rows = nd.rows, after = nd.after;
  const int32_t ncols = (int32_t)nd.ncols;
  const int64_t s_base = (int64_t)blockIdx.y * kG16Samples;
  const void *X = data[nd.tensor];
  const int32_t c_begin = (int32_t)blockIdx.z * kcols;
  const int32_t c_end = min(ncols, c_begin + kcols);
  // loads: slot lv of rows / samples lr + 16 p, p = 0..3
  const int lv = tid & 15, lr = tid >> 4;
  bool xok[4], gok[4];
  const G *grow[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    xok[p] = (int64_t)tl.row0 + lr + 16 * p < rows;
    gok[p] = s_base + lr + 16 * p < samples;
    grow[p] = gbuf + (gok[p] ? s_base + lr + 16 * p : 0) * g_row + nd.g_off;
  }
  const bool vec = (after % W) == 0 &&
                   (reinterpret_cast<uintptr_t>(X) & (uintptr_t)(W * sizeof(T) - 1)) == 0;
  const int32_t after32 = (int32_t)after;
  int32_t c = c_begin + W * lv;
  int32_t qd = c / after32, rm = c - qd * after32;
  const int32_t stepq = CC / after32, stepr = CC - stepq * after32;
  V xreg[4];
  VA greg[4];
  auto load_chunk = [&]() {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      xreg[p] = V{};
      greg[p] = VA{};
    }
    const int64_t x0 = ((int64_t)qd * rows + tl.row0 + lr) * after + rm;
    if (vec && c + W - 1 < c_end) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        if (xok[p]) xreg[p].load(X, x0 + 16 * p * after);
        if (gok[p]) greg[p].load(grow[p], c);
      }
    } else {
#pragma unroll
      for (int e = 0; e < W; ++e) {
        const int32_t ce = c + e;
        if (ce < c_end) {
          const int32_t qe = ce / after32;
          const int64_t xe = ((int64_t)qe * rows + tl.row0 + lr) * after + (ce - qe * after32);
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            if (xok[p]) xreg[p].set(e, X, xe + 16 * p * after);
            if (gok[p]) greg[p].set(e, grow[p], ce);
          }
        }
      }
    }
  };
  auto next_chunk = [&]() {
    c += CC;
    qd += stepq;
    rm += stepr;
    if (rm >= after32) { rm -= after32; ++qd; }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      Xs[((size_t)buf * kG16Rows + lr + 16 * p) * ROWV + lv] = xreg[p];
      Gs[((size_t)buf * kG16Samples + lr + 16 * p) * ROWV + lv] = greg[p];
    }
  };
  typedef double d4 __attribute__((ext_vector_type(4)));
  using Acc = typename std::conditional<PM == kProdF64, d4, gf32x4acc>::type;
  Acc acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = Acc{0, 0, 0, 0};
  int buf = 0;
  if (c_begin < c_end) {
    load_chunk();
    store_chunk(0);
  }
  __syncthreads();
  for (int32_t cb = c_begin; cb < c_end; cb += CC) {
    const bool more = cb + CC < c_end;  // the same in every thread
    if (more) {
      next_chunk();
      load_chunk();
    }
    const V *xb = Xs + ((size_t)buf * kG16Rows + wr * 32 + li) * ROWV + kk;
    const VA *gbp = Gs + ((size_t)buf * kG16Samples + ws * 32 + li) * ROWV + kk;
    if constexpr (BF) {
      // k-step st of 32 columns: lane (i, kk) packs its 8 / W vectors
      // kk + 4 (v + (8 / W) st), W values each, as elements 0..7 (contraction
      // index 8 kk + element), rounded to BF16 to nearest even via FP32.
      constexpr int NV = 8 / W;
#pragma unroll
      for (int st = 0; st < W / 2; ++st) {
        gbf16x8 xa[2], gv[2];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const int slot = 4 * (v + NV * st);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const V xv = xb[16 * ROWV * h + slot];
            const VA yv = gbp[16 * ROWV * h + slot];
#pragma unroll
            for (int e = 0; e < W; ++e) {
              xa[h][v * W + e] = (__bf16)(float)xv.get(e);
              gv[h][v * W + e] = (__bf16)(float)yv.get(e);
            }
          }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[a], gv[b], acc[a][b], 0, 0, 0);
      }
    } else if constexpr (PM == kProdF32) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const V a0 = xb[4 * q], a1 = xb[16 * ROWV + 4 * q];
        const VA b0 = gbp[4 * q], b1 = gbp[16 * ROWV + 4 * q];
#pragma unroll
        for (int e = 0; e < W; ++e) {
          const float x0 = (float)a0.get(e), x1 = (float)a1.get(e), y0 = (float)b0.get(e), y1 = (float)b1.get(e);
          acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(x0, y0, acc[0][0], 0, 0, 0);
          acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(x0, y1, acc[0][1], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(x1, y0, acc[1][0], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(x1, y1, acc[1][1], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const V a0 = xb[4 * q], a1 = xb[16 * ROWV + 4 * q];
        const VA b0 = gbp[4 * q], b1 = gbp[16 * ROWV + 4 * q];
#pragma unroll
        for (int e = 0; e < W; ++e) {
          const double x0 = a0.get(e), x1 = a1.get(e), y0 = b0.get(e), y1 = b1.get(e);
          acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y0, acc[0][0], 0, 0, 0);
          acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, y1, acc[0][1], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y0, acc[1][0], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, y1, acc[1][1], 0, 0, 0);
        }
      }
    }
    if (more) store_chunk(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // result tile through LDS (the operand buffers are free after the last barrier):
  // out[sample][row], row stride 65 doubles
  double *out = reinterpret_cast<double *>(g16_smem);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        out[(ws * 32 + b * 16 + li) * (kG16Rows + 1) + wr * 32 + a * 16 + (PM == kProdF64 ? kk + 4 * r : 4 * kk + r)] =
            (double)acc[a][b][r];
  __syncthreads();
  const int orl = tid & 63;  // tile row
  const int64_t orow = (int64_t)tl.row0 + orl;
  if (orow >= rows) return;
  for (int sl = tid >> 6; sl < kG16Samples; sl += kG16Threads / 64) {
    const int64_t smp = s_base + sl;
    if (smp >= samples) break;
    const double v = out[sl * (kG16Rows + 1) + orl];
    if (part)
      part[(((int64_t)blockIdx.z * n_tiles + blockIdx.x) * samples + smp) * kG16Rows + orl] = v;
    else if (nd.root)
      est[(int64_t)nd.net * S + sample0 + smp] = v;
    else
      wbuf[smp * w_row + nd.w_off + orow] = (A)v;
  }
}

// Roots (one row): y = sum_col X_o[col] g[col] per sample, a dot product bound
// by the reads of g, on the vector units in FP64.  Block: four waves, one
// sample each; a lane takes the vectors of W columns W lane + 64 W i,
// then the columns past the last full vector one by one; the wave sums its lanes
// with a fixed xor tree, so the result does not depend on timing.
constexpr int kRootSamples = 4;

template <typename T, typename A>
__global__ __launch_bounds__(256) void m2_root_kernel(const M2Node *__restrict__ nodes,
                                                      const M2Tile *__restrict__ tiles,
                                                      const void *const *data, const A *__restrict__ gbuf,
                                                      int64_t g_row, int64_t samples, double *__restrict__ est,
                                                      int64_t S, int64_t sample0) {
  constexpr int W = RawW<T>::W;
  const M2Node &nd = nodes[tiles[blockIdx.x].node];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t ncols = (int32_t)nd.ncols;
  const void *X = data[nd.tensor];
  const bool vec = (reinterpret_cast<uintptr_t>(X) & (uintptr_t)(W * sizeof(T) - 1)) == 0;
  const int32_t nvec = vec ? ncols / W : 0;  // full vectors; columns from W nvec on are scalar
  for (int k = 0; k < kRootSamples / 4; ++k) {
    const int64_t smp = (int64_t)blockIdx.y * kRootSamples + wave * (kRootSamples / 4) + k;
    if (smp >= samples) break;  // the same in every lane of the wave
    const A *g = gbuf + smp * g_row + nd.g_off;
    double acc = 0.0;
    for (int32_t v = lane; v < nvec; v += 64) {
      RawW<T> x;
      RawW<A> y;
      x.load(X, (int64_t)v * W);
      y.load(g, (int64_t)v * W);
#pragma unroll
      for (int e = 0; e < W; ++e) acc = fma(x.get(e), y.get(e), acc);
    }
    for (int32_t col = W * nvec + lane; col < ncols; col += 64)
      acc = fma(load_val<T>(X, col), (double)g[col], acc);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) est[(int64_t)nd.net * S + sample0 + smp] = acc;
  }
}

// Fixed-order sum of the column-split partials of one level.
template <typename A>
__global__ __launch_bounds__(256) void m2_reduce_kernel(const M2Node *__restrict__ nodes,
                                                        const M2Tile *__restrict__ tiles, int32_t n_tiles,
                                                        int32_t splits, int64_t samples,
                                                        const double *__restrict__ part,
                                                        A *__restrict__ wbuf, int64_t w_row,
                                                        double *__restrict__ est, int64_t S,
                                                        int64_t sample0) {
  const M2Tile tl = tiles[blockIdx.x];
  const M2Node &nd = nodes[tl.node];
  const int rloc = threadIdx.x & 63;
  const int64_t smp = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6);
  const int64_t orow = (int64_t)tl.row0 + rloc;
  if (smp >= samples || orow >= nd.rows) return;
  double v = 0.0;
  for (int z = 0; z < splits; ++z) v += part[(((int64_t)z * n_tiles + blockIdx.x) * samples + smp) * kG16Rows + rloc];
  if (nd.root)
    est[(int64_t)nd.net * S + sample0 + smp] = v;
  else
    wbuf[smp * w_row + nd.w_off + orow] = (A)v;
}


// Export hook: x_k = C_{parent,k} w_k for non-root tensors (w_k = X_k for leaves).
template <typename T, typename A>
__global__ void m2_export_kernel(const M2Node *__restrict__ nodes, int32_t n_nodes,
                                 const void *const *data, const int32_t *__restrict__ tables,
                                 int64_t W, int64_t sample0, int log2m,
                                 const A *__restrict__ wbuf, int64_t w_row, int64_t n_tensors,
                                 double *__restrict__ out) {
  extern __shared__ __align__(16) unsigned char smem[];
  double *x = reinterpret_cast<double *>(smem);
  const M2Node nd = nodes[blockIdx.x];
  const int64_t s = blockIdx.y;
  const uint32_t m = 1u << log2m, mask = m - 1;
  if (nd.root) return;  // the root's slot is written by the gather kernel
  for (uint32_t b = threadIdx.x; b < m; b += blockDim.x) x[b] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    const HashCoeffs cf = hash_coeffs(nd.seed, (uint64_t)(sample0 + s), (uint64_t)nd.parent_edge);
    for (int i = 0; i < nd.rows; ++i) {
      const uint32_t h = tables ? (uint32_t)tables[s * W + nd.parent_tab + i]
                                : hash_packed(cf, (uint32_t)i, mask);
      const double v = nd.nchild == 0 ? load_val<T>(data[nd.tensor], i)
                                      : (double)wbuf[s * w_row + nd.w_off + i];
      x[h & mask] += (h & 0x80000000u) ? -v : v;
    }
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < m; b += blockDim.x)
    out[(s * n_tensors + nd.tensor) * (int64_t)m + b] = x[b];
}

// G: storage type of g (BF16 bits for BF16 products on FP32 / BF16 data).
template <typename T, typename A, typename G>
int m2_run_t(tn_plan *p, hipStream_t st, int64_t c0, int64_t n, const int32_t *tables,
             double *est, double *export_out) {
  M2Plan *P = p->m2;
  const size_t lds = gather_lds<G>((uint32_t)p->m, P->tcap);
  auto gk = m2_gather_kernel<T, A, G>;
  auto gkp = m2_gather_kernel<T, A, G, true>;
  constexpr size_t g16 = g16_lds_bytes<T, G>();
  if (g16 > 65536) {
    if constexpr (sizeof(G) == sizeof(A)) {
      TN_HIP_CHECK(hipFuncSetAttribute((const void *)m2_gemm16_kernel<T, A, G, kProdF64>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)g16));
      TN_HIP_CHECK(hipFuncSetAttribute((const void *)m2_gemm16_kernel<T, A, G, kProdF32>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)g16));
    }
    TN_HIP_CHECK(hipFuncSetAttribute((const void *)m2_gemm16_kernel<T, A, G, kProdBF16>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)g16));
  }
  if (lds > 65536) {
    TN_HIP_CHECK(hipFuncSetAttribute((const void *)gk, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds));
    TN_HIP_CHECK(hipFuncSetAttribute((const void *)gkp, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds));
  }
  if (!P->all_nodes.empty()) {
    hipEvent_t ev = nullptr;
    int rc;
    if ((rc = prof_begin(p, st, &ev, TN_KERNEL_HASH)) != TN_OK) return rc;
    hipLaunchKernelGGL(m2_tables_kernel, dim3((unsigned)P->all_nodes.size(), (unsigned)((n + kTabSamples - 1) / kTabSamples)),
                       dim3(kTabThreads), 0, st,
                       P->d_nodes, P->d_all_nodes, tables, p->W, c0, n, p->log2m, P->d_ltab, P->tcap);
    TN_HIP_CHECK(hipGetLastError());
    if ((rc = prof_end(p, st, TN_KERNEL_HASH, ev)) != TN_OK) return rc;
  }
  for (int d = (int)P->level_nodes.size() - 1; d >= 0; --d) {
    if (P->level_nodes[(size_t)d].empty()) continue;
    hipEvent_t ev = nullptr;
    int rc;
    if ((rc = prof_begin(p, st, &ev, TN_KERNEL_COMBINE)) != TN_OK) return rc;
    // the children's depth left its products as column partials: summed here
    const bool cfuse = !export_out && (size_t)d + 1 < P->level_fuse.size() && P->level_fuse[(size_t)d + 1];
    // Every node of the depth with two children, the second of at most 256
    // values: the two-child kernel (74-80 registers against 116-123).
    bool pair = true;
    for (int32_t i : P->level_nodes[(size_t)d]) {
      const M2Node &nd = P->h_nodes[(size_t)i];
      pair = pair && nd.nchild == 2 && nd.child_dim[1] <= 256;
    }
    // Samples per block: about 1024 blocks per level (four resident per CU;
    // six for the two-child kernel with BF16 g's 32-bit sketches).
    const int64_t nn = (int64_t)P->level_nodes[(size_t)d].size();
    const int64_t target = P->gather_target > 0 ? P->gather_target : (pair && sizeof(G) == 2 ? 1536 : 1024);
    const int64_t gy = std::max<int64_t>(1, std::min<int64_t>(n, (target + nn - 1) / nn));
    dim3 g1((unsigned)nn, (unsigned)gy);
    hipLaunchKernelGGL(pair ? gkp : gk, g1, dim3(256), lds, st, P->d_nodes, P->d_level_nodes[(size_t)d],
                       (const void *const *)p->d_data, tables, p->W, c0, n, p->log2m, P->d_ltab, P->level_off[(size_t)d],
                       reinterpret_cast<const A *>(P->d_w), P->w_row,
                       reinterpret_cast<G *>(P->d_g), P->g_row,
                       export_out ? P->d_r : nullptr, (int64_t)p->n_nets * p->m, P->tcap,
                       P->d_part, cfuse ? P->level_splits[(size_t)d + 1] : 0,
                       cfuse ? (int32_t)P->level_tiles[(size_t)d + 1].size() : 0);
    TN_HIP_CHECK(hipGetLastError());
    if ((rc = prof_end(p, st, TN_KERNEL_COMBINE, ev)) != TN_OK) return rc;
    if ((rc = prof_begin(p, st, &ev, TN_KERNEL_SKETCH)) != TN_OK) return rc;
    const void *const *dp = (const void *const *)p->d_data;
    const G *gb = reinterpret_cast<const G *>(P->d_g);
    A *wb = reinterpret_cast<A *>(P->d_w);
    const M2Tile *tl = P->d_level_tiles[(size_t)d];
    const bool bf = (p->flags & TN_FLAG_MFMA_BF16) != 0;
    if (d == 0 && !bf) {  // roots only, one row each (g in A: without BF16 products)
      if constexpr (sizeof(G) == sizeof(A)) {
        dim3 g3((unsigned)P->level_tiles[0].size(), (unsigned)((n + kRootSamples - 1) / kRootSamples));
        hipLaunchKernelGGL((m2_root_kernel<T, A>), g3, dim3(256), 0, st, P->d_nodes, tl, dp, gb, P->g_row, n, est,
                           p->S, c0);
      }
    } else {
      const int32_t nt = (int32_t)P->level_tiles[(size_t)d].size();
      const int32_t z = P->level_splits[(size_t)d];
      dim3 g4((unsigned)nt, (unsigned)((n + kG16Samples - 1) / kG16Samples), (unsigned)z);
      double *part = z > 1 ? P->d_part : nullptr;
      if constexpr (sizeof(G) != sizeof(A)) {  // BF16 g: BF16 products only
        hipLaunchKernelGGL((m2_gemm16_kernel<T, A, G, kProdBF16>), g4, dim3(kG16Threads), g16, st, P->d_nodes, tl,
                           nt, dp, gb, P->g_row, n, wb, P->w_row, est, p->S, c0, P->level_kcols[(size_t)d], part);
      } else {
        if (bf)
          hipLaunchKernelGGL((m2_gemm16_kernel<T, A, G, kProdBF16>), g4, dim3(kG16Threads), g16, st, P->d_nodes,
                             tl, nt, dp, gb, P->g_row, n, wb, P->w_row, est, p->S, c0, P->level_kcols[(size_t)d],
                             part);
        else if (p->flags & TN_FLAG_MFMA_F32)
          hipLaunchKernelGGL((m2_gemm16_kernel<T, A, G, kProdF32>), g4, dim3(kG16Threads), g16, st, P->d_nodes,
                             tl, nt, dp, gb, P->g_row, n, wb, P->w_row, est, p->S, c0, P->level_kcols[(size_t)d],
                             part);
        else
          hipLaunchKernelGGL((m2_gemm16_kernel<T, A, G, kProdF64>), g4, dim3(kG16Threads), g16, st, P->d_nodes,
                             tl, nt, dp, gb, P->g_row, n, wb, P->w_row, est, p->S, c0, P->level_kcols[(size_t)d],
                             part);
      }
      TN_HIP_CHECK(hipGetLastError());
      if ((rc = prof_end(p, st, TN_KERNEL_SKETCH, ev)) != TN_OK) return rc;
      if (z > 1 && !(P->level_fuse[(size_t)d] && !export_out)) {  // the partials' sum is timed with the gathers
        if ((rc = prof_begin(p, st, &ev, TN_KERNEL_COMBINE)) != TN_OK) return rc;
        dim3 g5((unsigned)nt, (unsigned)((n + 3) / 4));
        hipLaunchKernelGGL((m2_reduce_kernel<A>), g5, dim3(256), 0, st, P->d_nodes, tl, nt, z, n, part, wb,
                           P->w_row, est, p->S, c0);
        TN_HIP_CHECK(hipGetLastError());
        if ((rc = prof_end(p, st, TN_KERNEL_COMBINE, ev)) != TN_OK) return rc;
      }
      continue;
    }
    TN_HIP_CHECK(hipGetLastError());
    if ((rc = prof_end(p, st, TN_KERNEL_SKETCH, ev)) != TN_OK) return rc;
  }
  if (export_out) {
    dim3 g3((unsigned)P->h_nodes.size(), (unsigned)n);
    hipLaunchKernelGGL((m2_export_kernel<T, A>), g3, dim3(256), (size_t)p->m * 8, st, P->d_nodes,
                       (int32_t)P->h_nodes.size(), (const void *const *)p->d_data, tables, p->W,
                       c0, p->log2m, reinterpret_cast<const A *>(P->d_w), P->w_row, p->n_tensors,
                       export_out);
    TN_HIP_CHECK(hipGetLastError());
  }
  return TN_OK;
}

int m2_run(tn_plan *p, hipStream_t st, int64_t c0, int64_t n, double *est, double *export_out) {
  const int32_t *tables = p->d_injected ? p->d_injected + c0 * p->W : nullptr;
  switch (p->dtype) {
    case TN_F64: return m2_run_t<double, double, double>(p, st, c0, n, tables, est, export_out);
    case TN_F32:
      return (p->flags & TN_FLAG_MFMA_BF16) ? m2_run_t<float, float, uint16_t>(p, st, c0, n, tables, est, export_out)
                                            : m2_run_t<float, float, float>(p, st, c0, n, tables, est, export_out);
    default:
      return (p->flags & TN_FLAG_MFMA_BF16)
                 ? m2_run_t<uint16_t, float, uint16_t>(p, st, c0, n, tables, est, export_out)
                 : m2_run_t<uint16_t, float, float>(p, st, c0, n, tables, est, export_out);
  }
}

template <typename V>
int upload_vec(V **ptr, const std::vector<V> &v) {
  *ptr = nullptr;
  if (v.empty()) return TN_OK;
  hipError_t e = hipMalloc((void **)ptr, v.size() * sizeof(V));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return set_error(TN_ERR_OOM, "hipMalloc(%zu bytes)", v.size() * sizeof(V));
  }
  TN_HIP_CHECK(hipMemcpy(*ptr, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice));
  return TN_OK;
}

}  // namespace

constexpr int32_t kSplitTargetMax = 2048;

// Column split of the products: a level with few 64 x 64 tiles spreads its
// columns over up to 8 blocks per tile, towards `target` blocks (512 by
// default: two per CU), each range still at least 8 chunks of 16 W columns.
// Returns the partials buffer this needs, [splits][tiles][chunk][64] doubles
// (below target x 2 x 64 x 64 entries: blocks x splits < target).  A split depth
// d >= 1 is consumed as partials by the gathers of depth d - 1 when each parent
// there has at most one non-leaf child, of at most 256 values (it is then loaded
// into registers ahead of its sample).
size_t m2_schedule(tn_plan *p, int32_t target) {
  M2Plan *P = p->m2;
  const int64_t chunk = P->chunk;
  const int64_t cc = p->dtype == TN_F64 ? 32 : 64;
  size_t part = 0;
  P->split_target = target;
  P->level_splits.assign(P->level_tiles.size(), 1);
  P->level_kcols.assign(P->level_tiles.size(), 0);
  for (size_t d = 0; d < P->level_tiles.size(); ++d) {
    const int64_t tiles = (int64_t)P->level_tiles[d].size();
    if (tiles == 0) continue;
    const int64_t blocks = tiles * ((chunk + kG16Samples - 1) / kG16Samples);
    const int64_t maxc = P->level_maxcols[d];
    int32_t z = 1;
    while (z < kMaxSplit && blocks * z < target && maxc >= 16 * cc * z) z *= 2;
    const int64_t kc = ((maxc + z - 1) / z + cc - 1) / cc * cc;
    P->level_splits[d] = z;
    P->level_kcols[d] = (int32_t)kc;
    if (z > 1) part = std::max(part, (size_t)z * (size_t)tiles * (size_t)chunk * kG16Rows);
  }
  P->level_fuse.assign(P->level_tiles.size(), 0);
  for (size_t d = 1; d < P->level_tiles.size(); ++d) {
    if (P->level_splits[d] <= 1 || P->level_splits[d] > kMaxSplit) continue;
    bool ok = true;
    for (int32_t ni : P->level_nodes[d - 1]) {
      const M2Node &nd = P->h_nodes[(size_t)ni];
      int nl = 0;
      for (int i = 0; i < nd.nchild; ++i)
        if (nd.child_tensor[i] < 0) {
          ++nl;
          ok = ok && nd.child_dim[i] <= 256;
        }
      ok = ok && nl <= 1;
    }
    P->level_fuse[d] = ok ? 1 : 0;
  }
  return part;
}

int m2_build(tn_plan *p, const tn_network *nets, const std::vector<NetCheck> &chk) {
  if (p->log2m > kM2MaxLog2M)
    return set_error(TN_ERR_UNSUPPORTED, "acyclic method: m = %lld exceeds %d", (long long)p->m,
                     1 << kM2MaxLog2M);
  M2Plan *P = new (std::nothrow) M2Plan();
  if (!P) return set_error(TN_ERR_OOM, "host allocation");
  p->m2 = P;
  P->node_of_tensor.assign((size_t)p->n_tensors, -1);
  const size_t as = p->dtype == TN_F64 ? 8 : 4;
  int64_t gtensor = 0;
  std::vector<int64_t> level_cols;
  for (int j = 0; j < p->n_nets; ++j) {
    const tn_network &n = nets[j];
    const NetCheck &c = chk[(size_t)j];
    // streams: the contractions first (stream e, domain n_e)
    std::vector<int64_t> edge_tab((size_t)n.t);
    for (int e = 0; e < n.t; ++e) {
      StreamDesc sd{};
      sd.seed = p->seed + (uint64_t)j;
      sd.stream = (uint64_t)e;
      sd.offset = p->W;
      sd.n = (int32_t)n.dims[n.edges[2 * e]];
      sd.net = j;
      edge_tab[(size_t)e] = p->W;
      p->W += sd.n;
      p->h_streams.push_back(sd);
    }
    std::vector<int> partner((size_t)c.q, -1);
    for (int e = 0; e < n.t; ++e) {
      partner[(size_t)n.edges[2 * e]] = n.edges[2 * e + 1];
      partner[(size_t)n.edges[2 * e + 1]] = n.edges[2 * e];
    }
    // orient breadth first from the root
    std::vector<int> parent_mode((size_t)n.p, -1), depth((size_t)n.p, 0);
    std::vector<std::vector<int>> child_modes((size_t)n.p);
    std::vector<int> order;
    std::queue<int> qu;
    qu.push(p->root);
    std::vector<char> seen((size_t)n.p, 0);
    seen[(size_t)p->root] = 1;
    while (!qu.empty()) {
      const int k = qu.front();
      qu.pop();
      order.push_back(k);
      for (int u = c.offsets[(size_t)k]; u < c.offsets[(size_t)k + 1]; ++u) {
        if (u == parent_mode[(size_t)k]) continue;
        const int l = c.tensor_of[(size_t)partner[(size_t)u]];
        seen[(size_t)l] = 1;
        parent_mode[(size_t)l] = partner[(size_t)u];
        depth[(size_t)l] = depth[(size_t)k] + 1;
        child_modes[(size_t)k].push_back(u);
        qu.push(l);
      }
    }
    // node descriptors
    const size_t base = P->h_nodes.size();
    for (int k = 0; k < n.p; ++k) {
      M2Node nd{};
      nd.tensor = (int32_t)(gtensor + k);
      nd.net = j;
      nd.local = k;
      nd.root = (k == p->root);
      nd.depth = depth[(size_t)k];
      nd.seed = p->seed + (uint64_t)j;
      const int cc = (int)child_modes[(size_t)k].size();
      if (cc > kM2MaxChildren)
        return set_error(TN_ERR_UNSUPPORTED, "acyclic method: network %d tensor %d has %d children (max %d)",
                         j, k, cc, kM2MaxChildren);
      nd.nchild = cc;
      int qt = 1;
      while (qt < cc) qt <<= 1;
      nd.qt = cc ? qt : 0;
      nd.ncols = 1;
      int64_t dsum = 0;
      for (int i = 0; i < cc; ++i) {
        const int u = child_modes[(size_t)k][(size_t)i];
        nd.child_dim[i] = (int32_t)n.dims[u];
        nd.ncols *= n.dims[u];
        dsum += n.dims[u];
        if (nd.ncols > 0x7fff0000ll)  // 32-bit column arithmetic with a chunk of headroom
          return set_error(TN_ERR_UNSUPPORTED,
                           "acyclic method: network %d tensor %d: more than 2^31 - 2^16 child index tuples", j, k);
        const int e = c.edge_of[(size_t)u];
        nd.child_edge[i] = e;
        nd.child_tab[i] = edge_tab[(size_t)e];
        nd.child_tensor[i] = -1;
      }
      if (dsum + (qt - cc) > kM2MaxTableSum)
        return set_error(TN_ERR_UNSUPPORTED,
                         "acyclic method: network %d tensor %d: child modes sum to %lld (max %d)", j, k,
                         (long long)dsum, kM2MaxTableSum);
      if (cc > 0) P->tcap = std::max<int32_t>(P->tcap, (int32_t)((dsum + (qt - cc) + 1) & ~1ll));
      if (nd.root) {
        nd.rows = 1;
        nd.after = nd.ncols;
      } else {
        const int pm = parent_mode[(size_t)k];
        nd.rows = (int32_t)n.dims[pm];
        nd.after = 1;
        for (int u = pm + 1; u < c.offsets[(size_t)k + 1]; ++u) nd.after *= n.dims[u];
        const int e = c.edge_of[(size_t)pm];
        nd.parent_edge = e;
        nd.parent_tab = edge_tab[(size_t)e];
      }
      P->h_nodes.push_back(nd);
    }
    // children's node links, tensor-sketch and padding streams
    for (int k = 0; k < n.p; ++k) {
      M2Node &nd = P->h_nodes[base + (size_t)k];
      for (int i = 0; i < nd.nchild; ++i) {
        const int u = child_modes[(size_t)k][(size_t)i];
        const int l = c.tensor_of[(size_t)partner[(size_t)u]];
        if (child_modes[(size_t)l].empty()) nd.child_tensor[i] = (int32_t)(gtensor + l);
      }
      if (nd.qt >= 2) {
        nd.t_tab = p->W;
        int tix = 0;
        for (int l = nd.qt; l >= 2; l /= 2)
          for (int jj = 0; jj < l / 2; ++jj, ++tix)
            for (int d = 0; d < 2; ++d) {
              StreamDesc sd{};
              sd.seed = nd.seed;
              sd.stream = (1ull << 62) + ((uint64_t)k << 32) + ((uint64_t)l << 16) + (uint64_t)(2 * jj + d);
              sd.offset = p->W;
              sd.n = (int32_t)p->m;
              sd.net = j;
              p->W += p->m;
              p->h_streams.push_back(sd);
            }
        for (int jj = nd.nchild; jj < nd.qt; ++jj) {
          StreamDesc sd{};
          sd.seed = nd.seed;
          sd.stream = (1ull << 63) + ((uint64_t)k << 32) + (uint64_t)jj;
          sd.offset = p->W;
          sd.n = 1;
          sd.net = j;
          nd.pad_tab[jj] = p->W;
          p->W += 1;
          p->h_streams.push_back(sd);
        }
      }
    }
    // w offsets for internal non-root tensors, then the children's w offsets
    for (int k = 0; k < n.p; ++k) {
      M2Node &nd = P->h_nodes[base + (size_t)k];
      if (!nd.root && nd.nchild > 0) {
        nd.w_off = P->w_row;
        P->w_row += nd.rows;
      }
      P->node_of_tensor[(size_t)(gtensor + k)] = (int32_t)(base + (size_t)k);
    }
    for (int k = 0; k < n.p; ++k) {
      M2Node &nd = P->h_nodes[base + (size_t)k];
      for (int i = 0; i < nd.nchild; ++i) {
        const int u = child_modes[(size_t)k][(size_t)i];
        const int l = c.tensor_of[(size_t)partner[(size_t)u]];
        nd.child_w_off[i] = P->h_nodes[base + (size_t)l].w_off;
        nd.child_tile0[i] = (int32_t)(base + (size_t)l);  // node index; first tile set below
      }
    }
    gtensor += n.p;
  }
  // levels: tensors with children, by depth; g offsets within each level
  int maxd = 0;
  for (const M2Node &nd : P->h_nodes) maxd = std::max(maxd, nd.depth);
  P->level_nodes.assign((size_t)maxd + 1, {});
  P->level_tiles.assign((size_t)maxd + 1, {});
  P->level_maxcols.assign((size_t)maxd + 1, 0);
  level_cols.assign((size_t)maxd + 1, 0);
  for (size_t i = 0; i < P->h_nodes.size(); ++i) {
    M2Node &nd = P->h_nodes[i];
    if (nd.nchild == 0) continue;
    nd.g_off = level_cols[(size_t)nd.depth];
    level_cols[(size_t)nd.depth] += (nd.ncols + 3) & ~3ll;  // 4-aligned rows of g
    P->level_nodes[(size_t)nd.depth].push_back((int32_t)i);
    P->level_maxcols[(size_t)nd.depth] = std::max(P->level_maxcols[(size_t)nd.depth], nd.ncols);
    for (int r0 = 0; r0 < nd.rows; r0 += kG16Rows) P->level_tiles[(size_t)nd.depth].push_back({(int32_t)i, r0});
  }
  for (int64_t v : level_cols) P->g_row = std::max(P->g_row, v);
  {
    std::vector<int32_t> first_tile(P->h_nodes.size(), -1);
    for (const auto &lt : P->level_tiles)
      for (size_t t = 0; t < lt.size(); ++t)
        if (first_tile[(size_t)lt[t].node] < 0) first_tile[(size_t)lt[t].node] = (int32_t)t;
    for (M2Node &nd : P->h_nodes)
      for (int i = 0; i < nd.nchild; ++i) nd.child_tile0[i] = first_tile[(size_t)nd.child_tile0[i]];
  }
  P->level_off.assign(P->level_nodes.size(), 0);
  for (size_t d = 0; d < P->level_nodes.size(); ++d) {
    P->level_off[d] = (int64_t)P->all_nodes.size();
    P->all_nodes.insert(P->all_nodes.end(), P->level_nodes[d].begin(), P->level_nodes[d].end());
  }
  if (P->g_row > 65535ll * 65536ll)
    return set_error(TN_ERR_UNSUPPORTED, "acyclic method: level too large");
  // sample chunk: g and w rows within a 2 GiB workspace, at most 65535 samples
  const size_t per_sample = (size_t)(P->g_row + P->w_row) * as + (size_t)p->n_nets * p->m * 8 +
                            P->all_nodes.size() * (size_t)P->tcap * 4;
  int64_t chunk = (int64_t)std::max<size_t>(1, ((size_t)2 << 30) / std::max<size_t>(1, per_sample));
  chunk = std::min<int64_t>({chunk, p->S, 65535});
  P->chunk = chunk;
  p->chunk = chunk;
  p->sb = 1;
  // The partials buffer holds the column split of the largest target the
  // autotuner may choose; the default target is then applied.
  const size_t part = m2_schedule(p, kSplitTargetMax);
  m2_schedule(p, 512);
  int rc;
  if ((rc = upload_vec(&p->d_streams, p->h_streams)) != TN_OK) return rc;
  if ((rc = upload_vec(&P->d_nodes, P->h_nodes)) != TN_OK) return rc;
  P->d_level_nodes.assign(P->level_nodes.size(), nullptr);
  P->d_level_tiles.assign(P->level_tiles.size(), nullptr);
  for (size_t d = 0; d < P->level_nodes.size(); ++d) {
    if ((rc = upload_vec(&P->d_level_nodes[d], P->level_nodes[d])) != TN_OK) return rc;
    if ((rc = upload_vec(&P->d_level_tiles[d], P->level_tiles[d])) != TN_OK) return rc;
  }
  auto alloc = [&](void **ptr, size_t bytes) -> int {
    *ptr = nullptr;
    if (bytes == 0) return TN_OK;
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *ptr = nullptr;
      return set_error(TN_ERR_OOM, "hipMalloc(%zu bytes)", bytes);
    }
    return TN_OK;
  };
  if ((rc = alloc(&P->d_g, (size_t)chunk * (size_t)P->g_row * as)) != TN_OK) return rc;
  if ((rc = alloc(&P->d_w, (size_t)chunk * (size_t)std::max<int64_t>(P->w_row, 1) * as)) != TN_OK) return rc;
  void *r = nullptr;
  if ((rc = alloc(&r, (size_t)chunk * (size_t)p->n_nets * (size_t)p->m * 8)) != TN_OK) return rc;
  P->d_r = reinterpret_cast<double *>(r);
  void *q = nullptr;
  if ((rc = alloc(&q, part * 8)) != TN_OK) return rc;
  P->d_part = reinterpret_cast<double *>(q);
  void *lt = nullptr;
  if ((rc = alloc(&lt, P->all_nodes.size() * (size_t)chunk * (size_t)P->tcap * 4)) != TN_OK) return rc;
  P->d_ltab = reinterpret_cast<uint32_t *>(lt);
  if ((rc = upload_vec(&P->d_all_nodes, P->all_nodes)) != TN_OK) return rc;
  return TN_OK;
}

int m2_estimate(tn_plan *p, hipStream_t st, double *est) {
  for (int64_t c0 = 0; c0 < p->S; c0 += p->m2->chunk) {
    const int64_t n = std::min(p->m2->chunk, p->S - c0);
    int rc = m2_run(p, st, c0, n, est, nullptr);
    if (rc != TN_OK) return rc;
  }
  return TN_OK;
}

// Launch shapes of the acyclic sweep (TN_FLAG_AUTOTUNE): the product levels'
// column-split target and the gather levels' block target, each candidate
// timed on the plan's first sample chunk (one warm-up run, then the faster of
// two), the fastest kept.  The column split only regroups FP64 partial sums,
// so estimates move by rounding alone.  Cached per plan shape.
namespace {
struct M2TuneKey {
  int64_t nodes, g_row, w_row, m, S, chunk;
  int dtype, device;
  uint32_t prec;
  bool operator==(const M2TuneKey &o) const {
    return nodes == o.nodes && g_row == o.g_row && w_row == o.w_row && m == o.m && S == o.S && chunk == o.chunk &&
           dtype == o.dtype && device == o.device && prec == o.prec;
  }
};
std::vector<std::pair<M2TuneKey, std::pair<int32_t, int32_t>>> g_m2_tuned;
std::mutex g_m2_tuned_mu;
}  // namespace

int m2_autotune(tn_plan *p, hipStream_t st) {
  M2Plan *P = p->m2;
  const M2TuneKey key{(int64_t)P->h_nodes.size(), P->g_row, P->w_row, p->m, p->S, P->chunk, p->dtype, p->device,
                      p->flags & (TN_FLAG_MFMA_BF16 | TN_FLAG_MFMA_F32)};
  auto apply = [&](std::pair<int32_t, int32_t> v) {
    m2_schedule(p, v.first);
    P->gather_target = v.second;
  };
  {
    std::lock_guard<std::mutex> lk(g_m2_tuned_mu);
    for (const auto &kv : g_m2_tuned)
      if (kv.first == key) {
        apply(kv.second);
        log_msg(1, "autotune: cached schedule, split target %d, gather target %d", kv.second.first,
                kv.second.second);
        return TN_OK;
      }
  }
  const int64_t n = std::min(P->chunk, p->S);
  const uint32_t saved_flags = p->flags;
  p->flags &= ~(uint32_t)(TN_FLAG_PROFILE | TN_FLAG_PROFILE_SKETCH);  // no events inside the timing runs
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = TN_OK;
  if (hipEventCreateWithFlags(&e0, hipEventDisableSystemFence) != hipSuccess ||
      hipEventCreateWithFlags(&e1, hipEventDisableSystemFence) != hipSuccess)
    rc = set_error(TN_ERR_HIP, "autotune: event create");
  std::pair<int32_t, int32_t> best{512, 0};
  float best_ms = 1e30f;
  for (int32_t split : {128, 256, 512, 1024, kSplitTargetMax}) {
    for (int32_t gather : {0, 512, 2048, 4096}) {
      if (rc != TN_OK) break;
      apply({split, gather});
      float ms_min = 1e30f;
      for (int rep = 0; rep < 3 && rc == TN_OK; ++rep) {
        float ms = 0.f;
        if (hipEventRecord(e0, st) != hipSuccess) rc = set_error(TN_ERR_HIP, "autotune: event record");
        if (rc == TN_OK) rc = m2_run(p, st, 0, n, p->d_est, nullptr);
        if (rc == TN_OK && hipEventRecord(e1, st) != hipSuccess) rc = set_error(TN_ERR_HIP, "autotune: event record");
        if (rc == TN_OK && hipEventSynchronize(e1) != hipSuccess) rc = set_error(TN_ERR_HIP, "autotune: sync");
        if (rc == TN_OK) (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) ms_min = std::min(ms_min, ms);
      }
      if (rc == TN_OK) log_msg(2, "autotune: split target %d, gather target %d: %.4f ms", split, gather, (double)ms_min);
      if (rc == TN_OK && ms_min < best_ms) {
        best_ms = ms_min;
        best = {split, gather};
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  p->flags = saved_flags;
  apply(best);
  if (rc != TN_OK) return rc;
  log_msg(1, "autotune: split target %d, gather target %d (%.4f ms for %lld samples)", best.first, best.second,
          (double)best_ms, (long long)n);
  std::lock_guard<std::mutex> lk(g_m2_tuned_mu);
  g_m2_tuned.push_back({key, best});
  return TN_OK;
}

int m2_get_sketches(tn_plan *p, int64_t first, int64_t count, hipStream_t st, double *out) {
  M2Plan *P = p->m2;
  for (int64_t c0 = first; c0 < first + count; c0 += P->chunk) {
    const int64_t n = std::min(P->chunk, first + count - c0);
    double *o = out + (c0 - first) * p->n_tensors * p->m;
    int rc = m2_run(p, st, c0, n, p->d_est, o);
    if (rc != TN_OK) return rc;
    // root slots: r_o, one per network
    for (int j = 0; j < p->n_nets; ++j) {
      const int64_t tensor = p->net_tensor0[(size_t)j] + p->root;
      TN_HIP_CHECK(hipMemcpy2DAsync(o + tensor * p->m, (size_t)p->n_tensors * p->m * 8,
                                    P->d_r + (int64_t)j * p->m, (size_t)p->n_nets * p->m * 8,
                                    (size_t)p->m * 8, (size_t)n, hipMemcpyDeviceToDevice, st));
    }
  }
  return TN_OK;
}

void m2_release(tn_plan *p) {
  M2Plan *P = p->m2;
  if (!P) return;
  if (P->d_nodes) (void)hipFree(P->d_nodes);
  for (auto *q : P->d_level_nodes)
    if (q) (void)hipFree(q);
  for (auto *q : P->d_level_tiles)
    if (q) (void)hipFree(q);
  if (P->d_g) (void)hipFree(P->d_g);
  if (P->d_w) (void)hipFree(P->d_w);
  if (P->d_r) (void)hipFree(P->d_r);
  if (P->d_part) (void)hipFree(P->d_part);
  if (P->d_ltab) (void)hipFree(P->d_ltab);
  if (P->d_all_nodes) (void)hipFree(P->d_all_nodes);
  delete P;
  p->m2 = nullptr;
}

}  // namespace tn
