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
//   m2_gemm   : w_k = mat(X_k) G over all samples of the chunk (operands in the
//               storage type, FP64 accumulation), rows tiled by 64, samples by 64.
#include <algorithm>
#include <new>
#include <queue>
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
};

namespace {

constexpr int kTR = 64;   // GEMM rows per tile
constexpr int kTS = 64;   // GEMM samples per tile
constexpr int kTK = 32;   // GEMM columns per step

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

// One sample's sketch r_k and gather g for tensor k (see the file comment).
// A: storage type of w and g (float for FP32/BF16 data, double for FP64).
template <typename T, typename A>
__global__ __launch_bounds__(256) void m2_gather_kernel(
    const M2Node *__restrict__ nodes, const int32_t *__restrict__ level, const void *const *data,
    const int32_t *__restrict__ tables, int64_t W, int64_t sample0, int log2m,
    const A *__restrict__ wbuf, int64_t w_row, A *__restrict__ gbuf, int64_t g_row,
    double *__restrict__ r_out, int64_t r_stride, int tcap) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ HashCoeffs coef[3 * kM2MaxChildren];
  __shared__ unsigned long long wmax[kM2MaxChildren];
  __shared__ int32_t tab_base[kM2MaxChildren + 1];

  const M2Node nd = nodes[level[blockIdx.x]];
  const int64_t s = blockIdx.y;
  const uint64_t sample = (uint64_t)(sample0 + s);
  const int tid = threadIdx.x;
  const uint32_t m = 1u << log2m, mask = m - 1;
  const int c = nd.nchild, qt = nd.qt;
  const int32_t *tab = tables ? tables + s * W : nullptr;

  unsigned long long *acc = reinterpret_cast<unsigned long long *>(smem);  // [m]
  uint32_t *dtab = reinterpret_cast<uint32_t *>(acc + m);                  // [tcap] slot tables
  double *wv = reinterpret_cast<double *>(dtab + tcap);                    // [tcap] children's w

  // Coefficients: child contractions [0, c), tensor sketches [c, c + 2(qt-1)),
  // padding slots after that.
  const int n_t = 2 * (qt - 1);
  if (!tab && tid < c + n_t + (qt - c)) {
    uint64_t stream;
    if (tid < c) {
      stream = (uint64_t)nd.child_edge[tid];
    } else if (tid < c + n_t) {
      const int k = tid - c, tix = k >> 1, d = k & 1;
      // tix enumerates (level l, index j) level-major from l = qt: tix = qt - l + j
      int l = qt, base = 0;
      while (tix - base >= l / 2) { base += l / 2; l /= 2; }
      stream = (1ull << 62) + ((uint64_t)nd.local << 32) + ((uint64_t)l << 16) +
               (uint64_t)(2 * (tix - base) + d);
    } else {
      stream = (1ull << 63) + ((uint64_t)nd.local << 32) + (uint64_t)(c + tid - c - n_t);
    }
    coef[tid] = hash_coeffs(nd.seed, sample, stream);
  }
  if (tid == 0) {
    int b = 0;
    for (int j = 0; j < qt; ++j) {
      tab_base[j] = b;
      b += j < c ? nd.child_dim[j] : 1;
    }
    tab_base[qt] = b;
  }
  if (tid < kM2MaxChildren) wmax[tid] = 0ull;
  for (uint32_t i = tid; i < m; i += 256) acc[i] = 0ull;
  __syncthreads();

  // Tensor-sketch lookup: packed value of T_{tix} side d at an m-valued index.
  auto tsk = [&](int tix, int d, uint32_t idx) -> uint32_t {
    if (tab) return (uint32_t)tab[nd.t_tab + (int64_t)(2 * tix + d) * m + idx];
    return hash_packed(coef[c + 2 * tix + d], idx, mask);
  };

  // Level-one slot tables: the child (or padding) count sketch, followed by the
  // first tensor sketch of its pair when qt >= 2.
  for (int j = 0; j < qt; ++j) {
    const int nj = tab_base[j + 1] - tab_base[j];
    for (int i = tid; i < nj; i += 256) {
      uint32_t v;
      if (j < c)
        v = tab ? (uint32_t)tab[nd.child_tab[j] + i] : hash_packed(coef[j], (uint32_t)i, mask);
      else
        v = tab ? (uint32_t)tab[nd.pad_tab[j]] : hash_packed(coef[c + n_t + (j - c)], 0u, mask);
      if (qt >= 2) {
        const uint32_t t = tsk(j >> 1, j & 1, v & 0x7fffffffu);
        v = (t & 0x7fffffffu) | ((v ^ t) & 0x80000000u);
      }
      dtab[tab_base[j] + i] = v;
    }
  }
  // Children's w vectors and their max |w|.
  for (int j = 0; j < c; ++j) {
    double lm = 0.0;
    for (int i = tid; i < nd.child_dim[j]; i += 256) {
      const double x = nd.child_tensor[j] >= 0
                           ? load_val<T>(data[nd.child_tensor[j]], i)
                           : (double)wbuf[s * w_row + nd.child_w_off[j] + i];
      wv[tab_base[j] + i] = x;
      lm = fmax(lm, fabs(x));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) lm = fmax(lm, __shfl_xor(lm, off, 64));
    if ((tid & 63) == 0) atomicMax(&wmax[j], (unsigned long long)__double_as_longlong(lm));
  }
  __syncthreads();

  // Fixed-point scale: every product is below prod_j max|w_j| < 2^e; ncols terms.
  double pmax = 1.0;
  for (int j = 0; j < c; ++j) pmax *= __longlong_as_double((long long)wmax[j]);
  const int lgN = max(nd.ncols > 1 ? 64 - __clzll((unsigned long long)(nd.ncols - 1)) : 0, 11);
  int e = 0;
  if (pmax > 0.0) (void)frexp(pmax, &e);
  const double sc = ldexp(1.0, 62 - lgN - e);
  const double inv_sc = ldexp(1.0, -(62 - lgN - e));
  const double kMagic = 6755399441055744.0;

  // Recursive-sketch hash (Algorithm 4) of the child index tuple of column col.
  auto rs_hash = [&](int64_t col, int32_t *idx) -> uint32_t {
    for (int j = c - 1; j >= 0; --j) {
      idx[j] = (int32_t)(col % nd.child_dim[j]);
      col /= nd.child_dim[j];
    }
    if (qt == 1) return dtab[idx[0]];
    uint32_t b[kM2MaxChildren / 2];
    for (int t = 0; t < qt / 2; ++t) {
      const int jl = 2 * t, jr = 2 * t + 1;
      const uint32_t vl = dtab[tab_base[jl] + (jl < c ? idx[jl] : 0)];
      const uint32_t vr = dtab[tab_base[jr] + (jr < c ? idx[jr] : 0)];
      b[t] = sum_packed(vl, vr, mask);
    }
    for (int l = qt / 2; l >= 2; l /= 2) {
      for (int t = 0; t < l / 2; ++t) {
        const int tix = qt - l + t;
        const uint32_t t0 = tsk(tix, 0, b[2 * t] & 0x7fffffffu);
        const uint32_t t1 = tsk(tix, 1, b[2 * t + 1] & 0x7fffffffu);
        const uint32_t sg = (b[2 * t] ^ b[2 * t + 1] ^ t0 ^ t1) & 0x80000000u;
        b[t] = (((t0 & 0x7fffffffu) + (t1 & 0x7fffffffu)) & mask) | sg;
      }
    }
    return b[0];
  };

  // r_k = R_k (kron_l w_l): scatter of the products.
  for (int64_t col = tid; col < nd.ncols; col += 256) {
    int32_t idx[kM2MaxChildren];
    const uint32_t h = rs_hash(col, idx);
    double p = 1.0;
    for (int j = 0; j < c; ++j) p *= wv[tab_base[j] + idx[j]];
    const long long v = __double_as_longlong(fma(p, sc, kMagic)) - __double_as_longlong(kMagic);
    atomicAdd(&acc[h & mask], (unsigned long long)((h & 0x80000000u) ? -v : v));
  }
  __syncthreads();

  // g[col] = sigma(col) r_k[b(col)].
  A *g = gbuf + s * g_row + nd.g_off;
  for (int64_t col = tid; col < nd.ncols; col += 256) {
    int32_t idx[kM2MaxChildren];
    const uint32_t h = rs_hash(col, idx);
    const double r = (double)(long long)acc[h & mask] * inv_sc;
    g[col] = (A)((h & 0x80000000u) ? -r : r);
  }
  if (r_out && nd.root) {
    for (uint32_t b = tid; b < m; b += 256)
      r_out[s * r_stride + (int64_t)nd.net * m + b] = (double)(long long)acc[b] * inv_sc;
  }
}

// w_k[row] = sum_col X_k(row, col) g[col] for a tile of 64 rows x 64 samples.
template <typename T, typename A>
__global__ __launch_bounds__(256) void m2_gemm_kernel(
    const M2Node *__restrict__ nodes, const M2Tile *__restrict__ tiles, const void *const *data,
    const A *__restrict__ gbuf, int64_t g_row, int64_t samples, A *__restrict__ wbuf,
    int64_t w_row, double *__restrict__ est, int64_t S, int64_t sample0) {
  __shared__ A As[kTK][kTR + 4];
  __shared__ A Bs[kTK][kTS + 4];
  const M2Tile tl = tiles[blockIdx.x];
  const M2Node nd = nodes[tl.node];
  const int tid = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.y * kTS;
  const int tr = tid >> 4, ts = tid & 15;  // 16 x 16 threads, 4 x 4 outputs each
  const void *X = data[nd.tensor];
  double accv[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) accv[i][j] = 0.0;

  for (int64_t c0 = 0; c0 < nd.ncols; c0 += kTK) {
    for (int i = tid; i < kTR * kTK; i += 256) {
      const int r = i / kTK, k = i % kTK;
      const int64_t row = tl.row0 + r, col = c0 + k;
      A v = (A)0;
      if (row < nd.rows && col < nd.ncols) {
        const int64_t off = ((col / nd.after) * nd.rows + row) * nd.after + col % nd.after;
        v = (A)load_val<T>(X, off);
      }
      As[k][r] = v;
    }
    for (int i = tid; i < kTS * kTK; i += 256) {
      const int sl = i / kTK, k = i % kTK;
      const int64_t smp = s0 + sl, col = c0 + k;
      Bs[k][sl] = (smp < samples && col < nd.ncols) ? gbuf[smp * g_row + nd.g_off + col] : (A)0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < kTK; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = (double)As[k][tr * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = (double)Bs[k][ts * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) accv[i][j] = fma(a[i], b[j], accv[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t row = tl.row0 + tr * 4 + i;
    if (row >= nd.rows) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t smp = s0 + ts * 4 + j;
      if (smp >= samples) continue;
      if (nd.root)
        est[(int64_t)nd.net * S + sample0 + smp] = accv[i][j];
      else
        wbuf[smp * w_row + nd.w_off + row] = (A)accv[i][j];
    }
  }
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

template <typename T, typename A>
int m2_run_t(tn_plan *p, hipStream_t st, int64_t c0, int64_t n, const int32_t *tables,
             double *est, double *export_out) {
  M2Plan *P = p->m2;
  const size_t lds = (size_t)p->m * 8 + (size_t)P->tcap * 12;
  auto gk = m2_gather_kernel<T, A>;
  if (lds > 65536)
    TN_HIP_CHECK(hipFuncSetAttribute((const void *)gk, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds));
  for (int d = (int)P->level_nodes.size() - 1; d >= 0; --d) {
    if (P->level_nodes[(size_t)d].empty()) continue;
    hipEvent_t ev = nullptr;
    int rc;
    if ((rc = prof_begin(p, st, &ev)) != TN_OK) return rc;
    dim3 g1((unsigned)P->level_nodes[(size_t)d].size(), (unsigned)n);
    hipLaunchKernelGGL(gk, g1, dim3(256), lds, st, P->d_nodes, P->d_level_nodes[(size_t)d],
                       (const void *const *)p->d_data, tables, p->W, c0, p->log2m,
                       reinterpret_cast<const A *>(P->d_w), P->w_row,
                       reinterpret_cast<A *>(P->d_g), P->g_row,
                       export_out ? P->d_r : nullptr, (int64_t)p->n_nets * p->m, P->tcap);
    TN_HIP_CHECK(hipGetLastError());
    if ((rc = prof_end(p, st, TN_KERNEL_COMBINE, ev)) != TN_OK) return rc;
    if ((rc = prof_begin(p, st, &ev)) != TN_OK) return rc;
    dim3 g2((unsigned)P->level_tiles[(size_t)d].size(), (unsigned)((n + kTS - 1) / kTS));
    hipLaunchKernelGGL((m2_gemm_kernel<T, A>), g2, dim3(256), 0, st, P->d_nodes,
                       P->d_level_tiles[(size_t)d], (const void *const *)p->d_data,
                       reinterpret_cast<const A *>(P->d_g), P->g_row, n,
                       reinterpret_cast<A *>(P->d_w), P->w_row, est, p->S, c0);
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
    case TN_F64: return m2_run_t<double, double>(p, st, c0, n, tables, est, export_out);
    case TN_F32: return m2_run_t<float, float>(p, st, c0, n, tables, est, export_out);
    default: return m2_run_t<uint16_t, float>(p, st, c0, n, tables, est, export_out);
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
      }
    }
    gtensor += n.p;
  }
  // levels: tensors with children, by depth; g offsets within each level
  int maxd = 0;
  for (const M2Node &nd : P->h_nodes) maxd = std::max(maxd, nd.depth);
  P->level_nodes.assign((size_t)maxd + 1, {});
  P->level_tiles.assign((size_t)maxd + 1, {});
  level_cols.assign((size_t)maxd + 1, 0);
  for (size_t i = 0; i < P->h_nodes.size(); ++i) {
    M2Node &nd = P->h_nodes[i];
    if (nd.nchild == 0) continue;
    nd.g_off = level_cols[(size_t)nd.depth];
    level_cols[(size_t)nd.depth] += nd.ncols;
    P->level_nodes[(size_t)nd.depth].push_back((int32_t)i);
    for (int r0 = 0; r0 < nd.rows; r0 += kTR) P->level_tiles[(size_t)nd.depth].push_back({(int32_t)i, r0});
  }
  for (int64_t v : level_cols) P->g_row = std::max(P->g_row, v);
  if (P->g_row > 65535ll * 65536ll)
    return set_error(TN_ERR_UNSUPPORTED, "acyclic method: level too large");
  // sample chunk: g and w rows within a 2 GiB workspace, at most 65535 samples
  const size_t per_sample = (size_t)(P->g_row + P->w_row) * as + (size_t)p->n_nets * p->m * 8;
  int64_t chunk = (int64_t)std::max<size_t>(1, ((size_t)2 << 30) / std::max<size_t>(1, per_sample));
  chunk = std::min<int64_t>({chunk, p->S, 65535});
  P->chunk = chunk;
  p->chunk = chunk;
  p->sb = 1;
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
  delete P;
  p->m2 = nullptr;
}

}  // namespace tn
