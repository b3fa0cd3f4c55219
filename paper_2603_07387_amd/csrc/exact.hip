// Exact full tensor network contraction in FP64 on the device (Def. 1-3).
//
// Intermediates carry one label per mode (the contraction it belongs to).  A
// tensor whose label appears twice is first traced (a contraction inside one
// tensor, WLOG 2) by a per-element walker.  The tensors of each connected
// component are then contracted pairwise along a contraction tree: for at most
// kDpMaxTensors tensors the tree of fewest multiply-adds (dynamic programming
// over subsets, every intermediate within a size cap), else a greedy tree
// (smallest result first).  The components' scalars multiply.
//
// A pairwise step is a matrix product.  With the shared labels summed (K
// entries), A's other labels as rows (M) and B's as columns (N), C = A B is
// M x N with A's remaining labels, then B's, in their operands' order.  An
// operand whose summed labels already form a contiguous block at either end is
// used in place (as M x K or K x M, K x N or N x K); otherwise, or when the two
// operands order their summed labels differently, it is first permuted into
// such a layout (a gather kernel; the smaller operand when only the order
// differs).  Products with at least kSkinny rows and columns run on the FP64
// matrix cores (v_mfma_f64_16x16x4f64) in 128 x 128 tiles, split along K when
// the tiles alone would not fill the chip; thinner ones as one dot product per
// wave, split along K likewise.  Partial sums over K meet in a fixed order, so
// the result does not depend on timing.
//
// Device memory: the tree is first run on labels alone to find the peak of
// live intermediates and permuted copies; a tree that would not fit in the
// free device memory is refused before any allocation (TN_ERR_OOM).
#include <algorithm>
#include <cmath>
#include <functional>
#include <memory>
#include <vector>

#include "plan.h"

namespace tn {
namespace {

constexpr int kMaxLabels = 24;
constexpr int kDpMaxTensors = 16;
constexpr int kSkinny = 16;  // products with fewer rows or columns: one dot product per wave

// ---------------------------------------------------------------------------
// Traces inside one tensor: a thread per output element walks the summed
// labels (a label repeated inside the operand gets the sum of its strides,
// i.e. the diagonal).
struct TraceDesc {
  int n_out, n_sum;
  int64_t out_dims[kMaxLabels];
  int64_t sum_dims[kMaxLabels];
  int64_t a_out[kMaxLabels];
  int64_t a_sum[kMaxLabels];
};

__global__ void trace_kernel(TraceDesc d, const double *__restrict__ A, int64_t out_size, double *__restrict__ C) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < out_size;
       o += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = o, ao = 0;
    for (int i = d.n_out - 1; i >= 0; --i) {
      const int64_t digit = rem % d.out_dims[i];
      rem /= d.out_dims[i];
      ao += digit * d.a_out[i];
    }
    int64_t idx[kMaxLabels];
    for (int i = 0; i < d.n_sum; ++i) idx[i] = 0;
    double acc = 0.0;
    int64_t as = 0;
    while (true) {
      acc += A[ao + as];
      int i = d.n_sum - 1;
      for (; i >= 0; --i) {
        if (++idx[i] < d.sum_dims[i]) {
          as += d.a_sum[i];
          break;
        }
        as -= (d.sum_dims[i] - 1) * d.a_sum[i];
        idx[i] = 0;
      }
      if (i < 0) break;
    }
    C[o] = acc;
  }
}

template <typename T>
__global__ void to_f64_kernel(const T *__restrict__ x, int64_t n, double *__restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

__global__ void bf16_to_f64_kernel(const uint16_t *__restrict__ x, int64_t n, double *__restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (double)__uint_as_float(((uint32_t)x[i]) << 16);
}

// ---------------------------------------------------------------------------
// Permutation: out (dims out_dims, row-major) [o] = in [sum_i digit_i(o) in_stride_i].
struct PermDesc {
  int rank;
  int64_t out_dims[kMaxLabels];
  int64_t in_stride[kMaxLabels];
};

__global__ void permute_f64_kernel(PermDesc d, const double *__restrict__ in, int64_t n, double *__restrict__ out) {
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = o, off = 0;
    for (int i = d.rank - 1; i >= 0; --i) {
      const int64_t digit = rem % d.out_dims[i];
      rem /= d.out_dims[i];
      off += digit * d.in_stride[i];
    }
    out[o] = in[off];
  }
}

// ---------------------------------------------------------------------------
// C = A B on the FP64 matrix cores.  v_mfma_f64_16x16x4f64: A[i][k] in lane
// i + 16 k, B[k][j] in lane j + 16 k, D[i][j] element i / 4 of lane j + 16 (i % 4).
// Block: 256 threads, a 128 x 128 tile of C; wave w a 64 x 64 quarter (rows
// 64 (w / 2), columns 64 (w % 2)), 4 x 4 accumulators.  K in chunks of 16,
// staged in double-buffered LDS as [k][row] with the next chunk's global loads
// in flight during the products.  AT: A stored K x M (else M x K); BT: B stored
// N x K (else K x N).  Each load instruction reads whole 128-byte runs along
// the operand's contiguous dimension.  Blocks z of a split along K write
// partial tiles part[z][M][N] (summed by gemm_reduce_kernel).
constexpr int kGT = 128, kGK = 16, kGPad = 2, kGStr = kGT + kGPad;

template <bool AT, bool BT>
__global__ __launch_bounds__(256) void gemm_f64_kernel(const double *__restrict__ A, const double *__restrict__ B,
                                                       double *__restrict__ C, int64_t M, int64_t N, int64_t K,
                                                       int64_t tiles_m, int64_t tiles_n, int64_t kchunk,
                                                       double *__restrict__ part) {
  __shared__ __align__(16) double As[2][kGK][kGStr];
  __shared__ __align__(16) double Bs[2][kGK][kGStr];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1, li = lane & 15, kq = lane >> 4;
  // Tile order: consecutive block numbers land on different XCDs (round robin
  // over 8), so each XCD is given a contiguous run of tile numbers, and runs
  // walk groups of 8 tile rows column by column (neighbouring tiles share
  // operand panels in that XCD's L2).
  const int64_t nblk = tiles_m * tiles_n;
  int64_t lin = blockIdx.x;
  if ((nblk & 7) == 0) lin = (lin & 7) * (nblk >> 3) + (lin >> 3);
  const int64_t group = lin / (8 * tiles_n), first_m = group * 8;
  const int64_t gm = min((int64_t)8, tiles_m - first_m);
  const int64_t within = lin - group * 8 * tiles_n;
  const int64_t tm = first_m + within % gm, tn = within / gm;
  const int64_t m0 = tm * kGT, n0 = tn * kGT;
  const int64_t kb = (int64_t)blockIdx.y * kchunk, ke = min(K, kb + kchunk);

  // Loader: 8 values of A and of B per thread per chunk.  Along K contiguous:
  // k = tid % 16, rows tid / 16 + 16 j; along rows contiguous: row = tid % 128,
  // k = tid / 128 + 2 j.
  double ra[8], rb[8];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (!AT) {  // M x K
        const int64_t m = m0 + (tid >> 4) + 16 * j, k = k0 + (tid & 15);
        ra[j] = (m < M && k < ke) ? A[m * K + k] : 0.0;
      } else {  // K x M
        const int64_t m = m0 + (tid & 127), k = k0 + (tid >> 7) + 2 * j;
        ra[j] = (m < M && k < ke) ? A[k * M + m] : 0.0;
      }
      if (!BT) {  // K x N
        const int64_t n = n0 + (tid & 127), k = k0 + (tid >> 7) + 2 * j;
        rb[j] = (n < N && k < ke) ? B[k * N + n] : 0.0;
      } else {  // N x K
        const int64_t n = n0 + (tid >> 4) + 16 * j, k = k0 + (tid & 15);
        rb[j] = (n < N && k < ke) ? B[n * K + k] : 0.0;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (!AT) As[buf][tid & 15][(tid >> 4) + 16 * j] = ra[j];
      else As[buf][(tid >> 7) + 2 * j][tid & 127] = ra[j];
      if (!BT) Bs[buf][(tid >> 7) + 2 * j][tid & 127] = rb[j];
      else Bs[buf][tid & 15][(tid >> 4) + 16 * j] = rb[j];
    }
  };
  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  int buf = 0;
  if (kb < ke) {
    load(kb);
    store(0);
  }
  __syncthreads();
  for (int64_t k0 = kb; k0 < ke; k0 += kGK) {
    const bool more = k0 + kGK < ke;  // the same in every thread
    if (more) load(k0 + kGK);
#pragma unroll
    for (int ks = 0; ks < kGK / 4; ++ks) {
      double fa[4], fb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) fa[a] = As[buf][4 * ks + kq][64 * wm + 16 * a + li];
#pragma unroll
      for (int b = 0; b < 4; ++b) fb[b] = Bs[buf][4 * ks + kq][64 * wn + 16 * b + li];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  double *out = part ? part + (int64_t)blockIdx.y * M * N : C;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t m = m0 + 64 * wm + 16 * a + kq + 4 * r, n = n0 + 64 * wn + 16 * b + li;
        if (m < M && n < N) out[m * N + n] = acc[a][b][r];
      }
}

// C[i] = sum_z part[z][i], z in order.
__global__ void gemm_reduce_kernel(const double *__restrict__ part, int64_t n, int64_t splits, double *__restrict__ C) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t z = 0; z < splits; ++z) s += part[z * n + i];
    C[i] = s;
  }
}

// Thin products: one wave per (output, K range), both operands K-contiguous
// (A M x K, B N x K); lane l takes k = kb + l + 64 i, the wave sums its lanes
// with a fixed xor tree.  Output part[z][m][n] (C itself when not split).
__global__ __launch_bounds__(256) void gemm_thin_kernel(const double *__restrict__ A, const double *__restrict__ B,
                                                        int64_t M, int64_t N, int64_t K, int64_t kchunk,
                                                        double *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t o = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (o >= M * N) return;
  const int64_t m = o / N, n = o - m * N;
  const int64_t kb = (int64_t)blockIdx.y * kchunk, ke = min(K, kb + kchunk);
  const double *a = A + m * K, *b = B + n * K;
  double s = 0.0;
  for (int64_t k = kb + lane; k < ke; k += 64) s = fma(a[k], b[k], s);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) out[(int64_t)blockIdx.y * M * N + o] = s;
}

// ---------------------------------------------------------------------------
struct DTensor {
  double *ptr = nullptr;
  std::vector<int> labels;
  std::vector<int64_t> dims;
  int64_t size = 1;
};

unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 16));
}

// Device memory for one run: every allocation is counted, so that a dry run
// (no device calls) gives the peak of the real one.
struct Mem {
  bool dry = false;
  hipStream_t st = nullptr;
  int64_t live = 0, peak = 0;
  int alloc(DTensor *t) {
    live += t->size * 8;
    peak = std::max(peak, live);
    if (dry) return TN_OK;
    hipError_t e = hipMalloc((void **)&t->ptr, (size_t)std::max<int64_t>(1, t->size) * sizeof(double));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      t->ptr = nullptr;
      return set_error(TN_ERR_OOM, "exact contraction: hipMalloc(%lld doubles)", (long long)t->size);
    }
    return TN_OK;
  }
  int scratch(double **p, int64_t n) {  // released with drop_scratch
    live += n * 8;
    peak = std::max(peak, live);
    if (dry) return TN_OK;
    hipError_t e = hipMalloc((void **)p, (size_t)std::max<int64_t>(1, n) * sizeof(double));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return set_error(TN_ERR_OOM, "exact contraction: hipMalloc(%lld doubles)", (long long)n);
    }
    return TN_OK;
  }
  void drop_scratch(double *p, int64_t n) {
    live -= n * 8;
    if (!dry && p) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(p);
    }
  }
  void release(DTensor *t) {
    live -= t->size * 8;
    if (!dry && t->ptr) {
      (void)hipStreamSynchronize(st);
      (void)hipFree(t->ptr);
    }
    t->ptr = nullptr;
  }
};

// Permute T's modes into the label order `to` (a permutation of T.labels).
int permute(Mem &mem, DTensor *T, const std::vector<int> &to) {
  if (to == T->labels) return TN_OK;
  const int r = (int)to.size();
  if (r > kMaxLabels) return set_error(TN_ERR_UNSUPPORTED, "exact contraction: more than %d labels", kMaxLabels);
  std::vector<int64_t> stride(T->labels.size());
  int64_t acc = 1;
  for (int i = (int)T->labels.size() - 1; i >= 0; --i) {
    stride[(size_t)i] = acc;
    acc *= T->dims[(size_t)i];
  }
  DTensor out;
  out.labels = to;
  out.size = T->size;
  PermDesc d{};
  d.rank = r;
  for (int i = 0; i < r; ++i) {
    const size_t j = (size_t)(std::find(T->labels.begin(), T->labels.end(), to[(size_t)i]) - T->labels.begin());
    d.out_dims[i] = T->dims[j];
    d.in_stride[i] = stride[j];
    out.dims.push_back(T->dims[j]);
  }
  int rc = mem.alloc(&out);
  if (rc != TN_OK) {
    mem.release(&out);
    return rc;
  }
  if (!mem.dry) {
    hipLaunchKernelGGL(permute_f64_kernel, dim3(grid_for(out.size)), dim3(256), 0, mem.st, d, T->ptr, out.size,
                       out.ptr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
      mem.release(&out);
      return set_error(TN_ERR_HIP, "exact contraction: %s", hipGetErrorString(e));
    }
  }
  mem.release(T);
  *T = out;
  return TN_OK;
}

// Where T's summed labels sit: +1 a trailing block, -1 a leading block, 0
// neither (with the block's internal order in *order).
int sum_block(const DTensor &T, const std::vector<int> &sum, std::vector<int> *order) {
  const size_t ns = sum.size(), nl = T.labels.size();
  auto is_sum = [&](int l) { return std::find(sum.begin(), sum.end(), l) != sum.end(); };
  bool tail = true, head = true;
  for (size_t i = 0; i < nl; ++i) {
    const bool s = is_sum(T.labels[i]);
    if (s != (i >= nl - ns)) tail = false;
    if (s != (i < ns)) head = false;
  }
  if (ns == 0 || ns == nl) tail = true;
  order->clear();
  for (int l : T.labels)
    if (is_sum(l)) order->push_back(l);
  return tail ? 1 : head ? -1 : 0;
}

// C = contraction of A and B over their shared labels.  A and B are consumed
// on every path; on an error C holds nothing.
int contract_pair(Mem &mem, DTensor *A, DTensor *B, DTensor *C) {
  std::vector<int> sum, keep_a, keep_b;
  std::vector<int64_t> kd_a, kd_b;
  int64_t M = 1, N = 1, K = 1;
  for (size_t i = 0; i < A->labels.size(); ++i) {
    if (std::find(B->labels.begin(), B->labels.end(), A->labels[i]) != B->labels.end()) {
      sum.push_back(A->labels[i]);
      K *= A->dims[i];
    } else {
      keep_a.push_back(A->labels[i]);
      kd_a.push_back(A->dims[i]);
      M *= A->dims[i];
    }
  }
  for (size_t i = 0; i < B->labels.size(); ++i)
    if (std::find(A->labels.begin(), A->labels.end(), B->labels[i]) == A->labels.end()) {
      keep_b.push_back(B->labels[i]);
      kd_b.push_back(B->dims[i]);
      N *= B->dims[i];
    }
  double *part = nullptr;
  int64_t splits = 1, kchunk = K;
  bool c_held = false;  // C counted by mem (allocated, or its allocation attempted)
  // every exit releases what the step holds
  auto finish = [&](int rc) {
    if (part || (mem.dry && splits > 1)) mem.drop_scratch(part, splits * M * N);
    part = nullptr;
    splits = 1;
    if (rc != TN_OK && c_held) mem.release(C);
    mem.release(A);
    mem.release(B);
    return rc;
  };
  auto launched = [&]() {
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? TN_OK : set_error(TN_ERR_HIP, "exact contraction: %s", hipGetErrorString(e));
  };
  if (keep_a.size() + keep_b.size() > (size_t)kMaxLabels)
    return finish(set_error(TN_ERR_UNSUPPORTED, "exact contraction: more than %d labels", kMaxLabels));
  const bool thin = M < kSkinny || N < kSkinny;
  std::vector<int> oa, ob;
  int pa = sum_block(*A, sum, &oa), pb = sum_block(*B, sum, &ob);
  // Thin products read both operands along K: summed labels trailing.
  if (thin) {
    if (M == 1) pa = 1;  // a vector is its own transpose
    if (N == 1) pb = 1;
  }
  int rc;
  auto concat = [](const std::vector<int> &x, const std::vector<int> &y) {
    std::vector<int> r = x;
    r.insert(r.end(), y.begin(), y.end());
    return r;
  };
  const bool a_ok = thin ? pa == 1 : pa != 0, b_ok = thin ? pb == 1 : pb != 0;
  if (a_ok && b_ok && oa != ob) {
    // same blocks, different internal order: permute the smaller operand
    if (A->size <= B->size) {
      if ((rc = permute(mem, A, pa == 1 ? concat(keep_a, ob) : concat(ob, keep_a))) != TN_OK) return finish(rc);
      oa = ob;
    } else {
      if ((rc = permute(mem, B, pb == 1 ? concat(keep_b, oa) : concat(oa, keep_b))) != TN_OK) return finish(rc);
      ob = oa;
    }
  } else {
    if (!a_ok) {
      const std::vector<int> &o = b_ok ? ob : oa;
      if ((rc = permute(mem, A, concat(keep_a, o))) != TN_OK) return finish(rc);
      pa = 1;
      oa = o;
    }
    if (!b_ok) {
      if ((rc = permute(mem, B, thin ? concat(keep_b, oa) : concat(oa, keep_b))) != TN_OK) return finish(rc);
      pb = thin ? 1 : -1;
      ob = oa;
    }
  }
  C->labels = concat(keep_a, keep_b);
  C->dims = kd_a;
  C->dims.insert(C->dims.end(), kd_b.begin(), kd_b.end());
  C->size = M * N;
  const bool at = pa == -1 && M > 1, bt = pb == 1 && N > 1;  // A as K x M; B as N x K
  const int64_t tiles_m = (M + kGT - 1) / kGT, tiles_n = (N + kGT - 1) / kGT, tiles = tiles_m * tiles_n;
  if (thin) {
    const int64_t waves = M * N;
    splits = std::max<int64_t>(1, std::min<int64_t>((K + 4095) / 4096, (8192 + waves - 1) / waves));
    kchunk = (K + splits - 1) / splits;
    splits = std::max<int64_t>(1, (K + kchunk - 1) / kchunk);
    if (splits > 65535 || (M * N + 3) / 4 > 0x7fffffffLL) {
      splits = 1;
      return finish(set_error(TN_ERR_UNSUPPORTED, "exact contraction: thin product %lld x %lld x %lld",
                              (long long)M, (long long)N, (long long)K));
    }
  } else {
    if (tiles > 0x7fffffffLL)
      return finish(set_error(TN_ERR_UNSUPPORTED, "exact contraction: %lld tiles", (long long)tiles));
    if (tiles < 1024 && K >= 1024) {
      splits = std::min<int64_t>((1024 + tiles - 1) / tiles, K / 512);
      kchunk = ((K + splits - 1) / splits + kGK - 1) / kGK * kGK;
      splits = (K + kchunk - 1) / kchunk;
    }
  }
  c_held = true;
  if ((rc = mem.alloc(C)) != TN_OK) {
    splits = 1;
    return finish(rc);
  }
  if (splits > 1 && (rc = mem.scratch(&part, splits * M * N)) != TN_OK) {
    splits = 1;
    return finish(rc);
  }
  if (!mem.dry) {
    if (thin) {
      hipLaunchKernelGGL(gemm_thin_kernel, dim3((unsigned)((M * N + 3) / 4), (unsigned)splits), dim3(256), 0, mem.st,
                         A->ptr, B->ptr, M, N, K, kchunk, part ? part : C->ptr);
    } else {
      const dim3 g((unsigned)tiles, (unsigned)splits);
      auto k = at ? (bt ? gemm_f64_kernel<true, true> : gemm_f64_kernel<true, false>)
                  : (bt ? gemm_f64_kernel<false, true> : gemm_f64_kernel<false, false>);
      hipLaunchKernelGGL(k, g, dim3(256), 0, mem.st, A->ptr, B->ptr, C->ptr, M, N, K, tiles_m, tiles_n, kchunk,
                         part);
    }
    if ((rc = launched()) != TN_OK) return finish(rc);
    if (part) {
      hipLaunchKernelGGL(gemm_reduce_kernel, dim3(grid_for(M * N)), dim3(256), 0, mem.st, part, M * N, splits,
                         C->ptr);
      if ((rc = launched()) != TN_OK) return finish(rc);
    }
  }
  return finish(TN_OK);
}

// Contraction tree over the tensors of one component: node i < n is tensor i,
// nodes n.. are pairs (left, right).
struct Tree {
  std::vector<int> left, right;
  int root = -1;
};

typedef unsigned __int128 LabelSet;

// Fewest multiply-adds over all trees (pairs share a label), every
// intermediate at most `cap` entries.  Returns false if no tree fits.
bool dp_tree(const std::vector<LabelSet> &lab, const std::vector<double> &ldim, double cap, Tree *tree) {
  const int n = (int)lab.size();
  const uint32_t full = (1u << n) - 1;
  std::vector<LabelSet> open(full + 1, 0);
  std::vector<double> sz(full + 1, 1.0), cost(full + 1, INFINITY);
  std::vector<uint32_t> split(full + 1, 0);
  for (uint32_t S = 1; S <= full; ++S) {
    const int low = __builtin_ctz(S);
    open[S] = open[S & (S - 1)] ^ lab[(size_t)low];  // labels with one end inside S
    double s = 1.0;
    LabelSet o = open[S];
    for (int b = 0; o; ++b, o >>= 1)
      if (o & 1) s *= ldim[(size_t)b];
    sz[S] = s;
  }
  for (int k = 0; k < n; ++k) cost[1u << k] = 0.0;
  for (uint32_t S = 1; S <= full; ++S) {
    if ((S & (S - 1)) == 0 || sz[S] > cap) continue;
    double best = INFINITY;
    uint32_t bs = 0;
    for (uint32_t S1 = (S - 1) & S; S1; S1 = (S1 - 1) & S) {
      const uint32_t S2 = S ^ S1;
      if (S1 > S2 || !(cost[S1] < INFINITY) || !(cost[S2] < INFINITY) || !(open[S1] & open[S2])) continue;
      // multiply-adds: every label of either operand once, = sqrt(|S1| |S2| |S|)
      const double c = cost[S1] + cost[S2] + std::sqrt(sz[S1] * sz[S2] * sz[S]);
      if (c < best) {
        best = c;
        bs = S1;
      }
    }
    cost[S] = best;
    split[S] = bs;
  }
  if (!(cost[full] < INFINITY)) return false;
  tree->left.assign((size_t)n, -1);
  tree->right.assign((size_t)n, -1);
  std::function<int(uint32_t)> build = [&](uint32_t S) -> int {
    if ((S & (S - 1)) == 0) return __builtin_ctz(S);
    const int l = build(split[S]), r = build(S ^ split[S]);
    tree->left.push_back(l);
    tree->right.push_back(r);
    return (int)tree->left.size() - 1;
  };
  tree->root = build(full);
  return true;
}

// Greedy: repeatedly join the pair (sharing a label) with the smallest result.
void greedy_tree(const std::vector<std::vector<int>> &labels, const std::vector<double> &ldim, Tree *tree) {
  const int n = (int)labels.size();
  tree->left.assign((size_t)n, -1);
  tree->right.assign((size_t)n, -1);
  std::vector<std::vector<int>> cur = labels;
  std::vector<int> node(n);
  for (int i = 0; i < n; ++i) node[(size_t)i] = i;
  while (cur.size() > 1) {
    int ba = -1, bb = -1;
    double bsz = 0.0, bfl = 0.0;
    for (size_t a = 0; a < cur.size(); ++a)
      for (size_t b = a + 1; b < cur.size(); ++b) {
        double osz = 1.0, shared = 1.0;
        bool share = false;
        for (int l : cur[a]) {
          if (std::find(cur[b].begin(), cur[b].end(), l) != cur[b].end()) {
            share = true;
            shared *= ldim[(size_t)l];
          } else {
            osz *= ldim[(size_t)l];
          }
        }
        if (!share) continue;
        for (int l : cur[b])
          if (std::find(cur[a].begin(), cur[a].end(), l) == cur[a].end()) osz *= ldim[(size_t)l];
        if (ba < 0 || osz < bsz || (osz == bsz && osz * shared < bfl)) {
          ba = (int)a;
          bb = (int)b;
          bsz = osz;
          bfl = osz * shared;
        }
      }
    std::vector<int> merged;
    for (int l : cur[(size_t)ba])
      if (std::find(cur[(size_t)bb].begin(), cur[(size_t)bb].end(), l) == cur[(size_t)bb].end()) merged.push_back(l);
    for (int l : cur[(size_t)bb])
      if (std::find(cur[(size_t)ba].begin(), cur[(size_t)ba].end(), l) == cur[(size_t)ba].end()) merged.push_back(l);
    tree->left.push_back(node[(size_t)ba]);
    tree->right.push_back(node[(size_t)bb]);
    node[(size_t)ba] = (int)tree->left.size() - 1;
    cur[(size_t)ba] = merged;
    cur.erase(cur.begin() + bb);
    node.erase(node.begin() + bb);
  }
  tree->root = node[0];
}

// Tensor sizes below each tree node (to evaluate the larger subtree first).
double subtree_size(const Tree &t, int v, const std::vector<DTensor> &ts, std::vector<double> *memo) {
  if (v < (int)ts.size()) return (double)ts[(size_t)v].size;
  double &m = (*memo)[(size_t)v];
  if (m < 0) m = subtree_size(t, t.left[(size_t)v], ts, memo) + subtree_size(t, t.right[(size_t)v], ts, memo);
  return m;
}

int run_tree(Mem &mem, const Tree &t, int v, std::vector<DTensor> &ts, std::vector<double> *memo, DTensor *out) {
  if (v < (int)ts.size()) {
    *out = ts[(size_t)v];
    ts[(size_t)v].ptr = nullptr;  // ownership moves to the caller
    return TN_OK;
  }
  int a = t.left[(size_t)v], b = t.right[(size_t)v];
  if (subtree_size(t, b, ts, memo) > subtree_size(t, a, ts, memo)) std::swap(a, b);
  DTensor A, B;
  int rc = run_tree(mem, t, a, ts, memo, &A);
  if (rc == TN_OK) rc = run_tree(mem, t, b, ts, memo, &B);
  if (rc != TN_OK) {
    mem.release(&A);
    mem.release(&B);
    return rc;
  }
  return contract_pair(mem, &A, &B, out);
}

}  // namespace

int contract_exact(const tn_network *net, hipStream_t st, double *out) {
  NetCheck chk;
  int rc = validate_network(net, 0, &chk);
  if (rc != TN_OK) return rc;
  if (!net->data) return set_error(TN_ERR_ARG, "null data array");
  for (int k = 0; k < net->p; ++k)
    if (!net->data[k]) return set_error(TN_ERR_ARG, "tensor %d: null data", k);
  // Labels after the traces, per tensor (host only, for the plan).
  const int p = net->p;
  std::vector<DTensor> shape((size_t)p);
  std::vector<double> ldim((size_t)std::max(1, net->t), 1.0);
  for (int k = 0; k < p; ++k) {
    DTensor &T = shape[(size_t)k];
    std::vector<int> all;
    for (int u = chk.offsets[(size_t)k]; u < chk.offsets[(size_t)k + 1]; ++u) {
      all.push_back(chk.edge_of[(size_t)u]);
      ldim[(size_t)chk.edge_of[(size_t)u]] = (double)net->dims[u];
    }
    for (size_t i = 0; i < all.size(); ++i)
      if (std::count(all.begin(), all.end(), all[i]) == 1) {
        T.labels.push_back(all[i]);
        T.dims.push_back(net->dims[chk.offsets[(size_t)k] + (int)i]);
        T.size *= net->dims[chk.offsets[(size_t)k] + (int)i];
      }
  }
  // Connected components over shared labels.
  std::vector<int> comp((size_t)p, -1);
  int n_comp = 0;
  for (int k = 0; k < p; ++k) {
    if (comp[(size_t)k] >= 0) continue;
    std::vector<int> stack{k};
    comp[(size_t)k] = n_comp;
    while (!stack.empty()) {
      const int a = stack.back();
      stack.pop_back();
      for (int b = 0; b < p; ++b) {
        if (comp[(size_t)b] >= 0) continue;
        bool share = false;
        for (int l : shape[(size_t)a].labels)
          share = share || std::find(shape[(size_t)b].labels.begin(), shape[(size_t)b].labels.end(), l) !=
                               shape[(size_t)b].labels.end();
        if (share) {
          comp[(size_t)b] = n_comp;
          stack.push_back(b);
        }
      }
    }
    ++n_comp;
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(TN_ERR_HIP, "exact contraction: hipMemGetInfo failed");
  }
  const double cap = (double)free_b / 8.0 / 3.0;
  std::vector<std::vector<int>> members((size_t)n_comp);
  std::vector<Tree> trees((size_t)n_comp);
  for (int k = 0; k < p; ++k) members[(size_t)comp[(size_t)k]].push_back(k);
  for (int c = 0; c < n_comp; ++c) {
    const std::vector<int> &mb = members[(size_t)c];
    std::vector<std::vector<int>> labs;
    for (int k : mb) labs.push_back(shape[(size_t)k].labels);
    bool ok = false;
    if (mb.size() <= (size_t)kDpMaxTensors && net->t <= 128) {
      std::vector<LabelSet> ls;
      for (const auto &l : labs) {
        LabelSet s = 0;
        for (int x : l) s |= (LabelSet)1 << x;
        ls.push_back(s);
      }
      ok = dp_tree(ls, ldim, cap, &trees[(size_t)c]);
    }
    if (!ok) greedy_tree(labs, ldim, &trees[(size_t)c]);
    log_msg(2, "exact: component %d: %zu tensors, %s tree", c, mb.size(), ok ? "fewest-flop (subset DP)" : "greedy");
  }
  // Dry run: the peak of live device memory.
  {
    Mem dry;
    dry.dry = true;
    for (int k = 0; k < p; ++k) {
      DTensor full;
      full.size = chk.sizes[(size_t)k];
      dry.alloc(&full);
      if (full.size != shape[(size_t)k].size) {  // traced: the result replaces it
        DTensor tr = shape[(size_t)k];
        dry.alloc(&tr);
        dry.release(&full);
      }
    }
    for (int c = 0; c < n_comp; ++c) {
      std::vector<DTensor> ts;
      for (int k : members[(size_t)c]) ts.push_back(shape[(size_t)k]);
      std::vector<double> memo(trees[(size_t)c].left.size(), -1.0);
      DTensor r;
      if ((rc = run_tree(dry, trees[(size_t)c], trees[(size_t)c].root, ts, &memo, &r)) != TN_OK) return rc;
    }
    log_msg(1, "exact: %d tensors in %d components, peak %.3g GB of device memory (%.3g GB free)", p, n_comp,
            (double)dry.peak / 1e9, (double)free_b / 1e9);
    if ((double)dry.peak > 0.92 * (double)free_b)
      return set_error(TN_ERR_OOM, "exact contraction needs %.3g GB of device memory at its peak, %.3g GB free",
                       (double)dry.peak / 1e9, (double)free_b / 1e9);
  }
  Mem mem;
  mem.st = st;
  std::vector<DTensor> ts((size_t)p);
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    for (DTensor &t : ts)
      if (t.ptr) (void)hipFree(t.ptr);
  };
  for (int k = 0; k < p; ++k) {
    DTensor &T = ts[(size_t)k];
    for (int u = chk.offsets[(size_t)k]; u < chk.offsets[(size_t)k + 1]; ++u) {
      T.labels.push_back(chk.edge_of[(size_t)u]);
      T.dims.push_back(net->dims[u]);
    }
    T.size = chk.sizes[(size_t)k];
    if ((rc = mem.alloc(&T)) != TN_OK) {
      cleanup();
      return rc;
    }
    const unsigned g = grid_for(T.size);
    if (net->dtype == TN_F64)
      hipLaunchKernelGGL(to_f64_kernel<double>, dim3(g), dim3(256), 0, st, (const double *)net->data[k], T.size, T.ptr);
    else if (net->dtype == TN_F32)
      hipLaunchKernelGGL(to_f64_kernel<float>, dim3(g), dim3(256), 0, st, (const float *)net->data[k], T.size, T.ptr);
    else
      hipLaunchKernelGGL(bf16_to_f64_kernel, dim3(g), dim3(256), 0, st, (const uint16_t *)net->data[k], T.size,
                         T.ptr);
    if (const hipError_t e = hipGetLastError(); e != hipSuccess) {
      cleanup();
      return set_error(TN_ERR_HIP, "exact contraction: %s", hipGetErrorString(e));
    }
    // Traces inside the tensor.
    std::vector<int> sum;
    std::vector<int64_t> sd;
    for (size_t i = 0; i < T.labels.size(); ++i)
      if (std::count(T.labels.begin(), T.labels.end(), T.labels[i]) == 2 &&
          std::find(sum.begin(), sum.end(), T.labels[i]) == sum.end()) {
        sum.push_back(T.labels[i]);
        sd.push_back(T.dims[i]);
      }
    if (sum.empty()) continue;
    if ((int)shape[(size_t)k].labels.size() > kMaxLabels || (int)sum.size() > kMaxLabels) {
      cleanup();
      return set_error(TN_ERR_UNSUPPORTED, "exact contraction: more than %d labels", kMaxLabels);
    }
    TraceDesc d{};
    std::vector<int64_t> stride(T.labels.size());
    int64_t acc = 1;
    for (int i = (int)T.labels.size() - 1; i >= 0; --i) {
      stride[(size_t)i] = acc;
      acc *= T.dims[(size_t)i];
    }
    auto stride_of = [&](int label) {
      int64_t v = 0;
      for (size_t i = 0; i < T.labels.size(); ++i)
        if (T.labels[i] == label) v += stride[i];
      return v;
    };
    const DTensor &sh = shape[(size_t)k];
    d.n_out = (int)sh.labels.size();
    d.n_sum = (int)sum.size();
    for (int i = 0; i < d.n_out; ++i) {
      d.out_dims[i] = sh.dims[(size_t)i];
      d.a_out[i] = stride_of(sh.labels[(size_t)i]);
    }
    for (int i = 0; i < d.n_sum; ++i) {
      d.sum_dims[i] = sd[(size_t)i];
      d.a_sum[i] = stride_of(sum[(size_t)i]);
    }
    DTensor C = sh;
    C.ptr = nullptr;
    if ((rc = mem.alloc(&C)) != TN_OK) {  // (C.ptr stays null on failure)
      cleanup();
      return rc;
    }
    hipLaunchKernelGGL(trace_kernel, dim3(grid_for(C.size)), dim3(256), 0, st, d, T.ptr, C.size, C.ptr);
    mem.release(&T);
    T = C;  // owned by ts from here, so cleanup() frees it on any later error
    if (const hipError_t e = hipGetLastError(); e != hipSuccess) {
      cleanup();
      return set_error(TN_ERR_HIP, "exact contraction: %s", hipGetErrorString(e));
    }
  }
  double result = 1.0;
  for (int c = 0; c < n_comp && rc == TN_OK; ++c) {
    std::vector<DTensor> part;
    for (int k : members[(size_t)c]) {
      part.push_back(ts[(size_t)k]);
      ts[(size_t)k].ptr = nullptr;
    }
    std::vector<double> memo(trees[(size_t)c].left.size(), -1.0);
    DTensor r;
    rc = run_tree(mem, trees[(size_t)c], trees[(size_t)c].root, part, &memo, &r);
    for (DTensor &t : part)
      if (t.ptr) mem.release(&t);
    if (rc != TN_OK) break;
    if (r.size != 1) {
      mem.release(&r);
      rc = set_error(TN_ERR_HIP, "exact contraction left an open tensor");
      break;
    }
    double v = 0.0;
    hipError_t e = hipMemcpyAsync(&v, r.ptr, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    mem.release(&r);
    if (e != hipSuccess) {
      rc = set_error(TN_ERR_HIP, "exact contraction: %s", hipGetErrorString(e));
      break;
    }
    result *= v;
  }
  cleanup();
  if (rc != TN_OK) return rc;
  *out = result;
  return TN_OK;
}

}  // namespace tn
