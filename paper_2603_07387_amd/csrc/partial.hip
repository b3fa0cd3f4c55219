// Partial tensor network contraction (Corollary 1) with the cyclic-network
// estimator.
//
// The output tensor Y is indexed by the free modes K' (Def. 1), row-major in
// increasing mode order.  By the corollary's proof, entry r is estimated by
// Eq. (1) applied to the full TNC of the sub-tensors X_k(s_k): every free mode
// fixed at r's index, every contracted mode kept.  The plan therefore turns
// tensor k into one "virtual" tensor per assignment of its own free modes (a
// contiguous sub-tensor once those modes lead; a tensor whose free modes do
// not lead is first copied with them moved to the front), scatters every
// virtual tensor once per sample, and combines, for each entry, the sketches
// of the virtual tensors that entry selects.  Every entry uses the same count
// sketches (the network's hash streams), so each tensor is read once per
// sample pass however many entries it feeds: cost O(q N + n_out p m log m)
// per sample, within the corollary's O(n^q' p m log m + q N).
#include <algorithm>
#include <cstring>
#include <memory>
#include <new>

#include "plan.h"

namespace tn {
namespace {

constexpr int64_t kMaxPartialOut = (int64_t)1 << 20;  // output entries per plan

// out[o] = in[permuted index]: out is the tensor with its free modes first
// (in mode order) and its contracted modes after them (in mode order).
struct PermDesc {
  int q;
  int64_t n;                  // entries
  int64_t out_dims[kMaxOrder];
  int64_t in_stride[kMaxOrder];  // input stride of the mode at each output position
};

template <typename T>
__global__ __launch_bounds__(256) void permute_kernel(PermDesc d, const void *const *__restrict__ src, int idx,
                                                      T *__restrict__ out) {
  const T *__restrict__ in = reinterpret_cast<const T *>(src[idx]);
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < d.n; o += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = o, off = 0;
    for (int i = d.q - 1; i >= 0; --i) {
      const int64_t dg = rem % d.out_dims[i];
      rem /= d.out_dims[i];
      off += dg * d.in_stride[i];
    }
    out[o] = in[off];
  }
}

size_t elem_size(int dtype) { return dtype == TN_F64 ? 8 : dtype == TN_F32 ? 4 : 2; }

template <typename T>
int dev_alloc_p(T **ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) return TN_OK;
  hipError_t e = hipMalloc((void **)ptr, count * sizeof(T));
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return set_error(e == hipErrorOutOfMemory ? TN_ERR_OOM : TN_ERR_HIP, "hipMalloc(%zu bytes): %s",
                     count * sizeof(T), hipGetErrorString(e));
  }
  return TN_OK;
}

}  // namespace

int partial_build(tn_plan *p, const tn_network *net) {
  NetCheck c;
  int rc = validate_network(net, 0, &c, /*allow_free=*/true);
  if (rc != TN_OK) return rc;
  // host-only checks first: a tensor with no contracted mode, the output size
  for (int k = 0; k < net->p; ++k) {
    bool any = false;
    for (int u = c.offsets[(size_t)k]; u < c.offsets[(size_t)k + 1]; ++u) any = any || c.edge_of[(size_t)u] >= 0;
    if (!any)
      return set_error(TN_ERR_UNSUPPORTED, "partial TNC: tensor %d has no contracted mode (an outer factor)", k);
  }
  {
    int64_t n_out = 1;
    for (int u = 0; u < c.q; ++u)
      if (c.edge_of[(size_t)u] < 0 && (n_out *= net->dims[u]) > kMaxPartialOut)
        return set_error(TN_ERR_UNSUPPORTED, "partial TNC: more than %lld output entries", (long long)kMaxPartialOut);
  }
  p->dtype = net->dtype;
  if ((rc = plan_common(p)) != TN_OK) return rc;
  if ((rc = m1_check_m(p)) != TN_OK) return rc;
  if (p->two_pass)
    return set_error(TN_ERR_UNSUPPORTED, "partial TNC: m = %lld needs the two-pass combine (not offered)",
                     (long long)p->m);
  const tn_network &n = *net;
  p->partial = true;
  p->dtype = n.dtype;
  // free modes, in global mode order
  std::vector<int> free_modes;
  for (int u = 0; u < c.q; ++u)
    if (c.edge_of[(size_t)u] < 0) free_modes.push_back(u);
  p->n_free = (int32_t)free_modes.size();
  int64_t n_out = 1;
  for (int u : free_modes) {
    n_out *= n.dims[u];
    if (n_out > kMaxPartialOut)
      return set_error(TN_ERR_UNSUPPORTED, "partial TNC: more than %lld output entries", (long long)kMaxPartialOut);
  }
  p->n_out = n_out;
  p->n_nets = (int)n_out;
  if ((int64_t)n_out * n.p > 0x7fffffff) return set_error(TN_ERR_UNSUPPORTED, "partial TNC: output too large");

  // one hash stream per contraction (the network's seed, as network 0 of a plan)
  std::vector<int64_t> stream_off((size_t)n.t);
  for (int e = 0; e < n.t; ++e) {
    StreamDesc sd{};
    sd.seed = p->seed;
    sd.stream = (uint64_t)e;
    sd.offset = p->W;
    sd.n = (int32_t)n.dims[n.edges[2 * e]];
    sd.net = 0;
    stream_off[(size_t)e] = p->W;
    p->W += sd.n;
    p->h_streams.push_back(sd);
  }

  // per tensor: its contracted modes (their count sketches), its sub-tensors
  const size_t es = elem_size(n.dtype);
  int64_t perm_bytes = 0;
  int32_t n_virtual = 0, n_perm = 0;
  p->pt.assign((size_t)n.p, tn_plan::PartialTensor{});
  for (int k = 0; k < n.p; ++k) {
    tn_plan::PartialTensor &T = p->pt[(size_t)k];
    const int q = n.order[k], u0 = c.offsets[(size_t)k];
    std::vector<int64_t> cdims;
    const int32_t mode0 = (int32_t)p->h_modes.size();
    bool seen_contracted = false;
    for (int i = 0; i < q; ++i) {
      const int u = u0 + i;
      T.dims.push_back(n.dims[u]);
      const int e = c.edge_of[(size_t)u];
      T.free.push_back(e < 0 ? 1 : 0);
      if (e < 0) {
        T.n_slices *= n.dims[u];
        if (seen_contracted) T.permute = true;  // a free mode after a contracted one
        continue;
      }
      seen_contracted = true;
      cdims.push_back(n.dims[u]);
      ModeDesc md{};
      md.table_off = stream_off[(size_t)e];
      md.n = (int32_t)n.dims[u];
      if (p->flags & TN_FLAG_PRIOR_XCORR)
        md.comp = ((n.p - 1 - k) & 1) ? 1 : 0;
      else
        md.comp = (n.edges[2 * e + 1] == u) ? 1 : 0;
      p->h_modes.push_back(md);
    }
    if (cdims.empty())
      return set_error(TN_ERR_UNSUPPORTED, "partial TNC: tensor %d has no contracted mode (an outer factor)", k);
    T.size = c.sizes[(size_t)k];
    T.slice = T.size / T.n_slices;
    T.first_virtual = n_virtual;
    if (T.permute) {
      T.perm_off = perm_bytes;
      T.perm_index = n_perm++;
      perm_bytes += (T.size * (int64_t)es + 255) / 256 * 256;
    }
    for (int64_t v = 0; v < T.n_slices; ++v, ++n_virtual) {
      if ((rc = add_tensor_slots(p, n_virtual, mode0, (int)cdims.size(), cdims.data(), T.slice, 0, k)) != TN_OK)
        return rc;
    }
  }
  p->n_tensors = n_virtual;
  p->net_p.push_back(n.p);
  p->net_orders.emplace_back(n.order, n.order + n.p);
  p->net_tensor0.push_back(0);

  // output entries: entry r takes, of every tensor, the sub-tensor at r's
  // indices of that tensor's free modes
  p->h_nets.clear();
  for (int64_t r = 0; r < n_out; ++r) p->h_nets.push_back(NetDesc{(int32_t)(r * n.p), (int32_t)((r + 1) * n.p)});
  if ((rc = m1_layout(p, nullptr)) != TN_OK) return rc;  // completes h_tslot with its end sentinel
  std::vector<int32_t> cbeg((size_t)(n_out * n.p)), cend((size_t)(n_out * n.p));
  std::vector<int64_t> digit(free_modes.size());
  for (int64_t r = 0; r < n_out; ++r) {
    int64_t rem = r;
    for (int i = (int)free_modes.size() - 1; i >= 0; --i) {
      digit[(size_t)i] = rem % n.dims[free_modes[(size_t)i]];
      rem /= n.dims[free_modes[(size_t)i]];
    }
    size_t fi = 0;  // free modes are visited in global order, tensor by tensor
    for (int k = 0; k < n.p; ++k) {
      const tn_plan::PartialTensor &T = p->pt[(size_t)k];
      int64_t proj = 0;
      for (size_t i = 0; i < T.free.size(); ++i)
        if (T.free[i]) proj = proj * T.dims[i] + digit[fi++];
      const int32_t vt = T.first_virtual + (int32_t)proj;
      cbeg[(size_t)(r * n.p + k)] = p->h_tslot[(size_t)vt];
      cend[(size_t)(r * n.p + k)] = p->h_tslot[(size_t)vt + 1];
    }
  }
  if ((rc = dev_alloc_p(&p->d_cbeg, cbeg.size())) != TN_OK) return rc;
  if ((rc = dev_alloc_p(&p->d_cend, cend.size())) != TN_OK) return rc;
  TN_HIP_CHECK(hipMemcpy(p->d_cbeg, cbeg.data(), cbeg.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  TN_HIP_CHECK(hipMemcpy(p->d_cend, cend.data(), cend.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  if (n_perm > 0) {
    unsigned char *buf = nullptr;
    if ((rc = dev_alloc_p(&buf, (size_t)perm_bytes)) != TN_OK) return rc;
    p->d_perm = buf;
    if ((rc = dev_alloc_p(&p->d_psrc, (size_t)n_perm)) != TN_OK) return rc;
    p->psrc.assign((size_t)n_perm, nullptr);
  }
  return TN_OK;
}

int partial_bind(tn_plan *p, const tn_network *nets, hipStream_t st) {
  const tn_network &n = nets[0];
  if (n.p != p->net_p[0] || n.dtype != p->dtype || !n.order || !n.data)
    return set_error(TN_ERR_ARG, "the network does not match the partial plan");
  const size_t es = elem_size(p->dtype);
  bool changed = false, pchanged = false;
  for (int k = 0; k < n.p; ++k) {
    if (n.order[k] != p->net_orders[0][(size_t)k])
      return set_error(TN_ERR_ARG, "tensor %d: order differs from the plan", k);
    if (!n.data[k]) return set_error(TN_ERR_ARG, "tensor %d: null data", k);
    const tn_plan::PartialTensor &T = p->pt[(size_t)k];
    const unsigned char *base = reinterpret_cast<const unsigned char *>(n.data[k]);
    if (T.permute) {
      if (p->psrc[(size_t)T.perm_index] != n.data[k]) {
        p->psrc[(size_t)T.perm_index] = n.data[k];
        pchanged = true;
      }
      base = reinterpret_cast<const unsigned char *>(p->d_perm) + T.perm_off;
    }
    for (int64_t v = 0; v < T.n_slices; ++v) {
      const void *ptr = base + (size_t)(v * T.slice) * es;
      const size_t g = (size_t)(T.first_virtual + v);
      if (p->bound[g] != ptr) {
        p->bound[g] = ptr;
        changed = true;
      }
    }
  }
  if (changed)
    TN_HIP_CHECK(hipMemcpyAsync(p->d_data, p->bound.data(), p->bound.size() * sizeof(void *),
                                hipMemcpyHostToDevice, st));
  if (pchanged)
    TN_HIP_CHECK(hipMemcpyAsync(p->d_psrc, p->psrc.data(), p->psrc.size() * sizeof(void *),
                                hipMemcpyHostToDevice, st));
  return TN_OK;
}

// Copy every tensor whose free modes do not lead into its permuted layout
// (free modes first); runs before each sketching pass, since the data may
// have changed in place.
int partial_prepare(tn_plan *p, hipStream_t st) {
  for (const tn_plan::PartialTensor &T : p->pt) {
    if (!T.permute) continue;
    PermDesc d{};
    const int q = (int)T.dims.size();
    d.q = q;
    d.n = T.size;
    std::vector<int64_t> stride((size_t)q);
    int64_t s = 1;
    for (int i = q - 1; i >= 0; --i) {
      stride[(size_t)i] = s;
      s *= T.dims[(size_t)i];
    }
    int o = 0;
    for (int pass = 1; pass >= 0; --pass)  // free modes first, then contracted, each in mode order
      for (int i = 0; i < q; ++i)
        if ((int)T.free[(size_t)i] == pass) {
          d.out_dims[o] = T.dims[(size_t)i];
          d.in_stride[o] = stride[(size_t)i];
          ++o;
        }
    void *out = reinterpret_cast<unsigned char *>(p->d_perm) + T.perm_off;
    const unsigned blocks = (unsigned)std::min<int64_t>((T.size + 255) / 256, 16384);
    if (p->dtype == TN_F64)
      hipLaunchKernelGGL(permute_kernel<double>, dim3(blocks), dim3(256), 0, st, d, p->d_psrc, T.perm_index,
                         reinterpret_cast<double *>(out));
    else if (p->dtype == TN_F32)
      hipLaunchKernelGGL(permute_kernel<float>, dim3(blocks), dim3(256), 0, st, d, p->d_psrc, T.perm_index,
                         reinterpret_cast<float *>(out));
    else
      hipLaunchKernelGGL(permute_kernel<uint16_t>, dim3(blocks), dim3(256), 0, st, d, p->d_psrc, T.perm_index,
                         reinterpret_cast<uint16_t *>(out));
    TN_HIP_CHECK(hipGetLastError());
  }
  return TN_OK;
}

void partial_release(tn_plan *p) {
  void *ptrs[] = {p->d_perm, (void *)p->d_psrc, p->d_cbeg, p->d_cend};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  p->d_perm = nullptr;
  p->d_psrc = nullptr;
  p->d_cbeg = p->d_cend = nullptr;
}

}  // namespace tn

using namespace tn;

extern "C" int tn_partial_plan(const tn_network *net, int64_t m, int64_t samples, uint64_t seed, uint32_t flags,
                               tn_plan **out) {
  clear_error();
  if (!out) return set_error(TN_ERR_ARG, "out is null");
  *out = nullptr;
  if (!net) return set_error(TN_ERR_ARG, "null network");
  if (samples < 1) return set_error(TN_ERR_ARG, "samples = %lld", (long long)samples);
  if (m < 1 || (m & (m - 1)) != 0) return set_error(TN_ERR_ARG, "m = %lld is not a power of two", (long long)m);
  if (flags & ~(uint32_t)(TN_FLAG_GRAPH | TN_FLAG_PROFILE | TN_FLAG_AUTOTUNE | TN_FLAG_PROFILE_SKETCH |
                          TN_FLAG_PRIOR_XCORR | TN_FLAG_DFT_BF16 | TN_FLAG_DFT_FP8))
    return set_error(TN_ERR_ARG, "flags 0x%x not offered for partial plans", flags);
  if ((flags & TN_FLAG_PROFILE_SKETCH) && !(flags & TN_FLAG_PROFILE))
    return set_error(TN_ERR_ARG, "TN_FLAG_PROFILE_SKETCH needs TN_FLAG_PROFILE");
  if ((flags & TN_FLAG_GRAPH) && (flags & TN_FLAG_PROFILE))
    return set_error(TN_ERR_ARG, "TN_FLAG_PROFILE cannot be combined with TN_FLAG_GRAPH");
  std::unique_ptr<tn_plan> plan(new (std::nothrow) tn_plan());
  if (!plan) return set_error(TN_ERR_OOM, "host allocation");
  tn_plan *p = plan.get();
  p->method = TN_CYCLIC;
  p->m = m;
  while ((1ll << p->log2m) < m) ++p->log2m;
  p->S = samples;
  p->seed = seed;
  p->flags = flags;
  int rc = partial_build(p, net);
  if (rc == TN_OK) rc = plan_alloc_tail(p);
  if (rc != TN_OK) {
    plan_release(p);
    return rc;
  }
  log_plan(p);
  *out = plan.release();
  return TN_OK;
}
