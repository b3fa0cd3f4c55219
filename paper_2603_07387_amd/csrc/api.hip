// C ABI of the tn_sketch library: validation, planning and launch sequencing.
//
// Validation follows the problem statement of Def. 1 (u != v, n_u = n_v) and
// WLOG 1 of the Methods section (every mode in exactly one contraction); the
// acyclic method further needs a tree (Section "Improved approximation for
// acyclic tensor network contraction").  All checks run on the host before any
// device allocation or launch.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "plan.h"

namespace tn {

static thread_local char g_err[1024] = "";

int set_error(int code, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_err[0] = '\0'; }

int log_level() {
  const char *e = std::getenv("TN_LOG");
  return e ? std::atoi(e) : 0;
}

void log_msg(int level, const char *fmt, ...) {
  if (log_level() < level) return;
  char line[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(line, sizeof(line), fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[tn] %s\n", line);
}

const char *last_error() { return g_err; }

int validate_network(const tn_network *n, int index, NetCheck *chk, bool allow_free) {
  if (!n) return set_error(TN_ERR_ARG, "network %d: null", index);
  if (n->p < 1) return set_error(TN_ERR_ARG, "network %d: p = %d", index, n->p);
  if (!n->order || !n->dims || (n->t > 0 && !n->edges))
    return set_error(TN_ERR_ARG, "network %d: null order/dims/edges", index);
  if (n->t < 0) return set_error(TN_ERR_ARG, "network %d: t = %d", index, n->t);
  if (n->dtype != TN_F64 && n->dtype != TN_F32 && n->dtype != TN_BF16)
    return set_error(TN_ERR_ARG, "network %d: dtype %d", index, n->dtype);
  int64_t q = 0;
  chk->offsets.assign((size_t)n->p + 1, 0);
  for (int k = 0; k < n->p; ++k) {
    if (n->order[k] < 1 || n->order[k] > kMaxOrder)
      return set_error(n->order[k] < 1 ? TN_ERR_ARG : TN_ERR_UNSUPPORTED,
                       "network %d: tensor %d has order %d (1..%d supported)", index, k,
                       n->order[k], kMaxOrder);
    q += n->order[k];
    chk->offsets[k + 1] = (int32_t)q;
  }
  chk->q = (int32_t)q;
  chk->sizes.assign((size_t)n->p, 1);
  for (int k = 0; k < n->p; ++k) {
    for (int u = chk->offsets[k]; u < chk->offsets[k + 1]; ++u) {
      if (n->dims[u] < 1) return set_error(TN_ERR_ARG, "network %d: mode %d has size %lld", index, u, (long long)n->dims[u]);
      if (n->dims[u] > kMaxDim)
        return set_error(TN_ERR_UNSUPPORTED, "network %d: mode %d has size %lld > %lld", index, u,
                         (long long)n->dims[u], (long long)kMaxDim);
      chk->sizes[k] *= n->dims[u];
      if (chk->sizes[k] > kMaxTensor)
        return set_error(TN_ERR_UNSUPPORTED, "network %d: tensor %d exceeds %lld entries", index,
                         k, (long long)kMaxTensor);
    }
  }
  chk->edge_of.assign((size_t)q, -1);
  chk->tensor_of.assign((size_t)q, 0);
  for (int k = 0; k < n->p; ++k)
    for (int u = chk->offsets[k]; u < chk->offsets[k + 1]; ++u) chk->tensor_of[u] = k;
  for (int e = 0; e < n->t; ++e) {
    const int u = n->edges[2 * e], v = n->edges[2 * e + 1];
    if (u < 0 || u >= q || v < 0 || v >= q)
      return set_error(TN_ERR_ARG, "network %d: edge %d names mode outside [0, %lld)", index, e, (long long)q);
    if (u == v) return set_error(TN_ERR_ARG, "network %d: edge %d contracts mode %d with itself", index, e, u);
    if (n->dims[u] != n->dims[v])
      return set_error(TN_ERR_DIMS, "network %d: edge %d joins modes of size %lld and %lld", index,
                       e, (long long)n->dims[u], (long long)n->dims[v]);
    if (chk->edge_of[u] >= 0 || chk->edge_of[v] >= 0)
      return set_error(TN_ERR_HYPEREDGE, "network %d: edge %d reuses a mode already contracted", index, e);
    chk->edge_of[u] = e;
    chk->edge_of[v] = e;
  }
  for (int u = 0; u < q && !allow_free; ++u)
    if (chk->edge_of[u] < 0)
      return set_error(TN_ERR_PARTIAL, "network %d: mode %d is not contracted (partial TNC)", index, u);
  return TN_OK;
}

int validate_tree(const tn_network *n, int index, const NetCheck &chk) {
  for (int e = 0; e < n->t; ++e)
    if (chk.tensor_of[n->edges[2 * e]] == chk.tensor_of[n->edges[2 * e + 1]])
      return set_error(TN_ERR_SELFLOOP, "network %d: edge %d contracts two modes of one tensor", index, e);
  if (n->t != n->p - 1)
    return set_error(TN_ERR_CYCLIC, "network %d: %d contractions for %d tensors is not a tree",
                     index, n->t, n->p);
  // connectivity (with t = p - 1, connected <=> acyclic)
  std::vector<int> parent(n->p);
  for (int k = 0; k < n->p; ++k) parent[k] = k;
  auto find = [&](int x) {
    while (parent[x] != x) x = parent[x] = parent[parent[x]];
    return x;
  };
  for (int e = 0; e < n->t; ++e) {
    const int a = find(chk.tensor_of[n->edges[2 * e]]), b = find(chk.tensor_of[n->edges[2 * e + 1]]);
    if (a == b) return set_error(TN_ERR_CYCLIC, "network %d: edge %d closes a cycle", index, e);
    parent[a] = b;
  }
  return TN_OK;
}

}  // namespace tn

using namespace tn;

extern "C" {

const char *tn_last_error(void) { return tn::last_error(); }

int tn_sketch_plan(const tn_network *nets, int32_t n_nets, int32_t method, int64_t m,
                   int64_t samples, uint64_t seed, int32_t root, uint32_t flags, tn_plan **out) {
  clear_error();
  if (!out) return set_error(TN_ERR_ARG, "out is null");
  *out = nullptr;
  if (!nets || n_nets < 1) return set_error(TN_ERR_ARG, "need at least one network");
  if (samples < 1 && m > 0) return set_error(TN_ERR_ARG, "samples = %lld", (long long)samples);
  if (m > 0 && (m & (m - 1)) != 0) return set_error(TN_ERR_ARG, "m = %lld is not a power of two", (long long)m);
  if (method != TN_CYCLIC && method != TN_ACYCLIC) return set_error(TN_ERR_ARG, "method %d", method);
  if ((flags & TN_FLAG_SIZE_PILOT) && (flags & TN_FLAG_SIZE_LEARNED))
    return set_error(TN_ERR_ARG, "TN_FLAG_SIZE_PILOT and TN_FLAG_SIZE_LEARNED exclude each other");
  if ((flags & (TN_FLAG_SIZE_PILOT | TN_FLAG_SIZE_LEARNED)) && m > 0)
    return set_error(TN_ERR_ARG, "sizing flags need m <= 0");
  if (flags & ~(uint32_t)(TN_FLAG_GRAPH | TN_FLAG_PROFILE | TN_FLAG_AUTOTUNE | TN_FLAG_MFMA_BF16 |
                          TN_FLAG_PERSISTENT | TN_FLAG_PROFILE_SKETCH | TN_FLAG_PRIOR_XCORR |
                          TN_FLAG_RESIDENT | TN_FLAG_SIZE_PILOT | TN_FLAG_SIZE_LEARNED | TN_FLAG_DFT_BF16 |
                          TN_FLAG_MFMA_F32 | TN_FLAG_DFT_FP8))
    return set_error(TN_ERR_ARG, "unknown flags 0x%x", flags);
  if ((flags & TN_FLAG_RESIDENT) && (method != TN_CYCLIC || (flags & TN_FLAG_PERSISTENT)))
    return set_error(TN_ERR_UNSUPPORTED, "TN_FLAG_RESIDENT applies to the cyclic method's slot kernels");
  if ((flags & TN_FLAG_DFT_BF16) && (method != TN_CYCLIC || (flags & TN_FLAG_PERSISTENT)))
    return set_error(TN_ERR_UNSUPPORTED, "TN_FLAG_DFT_BF16 applies to the cyclic method's two-kernel path");
  if ((flags & TN_FLAG_DFT_FP8) && (method != TN_CYCLIC || (flags & (TN_FLAG_PERSISTENT | TN_FLAG_DFT_BF16))))
    return set_error(TN_ERR_UNSUPPORTED,
                     "TN_FLAG_DFT_FP8 applies to the cyclic method's two-kernel path, without TN_FLAG_DFT_BF16");
  if ((flags & TN_FLAG_PRIOR_XCORR) && method != TN_CYCLIC)
    return set_error(TN_ERR_UNSUPPORTED, "TN_FLAG_PRIOR_XCORR applies to the cyclic method");
  if ((flags & TN_FLAG_PROFILE_SKETCH) && !(flags & TN_FLAG_PROFILE))
    return set_error(TN_ERR_ARG, "TN_FLAG_PROFILE_SKETCH needs TN_FLAG_PROFILE");
  if ((flags & TN_FLAG_PERSISTENT) && method != TN_CYCLIC)
    return set_error(TN_ERR_UNSUPPORTED, "TN_FLAG_PERSISTENT applies to the cyclic method");
  if ((flags & TN_FLAG_MFMA_BF16) && method != TN_ACYCLIC)
    return set_error(TN_ERR_UNSUPPORTED, "TN_FLAG_MFMA_BF16 applies to the acyclic method");
  if ((flags & TN_FLAG_MFMA_F32) && (method != TN_ACYCLIC || (flags & TN_FLAG_MFMA_BF16)))
    return set_error(TN_ERR_UNSUPPORTED, "TN_FLAG_MFMA_F32 applies to the acyclic method without BF16 products");
  if ((flags & TN_FLAG_MFMA_F32) && nets[0].dtype == TN_F64)
    return set_error(TN_ERR_UNSUPPORTED, "TN_FLAG_MFMA_F32 is for FP32 and BF16 data");
  if ((flags & TN_FLAG_GRAPH) && (flags & TN_FLAG_PROFILE))
    return set_error(TN_ERR_ARG, "TN_FLAG_PROFILE cannot be combined with TN_FLAG_GRAPH");
  if (m <= 0) {
    // validate before any device work, then choose (m, S)
    for (int j = 0; j < n_nets; ++j) {
      NetCheck c;
      int rc = validate_network(&nets[j], j, &c);
      if (rc == TN_OK && method == TN_ACYCLIC) rc = validate_tree(&nets[j], j, c);
      if (rc != TN_OK) return rc;
    }
    int64_t am = 0, aS = 0;
    const int rc = auto_size(nets, n_nets, method, flags, seed, samples, &am, &aS);
    if (rc != TN_OK) return rc;
    m = am;
    samples = aS;
    clear_error();
  }
  std::unique_ptr<tn_plan> plan(new (std::nothrow) tn_plan());
  if (!plan) return set_error(TN_ERR_OOM, "host allocation");
  int rc = plan_build(plan.get(), nets, n_nets, method, m, samples, seed, root,
                      flags & ~(uint32_t)(TN_FLAG_SIZE_PILOT | TN_FLAG_SIZE_LEARNED));
  if (rc != TN_OK) return rc;
  *out = plan.release();
  return TN_OK;
}

int tn_sketch_estimate(tn_plan *plan, const tn_network *nets, void *stream, double *stats,
                       double *samples_out) {
  clear_error();
  if (!plan || !nets || !stats) return set_error(TN_ERR_ARG, "null plan, networks or stats");
  return plan_estimate(plan, nets, (hipStream_t)stream, stats, samples_out);
}

int tn_contract_exact(const tn_network *net, void *stream, double *out) {
  clear_error();
  if (!net || !out) return set_error(TN_ERR_ARG, "null network or out");
  return contract_exact(net, (hipStream_t)stream, out);
}

void tn_plan_destroy(tn_plan *plan) {
  if (!plan) return;
  plan_release(plan);
  delete plan;
}

int64_t tn_plan_query(const tn_plan *plan, int32_t key) {
  clear_error();
  if (!plan) return set_error(TN_ERR_ARG, "null plan");
  return plan_query(plan, key);
}

int tn_plan_stream(const tn_plan *plan, int64_t i, int32_t *net, uint64_t *stream_id, int64_t *n,
                   int64_t *offset) {
  clear_error();
  if (!plan) return set_error(TN_ERR_ARG, "null plan");
  if (i < 0 || i >= (int64_t)plan->h_streams.size()) return set_error(TN_ERR_ARG, "stream %lld", (long long)i);
  const StreamDesc &sd = plan->h_streams[(size_t)i];
  if (net) *net = sd.net;
  if (stream_id) *stream_id = sd.stream;
  if (n) *n = sd.n;
  if (offset) *offset = sd.offset;
  return TN_OK;
}

int tn_plan_get_hashes(tn_plan *plan, int64_t first, int64_t count, void *stream, int32_t *out) {
  clear_error();
  if (!plan || !out) return set_error(TN_ERR_ARG, "null plan or out");
  return plan_get_hashes(plan, first, count, (hipStream_t)stream, out);
}

int tn_plan_set_hashes(tn_plan *plan, const int32_t *tables, void *stream) {
  clear_error();
  if (!plan) return set_error(TN_ERR_ARG, "null plan");
  return plan_set_hashes(plan, tables, (hipStream_t)stream);
}

int tn_plan_get_sketches(tn_plan *plan, const tn_network *nets, int64_t first, int64_t count,
                         void *stream, double *out) {
  clear_error();
  if (!plan || !nets || !out) return set_error(TN_ERR_ARG, "null plan, networks or out");
  return plan_get_sketches(plan, nets, first, count, (hipStream_t)stream, out);
}

int tn_sketch_update(tn_plan *plan, int32_t net, int32_t tensor, int64_t n, const int64_t *index,
                     const double *delta, void *stream) {
  clear_error();
  if (!plan) return set_error(TN_ERR_ARG, "null plan");
  return plan_update(plan, net, tensor, n, index, delta, (hipStream_t)stream);
}

int tn_sketch_combine(tn_plan *plan, void *stream, double *stats, double *samples_out) {
  clear_error();
  if (!plan || !stats) return set_error(TN_ERR_ARG, "null plan or stats");
  return plan_combine(plan, (hipStream_t)stream, stats, samples_out);
}

int tn_sketch_reset(tn_plan *plan, void *stream) {
  clear_error();
  if (!plan) return set_error(TN_ERR_ARG, "null plan");
  return plan_reset(plan, (hipStream_t)stream);
}

int tn_plan_kernel_time(tn_plan *plan, int32_t kind, double *ms, int64_t *launches) {
  clear_error();
  if (!plan || !ms || !launches) return set_error(TN_ERR_ARG, "null argument");
  return plan_kernel_time(plan, kind, ms, launches);
}

}  // extern "C"
