// Host-side plan of the tn_sketch library (not part of the public ABI).
#pragma once

#include <vector>

#include "tn_internal.h"

namespace tn {

constexpr int kMaxOrder = 16;
constexpr int64_t kMaxDim = 1 << 20;
constexpr int64_t kMaxTensor = (int64_t)1 << 31;

// Result of validating one network.
struct NetCheck {
  int32_t q = 0;
  std::vector<int32_t> offsets;    // p + 1
  std::vector<int64_t> sizes;      // entries per tensor
  std::vector<int32_t> edge_of;    // per mode
  std::vector<int32_t> tensor_of;  // per mode
};

int validate_network(const tn_network *n, int index, NetCheck *chk, bool allow_free = false);
int validate_tree(const tn_network *n, int index, const NetCheck &chk);
const char *last_error();

struct M2Plan;  // acyclic method, defined in m2.hip

}  // namespace tn

struct tn_plan {
  int device = 0;
  int method = 0;
  int64_t m = 0;
  int log2m = 0;
  int64_t S = 0;
  uint64_t seed = 0;
  uint32_t flags = 0;
  int root = 0;
  int dtype = 0;
  int n_nets = 0;
  int64_t n_tensors = 0;
  size_t max_lds = 65536;

  // structure, for checking the networks passed to estimate()
  std::vector<int32_t> net_p;
  std::vector<int64_t> net_tensor0;  // first global tensor of each network
  std::vector<int64_t> tensor_size;  // entries per global tensor
  std::vector<std::vector<int32_t>> net_orders;

  // hash streams
  std::vector<tn::StreamDesc> h_streams;
  int64_t max_stream = 0;  // the longest stream's indices
  int64_t W = 0;
  tn::StreamDesc *d_streams = nullptr;
  int32_t *d_tables = nullptr;    // [chunk][W]
  int32_t *d_injected = nullptr;  // [S][W] when tables are injected

  // data binding
  std::vector<const void *> bound;  // last pointers copied to d_data
  const void **d_data = nullptr;

  // cyclic method
  std::vector<tn::ModeDesc> h_modes;
  std::vector<tn::ScatterSlot> h_slots;
  std::vector<int32_t> h_tslot;  // per global tensor: first slot; n_tensors + 1 entries
  std::vector<tn::NetDesc> h_nets;
  tn::ModeDesc *d_modes = nullptr;
  tn::ScatterSlot *d_slots = nullptr;
  int32_t *d_tslot = nullptr;
  tn::NetDesc *d_nets = nullptr;
  void *d_tw = nullptr;
  void *d_ybuf = nullptr;
  double *d_slot_bound = nullptr;  // [slots]: power-of-two bound of |x| (see M1Launch)
  bool two_pass = false;        // the m-point FFT does not fit in LDS: two-pass combine
  int64_t n_pairs = 0;          // its tensor pairs (two real sketches per complex transform)
  int32_t *d_pairs = nullptr;   // [n_pairs][2]: tensors a, b (or -1)
  int32_t *d_pair0 = nullptr;   // [n_nets + 1]: first pair of each network
  void *d_cbuf = nullptr;       // the two-pass combine's transposed columns
  double *d_partial = nullptr;  // and its per-block row sums
  int32_t csplit = 1;           // in-LDS combine: blocks per (network, sample), each a share of the pairs
  double *d_csplit = nullptr;   // their partial product spectra [network][sample][block][m/2 + 1] (complex)
  int sb = 1;
  int banks = 1;            // scatter accumulator banks (autotuned: 1 or 2)
  size_t scatter_lds = 0;
  int64_t chunk = 0;        // samples per workspace pass
  int64_t chunk_alloc = 0;  // samples the workspace was sized for
  size_t worst_cols_rows = 0;
  bool tuned = false;
  bool tables_ready = false;  // d_tables holds every sample's tables (resident plans)

  // persistent fused kernel (TN_FLAG_PERSISTENT)
  bool fused = false;
  int fused_sb = 1;
  int fused_banks = 1;
  size_t fused_lds = 0;
  int64_t fused_chunk = 0;
  int64_t fused_chunk_cap = 0;       // samples per launch before rounding to fused_sb
  std::vector<int64_t> net_work;     // per network: entries + pair-FFT work
  int64_t fused_blocks = 0;
  int32_t n_items = 0;
  tn::FusedItem *d_items = nullptr;
  int32_t *d_counter = nullptr;
  int32_t *d_tensor_lgn = nullptr;

  // per-sample estimates [n_nets][S]
  double *d_est = nullptr;

  // partial TNC (Corollary 1; tn_partial_plan): the plan's "networks" are the
  // n_out entries of the output tensor.  Tensor k of the caller's network
  // becomes n_slices "virtual" tensors, the sub-tensors at each assignment of
  // its free modes; a tensor whose free modes are not its leading modes is
  // first copied with them moved to the front (perm_off into d_perm).
  struct PartialTensor {
    std::vector<int64_t> dims;   // the tensor's mode sizes
    std::vector<uint8_t> free;   // per mode: 1 if not contracted
    int64_t size = 0, slice = 0, n_slices = 1;
    int32_t first_virtual = 0;
    bool permute = false;
    int64_t perm_off = -1;       // byte offset of its copy in d_perm
    int32_t perm_index = -1;     // its entry in d_psrc
  };
  bool partial = false;
  int64_t n_out = 0;
  int32_t n_free = 0;
  std::vector<PartialTensor> pt;
  std::vector<const void *> psrc;  // bound source pointers of the permuted tensors
  const void **d_psrc = nullptr;
  void *d_perm = nullptr;
  int32_t *d_cbeg = nullptr;  // combine: per (entry, tensor) first slot ...
  int32_t *d_cend = nullptr;  // ... and end of slots

  // acyclic method
  tn::M2Plan *m2 = nullptr;

  // profiling events: (kind, start, stop) pending, and a pool of free events
  struct ProfRec {
    int kind;
    hipEvent_t start, stop;
  };
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> prof_pool;

  // graph replay
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t graph_stream = nullptr;
  double *graph_stats = nullptr;
  double *graph_samples = nullptr;
};

namespace tn {

int plan_build(tn_plan *p, const tn_network *nets, int n_nets, int method, int64_t m,
               int64_t S, uint64_t seed, int root, uint32_t flags);
int plan_estimate(tn_plan *p, const tn_network *nets, hipStream_t st, double *stats,
                  double *samples_out);
void plan_release(tn_plan *p);
int64_t plan_query(const tn_plan *p, int key);
int plan_get_hashes(tn_plan *p, int64_t first, int64_t count, hipStream_t st, int32_t *out);
int plan_set_hashes(tn_plan *p, const int32_t *tables, hipStream_t st);
int plan_get_sketches(tn_plan *p, const tn_network *nets, int64_t first, int64_t count,
                      hipStream_t st, double *out);
int plan_bind(tn_plan *p, const tn_network *nets, hipStream_t st);
// cyclic-method plan building blocks (plan.hip), shared with the partial planner
int m1_check_m(tn_plan *p);
int add_tensor_slots(tn_plan *p, int32_t gtensor, int32_t mode0, int q, const int64_t *dims, int64_t size,
                     int net, int k);
int m1_layout(tn_plan *p, const std::vector<NetCheck> *chk);
void log_plan(const tn_plan *p);
int plan_common(tn_plan *p);
int plan_alloc_tail(tn_plan *p);
// resident sketches (TN_FLAG_RESIDENT)
int plan_update(tn_plan *p, int net, int tensor, int64_t n, const int64_t *idx, const double *delta, hipStream_t st);
int plan_combine(tn_plan *p, hipStream_t st, double *stats, double *samples_out);
int plan_reset(tn_plan *p, hipStream_t st);
// automatic sketch size of tn_sketch_plan (sizing.hip)
int auto_size(const tn_network *nets, int n_nets, int method, uint32_t flags, uint64_t seed, int64_t samples,
              int64_t *m_out, int64_t *S_out);
// partial TNC (partial.hip)
int partial_build(tn_plan *p, const tn_network *net);
int partial_bind(tn_plan *p, const tn_network *nets, hipStream_t st);
int partial_prepare(tn_plan *p, hipStream_t st);
void partial_release(tn_plan *p);
int prof_begin(tn_plan *p, hipStream_t st, hipEvent_t *ev, int kind);
int prof_end(tn_plan *p, hipStream_t st, int kind, hipEvent_t start);
int plan_kernel_time(tn_plan *p, int kind, double *ms, int64_t *launches);

// acyclic method (m2.hip)
int m2_build(tn_plan *p, const tn_network *nets, const std::vector<NetCheck> &chk);
int m2_estimate(tn_plan *p, hipStream_t st, double *est);
int m2_autotune(tn_plan *p, hipStream_t st);
int m2_get_sketches(tn_plan *p, int64_t first, int64_t count, hipStream_t st, double *out);
void m2_release(tn_plan *p);

}  // namespace tn
