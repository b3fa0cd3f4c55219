// Planner and launch sequencing for the estimators.
//
// Cyclic method (Eq. (1), Algorithm 1): one hash stream per contraction e of
// network j (key seed + j, stream e).  The first mode of the contraction owns
// the count sketch, the second reads its complement (Def. 14).  Each tensor is
// viewed as a (rows x L) matrix whose L columns cover its trailing modes, and
// is cut into slots of at most kMaxSlotEntries entries; every slot is streamed
// once per batch of `sb` samples by the scatter kernel.
#include <algorithm>
#include <cstring>
#include <cstdlib>
#include <mutex>

#include "plan.h"
#include "m1_device.h"

namespace tn {
namespace {

constexpr int kMaxRowsPerSlot = 2048;
constexpr size_t kWorkspaceBudget = (size_t)1 << 30;  // tables + sketches per pass
constexpr int64_t kCombineSplitBlocks = 1024;            // combine blocks to aim for when splitting
constexpr size_t kCombineSplitBudget = (size_t)256 << 20;  // bytes of partial spectra
constexpr int64_t kCombineSplitWork = 65536;               // least (pairs x m) of a network worth splitting
constexpr size_t kResidentBudget = (size_t)16 << 30;  // all samples' sketches and tables (TN_FLAG_RESIDENT)

template <typename T>
int dev_alloc(T **ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) return TN_OK;
  hipError_t e = hipMalloc((void **)ptr, count * sizeof(T));
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return set_error(e == hipErrorOutOfMemory ? TN_ERR_OOM : TN_ERR_HIP,
                     "hipMalloc(%zu bytes): %s", count * sizeof(T), hipGetErrorString(e));
  }
  return TN_OK;
}

template <typename T>
int upload(T **ptr, const std::vector<T> &v) {
  int rc = dev_alloc(ptr, v.size());
  if (rc != TN_OK || v.empty()) return rc;
  TN_HIP_CHECK(hipMemcpy(*ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return TN_OK;
}

size_t acc_size(int dtype) { return dtype == TN_F64 ? sizeof(double) : sizeof(float); }

// LDS of one scatter block: the fixed-point accumulators (p->banks banks of m
// 8-byte words per sample) plus the packed tables.  (+64: the accumulator
// block is padded to 16 bytes and the kernel keeps a 16-byte running maximum
// in static LDS.)
size_t scatter_lds_for(const tn_plan *p, int sb) {
  const int64_t ma = std::min<int64_t>(p->m, (int64_t)1 << kMaxLog2Acc);  // bucket ranges above
  const size_t acc = p->banks == 2 ? m1dev::sign_bank_bytes(sb, (uint32_t)p->m) : (size_t)sb * 8 * ma;
  return acc + (size_t)sb * 4 * p->worst_cols_rows + 64;
}

constexpr size_t kFusedStatic = 128;  // static LDS of the persistent kernel

// Configure the persistent kernel for `sb` samples per item and `banks`
// accumulator banks: LDS, chunk (a multiple of sb), the work items of one
// chunk sorted by decreasing network work, and the grid (CUs x blocks per CU).
int fused_configure(tn_plan *p, int sb, int banks) {
  const size_t lds = m1_fused_lds(sb, banks, p->m, (int32_t)p->worst_cols_rows);
  if (lds + kFusedStatic > p->max_lds)
    return set_error(TN_ERR_UNSUPPORTED, "persistent kernel needs %zu bytes of LDS", lds + kFusedStatic);
  int64_t fc = p->fused_chunk_cap;
  if (fc > sb) fc = fc / sb * sb;
  std::vector<FusedItem> items;
  for (int j = 0; j < p->n_nets; ++j)
    for (int64_t s0 = 0; s0 < fc; s0 += sb) items.push_back(FusedItem{j, (int32_t)s0});
  std::stable_sort(items.begin(), items.end(), [&](const FusedItem &a, const FusedItem &b) {
    return p->net_work[(size_t)a.net] > p->net_work[(size_t)b.net];
  });
  if (items.size() > 0x7fffffff) return set_error(TN_ERR_UNSUPPORTED, "persistent kernel: too many items");
  if (p->d_items) (void)hipFree(p->d_items);
  p->d_items = nullptr;
  int rc = upload(&p->d_items, items);
  if (rc != TN_OK) return rc;
  int cus = 0;
  TN_HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device));
  const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(8, (int64_t)(160 * 1024) / (int64_t)(lds + kFusedStatic)));
  p->fused_sb = sb;
  p->fused_banks = banks;
  p->fused_lds = lds;
  p->fused_chunk = fc;
  p->n_items = (int32_t)items.size();
  p->fused_blocks = std::max<int64_t>(1, std::min<int64_t>((int64_t)items.size(), (int64_t)cus * per_cu));
  return TN_OK;
}

}  // namespace

// Cut tensor `gtensor` (q modes at plan modes mode0.., sizes dims[0..q), `size`
// entries) into scatter slots: a (rows x L) matrix view whose L <= kMaxCols
// columns are its trailing modes, at most kMaxSlotEntries entries per slot.
int add_tensor_slots(tn_plan *p, int32_t gtensor, int32_t mode0, int q, const int64_t *dims, int64_t size,
                     int net, int k) {
  int split = q;
  int64_t L = 1;
  while (split > 0 && L * dims[split - 1] <= kMaxCols) {
    L *= dims[split - 1];
    --split;
  }
  if (split == q)
    return set_error(TN_ERR_UNSUPPORTED, "cyclic method: network %d tensor %d has a last mode of size %lld > %d",
                     net, k, (long long)dims[q - 1], kMaxCols);
  const int64_t R = size / L;
  const int64_t rows_per = std::max<int64_t>(1, std::min<int64_t>(kMaxRowsPerSlot, kMaxSlotEntries / L));
  p->h_tslot.push_back((int32_t)p->h_slots.size());
  for (int64_t r0 = 0; r0 < R; r0 += rows_per) {
    ScatterSlot sl{};
    sl.tensor = gtensor;
    sl.q = q;
    sl.split = split;
    sl.L = (int32_t)L;
    sl.mode0 = mode0;
    sl.rows = (int32_t)std::min<int64_t>(rows_per, R - r0);
    sl.row0 = r0;
    sl.magic = L > 1 ? (uint32_t)(((uint64_t)1 << 32) / (uint64_t)L + 1) : 0u;
    p->h_slots.push_back(sl);
  }
  return TN_OK;
}

// The m-dependent limits of the cyclic method: m <= 2^16, and the combine's
// FFT in LDS or (from 2^14 points) in two passes through HBM.
int m1_check_m(tn_plan *p) {
  const size_t as = acc_size(p->dtype);
  if (p->log2m > kMaxLog2M1)
    return set_error(TN_ERR_UNSUPPORTED, "cyclic method: m = %lld exceeds %d", (long long)p->m,
                     1 << kMaxLog2M1);
  if ((p->flags & (TN_FLAG_DFT_BF16 | TN_FLAG_DFT_FP8)) && (p->m != 1024 || p->dtype == TN_F64))
    return set_error(TN_ERR_UNSUPPORTED, "TN_FLAG_DFT_BF16 / TN_FLAG_DFT_FP8: m = 1024 with FP32 or BF16 data only");
  p->two_pass = (size_t)p->m * 2 * as > p->max_lds;
  if (p->two_pass && p->log2m < kMaxLog2Acc)
    return set_error(TN_ERR_UNSUPPORTED, "cyclic method: the m-point FFT needs %zu bytes of LDS",
                     (size_t)p->m * 2 * as);
  return TN_OK;
}

int m1_build(tn_plan *p, const tn_network *nets, const std::vector<NetCheck> &chk) {
  int rc0 = m1_check_m(p);
  if (rc0 != TN_OK) return rc0;
  int64_t gmode = 0, gtensor = 0;
  for (int j = 0; j < p->n_nets; ++j) {
    const tn_network &n = nets[j];
    const NetCheck &c = chk[(size_t)j];
    std::vector<int64_t> stream_off((size_t)n.t);
    for (int e = 0; e < n.t; ++e) {
      StreamDesc sd{};
      sd.seed = p->seed + (uint64_t)j;
      sd.stream = (uint64_t)e;
      sd.offset = p->W;
      sd.n = (int32_t)n.dims[n.edges[2 * e]];
      sd.net = j;
      stream_off[(size_t)e] = p->W;
      p->W += sd.n;
      p->h_streams.push_back(sd);
    }
    NetDesc nd{(int32_t)gtensor, (int32_t)(gtensor + n.p)};
    p->h_nets.push_back(nd);
    for (int u = 0; u < c.q; ++u) {
      const int e = c.edge_of[(size_t)u];
      ModeDesc md{};
      md.table_off = stream_off[(size_t)e];
      md.n = (int32_t)n.dims[u];
      // Eq. (1): the second mode of each contraction takes the complement
      // (Def. 14).  The earlier cross-correlation chain instead conjugates the
      // whole spectrum of every tensor at an odd distance from the last one,
      // which by Lemma 5 is the complement on all of that tensor's modes.
      if (p->flags & TN_FLAG_PRIOR_XCORR)
        md.comp = ((n.p - 1 - c.tensor_of[(size_t)u]) & 1) ? 1 : 0;
      else
        md.comp = (n.edges[2 * e + 1] == u) ? 1 : 0;
      p->h_modes.push_back(md);
    }
    for (int k = 0; k < n.p; ++k, ++gtensor) {
      const int32_t mode0 = (int32_t)(gmode + c.offsets[(size_t)k]);
      const int rc = add_tensor_slots(p, (int32_t)gtensor, mode0, n.order[k], n.dims + c.offsets[(size_t)k],
                                      c.sizes[(size_t)k], j, k);
      if (rc != TN_OK) return rc;
    }
    gmode += c.q;
  }
  return m1_layout(p, &chk);
}

// Schedule, workspace and device tables of a cyclic plan whose slots, modes,
// streams and networks are in place.  chk (the networks' checks) is needed by
// the persistent kernel only.
int m1_layout(tn_plan *p, const std::vector<NetCheck> *chkp) {
  const size_t as = acc_size(p->dtype);
  const bool big = p->log2m > kMaxLog2Acc;  // bucket ranges in the scatter
  p->h_tslot.push_back((int32_t)p->h_slots.size());

  // Samples per scatter block: as many as fit 64 KB of LDS (two blocks per CU),
  // else one.
  size_t worst_cols_rows = 0;
  for (const ScatterSlot &sl : p->h_slots)
    worst_cols_rows = std::max(worst_cols_rows, (size_t)(sl.L + kColPad + sl.rows + 1));
  // 64-bit fixed-point accumulators (two banks of 8-byte words per sample)
  // plus packed tables.  (+64: the accumulator block is padded to 16 bytes and
  // the kernel keeps a 16-byte running maximum in static LDS.)
  // One bank with signed adds by default; TN_FLAG_AUTOTUNE also times two
  // banks (the sign in the address: fewer ALU operations, twice the LDS).
  p->worst_cols_rows = worst_cols_rows;
  p->banks = 1;
  auto lds_for = [&](int sb) { return scatter_lds_for(p, sb); };
  p->sb = 1;
  for (int sb : {8, 4, 2}) {
    if (sb <= p->S && lds_for(sb) <= 81920) { p->sb = sb; break; }
  }
  // Overrides of the untuned schedule (tests and tuning experiments; the
  // autotuner, when requested, still decides).
  if (big) p->sb = 1;  // bucket ranges: one bank, one sample per pass
  if (const char *env = getenv("TN_SCATTER_BANKS"); env && !big) {
    const int banks = atoi(env);
    if (banks == 1 || banks == 2) {
      const int save = p->banks;
      p->banks = banks;
      if (lds_for(1) > p->max_lds) p->banks = save;
      else if (lds_for(p->sb) > 81920) p->sb = 1;
    }
  }
  if (const char *env = getenv("TN_SCATTER_SB"); env && !big) {
    const int sb = atoi(env);
    if ((sb == 1 || sb == 2 || sb == 4 || sb == 8 || sb == 16) && lds_for(sb) <= p->max_lds &&
        scatter_words(sb, p->dtype) <= kMaxScatterWords)
      p->sb = sb;
  }
  p->scatter_lds = lds_for(p->sb);
  p->worst_cols_rows = worst_cols_rows;
  if (p->scatter_lds > p->max_lds)
    return set_error(TN_ERR_UNSUPPORTED, "cyclic method: scatter needs %zu bytes of LDS", p->scatter_lds);

  const size_t per_sample = (size_t)p->W * 4 + p->h_slots.size() * (size_t)p->m * as +
                            (p->two_pass ? (size_t)(p->n_tensors + p->n_nets) / 2 * (size_t)p->m * 2 * as +
                                               (size_t)p->n_nets * kBigPartials * 8
                                         : 0);
  int64_t chunk = (int64_t)std::max<size_t>(1, kWorkspaceBudget / std::max<size_t>(1, per_sample));
  chunk = std::min<int64_t>(chunk, p->S);
  chunk = std::min<int64_t>(chunk, 65535);
  if (p->flags & TN_FLAG_RESIDENT) {
    // every sample's sketches and hash tables stay in device memory
    if (p->S > 65535 || (double)per_sample * (double)p->S > (double)kResidentBudget)
      return set_error(TN_ERR_UNSUPPORTED, "resident sketches: %lld samples of %zu bytes exceed the %zu-byte limit",
                       (long long)p->S, per_sample, kResidentBudget);
    chunk = p->S;
  }
  p->chunk_alloc = chunk;
  if (chunk > 16 && !(p->flags & TN_FLAG_RESIDENT)) chunk = chunk / 16 * 16;  // a multiple of every samples-per-pass choice
  p->chunk = chunk;
  int64_t table_samples = chunk;

  // Persistent fused kernel: per-tensor headroom, per-network work (items are
  // handed out largest first), then a default configuration (one bank, as
  // many samples per item as fit 80 KB of LDS); TN_FLAG_AUTOTUNE may retune.
  if (p->flags & TN_FLAG_PERSISTENT) {
    if (!chkp) return set_error(TN_ERR_UNSUPPORTED, "persistent kernel: not for this plan");
    const std::vector<NetCheck> &chk = *chkp;
    if (p->log2m < 6 || p->log2m > 12)
      return set_error(TN_ERR_UNSUPPORTED, "persistent kernel: m = %lld outside 64..4096", (long long)p->m);
    p->fused = true;
    p->net_work.assign((size_t)p->n_nets, 0);
    std::vector<int32_t> lgn;
    for (int j = 0; j < p->n_nets; ++j) {
      const NetCheck &c = chk[(size_t)j];
      for (size_t k = 0; k < c.sizes.size(); ++k) {
        const int64_t N = c.sizes[k];
        int lg = 0;
        while (lg < 62 && ((int64_t)1 << lg) < N) ++lg;
        lgn.push_back(std::max(lg, 11));
        p->net_work[(size_t)j] += N;
      }
      p->net_work[(size_t)j] += (int64_t)(c.sizes.size() + 1) / 2 * p->m * p->log2m;  // the pair FFTs
    }
    int64_t fc = (int64_t)std::max<size_t>(1, kWorkspaceBudget / std::max<size_t>(1, (size_t)p->W * 4));
    p->fused_chunk_cap = std::min<int64_t>({fc, p->S, 65535});
    table_samples = std::max(table_samples, p->fused_chunk_cap);
    int rc0;
    if ((rc0 = upload(&p->d_tensor_lgn, lgn)) != TN_OK) return rc0;
    if ((rc0 = dev_alloc(&p->d_counter, 1)) != TN_OK) return rc0;
    int fsb = 0;
    for (int c : {4, 2, 1})
      if (c <= p->S && m1_fused_lds(c, 1, p->m, (int32_t)worst_cols_rows) + kFusedStatic <= 81920) {
        fsb = c;
        break;
      }
    if ((rc0 = fused_configure(p, fsb ? fsb : 1, 1)) != TN_OK) return rc0;
  }

  int rc;
  if ((rc = upload(&p->d_streams, p->h_streams)) != TN_OK) return rc;
  if ((rc = upload(&p->d_modes, p->h_modes)) != TN_OK) return rc;
  if ((rc = upload(&p->d_slots, p->h_slots)) != TN_OK) return rc;
  if ((rc = upload(&p->d_tslot, p->h_tslot)) != TN_OK) return rc;
  if ((rc = upload(&p->d_nets, p->h_nets)) != TN_OK) return rc;
  if ((rc = dev_alloc(&p->d_tables, (size_t)table_samples * (size_t)p->W)) != TN_OK) return rc;
  unsigned char *yb = nullptr;
  if ((rc = dev_alloc(&yb, (size_t)chunk * p->h_slots.size() * (size_t)p->m * as)) != TN_OK) return rc;
  p->d_ybuf = yb;
  if ((rc = dev_alloc(&p->d_slot_bound, p->h_slots.size())) != TN_OK) return rc;
  if (p->two_pass) {
    // the tensors of each network two by two (an odd one out alone)
    std::vector<int32_t> pairs, pair0;
    for (const NetDesc &nd : p->h_nets) {
      pair0.push_back((int32_t)(pairs.size() / 2));
      for (int32_t k = nd.t0; k < nd.t1; k += 2) {
        pairs.push_back(k);
        pairs.push_back(k + 1 < nd.t1 ? k + 1 : -1);
      }
    }
    pair0.push_back((int32_t)(pairs.size() / 2));
    p->n_pairs = (int64_t)pairs.size() / 2;
    if ((rc = upload(&p->d_pairs, pairs)) != TN_OK) return rc;
    if ((rc = upload(&p->d_pair0, pair0)) != TN_OK) return rc;
    unsigned char *cb = nullptr;
    if ((rc = dev_alloc(&cb, (size_t)chunk * (size_t)p->n_pairs * (size_t)p->m * 2 * as)) != TN_OK) return rc;
    p->d_cbuf = cb;
    if ((rc = dev_alloc(&p->d_partial, (size_t)chunk * (size_t)p->n_nets * kBigPartials)) != TN_OK) return rc;
  }
  // In-LDS combine with too few (network, sample) blocks to fill the GPU (one
  // network with many tensors, as the ladder): each (network, sample) takes
  // csplit blocks, each the product over a share of the tensor pairs, and a
  // join kernel multiplies the partial spectra.
  p->csplit = 1;
  if (!p->two_pass && !p->fused && !(p->flags & (TN_FLAG_DFT_BF16 | TN_FLAG_DFT_FP8))) {
    int64_t max_pairs = 0;
    for (const NetDesc &nd : p->h_nets) max_pairs = std::max<int64_t>(max_pairs, (nd.t1 - nd.t0 + 1) / 2);
    const int64_t blocks = (int64_t)p->n_nets * p->chunk_alloc;
    // (only for long products: the join is one more launch, which small
    // networks, launch-bound, do not repay)
    if (blocks > 0 && blocks < kCombineSplitBlocks / 2 && max_pairs >= 2 && max_pairs * p->m >= kCombineSplitWork) {
      const size_t H = (size_t)p->m / 2 + 1;
      int64_t gs = std::min<int64_t>({(kCombineSplitBlocks + blocks - 1) / blocks, max_pairs, 64});
      while (gs > 1 && (size_t)blocks * (size_t)gs * H * 16 > kCombineSplitBudget) --gs;
      if (gs > 1) {
        if ((rc = dev_alloc(&p->d_csplit, (size_t)blocks * (size_t)gs * H * 2)) != TN_OK) return rc;
        p->csplit = (int32_t)gs;
      }
    }
  }
  if (p->m >= 2) {
    unsigned char *tw = nullptr;
    if ((rc = dev_alloc(&tw, (size_t)(p->m / 2) * 2 * as)) != TN_OK) return rc;
    p->d_tw = tw;
    if ((rc = launch_twiddles(p->m, p->dtype, p->d_tw, 0)) != TN_OK) return rc;
    TN_HIP_CHECK(hipDeviceSynchronize());
  }
  return TN_OK;
}

namespace {

int m1_tables(tn_plan *p, int64_t c0, int64_t n, hipStream_t st, const int32_t **tables) {
  if (p->d_injected) {
    *tables = p->d_injected + c0 * p->W;
    return TN_OK;
  }
  p->tables_ready = c0 == 0 && n == p->S;  // a resident plan's tables cover every sample
  *tables = p->d_tables;
  hipEvent_t ev = nullptr;
  int rc = prof_begin(p, st, &ev, TN_KERNEL_HASH);
  if (rc == TN_OK)
    rc = launch_hashgen(p->d_streams, (int64_t)p->h_streams.size(), p->W, c0, n, p->m, p->max_stream,
                        p->d_tables, st);
  if (rc == TN_OK) rc = prof_end(p, st, TN_KERNEL_HASH, ev);
  return rc;
}

int m1_run_fused(tn_plan *p, hipStream_t st, double *est) {
  for (int64_t c0 = 0; c0 < p->S; c0 += p->fused_chunk) {
    const int64_t n = std::min(p->fused_chunk, p->S - c0);
    const int32_t *tables = nullptr;
    int rc = m1_tables(p, c0, n, st, &tables);
    if (rc != TN_OK) return rc;
    M1FusedLaunch L{};
    L.items = p->d_items;
    L.n_items = p->n_items;
    L.counter = p->d_counter;
    L.nets = p->d_nets;
    L.tslot = p->d_tslot;
    L.slots = p->d_slots;
    L.tensor_lgn = p->d_tensor_lgn;
    L.modes = p->d_modes;
    L.data = p->d_data;
    L.dtype = p->dtype;
    L.tables = tables;
    L.W = p->W;
    L.chunk = n;
    L.sample0 = c0;
    L.S = p->S;
    L.worst = (int32_t)p->worst_cols_rows;
    L.sb = p->fused_sb;
    L.banks = p->fused_banks;
    L.log2m = p->log2m;
    L.lds_bytes = p->fused_lds;
    L.blocks = p->fused_blocks;
    L.twiddles = p->d_tw;
    L.est = est;
    hipEvent_t ev = nullptr;
    if ((rc = prof_begin(p, st, &ev, TN_KERNEL_SKETCH)) != TN_OK) return rc;
    if ((rc = launch_m1_fused(L, st)) != TN_OK) return rc;
    if ((rc = prof_end(p, st, TN_KERNEL_SKETCH, ev)) != TN_OK) return rc;
  }
  return TN_OK;
}

int m1_run(tn_plan *p, hipStream_t st, double *est) {
  if (p->fused) return m1_run_fused(p, st, est);
  for (int64_t c0 = 0; c0 < p->S; c0 += p->chunk) {
    const int64_t n = std::min(p->chunk, p->S - c0);
    const int32_t *tables = nullptr;
    int rc = m1_tables(p, c0, n, st, &tables);
    if (rc != TN_OK) return rc;
    M1Launch L{};
    L.slots = p->d_slots;
    L.n_slots = (int64_t)p->h_slots.size();
    L.modes = p->d_modes;
    L.data = p->d_data;
    L.dtype = p->dtype;
    L.tables = tables;
    L.W = p->W;
    L.samples = n;
    L.sb = p->sb;
    L.banks = p->banks;
    L.log2m = p->log2m;
    L.lds_bytes = p->scatter_lds;
    L.ybuf = p->d_ybuf;
    L.slot_bound = p->d_slot_bound;
    L.record_bound = c0 == 0;  // the data may have changed since the last call
    hipEvent_t ev = nullptr;
    if ((rc = prof_begin(p, st, &ev, TN_KERNEL_SKETCH)) != TN_OK) return rc;
    if ((rc = launch_m1_scatter(L, st)) != TN_OK) return rc;
    if ((rc = prof_end(p, st, TN_KERNEL_SKETCH, ev)) != TN_OK) return rc;
    if ((rc = prof_begin(p, st, &ev, TN_KERNEL_COMBINE)) != TN_OK) return rc;
    if (p->two_pass)
      rc = launch_m1_combine_big(p->n_nets, p->d_tslot, p->d_pairs, p->d_pair0, p->n_pairs, p->dtype, p->d_ybuf,
                                 (int64_t)p->h_slots.size(), n, c0, p->S, p->log2m, p->d_tw, p->d_cbuf,
                                 p->d_partial, est, st);
    else
      rc = (p->flags & (TN_FLAG_DFT_BF16 | TN_FLAG_DFT_FP8))
               ? launch_m1_combine_dft32(p->d_nets, p->n_nets, p->d_cbeg ? p->d_cbeg : p->d_tslot,
                                         p->d_cbeg ? p->d_cend : p->d_tslot + 1, p->d_ybuf,
                                         (int64_t)p->h_slots.size(), n, c0, p->S, p->d_tw, est,
                                         (p->flags & TN_FLAG_DFT_FP8) != 0, st)
               : launch_m1_combine(p->d_nets, p->n_nets, p->d_cbeg ? p->d_cbeg : p->d_tslot,
                                   p->d_cbeg ? p->d_cend : p->d_tslot + 1, p->dtype, p->d_ybuf,
                                   (int64_t)p->h_slots.size(), n, c0, p->S, p->log2m, p->d_tw, est, p->csplit,
                                   p->d_csplit, st);
    if (rc != TN_OK) return rc;
    if ((rc = prof_end(p, st, TN_KERNEL_COMBINE, ev)) != TN_OK) return rc;
  }
  return TN_OK;
}

// Autotuner of the sketching pass.  Samples per pass trade one HBM read of the
// tensors per pass against LDS size (hence blocks per CU); two accumulator
// banks trade ALU work per term against twice the accumulator LDS.  Each
// feasible (samples per pass, banks) is timed on the plan's first workspace
// chunk with the bound data, for the slot kernel or, with TN_FLAG_PERSISTENT,
// for the persistent kernel.
struct TuneKey {
  int64_t slots, entries_hint, m, S, W;
  int dtype, device;
  bool fused;
  bool operator==(const TuneKey &o) const {
    return slots == o.slots && entries_hint == o.entries_hint && m == o.m && S == o.S && W == o.W &&
           dtype == o.dtype && device == o.device && fused == o.fused;
  }
};
// Process-wide cache of tuned schedules; plans on several host threads may
// tune at once, hence the lock (held only to look up or insert).
static std::vector<std::pair<TuneKey, std::pair<int, int>>> g_tuned;
static std::mutex g_tuned_mu;

int m1_autotune(tn_plan *p, hipStream_t st) {
  if (p->log2m > kMaxLog2Acc) return TN_OK;  // bucket ranges: one schedule only
  if (p->partial) {  // the timing launches read the sub-tensors
    int rc = partial_prepare(p, st);
    if (rc != TN_OK) return rc;
  }
  int64_t entries = 0;
  for (const ScatterSlot &sl : p->h_slots) entries += (int64_t)sl.rows * sl.L;
  const TuneKey key{(int64_t)p->h_slots.size(), entries, p->m, p->S, p->W, p->dtype, p->device, p->fused};
  auto apply = [&](int sb, int banks) -> int {
    if (p->fused) return fused_configure(p, sb, banks);
    p->sb = sb;
    p->banks = banks;
    p->scatter_lds = scatter_lds_for(p, sb);
    return TN_OK;
  };
  {
    std::pair<int, int> hit{0, 0};
    {
      std::lock_guard<std::mutex> lk(g_tuned_mu);
      for (const auto &kv : g_tuned)
        if (kv.first == key) hit = kv.second;
    }
    if (hit.first > 0) {
      log_msg(1, "autotune: cached schedule, samples per pass %d, banks %d", hit.first, hit.second);
      return apply(hit.first, hit.second);
    }
  }
  const int64_t n = std::min(p->fused ? p->fused_chunk_cap : p->chunk, p->S);
  const int32_t *tables = nullptr;
  int rc = m1_tables(p, 0, n, st, &tables);
  if (rc != TN_OK) return rc;
  hipEvent_t e0, e1;
  TN_HIP_CHECK(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
  TN_HIP_CHECK(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
  std::pair<int, int> best{p->fused ? p->fused_sb : p->sb, p->fused ? p->fused_banks : p->banks};
  float best_ms = 1e30f;
  const int sbs_slot[] = {1, 2, 4, 8, 16}, sbs_fused[] = {1, 2, 4};
  for (int banks : {1, 2}) {
    for (int sb : p->fused ? std::vector<int>(sbs_fused, sbs_fused + 3) : std::vector<int>(sbs_slot, sbs_slot + 5)) {
      if (sb > 1 && sb > n) break;
      float ms = 0.f;
      if (p->fused) {
        if (m1_fused_lds(sb, banks, p->m, (int32_t)p->worst_cols_rows) + kFusedStatic > p->max_lds) break;
        if ((rc = fused_configure(p, sb, banks)) != TN_OK) break;
      } else {
        const int save = p->banks;
        p->banks = banks;
        const size_t lds = scatter_lds_for(p, sb);
        p->banks = save;
        if (lds > p->max_lds || scatter_words(sb, p->dtype) > kMaxScatterWords) break;
      }
      // one warm-up launch, then the faster of two timed ones
      float ms_min = 1e30f;
      for (int rep = 0; rep < 3 && rc == TN_OK; ++rep) {
        if (hipEventRecord(e0, st) != hipSuccess) rc = set_error(TN_ERR_HIP, "autotune: event record");
        if (rc == TN_OK) {
          if (p->fused) {
            M1FusedLaunch L{};
            L.items = p->d_items;
            L.n_items = p->n_items;
            L.counter = p->d_counter;
            L.nets = p->d_nets;
            L.tslot = p->d_tslot;
            L.slots = p->d_slots;
            L.tensor_lgn = p->d_tensor_lgn;
            L.modes = p->d_modes;
            L.data = p->d_data;
            L.dtype = p->dtype;
            L.tables = tables;
            L.W = p->W;
            L.chunk = std::min(n, p->fused_chunk);
            L.sample0 = 0;
            L.S = p->S;
            L.worst = (int32_t)p->worst_cols_rows;
            L.sb = sb;
            L.banks = banks;
            L.log2m = p->log2m;
            L.lds_bytes = p->fused_lds;
            L.blocks = p->fused_blocks;
            L.twiddles = p->d_tw;
            L.est = p->d_est;  // scratch: overwritten by the estimate that follows
            rc = launch_m1_fused(L, st);
          } else {
            M1Launch L{};
                    L.slots = p->d_slots;
            L.n_slots = (int64_t)p->h_slots.size();
            L.modes = p->d_modes;
            L.data = p->d_data;
            L.dtype = p->dtype;
            L.tables = tables;
            L.W = p->W;
            L.samples = n;
            L.sb = sb;
            L.banks = banks;
            L.log2m = p->log2m;
            p->banks = banks;
            L.lds_bytes = scatter_lds_for(p, sb);
            L.ybuf = p->d_ybuf;
            L.slot_bound = p->d_slot_bound;
            L.record_bound = true;
            rc = launch_m1_scatter(L, st);
          }
        }
        if (rc == TN_OK && hipEventRecord(e1, st) != hipSuccess) rc = set_error(TN_ERR_HIP, "autotune: event record");
        if (rc == TN_OK && hipEventSynchronize(e1) != hipSuccess) rc = set_error(TN_ERR_HIP, "autotune: sync");
        if (rc == TN_OK) (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) ms_min = std::min(ms_min, ms);
      }
      if (rc != TN_OK) break;
      // per sample of the chunk, so that candidates with different chunks compare
      const float per = ms_min / (float)(p->fused ? std::min(n, p->fused_chunk) : n);
      log_msg(2, "autotune: samples per pass %d, banks %d: %.4f ms per sample", sb, banks, (double)per);
      if (per < best_ms) { best_ms = per; best = {sb, banks}; }
    }
    if (rc != TN_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != TN_OK) return rc;
  if ((rc = apply(best.first, best.second)) != TN_OK) return rc;
  log_msg(1, "autotune: samples per pass %d, banks %d (%.4f ms per sample)", best.first, best.second,
          (double)best_ms);
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    g_tuned.push_back({key, best});
  }
  return TN_OK;
}

int run_all(tn_plan *p, hipStream_t st, double *stats, double *est) {
  int rc = p->partial ? partial_prepare(p, st) : TN_OK;
  if (rc != TN_OK) return rc;
  rc = (p->method == TN_CYCLIC) ? m1_run(p, st, est) : m2_estimate(p, st, est);
  if (rc != TN_OK) return rc;
  hipEvent_t ev = nullptr;
  if ((rc = prof_begin(p, st, &ev, TN_KERNEL_STATS)) != TN_OK) return rc;
  if ((rc = launch_sample_stats(est, p->n_nets, p->S, stats, st)) != TN_OK) return rc;
  return prof_end(p, st, TN_KERNEL_STATS, ev);
}

}  // namespace

// Timing events carry no system-scope fence: they only time kernels, and a
// fence per record (a cache write-back) would slow the work being timed.
int prof_begin(tn_plan *p, hipStream_t st, hipEvent_t *ev, int kind) {
  *ev = nullptr;
  if (!(p->flags & TN_FLAG_PROFILE)) return TN_OK;
  if ((p->flags & TN_FLAG_PROFILE_SKETCH) && kind != TN_KERNEL_SKETCH) return TN_OK;
  if (p->prof_pool.empty()) {
    hipEvent_t e;
    TN_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    p->prof_pool.push_back(e);
  }
  *ev = p->prof_pool.back();
  p->prof_pool.pop_back();
  TN_HIP_CHECK(hipEventRecord(*ev, st));
  return TN_OK;
}

int prof_end(tn_plan *p, hipStream_t st, int kind, hipEvent_t start) {
  if (!(p->flags & TN_FLAG_PROFILE) || !start) return TN_OK;
  if (p->prof_pool.empty()) {
    hipEvent_t e;
    TN_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    p->prof_pool.push_back(e);
  }
  hipEvent_t stop = p->prof_pool.back();
  p->prof_pool.pop_back();
  TN_HIP_CHECK(hipEventRecord(stop, st));
  p->prof_pending.push_back({kind, start, stop});
  return TN_OK;
}

int plan_kernel_time(tn_plan *p, int kind, double *ms, int64_t *launches) {
  *ms = 0.0;
  *launches = 0;
  if (!(p->flags & TN_FLAG_PROFILE)) return set_error(TN_ERR_ARG, "plan was built without TN_FLAG_PROFILE");
  std::vector<tn_plan::ProfRec> keep;
  for (const auto &r : p->prof_pending) {
    if (r.kind != kind) {
      keep.push_back(r);
      continue;
    }
    TN_HIP_CHECK(hipEventSynchronize(r.stop));
    float t = 0.f;
    TN_HIP_CHECK(hipEventElapsedTime(&t, r.start, r.stop));
    *ms += t;
    *launches += 1;
    p->prof_pool.push_back(r.start);
    p->prof_pool.push_back(r.stop);
  }
  p->prof_pending.swap(keep);
  return TN_OK;
}

int plan_build(tn_plan *p, const tn_network *nets, int n_nets, int method, int64_t m, int64_t S,
               uint64_t seed, int root, uint32_t flags) {
  p->method = method;
  p->m = m;
  p->log2m = 0;
  while ((1ll << p->log2m) < m) ++p->log2m;
  p->S = S;
  p->seed = seed;
  p->flags = flags;
  p->root = root < 0 ? 0 : root;
  p->n_nets = n_nets;
  std::vector<NetCheck> chk((size_t)n_nets);
  for (int j = 0; j < n_nets; ++j) {
    int rc = validate_network(&nets[j], j, &chk[(size_t)j]);
    if (rc != TN_OK) return rc;
    if (j > 0 && nets[j].dtype != nets[0].dtype)
      return set_error(TN_ERR_ARG, "network %d: every network of a plan must share one dtype", j);
    if (method == TN_ACYCLIC) {
      if ((rc = validate_tree(&nets[j], j, chk[(size_t)j])) != TN_OK) return rc;
      if (p->root >= nets[j].p)
        return set_error(TN_ERR_ARG, "network %d: root %d outside [0, %d)", j, p->root, nets[j].p);
    }
    p->net_p.push_back(nets[j].p);
    p->net_tensor0.push_back(p->n_tensors);
    p->net_orders.emplace_back(nets[j].order, nets[j].order + nets[j].p);
    for (int k = 0; k < nets[j].p; ++k) p->tensor_size.push_back(chk[(size_t)j].sizes[(size_t)k]);
    p->n_tensors += nets[j].p;
  }
  p->dtype = nets[0].dtype;
  if (method == TN_ACYCLIC && (m < 2 || m > 65536))
    return set_error(TN_ERR_UNSUPPORTED, "acyclic method: m = %lld outside [2, 65536]", (long long)m);
  if (n_nets > 65535 && method == TN_CYCLIC)
    return set_error(TN_ERR_UNSUPPORTED, "at most 65535 networks per plan");
  int rc = plan_common(p);
  if (rc != TN_OK) return rc;
  rc = (method == TN_CYCLIC) ? m1_build(p, nets, chk) : m2_build(p, nets, chk);
  if (rc == TN_OK) rc = plan_alloc_tail(p);
  if (rc != TN_OK) {
    plan_release(p);
    return rc;
  }
  log_plan(p);
  return rc;
}

void log_plan(const tn_plan *p) {
  if (log_level() < 1) return;
  if (p->method == TN_CYCLIC)
    log_msg(1,
            "plan: cyclic, %d networks (%d outputs), %d tensors, %zu slots, m %lld, S %lld, chunk %lld, %s, "
            "samples per pass %d, banks %d, flags 0x%x",
            p->partial ? 1 : p->n_nets, p->n_nets, p->n_tensors, p->h_slots.size(), (long long)p->m,
            (long long)p->S, (long long)p->chunk,
            p->fused ? "persistent kernel" : p->two_pass ? "two-pass combine" : "in-LDS combine",
            p->fused ? p->fused_sb : p->sb, p->fused ? p->fused_banks : p->banks, p->flags);
  else
    log_msg(1, "plan: acyclic, %d networks, %d tensors, m %lld, S %lld, chunk %lld, root %d, flags 0x%x", p->n_nets,
            p->n_tensors, (long long)p->m, (long long)p->S, (long long)p->chunk, p->root, p->flags);
}

// Device and its LDS limit.
int plan_common(tn_plan *p) {
  TN_HIP_CHECK(hipGetDevice(&p->device));
  int lds = 0;
  TN_HIP_CHECK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device));
  p->max_lds = (size_t)lds;
  return TN_OK;
}

// Buffers every plan has: per-sample estimates and the device pointer table
// of its (virtual) tensors.
int plan_alloc_tail(tn_plan *p) {
  p->max_stream = 0;
  for (const StreamDesc &sd : p->h_streams) p->max_stream = std::max<int64_t>(p->max_stream, (int64_t)sd.n);
  int rc;
  if ((rc = dev_alloc(&p->d_est, (size_t)p->n_nets * (size_t)p->S)) != TN_OK) return rc;
  if ((rc = dev_alloc(&p->d_data, (size_t)p->n_tensors)) != TN_OK) return rc;
  p->bound.assign((size_t)p->n_tensors, nullptr);
  TN_HIP_CHECK(hipMemset(p->d_data, 0, (size_t)p->n_tensors * sizeof(void *)));
  TN_HIP_CHECK(hipDeviceSynchronize());
  return TN_OK;
}

int plan_bind(tn_plan *p, const tn_network *nets, hipStream_t st) {
  if (p->partial) return partial_bind(p, nets, st);
  bool changed = false;
  for (int j = 0; j < p->n_nets; ++j) {
    const tn_network &n = nets[j];
    if (n.p != p->net_p[(size_t)j] || n.dtype != p->dtype || !n.order || !n.data)
      return set_error(TN_ERR_ARG, "network %d does not match the plan", j);
    for (int k = 0; k < n.p; ++k) {
      if (n.order[k] != p->net_orders[(size_t)j][(size_t)k])
        return set_error(TN_ERR_ARG, "network %d tensor %d: order differs from the plan", j, k);
      if (!n.data[k]) return set_error(TN_ERR_ARG, "network %d tensor %d: null data", j, k);
      const size_t g = (size_t)(p->net_tensor0[(size_t)j] + k);
      if (p->bound[g] != n.data[k]) {
        p->bound[g] = n.data[k];
        changed = true;
      }
    }
  }
  if (changed) {
    // Pageable source: the copy is staged before the call returns, so the host
    // array may change right after.
    TN_HIP_CHECK(hipMemcpyAsync(p->d_data, p->bound.data(), p->bound.size() * sizeof(void *),
                                hipMemcpyHostToDevice, st));
  }
  return TN_OK;
}

int plan_estimate(tn_plan *p, const tn_network *nets, hipStream_t st, double *stats,
                  double *samples_out) {
  int rc = plan_bind(p, nets, st);
  if (rc != TN_OK) return rc;
  if ((p->flags & TN_FLAG_AUTOTUNE) && !p->tuned) {
    if ((rc = p->method == TN_CYCLIC ? m1_autotune(p, st) : m2_autotune(p, st)) != TN_OK) return rc;
    p->tuned = true;
  }
  double *est = samples_out ? samples_out : p->d_est;
  if (!(p->flags & TN_FLAG_GRAPH)) return run_all(p, st, stats, est);

  // Graph replay: capture once per (stream, output buffers), then relaunch.
  if (!p->graph_exec || p->graph_stream != st || p->graph_stats != stats || p->graph_samples != est) {
    if (p->graph_exec) {
      (void)hipGraphExecDestroy(p->graph_exec);
      p->graph_exec = nullptr;
    }
    if (p->graph) {
      (void)hipGraphDestroy(p->graph);
      p->graph = nullptr;
    }
    hipStream_t cap = st;
    bool own = false;
    if (cap == nullptr) {
      TN_HIP_CHECK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      own = true;
    }
    TN_HIP_CHECK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    rc = run_all(p, cap, stats, est);
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(cap, &g);
    if (own) (void)hipStreamDestroy(cap);
    if (rc != TN_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ee != hipSuccess) return set_error(TN_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ee));
    p->graph = g;
    TN_HIP_CHECK(hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0));
    p->graph_stream = st;
    p->graph_stats = stats;
    p->graph_samples = est;
  }
  TN_HIP_CHECK(hipGraphLaunch(p->graph_exec, st));
  return TN_OK;
}

void plan_release(tn_plan *p) {
  (void)hipDeviceSynchronize();
  for (const auto &r : p->prof_pending) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  for (hipEvent_t e : p->prof_pool) (void)hipEventDestroy(e);
  p->prof_pending.clear();
  p->prof_pool.clear();
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->graph_exec = nullptr;
  p->graph = nullptr;
  if (p->m2) m2_release(p);
  if (p->partial) partial_release(p);
  void *ptrs[] = {p->d_streams, p->d_tables, p->d_injected, p->d_data,    p->d_modes,
                  p->d_slots,   p->d_tslot,  p->d_nets,     p->d_tw,      p->d_ybuf,
                  p->d_est,     p->d_items,  p->d_counter,  p->d_tensor_lgn, p->d_cbuf, p->d_partial,
                  p->d_pairs,   p->d_pair0,  p->d_slot_bound, p->d_csplit};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  p->d_streams = nullptr;
  p->d_tables = p->d_injected = nullptr;
  p->d_data = nullptr;
  p->d_modes = nullptr;
  p->d_slots = nullptr;
  p->d_tslot = nullptr;
  p->d_nets = nullptr;
  p->d_tw = p->d_ybuf = p->d_cbuf = nullptr;
  p->d_partial = nullptr;
  p->d_pairs = p->d_pair0 = nullptr;
  p->d_slot_bound = nullptr;
  p->d_csplit = nullptr;
  p->d_est = nullptr;
  p->d_items = nullptr;
  p->d_counter = p->d_tensor_lgn = nullptr;
}

int64_t plan_query(const tn_plan *p, int key) {
  switch (key) {
    case 0: return p->W;
    case 1: return (int64_t)p->h_streams.size();
    case 2: return p->S;
    case 3: return p->m;
    case 4: return p->n_nets;
    case 5: return p->n_tensors;
    case 6: return p->n_tensors;
    case 7: return p->method;
    case 8: return p->fused ? p->fused_sb : p->sb;
    case 9: return p->fused ? p->fused_chunk : p->chunk;
    case 10: return p->method == TN_CYCLIC ? (p->fused ? p->fused_banks : p->banks) : 0;
    case 11: return p->fused ? 1 : 0;
    case 12: return p->partial ? p->n_out : p->n_nets;
    case 13: return p->partial ? p->n_free : 0;
    case 14: return p->m2 ? 0 : p->csplit;
    default: return set_error(TN_ERR_ARG, "unknown query key %d", key);
  }
}

// Resident sketches (TN_FLAG_RESIDENT): turnstile updates, the combine alone,
// and a reset to the sketches of all-zero tensors.
int resident_check(const tn_plan *p) {
  if (!(p->flags & TN_FLAG_RESIDENT) || p->method != TN_CYCLIC)
    return set_error(TN_ERR_ARG, "the plan was not built with TN_FLAG_RESIDENT (cyclic method)");
  return TN_OK;
}

int plan_update(tn_plan *p, int net, int tensor, int64_t n, const int64_t *idx, const double *delta, hipStream_t st) {
  int rc = resident_check(p);
  if (rc != TN_OK) return rc;
  if (net < 0 || net >= p->n_nets || tensor < 0 || tensor >= p->net_p[(size_t)net])
    return set_error(TN_ERR_ARG, "network %d tensor %d is not in the plan", net, tensor);
  if (n < 0 || (n > 0 && (!idx || !delta))) return set_error(TN_ERR_ARG, "bad update arrays");
  if (n == 0) return TN_OK;
  if (!p->d_injected && !p->tables_ready) {
    const int32_t *t = nullptr;
    if ((rc = m1_tables(p, 0, p->S, st, &t)) != TN_OK) return rc;
  }
  const int32_t *tables = p->d_injected ? p->d_injected : p->d_tables;
  const size_t g = (size_t)(p->net_tensor0[(size_t)net] + tensor);
  const int32_t slot0 = p->h_tslot[g];
  const ScatterSlot &sl = p->h_slots[(size_t)slot0];
  return launch_stream_update(p->d_modes, sl.mode0, sl.q, p->tensor_size[g], tables, p->W, p->S, p->log2m,
                              (int64_t)p->h_slots.size(), slot0, p->dtype, p->d_ybuf, n, idx, delta, st);
}

int plan_combine(tn_plan *p, hipStream_t st, double *stats, double *samples_out) {
  int rc = resident_check(p);
  if (rc != TN_OK) return rc;
  double *est = samples_out ? samples_out : p->d_est;
  if (p->two_pass)
    rc = launch_m1_combine_big(p->n_nets, p->d_tslot, p->d_pairs, p->d_pair0, p->n_pairs, p->dtype, p->d_ybuf,
                               (int64_t)p->h_slots.size(), p->S, 0, p->S, p->log2m, p->d_tw, p->d_cbuf,
                               p->d_partial, est, st);
  else if (p->flags & (TN_FLAG_DFT_BF16 | TN_FLAG_DFT_FP8))
    rc = launch_m1_combine_dft32(p->d_nets, p->n_nets, p->d_tslot, p->d_tslot + 1, p->d_ybuf,
                                 (int64_t)p->h_slots.size(), p->S, 0, p->S, p->d_tw, est,
                                 (p->flags & TN_FLAG_DFT_FP8) != 0, st);
  else
    rc = launch_m1_combine(p->d_nets, p->n_nets, p->d_tslot, p->d_tslot + 1, p->dtype, p->d_ybuf,
                           (int64_t)p->h_slots.size(), p->S, 0, p->S, p->log2m, p->d_tw, est, p->csplit,
                           p->d_csplit, st);
  if (rc != TN_OK) return rc;
  return launch_sample_stats(est, p->n_nets, p->S, stats, st);
}

int plan_reset(tn_plan *p, hipStream_t st) {
  int rc = resident_check(p);
  if (rc != TN_OK) return rc;
  const size_t bytes = (size_t)p->S * p->h_slots.size() * (size_t)p->m * acc_size(p->dtype);
  return launch_fill_zero(p->d_ybuf, bytes, st);
}

int plan_get_hashes(tn_plan *p, int64_t first, int64_t count, hipStream_t st, int32_t *out) {
  if (first < 0 || count < 0 || first + count > p->S)
    return set_error(TN_ERR_ARG, "samples [%lld, %lld) outside [0, %lld)", (long long)first,
                     (long long)(first + count), (long long)p->S);
  if (p->d_injected) {
    TN_HIP_CHECK(hipMemcpyAsync(out, p->d_injected + first * p->W,
                                (size_t)count * (size_t)p->W * sizeof(int32_t),
                                hipMemcpyDeviceToDevice, st));
    return TN_OK;
  }
  for (int64_t c = 0; c < count; c += 65535) {
    const int64_t n = std::min<int64_t>(65535, count - c);
    int rc = launch_hashgen(p->d_streams, (int64_t)p->h_streams.size(), p->W, first + c, n, p->m,
                            p->max_stream, out + c * p->W, st);
    if (rc != TN_OK) return rc;
  }
  return TN_OK;
}

int plan_set_hashes(tn_plan *p, const int32_t *tables, hipStream_t st) {
  if (p->graph_exec) {
    (void)hipGraphExecDestroy(p->graph_exec);
    p->graph_exec = nullptr;
    (void)hipGraphDestroy(p->graph);
    p->graph = nullptr;
  }
  if (!tables) {
    if (p->d_injected) {
      TN_HIP_CHECK(hipStreamSynchronize(st));
      TN_HIP_CHECK(hipFree(p->d_injected));
    }
    p->d_injected = nullptr;
    return TN_OK;
  }
  if (!p->d_injected) {
    int rc = dev_alloc(&p->d_injected, (size_t)p->S * (size_t)p->W);
    if (rc != TN_OK) return rc;
  }
  return launch_copy_i32(tables, p->d_injected, p->S * p->W, st);
}

int plan_get_sketches(tn_plan *p, const tn_network *nets, int64_t first, int64_t count,
                      hipStream_t st, double *out) {
  if (first < 0 || count < 0 || first + count > p->S)
    return set_error(TN_ERR_ARG, "samples [%lld, %lld) outside [0, %lld)", (long long)first,
                     (long long)(first + count), (long long)p->S);
  int rc = plan_bind(p, nets, st);
  if (rc != TN_OK) return rc;
  if (p->method == TN_ACYCLIC) return m2_get_sketches(p, first, count, st, out);
  if (p->partial && (rc = partial_prepare(p, st)) != TN_OK) return rc;
  for (int64_t c0 = first; c0 < first + count; c0 += p->chunk) {
    const int64_t n = std::min(p->chunk, first + count - c0);
    const int32_t *tables = nullptr;
    if ((rc = m1_tables(p, c0, n, st, &tables)) != TN_OK) return rc;
    M1Launch L{};
    L.slots = p->d_slots;
    L.n_slots = (int64_t)p->h_slots.size();
    L.modes = p->d_modes;
    L.data = p->d_data;
    L.dtype = p->dtype;
    L.tables = tables;
    L.W = p->W;
    L.samples = n;
    L.sb = p->sb;
    L.banks = p->banks;
    L.log2m = p->log2m;
    L.lds_bytes = p->scatter_lds;
    L.ybuf = p->d_ybuf;
    L.slot_bound = p->d_slot_bound;
    L.record_bound = c0 == first;
    if ((rc = launch_m1_scatter(L, st)) != TN_OK) return rc;
    if ((rc = launch_m1_slots_to_tensors(p->d_tslot, p->n_tensors, p->dtype, p->d_ybuf,
                                         (int64_t)p->h_slots.size(), n, p->log2m,
                                         out + (c0 - first) * p->n_tensors * p->m, st)) != TN_OK)
      return rc;
  }
  return TN_OK;
}

}  // namespace tn
