// Internal definitions of the tn_sketch library: device-visible descriptors,
// kernel launchers and error helpers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/tn_sketch.h"

namespace tn {

// ---------------------------------------------------------------------------
// Error reporting (thread-local text behind tn_last_error()).
// ---------------------------------------------------------------------------
int set_error(int code, const char *fmt, ...);
// Diagnostics on stderr, one "[tn] ..." line per call, printed when the
// environment variable TN_LOG is at least `level` (1: plan decisions and
// choices; 2: also every autotuner candidate).  Read at each call.
int log_level();
void log_msg(int level, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

#define TN_HIP_CHECK(call)                                                        \
  do {                                                                            \
    hipError_t _e = (call);                                                       \
    if (_e != hipSuccess)                                                         \
      return ::tn::set_error(TN_ERR_HIP, "%s failed: %s (%s:%d)", #call,          \
                             hipGetErrorString(_e), __FILE__, __LINE__);          \
  } while (0)

// ---------------------------------------------------------------------------
// Hash family (see tn_sketch.h): one descriptor per stream.
// ---------------------------------------------------------------------------
struct StreamDesc {
  uint64_t seed;     // network seed (plan seed + network index)
  uint64_t stream;   // stream id
  int64_t offset;    // first packed entry of this stream in a sample's table
  int32_t n;         // domain size
  int32_t net;       // owning network
};

// Packed hash entry: bucket in bits 0..30, bit 31 set for sign -1.
constexpr uint32_t kSignBit = 0x80000000u;

// ---------------------------------------------------------------------------
// Cyclic method (Eq. (1)).
// ---------------------------------------------------------------------------
// Per global mode: where its count sketch lives and whether it is the
// complement side of its contraction (Def. 14).
struct ModeDesc {
  int64_t table_off;  // offset of the edge's stream in a sample's table
  int32_t n;          // mode size
  int32_t comp;       // 1: second mode of the edge -> bucket (m - h) mod m
};

// One scatter work item: a block of rows of one tensor.  The tensor is viewed
// as a matrix: row index over modes [0, split), column index over modes
// [split, q) with L columns.
struct ScatterSlot {
  int32_t tensor;     // global tensor index (into the data pointer array)
  int32_t q;          // order
  int32_t split;      // first column mode
  int32_t L;          // number of columns
  int32_t mode0;      // global mode id of the tensor's first mode
  int32_t rows;       // rows in this block
  int64_t row0;       // first row of the block
  uint32_t magic;     // ceil(2^32 / L): row = umulhi(e, magic) for e < 2^21
  int32_t pad;
};

// Per network: its tensors [t0, t1) and, per tensor, slots
// [slot_begin[k], slot_begin[k+1]).
struct NetDesc {
  int32_t t0, t1;
};

// Limits of the cyclic scatter.
constexpr int kMaxCols = 1024;          // columns per slot (packed tables in LDS)
constexpr int kColPad = 8;              // words after each sample's column table (wrapped copy of its first columns)
constexpr int kMaxSlotEntries = 1 << 16;  // entries per scatter block
constexpr int kMaxLog2M1 = 16;          // m <= 65536
constexpr size_t kMaxLdsBytes = 160 * 1024;  // LDS per workgroup on gfx950
// Column-table words a scatter thread holds per load: samples per pass x
// entries per 16-byte load.  Above 64 the scatter would spill registers, so
// such schedules are not offered.
constexpr int kMaxScatterWords = 64;
inline int scatter_words(int sb, int dtype) { return sb * (dtype == TN_F64 ? 2 : dtype == TN_F32 ? 4 : 8); }
constexpr int kMaxLog2Acc = 14;         // sketch words in LDS per scatter block and FFT points in LDS;
                                        // larger m: bucket ranges and the two-pass FFT

struct M1Launch {
  const ScatterSlot *slots;
  int64_t n_slots;
  const ModeDesc *modes;
  const void *const *data;   // per global tensor
  int dtype;
  const int32_t *tables;     // [samples][W]
  int64_t W;
  int64_t samples;           // samples in this chunk
  int sb;                    // samples per scatter block
  int banks;                 // accumulator banks per sketch (1: signed adds, 2: sign in the address)
  int log2m;
  size_t lds_bytes;
  void *ybuf;                // [samples][n_slots][m] (double for F64, float otherwise)
  // Per-slot power-of-two bound of |x| ([n_slots]; null: every block keeps a
  // running maximum).  record_bound: this launch is the first to see the
  // data, its first sample batch records the bounds the others then use.
  double *slot_bound = nullptr;
  bool record_bound = false;
};

// Persistent fused kernel: one work item = (network, first sample of a batch
// of up to `sb` samples within the launch's chunk), sorted by decreasing work.
struct FusedItem {
  int32_t net;
  int32_t s0;
};

struct M1FusedLaunch {
  const FusedItem *items;
  int32_t n_items;
  int32_t *counter;           // one int of device memory (reset by the launch)
  const NetDesc *nets;
  const int32_t *tslot;       // per tensor: first slot; [n_tensors + 1]
  const ScatterSlot *slots;
  const int32_t *tensor_lgn;  // per tensor: max(ceil(log2(entries)), 11)
  const ModeDesc *modes;
  const void *const *data;
  int dtype;
  const int32_t *tables;      // [chunk][W]
  int64_t W;
  int64_t chunk;              // samples in this launch
  int64_t sample0;
  int64_t S;
  int32_t worst;              // table words per sample: max over slots of L + kColPad + rows + 1
  int sb;                     // samples per item (1, 2, 4)
  int banks;                  // accumulator banks per sketch (1 or 2, see the slot scatter)
  int log2m;
  size_t lds_bytes;
  int64_t blocks;             // persistent grid
  const void *twiddles;
  double *est;
};

size_t m1_fused_lds(int sb, int banks, int64_t m, int32_t worst);
int launch_m1_fused(const M1FusedLaunch &L, hipStream_t st);

// max_n: the longest stream (indices); all at most 64 take one thread per (stream, sample).
int launch_hashgen(const StreamDesc *streams, int64_t n_streams, int64_t W, int64_t sample0,
                   int64_t samples, int64_t m, int64_t max_n, int32_t *out, hipStream_t st);

int launch_m1_scatter(const M1Launch &L, hipStream_t st);

// Network j's tensors are the entries [nets[j].t0, nets[j].t1) of tbeg/tend:
// entry k's sketch sums the slots [tbeg[k], tend[k]).
int launch_m1_combine(const NetDesc *nets, int64_t n_nets, const int32_t *tbeg, const int32_t *tend,
                      int dtype, const void *ybuf, int64_t n_slots, int64_t samples,
                      int64_t sample0, int64_t S, int log2m, const void *twiddles,
                      double *est, int32_t csplit, double *cpart, hipStream_t st);
// The combine with its 1024-point DFTs on the BF16 matrix cores, or with fp8
// on the FP8 ones (dft.hip; FP32 sketches, m = 1024 only).
int launch_m1_combine_dft32(const NetDesc *nets, int64_t n_nets, const int32_t *tbeg, const int32_t *tend,
                            const void *ybuf, int64_t n_slots, int64_t samples, int64_t sample0, int64_t S,
                            const void *twiddles, double *est, bool fp8, hipStream_t st);
// The two-pass combine (the m-point FFT does not fit in LDS).  pairs: n_pairs x
// (tensor a, tensor b or -1), the tensors of each network two by two; pair0:
// n_nets + 1 offsets into pairs.  cbuf: samples x n_pairs x m complex (A);
// partial: n_nets x samples x 128 doubles.
int launch_m1_combine_big(int64_t n_nets, const int32_t *tensor_slot_begin, const int32_t *pairs,
                          const int32_t *pair0, int64_t n_pairs, int dtype, const void *ybuf, int64_t n_slots,
                          int64_t samples, int64_t sample0, int64_t S, int log2m, const void *tw, void *cbuf,
                          double *partial, double *est, hipStream_t st);
constexpr int kBigPartials = 128;  // partial sums per (network, sample) of the two-pass combine

int launch_m1_slots_to_tensors(const int32_t *tensor_slot_begin, int64_t n_tensors, int dtype,
                               const void *ybuf, int64_t n_slots, int64_t samples, int log2m,
                               double *out, hipStream_t st);

int launch_twiddles(int64_t m, int dtype, void *out, hipStream_t st);

int launch_sample_stats(const double *est, int64_t n_nets, int64_t S, double *stats,
                        hipStream_t st);

int launch_copy_i32(const int32_t *src, int32_t *dst, int64_t n, hipStream_t st);

// Turnstile updates of resident sketches (stream.hip): n updates X_k(idx[u])
// += delta[u] of the tensor whose modes are modes[mode0 .. mode0 + q) and whose
// first slot is slot0, applied to the [S][n_slots][m] sketches of every sample.
int launch_stream_update(const ModeDesc *modes, int mode0, int q, int64_t size, const int32_t *tables, int64_t W,
                         int64_t S, int log2m, int64_t n_slots, int32_t slot0, int dtype, void *ybuf, int64_t n,
                         const int64_t *idx, const double *delta, hipStream_t st);
int launch_fill_zero(void *buf, size_t bytes, hipStream_t st);

// ---------------------------------------------------------------------------
// Exact contraction.
// ---------------------------------------------------------------------------
int contract_exact(const tn_network *net, hipStream_t st, double *out);

}  // namespace tn
