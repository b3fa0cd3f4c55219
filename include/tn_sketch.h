/*
 * tn_sketch.h -- C ABI of the MI355X (gfx950) sketching estimators for full
 * tensor network contraction, after "Approximating Tensor Network Contraction
 * with Sketches" (arXiv 2603.07387).
 *
 * A network is the paper's tc(X_1 x ... x X_p, E) (Def. 1-3):
 *   - tensor k has order q_k and owns the consecutive global modes
 *     off_k .. off_k + q_k - 1 (off_0 = 0, off_{k+1} = off_k + q_k);
 *   - dims[u] is the size n_u of global mode u;
 *   - edges[2e], edges[2e+1] are the 0-based global modes (u, v) of
 *     contraction e, with u != v and n_u = n_v (Def. 1).  The paper counts
 *     modes from 1;
 *   - data[k] points to tensor k in DEVICE memory, row-major (vec() is
 *     lexicographic order, Preliminaries).
 * Every mode must take part in exactly one contraction: the estimators cover
 * full TNC (Theorem 1), under WLOG 1 of the Methods section.
 *
 * Environment: TN_LOG=1 prints each plan's layout, the autotuner's choices,
 * the size choices of auto-sized plans and the exact contraction's memory peak
 * on stderr, one "[tn] ..." line each; TN_LOG=2 also every autotuner
 * candidate and the exact contraction's tree kind.  TN_SCATTER_SB and
 * TN_SCATTER_BANKS fix the cyclic scatter's samples per pass and accumulator
 * banks of plans built without TN_FLAG_AUTOTUNE (test overrides).
 *
 * Estimators:
 *   TN_CYCLIC  -- the first method, for any network (Eq. (1), Algorithm 1):
 *                 edge e draws a count sketch C_u for its first mode u and
 *                 gives its complement C'_u (Def. 14) to the second mode v.
 *   TN_ACYCLIC -- the second method, for acyclic networks (Eq. (2),
 *                 Algorithms 2-5): recursive sketches built leaves-to-root.
 *
 * Hash family (Def. 10-11 ask for 2-wise independent buckets and 4-wise
 * independent signs; the paper fixes no construction).  Over P = 2^31 - 1,
 * with mix() the SplitMix64 output function (Steele, Lea, Flood 2014):
 *   key  = mix(mix(mix(seed_j) ^ sample) ^ stream),  raw_i = mix(key ^ i) >> 33
 *   h(i) = ((a1 i + a0) mod P) mod m,  a0 = raw_0 mod P, a1 = 1 + raw_1 mod (P-1)
 *   s(i) = +1 if (c3 i^3 + c2 i^2 + c1 i + c0) mod P is even else -1,
 *          c_i = raw_{2+i} mod P
 * seed_j = seed + j for network j of a plan.  Streams: edge e -> e; the
 * acyclic method's tensor-sketch count sketches T_{l,j} of tensor k, side d
 * -> 2^62 + k 2^32 + l 2^16 + 2j + d (domain [m]); padding sketches of
 * tensor k, slot j -> 2^63 + k 2^32 + j (domain [1]).
 *
 * Packed hash entry (int32): bits 0..30 bucket h, bit 31 set when s = -1.
 *
 * Buffers: the library trusts the pointers and sizes it is given.  Each data[k]
 * must hold prod(dims of tensor k) entries of `dtype` in memory of the plan's
 * device, and every output buffer must hold the element count its call states;
 * neither is checked (the device reads and writes through them as given).  The
 * Python binding checks device, dtype, contiguity and element counts before
 * each call.
 *
 * Errors: every entry point returns TN_OK (0) or a negative code; the text of
 * the last error on the calling thread is returned by tn_last_error().
 * Nothing throws across this boundary.  Validation runs on the host before any
 * device work, so argument errors never leave work queued.
 *
 * Streams: `stream` arguments are hipStream_t values (NULL = default stream).
 * Device work is queued asynchronously on that stream unless stated.
 */
#ifndef TN_SKETCH_H
#define TN_SKETCH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define TN_OK 0
#define TN_ERR_ARG (-1)         /* malformed argument (null, negative size, bad enum) */
#define TN_ERR_DIMS (-2)        /* contracted modes of different size (n_u != n_v) */
#define TN_ERR_HYPEREDGE (-3)   /* a mode in more than one contraction (WLOG 1) */
#define TN_ERR_SELFLOOP (-4)    /* acyclic method: a contraction inside one tensor */
#define TN_ERR_CYCLIC (-5)      /* acyclic method on a cyclic or disconnected network */
#define TN_ERR_PARTIAL (-6)     /* a free (uncontracted) mode: partial TNC is not supported */
#define TN_ERR_OOM (-7)         /* device or host allocation failed */
#define TN_ERR_HIP (-8)         /* a HIP runtime call failed */
#define TN_ERR_UNSUPPORTED (-9) /* a size outside the library's limits (see each call) */

/* Element types of tensor data. */
#define TN_F64 0
#define TN_F32 1
#define TN_BF16 2

/* Estimators. */
#define TN_CYCLIC 1
#define TN_ACYCLIC 2

/* Plan flags. */
#define TN_FLAG_GRAPH 0x1u      /* capture each estimate's launches in a hipGraph and replay it */
#define TN_FLAG_PROFILE 0x2u    /* record HIP events around every kernel launch (not with GRAPH) */
#define TN_FLAG_AUTOTUNE 0x4u   /* first estimate times launch shapes on the bound data and
                                   keeps the fastest (that call synchronizes its stream); cached
                                   per plan shape for the life of the process.  TN_CYCLIC: the
                                   scatter's samples per pass and accumulator banks (estimates
                                   unchanged bit for bit); TN_ACYCLIC: the products' column-split
                                   target and the gathers' blocks per level (the split regroups
                                   FP64 partial sums: estimates move by rounding only) */
#define TN_FLAG_MFMA_BF16 0x8u  /* TN_ACYCLIC only: the SMVP products w_k = mat(X_k) G run on the
                                   BF16 matrix cores (operands rounded to BF16 to nearest even,
                                   FP32 accumulation) instead of the FP64 ones; the hashes,
                                   sketches and combine are unchanged.  Rounding the operands
                                   perturbs each w_k by about 2^-8 relative per tree level; the
                                   estimate's error against exact arithmetic is measured and
                                   stated by the tests (TN_ERR_UNSUPPORTED with TN_CYCLIC) */
#define TN_FLAG_PERSISTENT 0x10u /* TN_CYCLIC only: one persistent kernel per estimate call takes
                                   (network, batch of samples) work items, largest first, from a
                                   device queue, and for each scatters the tensors, transforms
                                   and multiplies their sketches and writes the estimates, with
                                   the sketches held in LDS throughout (64 <= m <= 4096; else
                                   TN_ERR_UNSUPPORTED).  Same estimates as the two-kernel path
                                   up to FP rounding of the combine (TN_ERR_UNSUPPORTED with
                                   TN_ACYCLIC) */

#define TN_FLAG_PROFILE_SKETCH 0x20u /* with TN_FLAG_PROFILE: record the events around the
                                   TN_KERNEL_SKETCH launches only (each recorded event costs a
                                   few microseconds of device time; the other kinds then read
                                   0 launches).  TN_ERR_ARG without TN_FLAG_PROFILE */

#define TN_FLAG_PRIOR_XCORR 0x40u /* TN_CYCLIC only: run the earlier cross-correlation estimator the
                                   paper compares against (Examples 2-3) instead of Eq. (1):
                                   both modes of contraction e use the same count sketch C_e
                                   (no complement), and the tensor sketches are combined by the
                                   chain y_1 star y_2 star ... star y_p of circular
                                   cross-correlations (Def. 9) in tensor order.  By Lemma 5 this
                                   is Eq. (1)'s pipeline with every mode of tensor k (0-based)
                                   given the complement bucket when p - 1 - k is odd.  Unbiased
                                   when every contraction joins tensors of opposite parity (trees
                                   in chain order, even rings); otherwise biased (the triangle of
                                   Example 3).  A negative reference, not an estimator to use
                                   (TN_ERR_UNSUPPORTED with TN_ACYCLIC) */

#define TN_FLAG_RESIDENT 0x80u /* TN_CYCLIC only, not with TN_FLAG_PERSISTENT: keep the time-domain
                                   sketches of all S samples (and their hash tables) in device
                                   memory (S <= 65535 and at most 16 GiB for both, else
                                   TN_ERR_UNSUPPORTED), so that a stream of updates can change
                                   them (tn_sketch_update) and estimates can be read at any time
                                   (tn_sketch_combine) without rescanning the tensors */

#define TN_FLAG_DFT_BF16 0x400u /* TN_CYCLIC, m = 1024, FP32 or BF16 data, not with TN_FLAG_PERSISTENT:
                                   the combine takes each 1024-point DFT (Lemma 1's F y_k) as
                                   32 x 32 dense products on the BF16 matrix cores (four-step:
                                   32-point DFTs, twiddles, 32-point DFTs), operands rounded to
                                   BF16, FP32 accumulation, the product over tensors and the
                                   sum in FP64.  Each of the two stages rounds both factors of
                                   complex products whose magnitudes sum to at most
                                   sum_b |y_k[b]| <= U_k = sum |X_k|, so a spectrum value moves
                                   by at most about 6 2^-9 U_k to first order, and an estimate
                                   by at most 8 2^-9 (1/m) sum_j sum_k U_k prod_{k' != k}
                                   |Y_k'[j]| (the tests state the measured error) */
#define TN_FLAG_DFT_FP8 0x1000u /* as TN_FLAG_DFT_BF16 (and not with it), on the FP8 matrix cores:
                                   OCP E4M3 operands (3 mantissa bits), FP32 accumulation.
                                   The sketch and the twiddled intermediate are each scaled
                                   by a power of two so that their block maximum lies in
                                   [128, 256), then rounded stochastically (random bits from
                                   a hash of network, sample, tensor and element: unbiased,
                                   below one ulp, 2^-3 relative); the DFT constants are two
                                   E4M3 terms each (about 2^-8); the scales are undone
                                   exactly in FP64.  The estimator stays unbiased; its
                                   rounding noise, a fraction of the estimator's own
                                   spread, is stated by the tests */
#define TN_FLAG_MFMA_F32 0x800u /* TN_ACYCLIC only, FP32 or BF16 data, not with TN_FLAG_MFMA_BF16:
                                   the SMVP products w_k = mat(X_k) G run on the FP32 matrix
                                   cores (the operands are exact in FP32: the data, and g,
                                   which is stored in FP32 for such data; FP32 accumulation
                                   within a block's column range, FP64 across ranges) instead of
                                   the FP64 ones.  The accumulation over K columns adds about
                                   2^-24 sqrt(K) relative to each w_k per tree level; the tests
                                   state the measured error.  The FP64 products (no flag) stay
                                   the reference mode (TN_ERR_UNSUPPORTED with TN_CYCLIC or FP64
                                   data) */
#define TN_FLAG_SIZE_PILOT 0x100u   /* m <= 0: size the plan from a pilot (see tn_sketch_size) */
#define TN_FLAG_SIZE_LEARNED 0x200u /* m <= 0: size the plan from the registered regressor */

/* Kernel kinds for tn_plan_kernel_time. */
#define TN_KERNEL_HASH 0        /* count-sketch table generation */
#define TN_KERNEL_SKETCH 1      /* sketching pass: cyclic scatter / acyclic leaf+SMVP sweep */
#define TN_KERNEL_COMBINE 2     /* cyclic: DFT + product + sum; acyclic: tensor-sketch combine */
#define TN_KERNEL_STATS 3       /* per-network sample mean / variance */

typedef struct tn_network {
  int32_t p;                 /* number of tensors, >= 1 */
  const int32_t *order;      /* host, p entries: q_k >= 1 */
  const int64_t *dims;       /* host, sum_k q_k entries: n_u >= 1 */
  const void *const *data;   /* host array of p DEVICE pointers (row-major tensors) */
  int32_t dtype;             /* TN_F64 | TN_F32 | TN_BF16; all tensors alike */
  int32_t t;                 /* number of contractions |E| */
  const int32_t *edges;      /* host, 2t global 0-based mode ids */
} tn_network;

typedef struct tn_plan tn_plan;

/*
 * tn_sketch_plan -- validate a batch of networks and prepare an estimator.
 *   nets, n_nets : structures (orders, dims, edges, dtype; data may be NULL
 *                  here, it is bound by each tn_sketch_estimate call).
 *   method       : TN_CYCLIC (any network) or TN_ACYCLIC (trees only).
 *   m            : sketch size (the paper's m), a power of two, or m <= 0 to
 *                  let the plan choose it (and S too when samples <= 0) for
 *                  the target of tn_set_size_target (default eps = 1e-2,
 *                  delta = 0.25): the size of least work S (q N + p m log2 m)
 *                  over the method's ladder (2^6 .. 2^14 cyclic, .. 2^13
 *                  acyclic) with v_j(m) / S <= delta eps^2 for every network j
 *                  (Chebyshev on the plain mean), v from TN_FLAG_SIZE_PILOT,
 *                  TN_FLAG_SIZE_LEARNED or, with neither, the variance bound
 *                  of Lemma 6 / Lemma 9 (see tn_sketch_size).  Pilot and
 *                  learned sizing read the tensors (data must be bound here)
 *                  and synchronize the default stream.  tn_plan_query keys 3
 *                  and 2 return the chosen m and S.  Otherwise m is
 *                  1 <= m <= 65536 for TN_CYCLIC (above 16384 the scatter
 *                  splits each sketch's buckets over blocks and takes one
 *                  sample per pass; when the m-point FFT does not fit in LDS,
 *                  from 16384 with TN_F64 data and 32768 otherwise, the combine
 *                  runs in two passes through a device workspace of
 *                  tensors x m complex values per sample; when a launch has
 *                  under 512 (network, sample) pairs and a network's pairs of
 *                  tensors times m reach 65536, each (network, sample) is
 *                  combined by several blocks over shares of its pairs, with
 *                  a workspace of their m/2 + 1 complex products, at most
 *                  256 MB),
 *                  2 <= m <= 8192 for TN_ACYCLIC.
 *   samples      : S >= 1 independent sketch samples per network (S <= 0
 *                  only with m <= 0: chosen too); sample r
 *                  uses hash key (seed + j, r, stream) for network j.
 *   root         : TN_ACYCLIC root tensor o (Algorithm 2), same for every
 *                  network; -1 lets the planner pick tensor 0.  Ignored for
 *                  TN_CYCLIC.
 *   flags        : TN_FLAG_* bits.
 *   out          : receives the plan; the library owns it and its device
 *                  memory until tn_plan_destroy.
 * Errors: TN_ERR_ARG, TN_ERR_DIMS, TN_ERR_HYPEREDGE, TN_ERR_SELFLOOP,
 * TN_ERR_CYCLIC, TN_ERR_PARTIAL, TN_ERR_UNSUPPORTED (mode size > 2^20,
 * order > 16, m outside the limits; TN_CYCLIC: a tensor whose last mode
 * exceeds 1024; TN_ACYCLIC: a tensor with more than 8 children or whose child
 * modes sum to more than 4096), TN_ERR_OOM, TN_ERR_HIP.
 * Entries must be finite.
 * Uses the current HIP device; the plan is bound to it.
 */
int tn_sketch_plan(const tn_network *nets, int32_t n_nets, int32_t method, int64_t m,
                   int64_t samples, uint64_t seed, int32_t root, uint32_t flags,
                   tn_plan **out);

/*
 * tn_sketch_estimate -- run every sample of every network of the plan.
 *   nets      : the plan's networks again (same structure, same order); only
 *               their data pointers are read.  Buffers must stay valid until
 *               the queued work completes.
 *   stream    : hipStream_t for all device work.
 *   stats     : DEVICE, 2 * n_nets doubles: per network the sample mean of the
 *               S estimates (the averaged estimate) and their unbiased sample
 *               variance (0 when S = 1).  FP64.
 *   samples_out : DEVICE, n_nets * S doubles (network-major), each sample's
 *               estimate; may be NULL.
 * Work is asynchronous on `stream`; the call does not synchronize.  Calls on
 * one plan must not overlap (the plan's workspace is reused).
 */
int tn_sketch_estimate(tn_plan *plan, const tn_network *nets, void *stream, double *stats,
                       double *samples_out);

/*
 * tn_contract_exact -- exact full contraction of one network in FP64 on the
 * device (pairwise contractions in a greedy order; Def. 1-3).  Any network
 * whose every mode is contracted; self-contractions (traces) are allowed.
 *   out : HOST pointer to one double.  The call synchronizes `stream`.
 * Errors: TN_ERR_ARG, TN_ERR_DIMS, TN_ERR_HYPEREDGE, TN_ERR_PARTIAL,
 * TN_ERR_UNSUPPORTED (an intermediate over 2^31 entries), TN_ERR_OOM, TN_ERR_HIP.
 */
int tn_contract_exact(const tn_network *net, void *stream, double *out);

/*
 * Turnstile streaming (TN_FLAG_RESIDENT plans; the general turnstile setting
 * of Algorithm 1: the sketches x_k are kept, and an update, which may change
 * any entry by any amount, costs O(q_k) per sample).  A resident plan's
 * sketches start as those of tn_sketch_estimate's last scan of the bound
 * tensors, or zero after tn_sketch_reset (then the bound tensors are never
 * read); updates are linear, so the sketches always equal those of the
 * tensors the scan (or zero) plus all updates describe.
 *
 * tn_sketch_update -- X_k(index[u]) += delta[u], u < n, for tensor `tensor`
 *   of network `net`, in the sketches of every sample.  index: DEVICE, n int64
 *   row-major entry indices (entries outside [0, size) are ignored); delta:
 *   DEVICE, n doubles (added in the sketch precision: FP64 for TN_F64 data,
 *   FP32 otherwise, with device atomics, so the order of equal-bucket adds,
 *   and hence the low bits, may vary run to run).  The tensor data is not
 *   touched.  Asynchronous on `stream`.
 * tn_sketch_combine -- the estimates of the current sketches: the combine and
 *   per-network statistics of tn_sketch_estimate, without the scan.  stats /
 *   samples_out as for tn_sketch_estimate.
 * tn_sketch_reset -- zero every sketch (all-zero tensors).
 * TN_ERR_ARG on a plan without TN_FLAG_RESIDENT.
 */
int tn_sketch_update(tn_plan *plan, int32_t net, int32_t tensor, int64_t n, const int64_t *index,
                     const double *delta, void *stream);
int tn_sketch_combine(tn_plan *plan, void *stream, double *stats, double *samples_out);
int tn_sketch_reset(tn_plan *plan, void *stream);

/*
 * tn_partial_plan -- partial TNC (Corollary 1) with the estimator of Eq. (1).
 *   net     : one network (same layout as above) whose modes outside every
 *             contraction are free (K' of Def. 1); each tensor must keep at
 *             least one contracted mode (an outer factor is the caller's to
 *             multiply in), else TN_ERR_UNSUPPORTED.
 * The output Y has one entry per assignment of the free modes, row-major over
 * the free modes in increasing global mode order (Def. 1), n_out = prod of
 * their sizes <= 2^20 entries (tn_plan_query key 12; key 13 = free modes).
 * Entry r is estimated by Eq. (1) on the full TNC of the sub-tensors X_k(s_k)
 * at r's indices (the sub-tensors of the corollary's proof).  All entries of a
 * sample share one draw of the count sketches (seed `seed`, stream e for
 * contraction e, as network 0 of tn_sketch_plan): each entry is unbiased with
 * Lemma 6's variance bound for its sub-tensors, so the summed variance is at
 * most 3^t/m prod_k ||X_k||_F^2 as in the corollary's proof; the entries'
 * errors are correlated.  Each tensor is read once per sample pass; a tensor
 * whose free modes are not its leading modes is first copied into a plan
 * buffer with them moved to the front (every estimate call, on `stream`).
 *   m       : power of two, 1 <= m <= 16384 (8192 for TN_F64 data): the
 *             combine's transform stays in LDS.
 *   flags   : TN_FLAG_GRAPH, TN_FLAG_PROFILE, TN_FLAG_PROFILE_SKETCH,
 *             TN_FLAG_AUTOTUNE, TN_FLAG_PRIOR_XCORR; others TN_ERR_ARG.
 * Run it with tn_sketch_estimate(plan, net, stream, stats, samples_out):
 * stats holds 2 n_out doubles (per entry: mean, unbiased variance), samples_out
 * n_out S doubles (entry-major).  tn_plan_get_sketches exports one sketch per
 * sub-tensor (tensor by tensor, sub-tensors in row-major order of the
 * tensor's free modes; tn_plan_query key 6 counts them).
 * Errors as tn_sketch_plan (no TN_ERR_PARTIAL).
 */
int tn_partial_plan(const tn_network *net, int64_t m, int64_t samples, uint64_t seed, uint32_t flags,
                    tn_plan **out);

/* Release a plan and its device memory (synchronizes the device first). NULL is ignored. */
void tn_plan_destroy(tn_plan *plan);

/* Text of the last error raised on the calling thread ("" if none). */
const char *tn_last_error(void);

/*
 * tn_plan_query -- plan sizes.  key: 0 = hash-table width W (packed entries per
 * sample), 1 = number of hash streams, 2 = S, 3 = m, 4 = n_nets,
 * 5 = total tensors, 6 = sketch-vector slots per sample
 * (one per tensor; a partial plan: one per sub-tensor), 7 = method,
 * 8 = samples sketched per pass over the data,
 * 9 = samples per launch (workspace chunk), 10 = accumulator banks per sketch
 * of the cyclic sketching pass (1 or 2; 0 for TN_ACYCLIC), 11 = 1 when the
 * persistent kernel runs the plan (TN_FLAG_PERSISTENT), 12 = estimates per
 * sample (n_nets; a partial plan: its output entries), 13 = free modes of a
 * partial plan (0 otherwise), 14 = blocks per (network, sample) of the
 * cyclic in-LDS combine (1, or more when a plan of few networks has a long
 * product: see tn_sketch_plan; 0 for TN_ACYCLIC).  Keys 8 and 10 may
 * change after the first estimate of a TN_FLAG_AUTOTUNE plan.
 * Returns the value, or a negative code.
 */
int64_t tn_plan_query(const tn_plan *plan, int32_t key);

/*
 * tn_plan_stream -- describe hash stream i (0 <= i < tn_plan_query(plan, 1)):
 * its network index, stream id (as in the hash family above), domain size n
 * and offset of its n packed entries within one sample's table.
 */
int tn_plan_stream(const tn_plan *plan, int64_t i, int32_t *net, uint64_t *stream_id,
                   int64_t *n, int64_t *offset);

/*
 * tn_plan_get_hashes -- write the packed hash tables of samples
 * [first, first + count) to `out` (DEVICE, count * W int32, sample-major), as
 * the estimator uses them (drawn from the family, or the injected tables).
 */
int tn_plan_get_hashes(tn_plan *plan, int64_t first, int64_t count, void *stream, int32_t *out);

/*
 * tn_plan_set_hashes -- test hook: replace the hash family by explicit tables
 * for every sample (DEVICE, S * W packed int32, sample-major; copied on
 * `stream`).  Passing NULL returns the plan to the hash family.
 */
int tn_plan_set_hashes(tn_plan *plan, const int32_t *tables, void *stream);

/*
 * tn_plan_get_sketches -- test hook: the time-domain sketch vectors of samples
 * [first, first + count), as FP64 into `out` (DEVICE, count * slots * m
 * doubles, sample-major, slots as in tn_plan_query key 6).  TN_CYCLIC: y_k =
 * T_k vec(X_k) for every tensor (Algorithm 1's x_k before the DFT).
 * TN_ACYCLIC: x_l = C_{k,l} mat(X_l) R_l^T r_l for each non-root tensor l and
 * r_o = Q_o(kron_l x_l) in the root's slot (Algorithm 2; the estimate is
 * x_o^T r_o).
 */
int tn_plan_get_sketches(tn_plan *plan, const tn_network *nets, int64_t first, int64_t count,
                         void *stream, double *out);

/*
 * tn_plan_kernel_time -- with TN_FLAG_PROFILE: total device time in ms and the
 * number of launches of one kernel kind (TN_KERNEL_*) recorded since the
 * previous call for that kind.  The events are recorded on the stream each
 * kernel was launched on; the call waits for them.
 */
int tn_plan_kernel_time(tn_plan *plan, int32_t kind, double *ms, int64_t *launches);

/*
 * Sketch size for a target of Def. 4: P(|y - tc| > eps prod_k ||X_k||_F) <=
 * delta, following Theorem 1's proof.  One estimate at sketch size m has
 * variance v(m) prod_k ||X_k||_F^2; the mean of S estimates misses eps with
 * probability p <= v(m) / (S eps^2) (Chebyshev), and the median of G such
 * means (G odd) misses only when (G + 1) / 2 of them do, a binomial tail.
 *   mode TN_SIZE_BOUND   : v(m) from the bounds the theorem uses, 3^t / m
 *                          (Lemma 6, TN_CYCLIC) or (1 + 8/m)^{2t} - 1 (Lemma 9,
 *                          TN_ACYCLIC); needs no data;
 *        TN_SIZE_PILOT   : 16 estimates at m0 = 1024 (one batched plan, seed
 *                          `seed`), v(m) = v(m0) m0 / m (the 1/m law of Lemmas 2,
 *                          3 and 6);
 *        TN_SIZE_LEARNED : the regressor registered with tn_set_size_selector
 *                          (include/tn_mlp.h) predicts log v(m) from network
 *                          features (structure, sizes against m, the two bounds,
 *                          per-tensor data statistics), plus its margin.
 * For every network the choice over the ladder (2^6 .. 2^14 cyclic, .. 2^13
 * acyclic) minimizes the work G S (q N + p m log2 m) (q the mean order, N the
 * entries): with max_groups = 1, G = 1 and p = delta; otherwise p ranges over
 * 0.02 .. 0.48 and G is the smallest odd count, at most max_groups, with the
 * tail <= delta.  S <= 2^20; when no m meets the target, the m of least v with
 * S = 2^20.  out: HOST, n_nets choices.  Pilot and learned modes read the
 * tensors and synchronize `stream`.
 */
#define TN_SIZE_BOUND 0
#define TN_SIZE_PILOT 1
#define TN_SIZE_LEARNED 2
typedef struct tn_size_choice {
  int64_t m;        /* sketch size */
  int64_t samples;  /* S: estimates per group */
  int32_t groups;   /* G: the estimate is the median of G group means (odd; 1 = plain mean) */
  double p_group;   /* Chebyshev miss probability allowed per group */
  double v;         /* v(m) = Var(one estimate) / prod_k ||X_k||_F^2 used */
  double work;      /* G S (q N + p m log2 m) */
} tn_size_choice;
int tn_sketch_size(const tn_network *nets, int32_t n_nets, int32_t method, double eps, double delta,
                   int32_t max_groups, int32_t mode, uint64_t seed, void *stream, tn_size_choice *out);

/* Smallest odd G with P(Bin(G, p_group) >= (G + 1) / 2) <= delta (the median
 * trick of Theorem 1's proof), 0 < delta < 1, 0 < p_group < 1/2; at most 4095
 * (else TN_ERR_UNSUPPORTED). */
int tn_median_groups(double delta, double p_group, int32_t *groups);

/* Target (eps, delta) of plans sized by tn_sketch_plan (m <= 0), process-wide;
 * defaults eps = 1e-2, delta = 0.25 (with Chebyshev, two standard errors). */
int tn_set_size_target(double eps, double delta);

/*
 * tn_tensor_stats -- per-tensor statistics used as features by the sketch-size
 * selector: for every tensor of every network (network-major, tensor order),
 * four doubles sum x, sum x^2 (= ||X_k||_F^2), sum |x| and the count of entries
 * >= 0, written to `out` (HOST, 4 * total tensors doubles).  All networks must
 * share one dtype.  Synchronizes `stream`.
 */
int tn_tensor_stats(const tn_network *nets, int32_t n_nets, void *stream, double *out);

/*
 * tn_tensor_stats_noalloc -- tn_tensor_stats for callers that cannot allocate
 * device memory (code under stream capture, serving loops, hosts that forbid
 * hipMalloc): the same statistics, computed by the same kernel in the same
 * order (bit-identical results), with the pointer table, entry counts and
 * output staging in a fixed device array of the library (1.5 MiB per device,
 * held until the process ends) instead of per-call allocations.  It calls no
 * hipMalloc, hipFree or other allocating routine.
 * At most 32768 tensors over all networks, else TN_ERR_UNSUPPORTED (nothing
 * is queued).  Every call on a device shares that device's array: calls that
 * overlap on one device (from several host threads, or queued on different
 * streams) race; the library serializes its host side, and each call
 * synchronizes `stream` before returning.  out: HOST, 4 * total tensors
 * doubles.
 */
int tn_tensor_stats_noalloc(const tn_network *nets, int32_t n_nets, void *stream, double *out);

/*
 * tn_median_of_means -- the amplification of Theorem 1: per network, split its
 * S per-sample estimates (samples: DEVICE, n_nets * S doubles, network-major, as
 * written by tn_sketch_estimate's samples_out) into `groups` consecutive groups,
 * group g holding samples [floor(g S / G), floor((g + 1) S / G)), and write the
 * median of the G group means to out (DEVICE, n_nets doubles; for even G the
 * mean of the two middle ones; NaN if any group mean is NaN).  FP64.
 * 1 <= groups <= min(S, 1024), else TN_ERR_ARG.  Asynchronous on `stream`.
 */
int tn_median_of_means(const double *samples, int64_t n_nets, int64_t S, int32_t groups,
                       void *stream, double *out);

#ifdef __cplusplus
}
#endif

#endif /* TN_SKETCH_H */
