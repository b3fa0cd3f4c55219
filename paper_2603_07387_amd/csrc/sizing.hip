// Sketch-size choice for a target (eps, delta) of Def. 4, and the selector's
// regressor file format.
//
// Theorem 1's argument: an estimate whose variance is v prod_k ||X_k||_F^2
// misses eps prod_k ||X_k||_F with probability at most v / eps^2 (Chebyshev);
// the mean of S independent estimates at sketch size m has v = v(m) / S; the
// median of G such means misses only when at least (G + 1) / 2 of them miss,
// a binomial tail that falls exponentially in G (the median trick of the
// theorem's proof).  v(m) comes from one of three sources:
//   bound   -- the variance bounds the theorem uses: 3^t / m (Lemma 6) for the
//              cyclic method, (1 + 8/m)^{2t} - 1 (Lemma 9) for the acyclic one;
//   pilot   -- S0 estimates at m0, v(m) = v(m0) m0 / m (the 1/m law of Lemmas
//              2, 3 and 6);
//   learned -- the regressor's prediction of log v(m) from network features,
//              plus its calibration margin.
// Among the power-of-two sizes of the method's ladder the choice minimizes
// the work G S (q N + p m log2 m) (Theorem 1's cost terms, q the mean order).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "plan.h"
#include "../../include/tn_mlp.h"

namespace tn {
namespace {

constexpr int kFeatures = 32;
constexpr int64_t kMaxSamplesChoice = (int64_t)1 << 20;

// Power-of-two ladder of sketch sizes the choice ranges over.
std::vector<int64_t> ladder(int method) {
  std::vector<int64_t> out;
  for (int k = 6; k <= (method == TN_ACYCLIC ? 13 : 14); ++k) out.push_back((int64_t)1 << k);
  return out;
}

// P(Bin(G, p) >= (G + 1) / 2), G odd, in log space.
double median_miss(int G, double p) {
  double tail = 0.0;
  for (int i = (G + 1) / 2; i <= G; ++i)
    tail += std::exp(std::lgamma(G + 1.0) - std::lgamma(i + 1.0) - std::lgamma(G - i + 1.0) + i * std::log(p) +
                     (G - i) * std::log1p(-p));
  return tail;
}

// Smallest odd G with median_miss(G, p) <= delta (p < 1/2), or -1 past 4095.
int groups_for(double delta, double p) {
  if (!(p > 0.0 && p < 0.5)) return -1;
  for (int G = 1; G <= 4095; G += 2)
    if (median_miss(G, p) <= delta * (1.0 + 1e-12)) return G;  // (log-space rounding)
  return -1;
}

struct NetInfo {
  int p = 0, t = 0, depth = 0, leaves = 0;
  std::vector<double> orders, sizes, bonds;
  double N = 0.0, qmean = 0.0;
};

NetInfo net_info(const tn_network &n) {
  NetInfo I;
  I.p = n.p;
  I.t = n.t;
  std::vector<int> offs(1, 0), owner;
  for (int k = 0; k < n.p; ++k) {
    offs.push_back(offs.back() + n.order[k]);
    for (int i = 0; i < n.order[k]; ++i) owner.push_back(k);
    I.orders.push_back((double)n.order[k]);
    if (n.order[k] == 1) ++I.leaves;
    double s = 1.0;
    for (int u = offs[k]; u < offs[k + 1]; ++u) s *= (double)n.dims[u];
    I.sizes.push_back(s);
    I.N += s;
  }
  for (double q : I.orders) I.qmean += q;
  I.qmean /= n.p;
  for (int e = 0; e < n.t; ++e) I.bonds.push_back((double)n.dims[n.edges[2 * e]]);
  if (I.bonds.empty()) I.bonds.push_back(1.0);
  // breadth-first depth from tensor 0 over the contraction graph
  std::vector<std::vector<int>> adj((size_t)n.p);
  for (int e = 0; e < n.t; ++e) {
    const int a = owner[(size_t)n.edges[2 * e]], b = owner[(size_t)n.edges[2 * e + 1]];
    adj[(size_t)a].push_back(b);
    adj[(size_t)b].push_back(a);
  }
  std::vector<int> depth((size_t)n.p, -1), queue(1, 0);
  depth[0] = 0;
  for (size_t h = 0; h < queue.size(); ++h)
    for (int b : adj[(size_t)queue[h]])
      if (depth[(size_t)b] < 0) {
        depth[(size_t)b] = depth[(size_t)queue[h]] + 1;
        queue.push_back(b);
      }
  for (int d : depth) I.depth = std::max(I.depth, d);
  return I;
}

double work_per_sample(const NetInfo &I, int64_t m) {
  return I.qmean * I.N + I.p * (double)m * std::max(std::log2((double)m), 1.0);
}

double mean_of(const std::vector<double> &x) {
  double s = 0.0;
  for (double v : x) s += v;
  return s / (double)x.size();
}

// The regressor's features of one network at sketch size m (stats: per
// tensor sum x, sum x^2, sum |x|, count x >= 0).  Each is O(1): structure
// (sizes, orders, depth, bond and tensor sizes against m), the two variance
// bounds in log form, and data shape (coherence |sum x| / (||X||_F sqrt N),
// the mean-absolute to RMS ratio, the fraction of non-negative entries).
void features(const NetInfo &I, const double *stats, int method, int64_t m, float *f) {
  const int p = I.p, t = I.t;
  std::vector<double> coh((size_t)p), shape((size_t)p), lcoh((size_t)p), ls((size_t)p), lb, nnf((size_t)p);
  for (int k = 0; k < p; ++k) {
    const double s = stats[4 * k], s2 = stats[4 * k + 1], sa = stats[4 * k + 2], nn = stats[4 * k + 3];
    const double fro = std::sqrt(std::max(s2, 1e-300));
    const double sz = I.sizes[(size_t)k];
    coh[(size_t)k] = std::fabs(s) / (fro * std::sqrt(sz));
    shape[(size_t)k] = sa / (fro * std::sqrt(sz));
    lcoh[(size_t)k] = std::log2(1.0 + coh[(size_t)k] * coh[(size_t)k] * sz);
    ls[(size_t)k] = std::log2(sz);
    nnf[(size_t)k] = nn / sz;
  }
  for (double b : I.bonds) lb.push_back(std::log2(b));
  const double lm = std::log2((double)m);
  double maxo = 0, maxlb = -1e300, minlb = 1e300, maxls = -1e300, sumsz = 0, maxcoh = -1e300, mincoh = 1e300,
         mincoh_shape = 1e300, sumlcoh = 0, big = 0, lcohlog = 0;
  for (double o : I.orders) maxo = std::max(maxo, o);
  for (double v : lb) { maxlb = std::max(maxlb, v); minlb = std::min(minlb, v); }
  for (int k = 0; k < p; ++k) {
    maxls = std::max(maxls, ls[(size_t)k]);
    sumsz += I.sizes[(size_t)k];
    maxcoh = std::max(maxcoh, coh[(size_t)k]);
    mincoh = std::min(mincoh, coh[(size_t)k]);
    mincoh_shape = std::min(mincoh_shape, shape[(size_t)k]);
    sumlcoh += lcoh[(size_t)k];
    big += coh[(size_t)k] > 0.5 ? 1.0 : 0.0;
    lcohlog += std::log2(std::max(coh[(size_t)k], 1e-30));
  }
  const double v9 = std::pow(1.0 + 8.0 / (double)m, 2.0 * t) - 1.0;
  const double x[kFeatures] = {
      method == TN_ACYCLIC ? 1.0 : 0.0,
      lm / 10,
      lm * lm / 100,
      64.0 / (double)m,
      p / 10.0,
      t / 10.0,
      (t - p + 1) / 10.0,
      mean_of(I.orders) / 4,
      maxo / 4,
      I.depth / 10.0,
      (double)I.leaves / p,
      mean_of(lb) / 5,
      maxlb / 5,
      minlb / 5,
      mean_of(ls) / 10,
      maxls / 10,
      std::log2(sumsz) / 20,
      (maxls - lm) / 10,
      (mean_of(lb) - lm) / 10,
      mean_of(coh),
      maxcoh,
      mincoh,
      big / p,
      mean_of(lcoh) / 10,
      sumlcoh / std::max(t, 1) / 10,
      mean_of(nnf),
      mean_of(shape),
      mincoh_shape,
      (t * std::log2(3.0) - lm) / 10,
      std::log2(std::max(v9, 1e-300)) / 10,
      (sumlcoh - lm) / 100,
      lcohlog / p / 10,
  };
  for (int i = 0; i < kFeatures; ++i) f[i] = (float)x[i];
}

// The registered regressor (tn_set_size_selector) and the target of plans
// sized automatically (tn_set_size_target).
std::mutex g_size_mu;
const tn_mlp *g_sel = nullptr;
double g_sel_mu = 0.0, g_sel_sd = 1.0, g_sel_margin = 0.0;
double g_eps = 1e-2, g_delta = 0.25;

// log v(m) over the ladder for every network (n_nets x ladder, row-major).
int logv_ladder(const tn_network *nets, int n_nets, int method, int mode, uint64_t seed, hipStream_t st,
                std::vector<double> *out, std::vector<NetInfo> *infos) {
  const std::vector<int64_t> L = ladder(method);
  const size_t nl = L.size();
  out->assign((size_t)n_nets * nl, 0.0);
  infos->clear();
  for (int j = 0; j < n_nets; ++j) infos->push_back(net_info(nets[j]));
  if (mode == TN_SIZE_BOUND) {
    for (int j = 0; j < n_nets; ++j)
      for (size_t i = 0; i < nl; ++i) {
        const double t = (*infos)[(size_t)j].t;
        const double v = method == TN_CYCLIC ? std::pow(3.0, t) / (double)L[i]
                                             : std::pow(1.0 + 8.0 / (double)L[i], 2.0 * t) - 1.0;
        (*out)[(size_t)j * nl + i] = std::log(std::max(v, 1e-300));
      }
    return TN_OK;
  }
  int64_t nt = 0;
  for (int j = 0; j < n_nets; ++j) nt += nets[j].p;
  std::vector<double> stats((size_t)nt * 4);
  int rc = tn_tensor_stats(nets, n_nets, st, stats.data());
  if (rc != TN_OK) return rc;
  std::vector<double> norm2((size_t)n_nets, 1.0);
  {
    int64_t k0 = 0;
    for (int j = 0; j < n_nets; ++j)
      for (int k = 0; k < nets[j].p; ++k, ++k0) norm2[(size_t)j] *= stats[(size_t)k0 * 4 + 1];
  }
  if (mode == TN_SIZE_PILOT) {
    // S0 = 16 estimates at m0 = 1024 (or the ladder's top), one batched plan
    const int64_t m0 = std::min<int64_t>(1024, L.back()), S0 = 16;
    tn_plan *pl = nullptr;
    if ((rc = tn_sketch_plan(nets, n_nets, method, m0, S0, seed, -1, 0, &pl)) != TN_OK) return rc;
    double *d_stats = nullptr;
    if (hipMalloc((void **)&d_stats, (size_t)n_nets * 2 * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      tn_plan_destroy(pl);
      return set_error(TN_ERR_OOM, "pilot: hipMalloc");
    }
    std::vector<double> h((size_t)n_nets * 2);
    rc = tn_sketch_estimate(pl, nets, st, d_stats, nullptr);
    hipError_t e = hipSuccess;
    if (rc == TN_OK) e = hipMemcpyAsync(h.data(), d_stats, h.size() * 8, hipMemcpyDeviceToHost, st);
    if (rc == TN_OK && e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_stats);
    tn_plan_destroy(pl);
    if (rc != TN_OK) return rc;
    if (e != hipSuccess) return set_error(TN_ERR_HIP, "pilot: %s", hipGetErrorString(e));
    for (int j = 0; j < n_nets; ++j) {
      const double v0 = std::max(norm2[(size_t)j] > 0 ? h[(size_t)j * 2 + 1] / norm2[(size_t)j] : 0.0, 1e-300);
      for (size_t i = 0; i < nl; ++i) (*out)[(size_t)j * nl + i] = std::log(v0 * (double)m0 / (double)L[i]);
    }
    return TN_OK;
  }
  // learned: features on the host, the regressor on the device
  std::lock_guard<std::mutex> lk(g_size_mu);
  if (!g_sel) return set_error(TN_ERR_ARG, "learned sizing: no regressor registered (tn_set_size_selector)");
  std::vector<float> X((size_t)n_nets * nl * kFeatures);
  {
    int64_t k0 = 0;
    for (int j = 0; j < n_nets; ++j) {
      for (size_t i = 0; i < nl; ++i)
        features((*infos)[(size_t)j], stats.data() + k0 * 4, method, L[i], X.data() + ((size_t)j * nl + i) * kFeatures);
      k0 += nets[j].p;
    }
  }
  float *dX = nullptr, *dy = nullptr;
  const size_t rows = (size_t)n_nets * nl;
  if (hipMalloc((void **)&dX, X.size() * 4) != hipSuccess || hipMalloc((void **)&dy, rows * 4) != hipSuccess) {
    (void)hipGetLastError();
    if (dX) (void)hipFree(dX);
    return set_error(TN_ERR_OOM, "learned sizing: hipMalloc");
  }
  std::vector<float> y(rows);
  hipError_t e = hipMemcpyAsync(dX, X.data(), X.size() * 4, hipMemcpyHostToDevice, st);
  rc = e == hipSuccess ? tn_mlp_predict(const_cast<tn_mlp *>(g_sel), dX, (int64_t)rows, st, dy)
                       : set_error(TN_ERR_HIP, "learned sizing: %s", hipGetErrorString(e));
  if (rc == TN_OK) e = hipMemcpyAsync(y.data(), dy, rows * 4, hipMemcpyDeviceToHost, st);
  if (rc == TN_OK && e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dX);
  (void)hipFree(dy);
  if (rc != TN_OK) return rc;
  if (e != hipSuccess) return set_error(TN_ERR_HIP, "learned sizing: %s", hipGetErrorString(e));
  for (size_t r = 0; r < rows; ++r) (*out)[r] = (double)y[r] * g_sel_sd + g_sel_mu + g_sel_margin;
  return TN_OK;
}

// The least-work (m, S, G) for one network given log v over the ladder.
tn_size_choice choose_one(const NetInfo &I, const std::vector<int64_t> &L, const double *logv, double eps,
                          double delta, int max_groups) {
  tn_size_choice best{};
  best.work = -1.0;
  for (size_t i = 0; i < L.size(); ++i) {
    const double v = std::exp(std::min(logv[i], 700.0));
    // Group miss probability p (Chebyshev: v / (S eps^2) <= p) and median size
    // G.  G = 1 takes p = delta; with medians allowed, the p of least G S over
    // a grid, G the smallest odd count whose binomial tail is <= delta.
    double bp = delta;
    int bG = 1;
    double bS = std::ceil(v / (bp * eps * eps));
    if (max_groups > 1) {
      for (int gi = 1; gi <= 24; ++gi) {
        const double pg = 0.02 * gi;
        const int G = groups_for(delta, pg);
        if (G < 1 || G > max_groups) continue;
        const double Sg = std::ceil(v / (pg * eps * eps));
        if ((double)G * Sg < (double)bG * bS) { bG = G; bS = Sg; bp = pg; }
      }
    }
    const double Sg = std::max(1.0, bS);
    if (Sg > (double)kMaxSamplesChoice) continue;
    const double w = (double)bG * Sg * work_per_sample(I, L[i]);
    if (best.work < 0.0 || w < best.work) {
      best.m = L[i];
      best.samples = (int64_t)Sg;
      best.groups = bG;
      best.p_group = bp;
      best.v = v;
      best.work = w;
    }
  }
  if (best.work < 0.0) {  // no size meets the target within the sample cap: the least variance
    size_t ib = 0;
    for (size_t i = 1; i < L.size(); ++i)
      if (logv[i] < logv[ib]) ib = i;
    best.m = L[ib];
    best.samples = kMaxSamplesChoice;
    best.groups = 1;
    best.p_group = delta;
    best.v = std::exp(std::min(logv[ib], 700.0));
    best.work = (double)kMaxSamplesChoice * work_per_sample(I, L[ib]);
  }
  return best;
}

// CRC-32 of ISO 3309 / ITU-T V.42 (reflected polynomial 0xEDB88320, initial
// and final complement), bit by bit.
uint32_t crc32_update(uint32_t crc, const unsigned char *p, size_t n) {
  crc = ~crc;
  for (size_t i = 0; i < n; ++i) {
    crc ^= p[i];
    for (int b = 0; b < 8; ++b) crc = (crc >> 1) ^ (0xEDB88320u & (0u - (crc & 1u)));
  }
  return ~crc;
}

constexpr char kMagic[8] = {'T', 'N', 'M', 'L', 'P', '\0', '\0', '\1'};

}  // namespace

// Automatic (m, S) of a plan (tn_sketch_plan with m <= 0): the target of
// tn_set_size_target, the plain mean (G = 1), one m for every network.
int auto_size(const tn_network *nets, int n_nets, int method, uint32_t flags, uint64_t seed, int64_t samples,
              int64_t *m_out, int64_t *S_out) {
  const int mode = (flags & TN_FLAG_SIZE_LEARNED) ? TN_SIZE_LEARNED : (flags & TN_FLAG_SIZE_PILOT) ? TN_SIZE_PILOT
                                                                                                   : TN_SIZE_BOUND;
  double eps, delta;
  {
    std::lock_guard<std::mutex> lk(g_size_mu);
    eps = g_eps;
    delta = g_delta;
  }
  std::vector<double> lv;
  std::vector<NetInfo> info;
  int rc = logv_ladder(nets, n_nets, method, mode, seed, nullptr, &lv, &info);
  if (rc != TN_OK) return rc;
  const std::vector<int64_t> L = ladder(method);
  const size_t nl = L.size();
  const double cap = samples > 0 ? (double)samples : (double)kMaxSamplesChoice;
  double best_w = -1.0;
  int64_t bm = L.back(), bS = samples > 0 ? samples : kMaxSamplesChoice;
  for (size_t i = 0; i < nl; ++i) {
    double need = 1.0;
    for (int j = 0; j < n_nets; ++j)
      need = std::max(need, std::ceil(std::exp(std::min(lv[(size_t)j * nl + i], 700.0)) / (delta * eps * eps)));
    if (need > cap) continue;
    const double S = samples > 0 ? (double)samples : need;
    double w = 0.0;
    for (int j = 0; j < n_nets; ++j) w += S * work_per_sample(info[(size_t)j], L[i]);
    if (best_w < 0.0 || w < best_w) {
      best_w = w;
      bm = L[i];
      bS = (int64_t)S;
    }
  }
  if (best_w < 0.0) {  // the target is out of reach: the size of least summed variance
    double bv = 1e300;
    for (size_t i = 0; i < nl; ++i) {
      double v = 0.0;
      for (int j = 0; j < n_nets; ++j) v += std::exp(std::min(lv[(size_t)j * nl + i], 700.0));
      if (v < bv) { bv = v; bm = L[i]; }
    }
  }
  log_msg(1, "size: %s variance, eps %g, delta %g, %d networks: m %lld, S %lld%s",
          mode == TN_SIZE_LEARNED ? "learned" : mode == TN_SIZE_PILOT ? "pilot" : "bound", eps, delta, n_nets,
          (long long)bm, (long long)bS, best_w < 0.0 ? " (target out of reach: least variance)" : "");
  *m_out = bm;
  *S_out = bS;
  return TN_OK;
}

}  // namespace tn

using namespace tn;

extern "C" {

int tn_median_groups(double delta, double p_group, int32_t *groups) {
  clear_error();
  if (!groups || !(delta > 0.0 && delta < 1.0) || !(p_group > 0.0 && p_group < 0.5))
    return set_error(TN_ERR_ARG, "need 0 < delta < 1 and 0 < p_group < 1/2");
  const int G = groups_for(delta, p_group);
  if (G < 0) return set_error(TN_ERR_UNSUPPORTED, "more than 4095 groups needed");
  *groups = G;
  return TN_OK;
}

int tn_sketch_size(const tn_network *nets, int32_t n_nets, int32_t method, double eps, double delta,
                   int32_t max_groups, int32_t mode, uint64_t seed, void *stream, tn_size_choice *out) {
  clear_error();
  if (!nets || n_nets < 1 || !out) return set_error(TN_ERR_ARG, "null argument");
  if (method != TN_CYCLIC && method != TN_ACYCLIC) return set_error(TN_ERR_ARG, "method %d", method);
  if (!(eps > 0.0) || !(delta > 0.0 && delta < 1.0) || max_groups < 1)
    return set_error(TN_ERR_ARG, "need eps > 0, 0 < delta < 1, max_groups >= 1");
  if (mode != TN_SIZE_BOUND && mode != TN_SIZE_PILOT && mode != TN_SIZE_LEARNED)
    return set_error(TN_ERR_ARG, "mode %d", mode);
  for (int j = 0; j < n_nets; ++j) {
    NetCheck c;
    int rc = validate_network(&nets[j], j, &c);
    if (rc != TN_OK) return rc;
    if (method == TN_ACYCLIC && (rc = validate_tree(&nets[j], j, c)) != TN_OK) return rc;
  }
  std::vector<double> lv;
  std::vector<NetInfo> info;
  int rc = logv_ladder(nets, n_nets, method, mode, seed, (hipStream_t)stream, &lv, &info);
  if (rc != TN_OK) return rc;
  const std::vector<int64_t> L = ladder(method);
  for (int j = 0; j < n_nets; ++j)
    out[j] = choose_one(info[(size_t)j], L, lv.data() + (size_t)j * L.size(), eps, delta, max_groups);
  return TN_OK;
}

int tn_set_size_selector(const tn_mlp *net, double mu, double sd, double margin) {
  clear_error();
  if (net && (tn_mlp_num_params(net) <= 0 || !(sd > 0.0)))
    return set_error(TN_ERR_ARG, "selector: bad regressor or standard deviation");
  std::lock_guard<std::mutex> lk(g_size_mu);
  g_sel = net;
  g_sel_mu = mu;
  g_sel_sd = sd;
  g_sel_margin = margin;
  return TN_OK;
}

int tn_set_size_target(double eps, double delta) {
  clear_error();
  if (!(eps > 0.0) || !(delta > 0.0 && delta < 1.0)) return set_error(TN_ERR_ARG, "need eps > 0, 0 < delta < 1");
  std::lock_guard<std::mutex> lk(g_size_mu);
  g_eps = eps;
  g_delta = delta;
  return TN_OK;
}

int tn_mlp_save(const tn_mlp *net, const char *path, const double *meta, int32_t n_meta) {
  clear_error();
  if (!net || !path || n_meta < 0 || n_meta > 64 || (n_meta > 0 && !meta))
    return set_error(TN_ERR_ARG, "bad argument");
  const int64_t P = tn_mlp_num_params(net);
  std::vector<float> params((size_t)P);
  int rc = tn_mlp_get_params(net, params.data());
  if (rc != TN_OK) return rc;
  std::vector<unsigned char> buf;
  auto put = [&](const void *p, size_t n) {
    const unsigned char *c = static_cast<const unsigned char *>(p);
    buf.insert(buf.end(), c, c + n);
  };
  const uint32_t version = 1;
  int32_t d_in = 0, hidden = 0;
  if ((rc = tn_mlp_shape(net, &d_in, &hidden)) != TN_OK) return rc;
  put(kMagic, 8);
  put(&version, 4);
  put(&d_in, 4);
  put(&hidden, 4);
  put(&n_meta, 4);
  put(&P, 8);
  if (n_meta > 0) put(meta, (size_t)n_meta * 8);
  put(params.data(), (size_t)P * 4);
  const uint32_t crc = crc32_update(0, buf.data(), buf.size());
  put(&crc, 4);
  FILE *f = std::fopen(path, "wb");
  if (!f) return set_error(TN_ERR_ARG, "cannot open %s for writing", path);
  const size_t w = std::fwrite(buf.data(), 1, buf.size(), f);
  const int cl = std::fclose(f);
  if (w != buf.size() || cl != 0) return set_error(TN_ERR_ARG, "writing %s failed", path);
  return TN_OK;
}

int tn_mlp_load(const char *path, tn_mlp **out, double *meta, int32_t max_meta, int32_t *n_meta) {
  clear_error();
  if (!path || !out || max_meta < 0 || (max_meta > 0 && !meta)) return set_error(TN_ERR_ARG, "bad argument");
  *out = nullptr;
  FILE *f = std::fopen(path, "rb");
  if (!f) return set_error(TN_ERR_ARG, "cannot open %s", path);
  const size_t head = 8 + 4 + 4 + 4 + 4 + 8;
  const size_t largest = head + 64 * 8 + ((size_t)1 << 26) * 4 + 4;  // the largest legal file
  std::vector<unsigned char> buf;
  unsigned char tmp[65536];
  size_t r;
  while ((r = std::fread(tmp, 1, sizeof(tmp), f)) > 0 && buf.size() <= largest) buf.insert(buf.end(), tmp, tmp + r);
  std::fclose(f);
  if (buf.size() > largest) return set_error(TN_ERR_ARG, "%s is too large for a regressor file", path);
  if (buf.size() < head + 4 || std::memcmp(buf.data(), kMagic, 8) != 0)
    return set_error(TN_ERR_ARG, "%s is not a regressor file", path);
  uint32_t version, crc;
  int32_t d_in, hidden, nm;
  int64_t P;
  std::memcpy(&version, buf.data() + 8, 4);
  std::memcpy(&d_in, buf.data() + 12, 4);
  std::memcpy(&hidden, buf.data() + 16, 4);
  std::memcpy(&nm, buf.data() + 20, 4);
  std::memcpy(&P, buf.data() + 24, 8);
  if (version != 1 || nm < 0 || nm > 64 || P < 1 || P > (int64_t)1 << 26 ||
      buf.size() != head + (size_t)nm * 8 + (size_t)P * 4 + 4)
    return set_error(TN_ERR_ARG, "%s: bad header or size", path);
  std::memcpy(&crc, buf.data() + buf.size() - 4, 4);
  if (crc32_update(0, buf.data(), buf.size() - 4) != crc) return set_error(TN_ERR_ARG, "%s: CRC mismatch", path);
  if (nm > max_meta) return set_error(TN_ERR_ARG, "%s holds %d meta values, room for %d", path, nm, max_meta);
  tn_mlp *net = nullptr;
  int rc = tn_mlp_create(d_in, hidden, 0, &net);
  if (rc != TN_OK) return rc;
  if (tn_mlp_num_params(net) != P) {
    tn_mlp_destroy(net);
    return set_error(TN_ERR_ARG, "%s: parameter count does not match d_in %d, hidden %d", path, d_in, hidden);
  }
  std::vector<float> params((size_t)P);
  std::memcpy(params.data(), buf.data() + head + (size_t)nm * 8, (size_t)P * 4);
  if ((rc = tn_mlp_set_params(net, params.data())) != TN_OK) {
    tn_mlp_destroy(net);
    return rc;
  }
  if (nm > 0) std::memcpy(meta, buf.data() + head, (size_t)nm * 8);
  if (n_meta) *n_meta = nm;
  *out = net;
  return TN_OK;
}

}  // extern "C"
