/*
 * tn_oracle.c -- plain FP64 CPU oracle for the sketching estimators of
 * "Approximating Tensor Network Contraction with Sketches" (arXiv 2603.07387).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or table with the HIP path.
 *
 * Everything here is written for obviousness, not speed: index loops in the
 * order the definitions state them, FP64 throughout, no blocking or fusion.
 *
 * Networks (Def. 1-3): p tensors; tensor k owns the consecutive global modes
 * off[k] .. off[k]+order[k]-1; dims[u] is the size of global mode u; data[k]
 * is row-major (vec = lexicographic order, Preliminaries); edges[2e], edges[2e+1]
 * is the contracted mode pair (u, v) of edge e, 0-based.
 *
 * Hash family (Def. 10-11 need 2-wise independent buckets and 4-wise
 * independent signs; the paper gives no construction).  Over the prime
 * P = 2^31 - 1:
 *     mix(x)   = SplitMix64 output for state x (Steele, Lea, Flood 2014)
 *     key      = mix(mix(mix(seed) ^ sample) ^ stream)
 *     raw_j    = mix(key ^ j) >> 33                              (j = 0..5)
 *     a0 = raw_0 mod P,   a1 = 1 + raw_1 mod (P - 1)
 *     c_j = raw_{2+j} mod P                                      (j = 0..3)
 *     h(i) = ((a1 i + a0) mod P) mod m                  (degree-1: 2-wise)
 *     s(i) = +1 if (c3 i^3 + c2 i^2 + c1 i + c0) mod P is even, else -1
 *                                                      (degree-3: 4-wise)
 * Streams: edge e -> stream e.  Cyclic method: the first mode of edge e uses
 * (h, s); the second uses the complement count sketch (Def. 14), 0-based
 * bucket (m - h) mod m with the same sign.  Acyclic method: tensor sketch T_{l,j}
 * of node k, side d -> stream 2^62 + k 2^32 + l 2^16 + 2j + d (domain [m]);
 * padding sketch of node k, slot j -> stream 2^63 + k 2^32 + j (domain [1]).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_P 2147483647ULL

/* ------------------------------------------------------------------------- */
/* Hash family                                                               */
/* ------------------------------------------------------------------------- */

uint64_t orc_mix(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

void orc_hash_coeffs(uint64_t seed, uint64_t sample, uint64_t stream, uint64_t c[6]) {
  uint64_t key = orc_mix(orc_mix(orc_mix(seed) ^ sample) ^ stream);
  uint64_t raw[6];
  for (int j = 0; j < 6; ++j) raw[j] = orc_mix(key ^ (uint64_t)j) >> 33;
  c[0] = raw[0] % ORC_P;             /* a0 */
  c[1] = 1 + raw[1] % (ORC_P - 1);   /* a1 */
  c[2] = raw[2] % ORC_P;             /* sign polynomial c0 */
  c[3] = raw[3] % ORC_P;             /* c1 */
  c[4] = raw[4] % ORC_P;             /* c2 */
  c[5] = raw[5] % ORC_P;             /* c3 */
}

static int64_t hash_bucket(const uint64_t c[6], uint64_t i, int64_t m) {
  uint64_t v = ((c[1] * i) % ORC_P + c[0]) % ORC_P;
  return (int64_t)(v % (uint64_t)m);
}

static int hash_sign(const uint64_t c[6], uint64_t i) {
  uint64_t v = c[5];
  v = (v * i + c[4]) % ORC_P;
  v = (v * i + c[3]) % ORC_P;
  v = (v * i + c[2]) % ORC_P;
  return (v & 1ULL) ? -1 : 1;
}

/* Count sketch tables of one stream: h[i] in [0, m), s[i] in {-1, +1}. */
void orc_count_sketch(uint64_t seed, uint64_t sample, uint64_t stream, int64_t n, int64_t m,
                      int64_t *h, int32_t *s) {
  uint64_t c[6];
  orc_hash_coeffs(seed, sample, stream, c);
  for (int64_t i = 0; i < n; ++i) {
    h[i] = hash_bucket(c, (uint64_t)i, m);
    s[i] = hash_sign(c, (uint64_t)i);
  }
}

uint64_t orc_stream_tsketch(int64_t node, int64_t level, int64_t j, int side) {
  return (1ULL << 62) + ((uint64_t)node << 32) + ((uint64_t)level << 16) + (uint64_t)(2 * j + side);
}

uint64_t orc_stream_pad(int64_t node, int64_t slot) {
  return (1ULL << 63) + ((uint64_t)node << 32) + (uint64_t)slot;
}

/* ------------------------------------------------------------------------- */
/* Network helpers                                                           */
/* ------------------------------------------------------------------------- */

typedef struct {
  int p, t, q;
  const int *order;
  const int64_t *dims;
  const double *const *data;
  const int *edges;
  int off[4097];
} net_t;

static int net_init(net_t *N, int p, const int *order, const int64_t *dims,
                    const double *const *data, int t, const int *edges) {
  if (p <= 0 || p > 4096) return -1;
  N->p = p; N->t = t; N->order = order; N->dims = dims; N->data = data; N->edges = edges;
  N->off[0] = 0;
  for (int k = 0; k < p; ++k) N->off[k + 1] = N->off[k] + order[k];
  N->q = N->off[p];
  return 0;
}

static int64_t tensor_size(const net_t *N, int k) {
  int64_t s = 1;
  for (int u = N->off[k]; u < N->off[k + 1]; ++u) s *= N->dims[u];
  return s;
}

/* Advance a row-major multi-index; returns 0 when it wraps around. */
static int odometer(int64_t *idx, const int64_t *dims, int q) {
  for (int j = q - 1; j >= 0; --j) {
    if (++idx[j] < dims[j]) return 1;
    idx[j] = 0;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Exact contraction                                                         */
/* ------------------------------------------------------------------------- */

/*
 * Def. 1 read literally: sum over every index of every mode of the product
 * tensor, weighted by prod_{(u,v) in E} [i_u = i_v]; the result is indexed by
 * the free modes K' in increasing mode order (row-major).  Cost prod_u n_u:
 * tiny networks only.  out must hold prod_{u in K'} n_u doubles.
 */
int orc_tc_literal(int p, const int *order, const int64_t *dims, const double *const *data,
                   int t, const int *edges, double *out) {
  net_t N;
  if (net_init(&N, p, order, dims, data, t, edges)) return -1;
  int q = N.q;
  int *is_free = calloc((size_t)q, sizeof(int));
  int64_t *idx = calloc((size_t)q, sizeof(int64_t));
  int64_t outsize = 1;
  for (int u = 0; u < q; ++u) is_free[u] = 1;
  for (int e = 0; e < t; ++e) { is_free[edges[2 * e]] = 0; is_free[edges[2 * e + 1]] = 0; }
  for (int u = 0; u < q; ++u) if (is_free[u]) outsize *= dims[u];
  for (int64_t o = 0; o < outsize; ++o) out[o] = 0.0;
  do {
    int ok = 1;
    for (int e = 0; e < t; ++e) if (idx[edges[2 * e]] != idx[edges[2 * e + 1]]) { ok = 0; break; }
    if (!ok) continue;
    double prod = 1.0;
    for (int k = 0; k < p; ++k) {
      int64_t lin = 0;
      for (int u = N.off[k]; u < N.off[k + 1]; ++u) lin = lin * dims[u] + idx[u];
      prod *= data[k][lin];
    }
    int64_t o = 0;
    for (int u = 0; u < q; ++u) if (is_free[u]) o = o * dims[u] + idx[u];
    out[o] += prod;
  } while (odometer(idx, dims, q));
  free(is_free); free(idx);
  return 0;
}

/*
 * Full TNC with the Iverson brackets reduced (as in Example 1): one summation
 * index per contraction.  Requires every mode to be in exactly one edge.
 */
int orc_tc_full(int p, const int *order, const int64_t *dims, const double *const *data,
                int t, const int *edges, double *out) {
  net_t N;
  if (net_init(&N, p, order, dims, data, t, edges)) return -1;
  int q = N.q;
  int *edge_of = malloc((size_t)q * sizeof(int));
  for (int u = 0; u < q; ++u) edge_of[u] = -1;
  for (int e = 0; e < t; ++e) {
    for (int side = 0; side < 2; ++side) {
      int u = edges[2 * e + side];
      if (edge_of[u] != -1) { free(edge_of); return -2; }
      edge_of[u] = e;
    }
  }
  for (int u = 0; u < q; ++u) if (edge_of[u] < 0) { free(edge_of); return -3; }
  int64_t *edims = malloc((size_t)(t > 0 ? t : 1) * sizeof(int64_t));
  int64_t *eidx = calloc((size_t)(t > 0 ? t : 1), sizeof(int64_t));
  double terms = 1.0;
  for (int e = 0; e < t; ++e) { edims[e] = dims[edges[2 * e]]; terms *= (double)edims[e]; }
  if (terms > 17179869184.0) { free(edge_of); free(edims); free(eidx); return -7; }  /* > 2^34 */
  double acc = 0.0;
  do {
    double prod = 1.0;
    for (int k = 0; k < p; ++k) {
      int64_t lin = 0;
      for (int u = N.off[k]; u < N.off[k + 1]; ++u) lin = lin * dims[u] + eidx[edge_of[u]];
      prod *= data[k][lin];
    }
    acc += prod;
  } while (t > 0 && odometer(eidx, edims, t));
  *out = acc;
  free(edge_of); free(edims); free(eidx);
  return 0;
}

/*
 * Periodic R x C lattice (Def. 1-3 for the torus): tensor (r, c) is data[r C + c]
 * with modes (left, right, up, down), each of size D; right(r, c) meets
 * left(r, c+1) and down(r, c) meets up(r+1, c), indices mod C and R.  Summed
 * row by row: the row transfer matrix
 *   T_r[(u_0..u_{C-1}), (d_0..d_{C-1})]
 *     = sum over h_0..h_{C-1} of prod_c X_(r,c)[h_c, h_{c+1 mod C}, u_c, d_c]
 * (the horizontal contractions of row r), and the vertical contractions join
 * the rows' down and up indices: Z = trace(T_0 T_1 ... T_{R-1}).  Each T_r is
 * D^C x D^C, built by summing over every (u, d, h).  Requires D^(3C) <= 2^28.
 */
int orc_tc_torus(int R, int C, int64_t D, const double *const *data, double *out) {
  if (R < 1 || C < 1 || D < 1) return -1;
  double cells = pow((double)D, 3.0 * C);
  if (cells > 268435456.0) return -7;
  int64_t n = 1;
  for (int c = 0; c < C; ++c) n *= D;            /* D^C row states */
  int64_t *u = calloc((size_t)C, sizeof(int64_t));
  int64_t *d = calloc((size_t)C, sizeof(int64_t));
  int64_t *h = calloc((size_t)C, sizeof(int64_t));
  int64_t *dimsC = malloc((size_t)C * sizeof(int64_t));
  for (int c = 0; c < C; ++c) dimsC[c] = D;
  double *T = calloc((size_t)(n * n), sizeof(double));
  double *P = calloc((size_t)(n * n), sizeof(double));
  double *Q = calloc((size_t)(n * n), sizeof(double));
  for (int r = 0; r < R; ++r) {
    /* T_r */
    for (int64_t i = 0; i < n * n; ++i) T[i] = 0.0;
    for (int c = 0; c < C; ++c) u[c] = 0;
    do {
      for (int c = 0; c < C; ++c) d[c] = 0;
      do {
        double sum = 0.0;
        for (int c = 0; c < C; ++c) h[c] = 0;
        do {
          double prod = 1.0;
          for (int c = 0; c < C; ++c) {
            const double *X = data[r * C + c];
            int64_t lin = ((h[c] * D + h[(c + 1) % C]) * D + u[c]) * D + d[c];
            prod *= X[lin];
          }
          sum += prod;
        } while (odometer(h, dimsC, C));
        int64_t iu = 0, id = 0;
        for (int c = 0; c < C; ++c) { iu = iu * D + u[c]; id = id * D + d[c]; }
        T[iu * n + id] = sum;
      } while (odometer(d, dimsC, C));
    } while (odometer(u, dimsC, C));
    /* P = P T_r (P = T_0 for r = 0) */
    if (r == 0) {
      for (int64_t i = 0; i < n * n; ++i) P[i] = T[i];
    } else {
      for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
          double acc = 0.0;
          for (int64_t k = 0; k < n; ++k) acc += P[i * n + k] * T[k * n + j];
          Q[i * n + j] = acc;
        }
      for (int64_t i = 0; i < n * n; ++i) P[i] = Q[i];
    }
  }
  double tr = 0.0;
  for (int64_t i = 0; i < n; ++i) tr += P[i * n + i];
  *out = tr;
  free(u); free(d); free(h); free(dimsC); free(T); free(P); free(Q);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Discrete Fourier transform, F[j][b] = exp(-2 pi i j b / m)                 */
/* ------------------------------------------------------------------------- */

/* Plain O(m^2) DFT (the definition). */
void orc_dft(int64_t m, const double *re, const double *im, double *ore, double *oim, int inverse) {
  double sgn = inverse ? 1.0 : -1.0;
  for (int64_t j = 0; j < m; ++j) {
    double sr = 0.0, si = 0.0;
    for (int64_t b = 0; b < m; ++b) {
      double ang = sgn * 2.0 * M_PI * (double)((j * b) % m) / (double)m;
      double c = cos(ang), s = sin(ang);
      sr += re[b] * c - im[b] * s;
      si += re[b] * s + im[b] * c;
    }
    ore[j] = inverse ? sr / (double)m : sr;
    oim[j] = inverse ? si / (double)m : si;
  }
}

/* Iterative radix-2 FFT (Cooley-Tukey, decimation in time), in place.
 * m must be a power of two.  Same convention as orc_dft. */
void orc_fft(int64_t m, double *re, double *im, int inverse) {
  for (int64_t i = 1, j = 0; i < m; ++i) {
    int64_t bit = m >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      double tr = re[i]; re[i] = re[j]; re[j] = tr;
      double ti = im[i]; im[i] = im[j]; im[j] = ti;
    }
  }
  double sgn = inverse ? 1.0 : -1.0;
  for (int64_t len = 2; len <= m; len <<= 1) {
    for (int64_t i = 0; i < m; i += len) {
      for (int64_t k = 0; k < len / 2; ++k) {
        double ang = sgn * 2.0 * M_PI * (double)k / (double)len;
        double wr = cos(ang), wi = sin(ang);
        int64_t a = i + k, b = i + k + len / 2;
        double xr = re[b] * wr - im[b] * wi;
        double xi = re[b] * wi + im[b] * wr;
        re[b] = re[a] - xr; im[b] = im[a] - xi;
        re[a] += xr; im[a] += xi;
      }
    }
  }
  if (inverse) for (int64_t i = 0; i < m; ++i) { re[i] /= (double)m; im[i] /= (double)m; }
}

static int is_pow2(int64_t m) { return m > 0 && (m & (m - 1)) == 0; }

static void dft_any(int64_t m, const double *re, const double *im, double *ore, double *oim, int inverse) {
  if (is_pow2(m)) {
    memcpy(ore, re, (size_t)m * sizeof(double));
    memcpy(oim, im, (size_t)m * sizeof(double));
    orc_fft(m, ore, oim, inverse);
  } else {
    orc_dft(m, re, im, ore, oim, inverse);
  }
}

/* Circular convolution (Def. 8, 0-based): (x*y)_j = sum_i x_i y_{(j - i) mod m}. */
void orc_circ_conv(int64_t m, const double *x, const double *y, double *out) {
  for (int64_t j = 0; j < m; ++j) {
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) s += x[i] * y[((j - i) % m + m) % m];
    out[j] = s;
  }
}

/* ------------------------------------------------------------------------- */
/* Method 1 (cyclic networks): Eq. (1), Algorithm 1                          */
/* ------------------------------------------------------------------------- */

/*
 * Per-mode hash tables of one sample.  tables == NULL: drawn from the hash
 * family above (stream e for edge e).  Otherwise tables holds, per edge e,
 * dims[edge's mode] buckets followed by as many signs, concatenated over
 * edges (the "table mode" used for enumeration and injective pins).
 * Output: for every global mode u, mh[u][i] and ms[u][i] -- the owner gets
 * (h, s), the second mode of the edge the complement ((m - h) mod m, s).
 */
static int m1_mode_tables(const net_t *N, int64_t m, uint64_t seed, uint64_t sample,
                          const int64_t *tables, int64_t **mh, int32_t **ms) {
  const int64_t *tp = tables;
  for (int e = 0; e < N->t; ++e) {
    int u = N->edges[2 * e], v = N->edges[2 * e + 1];
    int64_t n = N->dims[u];
    if (N->dims[v] != n) return -1;
    if (u == v || mh[u] || mh[v]) return -3;   /* a mode in two contractions */
    mh[u] = malloc((size_t)n * sizeof(int64_t)); ms[u] = malloc((size_t)n * sizeof(int32_t));
    mh[v] = malloc((size_t)n * sizeof(int64_t)); ms[v] = malloc((size_t)n * sizeof(int32_t));
    if (tables) {
      for (int64_t i = 0; i < n; ++i) { mh[u][i] = tp[i]; ms[u][i] = (int32_t)tp[n + i]; }
      tp += 2 * n;
    } else {
      orc_count_sketch(seed, sample, (uint64_t)e, n, m, mh[u], ms[u]);
    }
    for (int64_t i = 0; i < n; ++i) {
      mh[v][i] = (m - mh[u][i]) % m;   /* complement count sketch (Def. 14) */
      ms[v][i] = ms[u][i];
    }
  }
  return 0;
}

/* Time-domain tensor sketch of tensor k: y[b] += (prod_u s_u(i_u)) X_k(i) at
 * b = (sum_u h_u(i_u)) mod m  (Def. 12 in the column form of Alg. 3). */
static void m1_sketch_tensor(const net_t *N, int k, int64_t m, int64_t *const *mh,
                             int32_t *const *ms, double *y) {
  int q = N->order[k];
  const int64_t *dims = N->dims + N->off[k];
  int64_t idx[64] = {0};
  for (int64_t b = 0; b < m; ++b) y[b] = 0.0;
  int64_t lin = 0;
  do {
    int64_t b = 0; int sg = 1;
    for (int j = 0; j < q; ++j) {
      int u = N->off[k] + j;
      b += mh[u][idx[j]];
      sg *= ms[u][idx[j]];
    }
    y[b % m] += (double)sg * N->data[k][lin];
    ++lin;
  } while (q > 0 && odometer(idx, dims, q));
}

/*
 * One Method-1 estimate.  combine: 0 = direct circular convolutions (Def. 8),
 * y_1 * ... * y_p evaluated at index 0; 1 = Eq. (1) with the DFT,
 * e_1^T F^{-1}(x_1 o ... o x_p).  sketches (p*m, may be NULL) receives the
 * time-domain sketches y_k.  scale (may be NULL) receives the first-order
 * rounding-error scale (1/m) sum_j sum_k U_k prod_{k' != k} |Y_k'[j]| with
 * U_k = sum_i |X_k(i)| and Y = F y.
 */
int orc_m1_estimate(int p, const int *order, const int64_t *dims, const double *const *data,
                    int t, const int *edges, int64_t m, uint64_t seed, uint64_t sample,
                    const int64_t *tables, int combine, double *est, double *sketches,
                    double *scale) {
  net_t N;
  if (m < 1 || net_init(&N, p, order, dims, data, t, edges)) return -1;
  int64_t **mh = calloc((size_t)N.q, sizeof(int64_t *));
  int32_t **ms = calloc((size_t)N.q, sizeof(int32_t *));
  int rc = m1_mode_tables(&N, m, seed, sample, tables, mh, ms);
  for (int u = 0; u < N.q && rc == 0; ++u) if (!mh[u]) rc = -2;   /* free mode */
  double *y = malloc((size_t)(p * m) * sizeof(double));
  if (rc == 0) {
    for (int k = 0; k < p; ++k) m1_sketch_tensor(&N, k, m, mh, ms, y + (int64_t)k * m);
    if (sketches) memcpy(sketches, y, (size_t)(p * m) * sizeof(double));
    if (combine == 0) {
      double *w = malloc((size_t)m * sizeof(double));
      double *tmp = malloc((size_t)m * sizeof(double));
      memcpy(w, y, (size_t)m * sizeof(double));
      for (int k = 1; k < p; ++k) {
        orc_circ_conv(m, w, y + (int64_t)k * m, tmp);
        memcpy(w, tmp, (size_t)m * sizeof(double));
      }
      *est = w[0];
      free(w); free(tmp);
    }
    if (combine == 1 || scale) {
      double *zr = malloc((size_t)m * sizeof(double)), *zi = malloc((size_t)m * sizeof(double));
      double *Yr = malloc((size_t)(p * m) * sizeof(double)), *Yi = malloc((size_t)(p * m) * sizeof(double));
      double *zero = calloc((size_t)m, sizeof(double));
      for (int k = 0; k < p; ++k) dft_any(m, y + (int64_t)k * m, zero, Yr + (int64_t)k * m, Yi + (int64_t)k * m, 0);
      if (combine == 1) {
        for (int64_t j = 0; j < m; ++j) {
          double ar = 1.0, ai = 0.0;
          for (int k = 0; k < p; ++k) {
            double br = Yr[k * m + j], bi = Yi[k * m + j];
            double nr = ar * br - ai * bi, ni = ar * bi + ai * br;
            ar = nr; ai = ni;
          }
          zr[j] = ar; zi[j] = ai;
        }
        double s = 0.0;
        for (int64_t j = 0; j < m; ++j) s += zr[j];
        *est = s / (double)m;           /* e_1^T F^{-1} z = (1/m) sum_j z_j */
      }
      if (scale) {
        double acc = 0.0;
        for (int k = 0; k < p; ++k) {
          double U = 0.0;
          int64_t sz = tensor_size(&N, k);
          for (int64_t i = 0; i < sz; ++i) U += fabs(data[k][i]);
          for (int64_t j = 0; j < m; ++j) {
            double prod = U;
            for (int kk = 0; kk < p; ++kk)
              if (kk != k) prod *= hypot(Yr[kk * m + j], Yi[kk * m + j]);
            acc += prod;
          }
        }
        *scale = acc / (double)m;
      }
      free(zr); free(zi); free(Yr); free(Yi); free(zero);
    }
  }
  for (int u = 0; u < N.q; ++u) { free(mh[u]); free(ms[u]); }
  free(mh); free(ms); free(y);
  return rc;
}

/*
 * Exact mean and variance of the Method-1 estimator over fully random hash
 * functions, by enumerating every assignment of (h_e, s_e) for every edge
 * (each h_e: [n_e] -> [m], each s_e: [n_e] -> {-1, +1}).  Count must stay small.
 */
int orc_m1_enumerate(int p, const int *order, const int64_t *dims, const double *const *data,
                     int t, const int *edges, int64_t m, double *mean, double *var,
                     int64_t *count) {
  int64_t total = 1, width = 0;
  for (int e = 0; e < t; ++e) {
    int64_t n = dims[edges[2 * e]];
    for (int64_t i = 0; i < n; ++i) { total *= 2 * m; if (total > 50000000) return -1; }
    width += 2 * n;
  }
  int64_t *tables = malloc((size_t)width * sizeof(int64_t));
  double s1 = 0.0, s2 = 0.0;
  for (int64_t a = 0; a < total; ++a) {
    int64_t code = a, pos = 0;
    for (int e = 0; e < t; ++e) {
      int64_t n = dims[edges[2 * e]];
      for (int64_t i = 0; i < n; ++i) {
        tables[pos + i] = code % m; code /= m;
        tables[pos + n + i] = (code % 2) ? -1 : 1; code /= 2;
      }
      pos += 2 * n;
    }
    double est;
    int rc = orc_m1_estimate(p, order, dims, data, t, edges, m, 0, 0, tables, 0, &est, NULL, NULL);
    if (rc) { free(tables); return rc; }
    s1 += est; s2 += est * est;
  }
  *mean = s1 / (double)total;
  *var = s2 / (double)total - (*mean) * (*mean);
  *count = total;
  free(tables);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* The prior cross-correlation method (Examples 2-3 of the Methods section)   */
/* ------------------------------------------------------------------------- */

/* Circular cross-correlation (Def. 9, 0-based, real vectors):
 * (x star y)_j = sum_i x_i y_{(i + j) mod m}. */
void orc_circ_xcorr(int64_t m, const double *x, const double *y, double *out) {
  for (int64_t j = 0; j < m; ++j) {
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) s += x[i] * y[(i + j) % m];
    out[j] = s;
  }
}

/*
 * One estimate of the earlier cross-correlation estimator the Methods section
 * compares against (Examples 2 and 3): contraction e draws one count sketch
 * C_e (stream e of the hash family, or the injected tables as in
 * orc_m1_estimate) that BOTH of its modes use -- no complement -- every tensor
 * is sketched with the tensor sketch of its modes' count sketches, and the
 * sketches are combined by a left-to-right chain of circular
 * cross-correlations in tensor order, y_1 star y_2 star ... star y_p, whose
 * first component is the estimate.  scale (may be NULL): the first-order
 * rounding scale of the Fourier route, (1/m) sum_j sum_k U_k prod_{k' != k}
 * |Y_k'[j]| with Y = F y and U_k = sum_i |X_k(i)| (conjugation does not change
 * a magnitude).
 */
int orc_xcorr_estimate(int p, const int *order, const int64_t *dims, const double *const *data,
                       int t, const int *edges, int64_t m, uint64_t seed, uint64_t sample,
                       const int64_t *tables, double *est, double *sketches, double *scale) {
  net_t N;
  if (m < 1 || net_init(&N, p, order, dims, data, t, edges)) return -1;
  int64_t **mh = calloc((size_t)N.q, sizeof(int64_t *));
  int32_t **ms = calloc((size_t)N.q, sizeof(int32_t *));
  int rc = 0;
  const int64_t *tp = tables;
  for (int e = 0; e < t && rc == 0; ++e) {
    int u = edges[2 * e], v = edges[2 * e + 1];
    int64_t n = dims[u];
    if (dims[v] != n) { rc = -1; break; }
    if (u == v || mh[u] || mh[v]) { rc = -3; break; }
    mh[u] = malloc((size_t)n * sizeof(int64_t)); ms[u] = malloc((size_t)n * sizeof(int32_t));
    mh[v] = malloc((size_t)n * sizeof(int64_t)); ms[v] = malloc((size_t)n * sizeof(int32_t));
    if (tables) {
      for (int64_t i = 0; i < n; ++i) { mh[u][i] = tp[i]; ms[u][i] = (int32_t)tp[n + i]; }
      tp += 2 * n;
    } else {
      orc_count_sketch(seed, sample, (uint64_t)e, n, m, mh[u], ms[u]);
    }
    for (int64_t i = 0; i < n; ++i) { mh[v][i] = mh[u][i]; ms[v][i] = ms[u][i]; }  /* the same C_e */
  }
  for (int u = 0; u < N.q && rc == 0; ++u) if (!mh[u]) rc = -2;   /* free mode */
  double *y = malloc((size_t)(p * m) * sizeof(double));
  if (rc == 0) {
    for (int k = 0; k < p; ++k) m1_sketch_tensor(&N, k, m, mh, ms, y + (int64_t)k * m);
    if (sketches) memcpy(sketches, y, (size_t)(p * m) * sizeof(double));
    double *w = malloc((size_t)m * sizeof(double)), *tmp = malloc((size_t)m * sizeof(double));
    memcpy(w, y, (size_t)m * sizeof(double));
    for (int k = 1; k < p; ++k) {
      orc_circ_xcorr(m, w, y + (int64_t)k * m, tmp);
      memcpy(w, tmp, (size_t)m * sizeof(double));
    }
    *est = w[0];
    free(w); free(tmp);
    if (scale) {
      double *Yr = malloc((size_t)(p * m) * sizeof(double)), *Yi = malloc((size_t)(p * m) * sizeof(double));
      double *zero = calloc((size_t)m, sizeof(double));
      for (int k = 0; k < p; ++k) dft_any(m, y + (int64_t)k * m, zero, Yr + (int64_t)k * m, Yi + (int64_t)k * m, 0);
      double acc = 0.0;
      for (int k = 0; k < p; ++k) {
        double U = 0.0;
        int64_t sz = tensor_size(&N, k);
        for (int64_t i = 0; i < sz; ++i) U += fabs(data[k][i]);
        for (int64_t j = 0; j < m; ++j) {
          double prod = U;
          for (int kk = 0; kk < p; ++kk)
            if (kk != k) prod *= hypot(Yr[kk * m + j], Yi[kk * m + j]);
          acc += prod;
        }
      }
      *scale = acc / (double)m;
      free(Yr); free(Yi); free(zero);
    }
  }
  for (int u = 0; u < N.q; ++u) { free(mh[u]); free(ms[u]); }
  free(mh); free(ms); free(y);
  return rc;
}

/* Exact mean and variance of the cross-correlation estimator over every fully
 * random hash assignment (as orc_m1_enumerate does for Method 1). */
int orc_xcorr_enumerate(int p, const int *order, const int64_t *dims, const double *const *data,
                        int t, const int *edges, int64_t m, double *mean, double *var,
                        int64_t *count) {
  int64_t total = 1, width = 0;
  for (int e = 0; e < t; ++e) {
    int64_t n = dims[edges[2 * e]];
    for (int64_t i = 0; i < n; ++i) { total *= 2 * m; if (total > 50000000) return -1; }
    width += 2 * n;
  }
  int64_t *tables = malloc((size_t)width * sizeof(int64_t));
  double s1 = 0.0, s2 = 0.0;
  for (int64_t a = 0; a < total; ++a) {
    int64_t code = a, pos = 0;
    for (int e = 0; e < t; ++e) {
      int64_t n = dims[edges[2 * e]];
      for (int64_t i = 0; i < n; ++i) {
        tables[pos + i] = code % m; code /= m;
        tables[pos + n + i] = (code % 2) ? -1 : 1; code /= 2;
      }
      pos += 2 * n;
    }
    double est;
    int rc = orc_xcorr_estimate(p, order, dims, data, t, edges, m, 0, 0, tables, &est, NULL, NULL);
    if (rc) { free(tables); return rc; }
    s1 += est; s2 += est * est;
  }
  *mean = s1 / (double)total;
  *var = s2 / (double)total - (*mean) * (*mean);
  *count = total;
  free(tables);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Method 2 (acyclic networks): Eq. (2), Algorithms 2-5                      */
/* ------------------------------------------------------------------------- */

typedef struct {
  const net_t *N;
  int64_t m;
  uint64_t seed, sample;
  int root;
  int *partner;       /* partner[u] = other mode of u's edge */
  int *edge_of;       /* edge index of mode u */
  int *tensor_of;     /* tensor owning mode u */
  int *parent_mode;   /* per tensor: its mode on the parent edge (-1 for the root) */
  int *nchild;        /* per tensor: number of children |Gamma(k)| */
  int **child_mode;   /* per tensor: its own modes leading to children, mode order */
  /* Hash tables, filled per sample. */
  int64_t **eh; int32_t **es;                 /* per edge: [n_e] */
  int64_t ***th; int32_t ***ts;               /* per tensor, per T (level-major), side 0/1: [m] */
  int64_t **ph; int32_t **ps;                 /* per tensor: pad slots, value at index 0 */
  /* Optional injected tables: stream ids, lengths, and [h..., s...] blocks. */
  int nover; const uint64_t *over_ids; const int64_t *over_len; const int64_t *over_tab;
  /* BF16-product variant: every product X(i) * (sigma z[b]) of the SMVP of a
   * tensor with children, and of the root's x_o^T r_o, takes both factors
   * rounded to BF16 (orc_bf16_round); sums stay FP64. */
  int bf16;
} m2_t;

/*
 * Round to the nearest BF16 value (ties to even), through FP32 first: the
 * operand rounding of the acyclic method's BF16-product variant (a double is
 * rounded to the nearest float, that float's low 16 bits to the nearest even
 * upper half).  Not used by the paper's estimators themselves.
 */
double orc_bf16_round(double x) {
  float f = (float)x;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (double)f;   /* inf / nan: unchanged */
  u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

/* Draw one stream's count sketch, or copy it from the injected tables. */
static void m2_stream(const m2_t *M, uint64_t stream, int64_t n, int64_t *h, int32_t *s) {
  const int64_t *tp = M->over_tab;
  for (int i = 0; i < M->nover; ++i) {
    if (M->over_ids[i] == stream) {
      for (int64_t j = 0; j < n; ++j) { h[j] = tp[j]; s[j] = (int32_t)tp[M->over_len[i] + j]; }
      return;
    }
    tp += 2 * M->over_len[i];
  }
  orc_count_sketch(M->seed, M->sample, stream, n, M->m, h, s);
}

static int next_pow2(int c) { int q = 1; while (q < c) q <<= 1; return q; }

/* Orient the tree from the root (breadth first).  Returns 0, or -4 for a cycle,
 * a self-contraction or a disconnected network. */
static int m2_orient(m2_t *M) {
  const net_t *N = M->N;
  int p = N->p, q = N->q;
  M->partner = malloc((size_t)q * sizeof(int));
  M->edge_of = malloc((size_t)q * sizeof(int));
  M->tensor_of = malloc((size_t)q * sizeof(int));
  M->parent_mode = malloc((size_t)p * sizeof(int));
  M->nchild = calloc((size_t)p, sizeof(int));
  M->child_mode = calloc((size_t)p, sizeof(int *));
  for (int u = 0; u < q; ++u) M->partner[u] = -1;
  for (int k = 0; k < p; ++k) for (int u = N->off[k]; u < N->off[k + 1]; ++u) M->tensor_of[u] = k;
  for (int e = 0; e < N->t; ++e) {
    int u = N->edges[2 * e], v = N->edges[2 * e + 1];
    if (M->partner[u] >= 0 || M->partner[v] >= 0) return -3;
    M->partner[u] = v; M->partner[v] = u;
    M->edge_of[u] = e; M->edge_of[v] = e;
    if (M->tensor_of[u] == M->tensor_of[v]) return -4;
  }
  for (int u = 0; u < q; ++u) if (M->partner[u] < 0) return -5;
  if (N->t != p - 1) return -4;
  int *seen = calloc((size_t)p, sizeof(int));
  int *queue = malloc((size_t)p * sizeof(int));
  int head = 0, tail = 0;
  queue[tail++] = M->root; seen[M->root] = 1; M->parent_mode[M->root] = -1;
  while (head < tail) {
    int k = queue[head++];
    M->child_mode[k] = malloc((size_t)(N->order[k] + 1) * sizeof(int));
    for (int u = N->off[k]; u < N->off[k + 1]; ++u) {
      if (u == M->parent_mode[k]) continue;
      int l = M->tensor_of[M->partner[u]];
      if (seen[l]) { free(seen); free(queue); return -4; }
      seen[l] = 1;
      M->parent_mode[l] = M->partner[u];
      M->child_mode[k][M->nchild[k]++] = u;
      queue[tail++] = l;
    }
  }
  int connected = (tail == p);
  free(seen); free(queue);
  return connected ? 0 : -4;
}

static void m2_draw_hashes(m2_t *M) {
  const net_t *N = M->N;
  int64_t m = M->m;
  for (int e = 0; e < N->t; ++e) {
    int64_t n = N->dims[N->edges[2 * e]];
    m2_stream(M, (uint64_t)e, n, M->eh[e], M->es[e]);
  }
  for (int k = 0; k < N->p; ++k) {
    int c = M->nchild[k];
    if (c == 0) continue;
    int qt = next_pow2(c);
    int tix = 0;
    for (int l = qt; l >= 2; l /= 2) {
      for (int j = 0; j < l / 2; ++j, ++tix) {
        for (int d = 0; d < 2; ++d)
          m2_stream(M, orc_stream_tsketch(k, l, j, d), m, M->th[k][2 * tix + d],
                    M->ts[k][2 * tix + d]);
      }
    }
    for (int j = c; j < qt; ++j) {
      int64_t hh; int32_t ss;
      m2_stream(M, orc_stream_pad(k, j), 1, &hh, &ss);
      M->ph[k][j] = hh; M->ps[k][j] = ss;
    }
  }
}

/* Algorithm 3 (0-based): sign and row of a tensor sketch column. */
static void tensor_sketch_hash(const int64_t *b, int qn, int64_t *const *h, int32_t *const *s,
                               int64_t m, int *sig, int64_t *row) {
  int sg = 1; int64_t acc = 0;
  for (int k = 0; k < qn; ++k) { sg *= s[k][b[k]]; acc += h[k][b[k]]; }
  *sig = sg; *row = acc % m;
}

/* Algorithm 4: sign and row of the recursive sketch R_k for the child-mode
 * indices idx[0..c-1] (children in mode order, padded to a power of two with
 * index 0 of the padding sketches). */
static void recursive_sketch_hash(const m2_t *M, int k, const int64_t *idx, int *sig, int64_t *row) {
  int c = M->nchild[k];
  int qt = next_pow2(c);
  int64_t b[64];
  int sg = 1;
  for (int j = 0; j < c; ++j) {
    int e = M->edge_of[M->child_mode[k][j]];
    sg *= M->es[e][idx[j]];
    b[j] = M->eh[e][idx[j]];
  }
  for (int j = c; j < qt; ++j) { sg *= M->ps[k][j]; b[j] = M->ph[k][j]; }
  int tix = 0;
  for (int l = qt; l >= 2; l /= 2) {
    for (int j = 0; j < l / 2; ++j, ++tix) {
      int64_t pair[2] = {b[2 * j], b[2 * j + 1]};
      int64_t *hh[2] = {M->th[k][2 * tix], M->th[k][2 * tix + 1]};
      int32_t *ss[2] = {M->ts[k][2 * tix], M->ts[k][2 * tix + 1]};
      int s2; int64_t r2;
      tensor_sketch_hash(pair, 2, hh, ss, M->m, &s2, &r2);
      sg *= s2;
      b[j] = r2;
    }
  }
  *sig = sg; *row = b[0];
}

/* Count sketch of an m-vector with a [m] -> [m] count sketch. */
static void count_sketch_vec(int64_t m, const int64_t *h, const int32_t *s, const double *x, double *out) {
  for (int64_t b = 0; b < m; ++b) out[b] = 0.0;
  for (int64_t i = 0; i < m; ++i) out[h[i]] += (double)s[i] * x[i];
}

/* Tensor sketch of a Kronecker product (Def. 12): T(a (x) b) = F^{-1}(F C1 a o F C2 b). */
static void tensor_sketch_pair(int64_t m, const int64_t *h1, const int32_t *s1, const int64_t *h2,
                               const int32_t *s2, const double *a, const double *b, double *out) {
  double *ca = malloc((size_t)m * sizeof(double)), *cb = malloc((size_t)m * sizeof(double));
  double *ar = malloc((size_t)m * sizeof(double)), *ai = malloc((size_t)m * sizeof(double));
  double *br = malloc((size_t)m * sizeof(double)), *bi = malloc((size_t)m * sizeof(double));
  double *zero = calloc((size_t)m, sizeof(double));
  count_sketch_vec(m, h1, s1, a, ca);
  count_sketch_vec(m, h2, s2, b, cb);
  dft_any(m, ca, zero, ar, ai, 0);
  dft_any(m, cb, zero, br, bi, 0);
  for (int64_t j = 0; j < m; ++j) {
    double r = ar[j] * br[j] - ai[j] * bi[j], i = ar[j] * bi[j] + ai[j] * br[j];
    ar[j] = r; ai[j] = i;
  }
  dft_any(m, ar, ai, ca, cb, 1);
  memcpy(out, ca, (size_t)m * sizeof(double));
  free(ca); free(cb); free(ar); free(ai); free(br); free(bi); free(zero);
}

/* Q_k applied to the Kronecker product of the child sketches xs[0..c-1]
 * (padding slots contribute C_pad e_1), level by level. */
static void apply_q(const m2_t *M, int k, double **xs, double *out) {
  int64_t m = M->m;
  int c = M->nchild[k], qt = next_pow2(c);
  double **v = malloc((size_t)qt * sizeof(double *));
  for (int j = 0; j < qt; ++j) {
    v[j] = calloc((size_t)m, sizeof(double));
    if (j < c) memcpy(v[j], xs[j], (size_t)m * sizeof(double));
    else v[j][M->ph[k][j]] = (double)M->ps[k][j];
  }
  int tix = 0;
  for (int l = qt; l >= 2; l /= 2) {
    for (int j = 0; j < l / 2; ++j, ++tix) {
      double *r = malloc((size_t)m * sizeof(double));
      tensor_sketch_pair(m, M->th[k][2 * tix], M->ts[k][2 * tix], M->th[k][2 * tix + 1],
                         M->ts[k][2 * tix + 1], v[2 * j], v[2 * j + 1], r);
      free(v[2 * j]); free(v[2 * j + 1]);
      v[j] = r;
    }
  }
  memcpy(out, v[0], (size_t)m * sizeof(double));
  free(v[0]); free(v);
}

/* Algorithm 5 for a non-root tensor k with parent-edge count sketch C:
 * y[h(i_parent)] += X(i) z[b] sigma s(i_parent), (sigma, b) from Algorithm 4 on
 * the child-mode indices.  A leaf (no children) gives the count sketch C X. */
static void smvp(const m2_t *M, int k, const double *z, double *y) {
  const net_t *N = M->N;
  int64_t m = M->m;
  int q = N->order[k];
  const int64_t *dims = N->dims + N->off[k];
  int pm = M->parent_mode[k] - N->off[k];
  int e = M->edge_of[M->parent_mode[k]];
  int c = M->nchild[k];
  int64_t idx[64] = {0}, cidx[64];
  for (int64_t b = 0; b < m; ++b) y[b] = 0.0;
  int64_t lin = 0;
  do {
    int64_t i1 = idx[pm];
    int64_t j = M->eh[e][i1];
    double zb = 1.0; int sg = 1;
    if (c > 0) {
      for (int cc = 0; cc < c; ++cc) cidx[cc] = idx[M->child_mode[k][cc] - N->off[k]];
      int64_t b;
      recursive_sketch_hash(M, k, cidx, &sg, &b);
      zb = z[b];
    }
    if (M->bf16 && c > 0)
      y[j] += orc_bf16_round(N->data[k][lin]) * orc_bf16_round(zb * (double)sg) * (double)M->es[e][i1];
    else
      y[j] += N->data[k][lin] * zb * (double)sg * (double)M->es[e][i1];
    ++lin;
  } while (odometer(idx, dims, q));
}

/* NeighborsSketch(k) of Algorithm 2: returns r_k = Q_k(kron_l x_l) in out. */
static void neighbors_sketch(m2_t *M, int k, double *out, double *trace) {
  int64_t m = M->m;
  int c = M->nchild[k];
  double **xs = malloc((size_t)(c > 0 ? c : 1) * sizeof(double *));
  for (int j = 0; j < c; ++j) {
    int l = M->tensor_of[M->partner[M->child_mode[k][j]]];
    double *rl = NULL;
    if (M->nchild[l] > 0) {
      rl = malloc((size_t)m * sizeof(double));
      neighbors_sketch(M, l, rl, trace);
    }
    xs[j] = malloc((size_t)m * sizeof(double));
    smvp(M, l, rl, xs[j]);
    if (trace) memcpy(trace + (int64_t)l * m, xs[j], (size_t)m * sizeof(double));
    free(rl);
  }
  apply_q(M, k, xs, out);
  for (int j = 0; j < c; ++j) free(xs[j]);
  free(xs);
}

static void m2_free(m2_t *M) {
  const net_t *N = M->N;
  if (M->eh) for (int e = 0; e < N->t; ++e) { free(M->eh[e]); free(M->es[e]); }
  free(M->eh); free(M->es);
  if (M->th) {
    for (int k = 0; k < N->p; ++k) {
      if (!M->th[k]) continue;
      int qt = next_pow2(M->nchild[k]);
      for (int i = 0; i < 2 * (qt - 1); ++i) { free(M->th[k][i]); free(M->ts[k][i]); }
      free(M->th[k]); free(M->ts[k]); free(M->ph[k]); free(M->ps[k]);
    }
  }
  free(M->th); free(M->ts); free(M->ph); free(M->ps);
  if (M->child_mode) for (int k = 0; k < N->p; ++k) free(M->child_mode[k]);
  free(M->partner); free(M->edge_of); free(M->tensor_of); free(M->parent_mode);
  free(M->nchild); free(M->child_mode);
}

/*
 * One Method-2 estimate: y = x_o^T r_o with x_o = R_o vec(X_o) and
 * r_o = NeighborsSketch(o) (Algorithm 2).  trace (p*m doubles, may be NULL)
 * receives x_l for every non-root tensor l and x_o in the root's slot;
 * rtrace (m, may be NULL) receives r_o.  nover > 0 injects hash tables: stream
 * over_ids[i] of length over_len[i] takes [h..., s...] from over_tab (blocks
 * concatenated in order); streams not listed are drawn from the family.
 */
int orc_m2_estimate(int p, const int *order, const int64_t *dims, const double *const *data,
                    int t, const int *edges, int64_t m, uint64_t seed, uint64_t sample,
                    int root, int nover, const uint64_t *over_ids, const int64_t *over_len,
                    const int64_t *over_tab, int bf16, double *est, double *trace, double *rtrace) {
  net_t N;
  if (m < 1 || net_init(&N, p, order, dims, data, t, edges)) return -1;
  if (root < 0 || root >= p) return -1;
  m2_t M;
  memset(&M, 0, sizeof(M));
  M.N = &N; M.m = m; M.seed = seed; M.sample = sample; M.root = root;
  M.nover = nover; M.over_ids = over_ids; M.over_len = over_len; M.over_tab = over_tab;
  M.bf16 = bf16;
  int rc = m2_orient(&M);
  if (rc) { m2_free(&M); return rc; }
  if (N.order[root] == 0) { m2_free(&M); return -1; }
  M.eh = calloc((size_t)t, sizeof(int64_t *)); M.es = calloc((size_t)t, sizeof(int32_t *));
  for (int e = 0; e < t; ++e) {
    int64_t n = dims[edges[2 * e]];
    if (dims[edges[2 * e + 1]] != n) { m2_free(&M); return -1; }
    M.eh[e] = malloc((size_t)n * sizeof(int64_t)); M.es[e] = malloc((size_t)n * sizeof(int32_t));
  }
  M.th = calloc((size_t)p, sizeof(int64_t **)); M.ts = calloc((size_t)p, sizeof(int32_t **));
  M.ph = calloc((size_t)p, sizeof(int64_t *)); M.ps = calloc((size_t)p, sizeof(int32_t *));
  for (int k = 0; k < p; ++k) {
    int c = M.nchild[k];
    if (c == 0) continue;
    if (c > 32) { m2_free(&M); return -1; }
    int qt = next_pow2(c);
    M.th[k] = calloc((size_t)(2 * qt), sizeof(int64_t *));
    M.ts[k] = calloc((size_t)(2 * qt), sizeof(int32_t *));
    for (int i = 0; i < 2 * (qt - 1); ++i) {
      M.th[k][i] = malloc((size_t)m * sizeof(int64_t));
      M.ts[k][i] = malloc((size_t)m * sizeof(int32_t));
    }
    M.ph[k] = calloc((size_t)qt, sizeof(int64_t)); M.ps[k] = calloc((size_t)qt, sizeof(int32_t));
  }
  m2_draw_hashes(&M);
  /* x_o = R_o vec(X_o): scatter every root entry with Algorithm 4 over all its modes. */
  double *xo = calloc((size_t)m, sizeof(double));
  {
    int q = N.order[root];
    const int64_t *rd = N.dims + N.off[root];
    int64_t idx[64] = {0}, cidx[64];
    int64_t lin = 0;
    do {
      for (int cc = 0; cc < M.nchild[root]; ++cc) cidx[cc] = idx[M.child_mode[root][cc] - N.off[root]];
      int sg; int64_t b;
      recursive_sketch_hash(&M, root, cidx, &sg, &b);
      xo[b] += (double)sg * N.data[root][lin];
      ++lin;
    } while (odometer(idx, rd, q));
  }
  double *ro = malloc((size_t)m * sizeof(double));
  neighbors_sketch(&M, root, ro, trace);
  double y = 0.0;
  if (!bf16) {
    for (int64_t b = 0; b < m; ++b) y += xo[b] * ro[b];
  } else {
    /* the same sum, sum_i X_o(i) sigma(i) r_o[b(i)], with both factors of each
     * product rounded to BF16 */
    int q = N.order[root];
    const int64_t *rd = N.dims + N.off[root];
    int64_t idx[64] = {0}, cidx[64];
    int64_t lin = 0;
    do {
      for (int cc = 0; cc < M.nchild[root]; ++cc) cidx[cc] = idx[M.child_mode[root][cc] - N.off[root]];
      int sg; int64_t b;
      recursive_sketch_hash(&M, root, cidx, &sg, &b);
      y += orc_bf16_round(N.data[root][lin]) * orc_bf16_round((double)sg * ro[b]);
      ++lin;
    } while (odometer(idx, rd, q));
  }
  *est = y;
  if (trace) memcpy(trace + (int64_t)root * m, xo, (size_t)m * sizeof(double));
  if (rtrace) memcpy(rtrace, ro, (size_t)m * sizeof(double));
  free(xo); free(ro);
  m2_free(&M);
  return 0;
}

/*
 * Lemma 8: exact acyclic full TNC, vec(X_o)^T g(o) with
 * g(k) = kron_{l in Gamma(k)} mat(X_l) g(l).  mat(X_l) takes the parent mode
 * as rows and the child modes (mode order) as columns (the footnote's
 * permutation), and g(l) is formed explicitly as a Kronecker product.
 */
static double *lemma8_matvec(m2_t *M, int l);

static double *lemma8_g(m2_t *M, int k, int64_t *len) {
  const net_t *N = M->N;
  int c = M->nchild[k];
  double *g = malloc(sizeof(double));
  g[0] = 1.0;
  int64_t glen = 1;
  for (int j = 0; j < c; ++j) {
    int u = M->child_mode[k][j];
    int l = M->tensor_of[M->partner[u]];
    double *v = lemma8_matvec(M, l);
    int64_t n = N->dims[u];
    double *ng = malloc((size_t)(glen * n) * sizeof(double));
    for (int64_t a = 0; a < glen; ++a)
      for (int64_t b = 0; b < n; ++b) ng[a * n + b] = g[a] * v[b];   /* g (x) v */
    free(g); free(v);
    g = ng; glen *= n;
  }
  *len = glen;
  return g;
}

static double *lemma8_matvec(m2_t *M, int l) {
  const net_t *N = M->N;
  int q = N->order[l];
  const int64_t *dims = N->dims + N->off[l];
  int pm = M->parent_mode[l] - N->off[l];
  int64_t glen;
  double *g = lemma8_g(M, l, &glen);
  double *out = calloc((size_t)dims[pm], sizeof(double));
  int64_t idx[64] = {0};
  int64_t lin = 0;
  do {
    int64_t col = 0;
    for (int j = 0; j < M->nchild[l]; ++j) {
      int jm = M->child_mode[l][j] - N->off[l];
      col = col * dims[jm] + idx[jm];
    }
    out[idx[pm]] += N->data[l][lin] * g[col];
    ++lin;
  } while (odometer(idx, dims, q));
  free(g);
  return out;
}

int orc_tc_tree(int p, const int *order, const int64_t *dims, const double *const *data,
                int t, const int *edges, int root, double *out) {
  net_t N;
  if (net_init(&N, p, order, dims, data, t, edges)) return -1;
  m2_t M;
  memset(&M, 0, sizeof(M));
  M.N = &N; M.root = root;
  int rc = m2_orient(&M);
  if (rc) { m2_free(&M); return rc; }
  int64_t glen;
  double *g = lemma8_g(&M, root, &glen);
  /* vec(X_o)^T g(o): the root's modes are all child modes, in mode order. */
  const int64_t *rd = N.dims + N.off[root];
  int64_t idx[64] = {0};
  int64_t lin = 0;
  double acc = 0.0;
  do {
    int64_t col = 0;
    for (int j = 0; j < M.nchild[root]; ++j) {
      int jm = M.child_mode[root][j] - N.off[root];
      col = col * rd[jm] + idx[jm];
    }
    acc += N.data[root][lin] * g[col];
    ++lin;
  } while (odometer(idx, rd, N.order[root]));
  *out = acc;
  free(g);
  m2_free(&M);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Sample statistics                                                         */
/* ------------------------------------------------------------------------- */

/* Welford mean and unbiased sample variance of n values. */
void orc_mean_var(int64_t n, const double *x, double *mean, double *var) {
  double mu = 0.0, m2 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double d = x[i] - mu;
    mu += d / (double)(i + 1);
    m2 += d * (x[i] - mu);
  }
  *mean = mu;
  *var = n > 1 ? m2 / (double)(n - 1) : 0.0;
}
