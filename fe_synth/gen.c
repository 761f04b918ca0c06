/*
 * Seeded synthetic inputs: graph edge streams and dense blocks.
 *
 * This module generates inputs only.  It holds none of the eigensolver's
 * arithmetic (no CSR construction, no products, no orthogonalisation); both
 * the GPU library and the CPU oracle consume what it writes.
 *
 * Every random value is a pure function of (seed, counter), drawn from the
 * Philox4x32-10 counter-based generator as published by Salmon, Moraes, Dror
 * and Shaw ("Parallel random numbers: as easy as 1, 2, 3", SC 2011): ten
 * rounds of two 32x32->64 multiplies (constants 0xD2511F53, 0xCD9E8D57) with a
 * Weyl key schedule (0x9E3779B9, 0xBB67AE85).  Because edge k depends only on
 * (seed, k), the stream can be produced in parallel and at any size.
 *
 * Graph families (none is defined by the paper, which measures on real
 * graphs that are not available; these stand in for them):
 *   - R-MAT (Chakrabarti, Zhan, Faloutsos 2004): each edge descends `scale`
 *     levels, choosing a quadrant with probabilities (a, b, c, 1-a-b-c).
 *   - Chung-Lu: vertex weights Pareto with density ~ w^-alpha (x_m = 1),
 *     rescaled to a target mean; endpoints drawn with P(i) ~ w_i.
 *   - Stochastic block model with equal blocks and an in-block fraction rho.
 * The generators emit raw directed samples (duplicates and self-loops
 * included); symmetrising and deduplicating is the consumer's job.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TAG_RMAT 0x524d4154u /* "RMAT" */
#define TAG_PERM 0x5045524du /* "PERM" */
#define TAG_CLW 0x434c5755u  /* "CLWU" */
#define TAG_CLE 0x434c4555u  /* "CLEU" */
#define TAG_SBM 0x53424d55u  /* "SBMU" */
#define TAG_NORM 0x4e4f524du /* "NORM" */
#define TAG_INT 0x494e5455u  /* "INTU" */

static inline void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                 uint32_t k0, uint32_t k1, uint32_t out[4]) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Exposed for the known-answer test. */
void synth_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  philox4x32_10(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1], out);
}

/* 53-bit uniform in [0,1) from two words. */
static inline double u53(uint32_t hi, uint32_t lo) {
  return ((double)(hi >> 5) * 67108864.0 + (double)(lo >> 6)) * (1.0 / 9007199254740992.0);
}

/* Uniform integer in [0, bound) from a 64-bit draw (bias below 2^-37 for bound < 2^27). */
static inline uint64_t below(uint32_t hi, uint32_t lo, uint64_t bound) {
  unsigned __int128 x = ((unsigned __int128)(((uint64_t)hi << 32) | lo)) * bound;
  return (uint64_t)(x >> 64);
}

/* Random permutation of [0, n) by Fisher-Yates; draw i uses counter (i, 0, 0, PERM). */
void synth_permutation(int64_t n, uint64_t seed, int32_t *perm) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    uint32_t w[4];
    philox4x32_10((uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0, TAG_PERM, k0, k1, w);
    int64_t j = (int64_t)below(w[0], w[1], (uint64_t)i + 1);
    int32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
}

/* R-MAT: n = 2^scale vertices, m edges.  perm (optional) relabels both ends. */
void synth_rmat(int32_t scale, int64_t m, double a, double b, double c, uint64_t seed,
                const int32_t *perm, int32_t *src, int32_t *dst) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint32_t u = 0, v = 0, w[4];
    for (int l = 0; l < scale; ++l) {
      if ((l & 3) == 0)
        philox4x32_10((uint32_t)e, (uint32_t)((uint64_t)e >> 32), (uint32_t)(l >> 2), TAG_RMAT,
                      k0, k1, w);
      double x = (double)w[l & 3] * (1.0 / 4294967296.0);
      uint32_t bu, bv;
      if (x < a) { bu = 0; bv = 0; }
      else if (x < ab) { bu = 0; bv = 1; }
      else if (x < abc) { bu = 1; bv = 0; }
      else { bu = 1; bv = 1; }
      u |= bu << (scale - 1 - l);
      v |= bv << (scale - 1 - l);
    }
    src[e] = perm ? perm[u] : (int32_t)u;
    dst[e] = perm ? perm[v] : (int32_t)v;
  }
}

/* Chung-Lu weights: w_i = (1-U_i)^(-1/(alpha-1)), then scaled so mean(w) = mean_deg. */
void synth_chung_lu_weights(int64_t n, double alpha, double mean_deg, uint64_t seed, double *w) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    uint32_t r[4];
    philox4x32_10((uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0, TAG_CLW, k0, k1, r);
    double U = u53(r[0], r[1]);
    w[i] = pow(1.0 - U, -1.0 / (alpha - 1.0));
    s += w[i];
  }
  double f = mean_deg * (double)n / s;
  for (int64_t i = 0; i < n; ++i) w[i] *= f;
}

/* Chung-Lu endpoints: 2m draws with P(i) = w_i / sum(w), edge e = (draw 2e, draw 2e+1). */
void synth_chung_lu(int64_t n, int64_t m, const double *w, uint64_t seed, int32_t *src,
                    int32_t *dst) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  double *cdf = (double *)malloc(sizeof(double) * (size_t)n);
  double acc = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    acc += w[i];
    cdf[i] = acc;
  }
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint32_t r[4];
    philox4x32_10((uint32_t)e, (uint32_t)((uint64_t)e >> 32), 0, TAG_CLE, k0, k1, r);
    for (int end = 0; end < 2; ++end) {
      double t = u53(r[2 * end], r[2 * end + 1]) * acc;
      int64_t lo = 0, hi = n - 1; /* first i with cdf[i] > t */
      while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cdf[mid] > t) hi = mid;
        else lo = mid + 1;
      }
      if (end == 0) src[e] = (int32_t)lo;
      else dst[e] = (int32_t)lo;
    }
  }
  free(cdf);
}

/* SBM: kb equal blocks (block of v = v*kb/n); with probability rho both ends in one
   uniformly chosen block, otherwise in two distinct uniformly chosen blocks. */
void synth_sbm(int64_t n, int32_t kb, double rho, int64_t m, uint64_t seed, int32_t *src,
               int32_t *dst) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    uint32_t r[4], q[4];
    philox4x32_10((uint32_t)e, (uint32_t)((uint64_t)e >> 32), 0, TAG_SBM, k0, k1, r);
    philox4x32_10((uint32_t)e, (uint32_t)((uint64_t)e >> 32), 1, TAG_SBM, k0, k1, q);
    int64_t B1 = (int64_t)below(r[1], r[2], (uint64_t)kb), B2;
    if ((double)r[0] * (1.0 / 4294967296.0) < rho || kb == 1) {
      B2 = B1;
    } else {
      B2 = (int64_t)below(r[3], r[1] ^ r[2], (uint64_t)(kb - 1));
      if (B2 >= B1) ++B2;
    }
    int64_t s1 = B1 * n / kb, e1 = (B1 + 1) * n / kb;
    int64_t s2 = B2 * n / kb, e2 = (B2 + 1) * n / kb;
    src[e] = (int32_t)(s1 + (int64_t)below(q[0], q[1], (uint64_t)(e1 - s1)));
    dst[e] = (int32_t)(s2 + (int64_t)below(q[2], q[3], (uint64_t)(e2 - s2)));
  }
}

/* N(0,1) by Box-Muller: values 2p, 2p+1 come from counter (p, stream, NORM). */
void synth_normal(int64_t count, uint64_t seed, uint32_t stream, double *out) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < (count + 1) / 2; ++p) {
    uint32_t r[4];
    philox4x32_10((uint32_t)p, (uint32_t)((uint64_t)p >> 32), stream, TAG_NORM, k0, k1, r);
    double u1 = 1.0 - u53(r[0], r[1]); /* (0, 1] */
    double u2 = u53(r[2], r[3]);
    double rad = sqrt(-2.0 * log(u1));
    out[2 * p] = rad * cos(two_pi * u2);
    if (2 * p + 1 < count) out[2 * p + 1] = rad * sin(two_pi * u2);
  }
}

/* Integers uniform in [lo, hi], for inputs whose sums are exact in every dtype. */
void synth_small_int(int64_t count, uint64_t seed, uint32_t stream, int32_t lo, int32_t hi,
                     double *out) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i) {
    uint32_t r[4];
    philox4x32_10((uint32_t)i, (uint32_t)((uint64_t)i >> 32), stream, TAG_INT, k0, k1, r);
    out[i] = (double)(lo + (int64_t)below(r[0], r[1], (uint64_t)(hi - lo + 1)));
  }
}
