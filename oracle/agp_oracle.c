/*
 * agp_oracle.c -- TEST INFRASTRUCTURE ONLY (see agp_oracle.h).
 *
 * A deliberately plain implementation of randomized graph propagation
 * (Approximate Graph Propagation, KDD'21, Section 4, Algorithm 2):
 *
 *   pi = sum_{i=0}^{L} w_i (D^-a A D^-b)^i x
 *
 * is estimated level by level through residue vectors r^(i) and reserves
 * q^(i) (Definition 3.2 and the recursion that follows it).  A push from u to
 * a neighbour v carries inc = (Y_{i+1}/Y_i) r(u) / (d_v^a d_u^b); it is added
 * exactly when inc >= theta and otherwise v is sampled with probability
 * inc/theta and receives theta.
 *
 * Readings of points the paper leaves open (each is also listed in the design
 * notes of the repository):
 *  - weights are normalised by S = sum w_k and the result rescaled by S
 *    (Section 3, assumptions on w_i); Y_i = sum_{k=i..L} w_k, so the estimand
 *    is the truncated sum and the last level keeps all of r^(L);
 *  - theta = eps * ||x||_1 per column (Section 3 assumes ||x||_1 = 1; running
 *    unscaled with this absolute threshold is the same as normalise, run at
 *    eps, rescale);
 *  - signed signals are pushed in one pass: decisions use |r|, contributions
 *    carry the sign of r (Section 3 splits x into x+ and x-);
 *  - adjacency lists are sorted by (d_v, v), so every correct sort agrees;
 *  - subset sampling (after Algorithm 2): the sampled suffix of N_u is cut
 *    into runs inside aligned windows of 64 positions.  In a run starting at
 *    position s the scheme draws Bernoulli(p*) per position, p* = p_{v_s}
 *    (the largest in the run), and keeps a drawn position j with probability
 *    p_{v_j}/p*.  The Bernoulli(p*) positions are produced by geometric skips,
 *    which has the same distribution as the paper's Binomial count plus
 *    uniform choice.  With a = 0 a run is the rest of the window.  With
 *    a > 0 a run ends with the degree group floor(log2 d_v) of its first
 *    position (so every kept probability is above 1/2), unless p* times the
 *    positions left in the window is at most ORC_MERGE_CANDIDATES: then the
 *    run takes the rest of the window (at most that many candidates are
 *    expected, fewer draws than one run per group).  Every position is still
 *    kept with probability p_{v_j}, independently;
 *  - randomness: Philox4x32-10 keyed by the 64-bit seed, counter
 *    (t, s, u, (qid << 8) | level), t = draw index in the run;
 *  - the residue of a node at the next level is the exact sum of all
 *    contributions it receives in the level, rounded once to the working
 *    precision (binary32 or binary64).  The paper visits the nodes of a level
 *    in no fixed order; the exact sum is the value every visiting order
 *    agrees on;
 *  - the reserve pi(u) is accumulated level after level in the working
 *    precision: pi(u) <- fl(pi(u) + fl(kappa_i r(u))).
 */
#include "agp_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------ degree sort */

static int cmp_deg_id(const void* pa, const void* pb, void* ctx) {
  const int32_t* fdeg = (const int32_t*)ctx; /* degree table of the comparison */
  int32_t va = *(const int32_t*)pa, vb = *(const int32_t*)pb;
  int32_t da = fdeg[va], db = fdeg[vb];
  if (da != db) return da < db ? -1 : 1;
  if (va != vb) return va < vb ? -1 : 1;
  return 0;
}

/* Row bounds of nthreads contiguous row ranges with about equal numbers of
 * arcs: bounds[t] .. bounds[t+1] for thread t. */
static void split_rows_by_arcs(int64_t n, const int64_t* rp, int nthreads, int64_t* bounds) {
  bounds[0] = 0;
  for (int t = 1; t < nthreads; ++t) { /* first row starting at or after the share's end */
    const int64_t target = rp[n] / nthreads * t;
    int64_t lo = bounds[t - 1], hi = n;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (rp[mid] < target) lo = mid + 1; else hi = mid;
    }
    bounds[t] = lo;
  }
  bounds[nthreads] = n;
}

typedef struct {
  const int64_t* rp;
  int32_t* col;
  const int32_t* fdeg;
  int64_t lo, hi;
} sort_job;

static void* sort_rows(void* arg) {
  sort_job* jb = (sort_job*)arg;
  for (int64_t u = jb->lo; u < jb->hi; ++u)
    qsort_r(jb->col + jb->rp[u], (size_t)(jb->rp[u + 1] - jb->rp[u]), sizeof(int32_t), cmp_deg_id,
            (void*)jb->fdeg);
  return NULL;
}

/* Pre-sorting adjacency lists by degree (Section 4): N_u ascending in the
 * degree of the neighbour that enters the factors d^-a, d^-b.  Undirected
 * graphs: that degree is the row length (at least 1).  Directed graphs pass
 * the out-degrees (Section 4, propagation on directed graphs).  Each row is
 * sorted on its own, so the rows are shared among nthreads threads. */
int orc_degree_sort(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* fdeg_in,
                    int32_t* out_col, int32_t* deg, int32_t* fdeg, int32_t nthreads) {
  if (n < 0 || nthreads < 1) return -1;
  for (int64_t u = 0; u < n; ++u) {
    deg[u] = (int32_t)(rp[u + 1] - rp[u]);
    const int32_t f = fdeg_in ? fdeg_in[u] : deg[u];
    fdeg[u] = f < 1 ? 1 : f;
  }
  memcpy(out_col, col, (size_t)rp[n] * sizeof(int32_t));
  if (n < 4096) nthreads = 1;
  pthread_t* th = malloc(sizeof(pthread_t) * (size_t)nthreads);
  sort_job* jobs = malloc(sizeof(sort_job) * (size_t)nthreads);
  int64_t* bounds = malloc(sizeof(int64_t) * ((size_t)nthreads + 1));
  split_rows_by_arcs(n, rp, nthreads, bounds);
  for (int t = 0; t < nthreads; ++t) {
    jobs[t].rp = rp;
    jobs[t].col = out_col;
    jobs[t].fdeg = fdeg;
    jobs[t].lo = bounds[t];
    jobs[t].hi = bounds[t + 1];
    pthread_create(&th[t], NULL, sort_rows, &jobs[t]);
  }
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th);
  free(jobs);
  free(bounds);
  return 0;
}

/* ------------------------------------------------------- weights, theta */

/* Partial sums Y_i = sum_{k>=i} w_k (Definition 3.2), with w_k = 0 for k > L,
 * added from k = L downwards; rho_i = Y_{i+1}/Y_i (recursion for r^(i+1));
 * kappa_i = (S * w_i) / Y_i (reserve q^(i) = (w_i/Y_i) r^(i), rescaled by S).
 *
 * tail != 0: the paper-literal infinite tail.  The weights are the first
 * terms of a sequence whose infinite sum is 1 (Section 3, assumptions on
 * w_i), so the terms beyond L hold T = 1 - (w_0 + ... + w_L) (the sum taken
 * from k = 0 upwards, T floored at 0) and Y_i = T + sum_{k=i..L} w_k, added
 * from k = L downwards onto Y_{L+1} = T; S = Y_0 (1 up to rounding), kappa
 * as above, rho_i = Y_{i+1}/Y_i for i < L and rho_L = 0: the last level keeps
 * (w_L / Y_L) r^(L) and drops the rest (Algorithm 2, final step).  Needs
 * w_0 + ... + w_L <= 1 + 1e-9.  With T = 0 the tables equal the default ones. */
int orc_level_tables(const double* w, int32_t L, int32_t tail, double* S, double* Y,
                     double* rho, double* kappa) {
  if (L < 0) return -1;
  double T = 0.0;
  if (tail) {
    double total = 0.0;
    for (int32_t k = 0; k <= L; ++k) total += w[k];
    if (!(total <= 1.0 + 1e-9)) return -1;
    T = total < 1.0 ? 1.0 - total : 0.0;
  }
  Y[L + 1] = T;
  for (int32_t k = L; k >= 0; --k) Y[k] = Y[k + 1] + w[k];
  *S = Y[0];
  for (int32_t i = 0; i <= L; ++i) {
    rho[i] = (Y[i] == 0.0 || i == L) ? 0.0 : Y[i + 1] / Y[i];
    kappa[i] = (Y[i] == 0.0) ? 0.0 : ((*S) * w[i]) / Y[i];
  }
  return 0;
}

/* ||x||_1 summed in binary64: sequentially inside blocks of 4096 consecutive
 * rows, then sequentially over the block sums; theta = eps * ||x||_1. */
double orc_theta(const double* x, int64_t n, double eps) {
  double total = 0.0;
  for (int64_t lo = 0; lo < n; lo += 4096) {
    double part = 0.0;
    int64_t hi = lo + 4096 < n ? lo + 4096 : n;
    for (int64_t i = lo; i < hi; ++i) part += fabs(x[i]);
    total += part;
  }
  return eps * total;
}

/* ------------------------------------------------------------ randomness */

/* Philox4x32 with 10 rounds: each round multiplies counter words 0 and 2 by
 * the two published multipliers, swaps and xors with the key, and the key is
 * bumped by the two Weyl constants between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* 53-bit uniform in [0, 1) from two 32-bit words. */
static double uniform53(uint32_t hi, uint32_t lo) {
  uint64_t bits = ((uint64_t)hi << 21) | (uint64_t)(lo >> 11);
  return (double)bits * (1.0 / 9007199254740992.0);
}

/* Number K of failures before the next success of Bernoulli(p) trials:
 * the largest K with 1 - (1-p)^K <= V.  With s_h = 1 - (1-p)^(2^h)
 * (s_0 = p, s_{h+1} = s_h * (2 - s_h)) the value 1-(1-p)^K is built by
 * binary lifting: sigma' = (sigma + s_h) - sigma * s_h.  K stays below 128,
 * which is more than any run of 64 positions needs. */
int32_t orc_skip(double p, double V) {
  double s[7];
  s[0] = p;
  for (int h = 0; h < 6; ++h) {
    double t = 2.0 - s[h];
    s[h + 1] = s[h] * t;
  }
  double sigma = 0.0;
  int32_t K = 0;
  for (int h = 6; h >= 0; --h) {
    double sum = sigma + s[h];
    double prod = sigma * s[h];
    double cand = sum - prod;
    if (cand <= V) {
      sigma = cand;
      K += (int32_t)1 << h;
    }
  }
  return K;
}

uint64_t orc_splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* ------------------------------------------------- exact accumulation */

/* A binary32 value is an integer multiple of 2^-149 below 2^128 and a
 * binary64 value a multiple of 2^-1074 below 2^1024.  Sums are kept as
 * two's-complement integers in those units, wide enough for 2^32 terms. */
#define W32 5
#define W64 34

typedef struct exact_acc {
  int words;
  int unit_exp;
  int prec;
} exact_fmt;

static exact_fmt fmt_for(int wp) {
  exact_fmt f;
  if (wp == 32) {
    f.words = W32;
    f.unit_exp = -149;
    f.prec = 24;
  } else {
    f.words = W64;
    f.unit_exp = -1074;
    f.prec = 53;
  }
  return f;
}

/* acc += v exactly (v must be a finite value of the working format). */
static void exact_add(uint64_t* acc, const exact_fmt* f, double v) {
  if (v == 0.0) return;
  int e;
  double fr = frexp(fabs(v), &e); /* |v| = fr * 2^e, fr in [0.5, 1) */
  uint64_t m = (uint64_t)ldexp(fr, 53);
  int pos = e - 53 - f->unit_exp;
  while (pos < 0) {
    if (m & 1u) abort(); /* not on the grid of the working format */
    m >>= 1;
    ++pos;
  }
  int wi = pos / 64, sh = pos % 64;
  uint64_t part[2];
  part[0] = m << sh;
  part[1] = sh ? (m >> (64 - sh)) : 0;
  if (v > 0) {
    uint64_t carry = 0;
    for (int k = wi; k < f->words; ++k) {
      uint64_t add = (k == wi) ? part[0] : (k == wi + 1) ? part[1] : 0;
      uint64_t s1 = acc[k] + add;
      uint64_t c1 = s1 < add;
      uint64_t s2 = s1 + carry;
      uint64_t c2 = s2 < carry;
      acc[k] = s2;
      carry = c1 | c2;
      if (k > wi && carry == 0) break;
    }
  } else {
    uint64_t borrow = 0;
    for (int k = wi; k < f->words; ++k) {
      uint64_t sub = (k == wi) ? part[0] : (k == wi + 1) ? part[1] : 0;
      uint64_t b1 = acc[k] < sub;
      uint64_t d1 = acc[k] - sub;
      uint64_t b2 = d1 < borrow;
      uint64_t d2 = d1 - borrow;
      acc[k] = d2;
      borrow = b1 | b2;
      if (k > wi && borrow == 0) break;
    }
  }
}

static int bit_of(const uint64_t* t, int k) { return (int)((t[k / 64] >> (k % 64)) & 1u); }

/* Round the integer in acc (units 2^unit_exp) to the working format,
 * round-to-nearest-even; a zero sum gives +0. */
static double exact_round(const uint64_t* acc, const exact_fmt* f) {
  uint64_t t[W64];
  int W = f->words;
  memcpy(t, acc, (size_t)W * sizeof(uint64_t));
  int neg = (int)(t[W - 1] >> 63);
  if (neg) { /* two's complement negate */
    uint64_t carry = 1;
    for (int k = 0; k < W; ++k) {
      t[k] = ~t[k] + carry;
      carry = (carry && t[k] == 0) ? 1 : 0;
    }
  }
  int nb = 0;
  for (int k = W - 1; k >= 0; --k) {
    if (t[k]) {
      nb = 64 * k + (64 - __builtin_clzll(t[k]));
      break;
    }
  }
  if (nb == 0) return 0.0;
  double r;
  if (nb <= f->prec) {
    uint64_t q = 0;
    for (int k = nb - 1; k >= 0; --k) q = (q << 1) | (uint64_t)bit_of(t, k);
    r = ldexp((double)q, f->unit_exp);
  } else {
    int shift = nb - f->prec;
    uint64_t q = 0;
    for (int k = nb - 1; k >= shift; --k) q = (q << 1) | (uint64_t)bit_of(t, k);
    int round_bit = bit_of(t, shift - 1);
    int sticky = 0;
    for (int k = shift - 2; k >= 0 && !sticky; --k) sticky = bit_of(t, k);
    if (round_bit && (sticky || (q & 1u))) {
      ++q;
      if (q == ((uint64_t)1 << f->prec)) {
        q >>= 1;
        ++shift;
      }
    }
    r = ldexp((double)q, f->unit_exp + shift);
  }
  if (f->prec == 24) r = (double)(float)r; /* exact, or +inf past FLT_MAX */
  return neg ? -r : r;
}

double orc_exact_sum(const double* vals, int64_t k, int32_t wp) {
  exact_fmt f = fmt_for(wp);
  uint64_t acc[W64];
  memset(acc, 0, sizeof(acc));
  for (int64_t i = 0; i < k; ++i) exact_add(acc, &f, vals[i]);
  return exact_round(acc, &f);
}

/* --------------------------------------------------------- propagation */

/* Round to the working precision. */
static double fl_w(double v, int wp) { return wp == 32 ? (double)(float)v : v; }

/* d^-e for d >= 1: exact forms 1, 1/sqrt(d), 1/d for e = 0, 1/2, 1. */
static double deg_pow(int32_t d, double e) {
  if (d <= 0) return 0.0;
  if (e == 0.0) return 1.0;
  if (e == 0.5) return 1.0 / sqrt((double)d);
  if (e == 1.0) return 1.0 / (double)d;
  return pow((double)d, -e);
}

static int group_of(int32_t d) { return 31 - __builtin_clz((unsigned)d); }

int orc_propagate(int64_t n, const int64_t* rp, const int32_t* col_sorted,
                  const int32_t* deg, double a, double b, const double* w,
                  int32_t L, int32_t tail, const double* x, double eps, uint64_t seed,
                  uint32_t qid, int32_t wp, double* out, orc_counters* cnt) {
  return orc_propagate_levels(n, rp, col_sorted, deg, a, b, w, L, tail, x, eps, seed, qid, wp, out, cnt, -1, 1);
}

int orc_propagate_levels(int64_t n, const int64_t* rp, const int32_t* col_sorted, const int32_t* deg, double a,
                         double b, const double* w, int32_t L, int32_t tail, const double* x, double eps,
                         uint64_t seed, uint32_t qid, int32_t wp, double* out, orc_counters* cnt, int32_t stop,
                         int32_t stride) {
  if (n < 0 || L < 0 || L > 255 || !(a >= 0.0 && a <= 1.0) || !(b >= 0.0 && b <= 1.0) ||
      !(eps >= 0.0) || (wp != 32 && wp != 64) || stride < 1)
    return -1;
  for (int32_t k = 0; k <= L; ++k)
    if (!(w[k] >= 0.0) || isinf(w[k])) return -1;

  int32_t maxdeg = 0;
  for (int64_t u = 0; u < n; ++u)
    if (deg[u] > maxdeg) maxdeg = deg[u];
  double* da = malloc(sizeof(double) * ((size_t)maxdeg + 1));
  double* db = malloc(sizeof(double) * ((size_t)maxdeg + 1));
  for (int32_t d = 0; d <= maxdeg; ++d) {
    da[d] = deg_pow(d, a);
    db[d] = deg_pow(d, b);
  }
  double S;
  double* Y = malloc(sizeof(double) * ((size_t)L + 2));
  double* rho = malloc(sizeof(double) * ((size_t)L + 1));
  double* kappa = malloc(sizeof(double) * ((size_t)L + 1));
  if (orc_level_tables(w, L, tail, &S, Y, &rho[0], &kappa[0])) {
    free(da);
    free(db);
    free(Y);
    free(rho);
    free(kappa);
    return -1;
  }

  const double theta = orc_theta(x, n, eps);
  const double theta_w = fl_w(theta, wp);
  exact_fmt f = fmt_for(wp);
  double* r = malloc(sizeof(double) * (size_t)(n ? n : 1));
  uint64_t* acc = calloc((size_t)(n ? n : 1) * (size_t)f.words, sizeof(uint64_t));
  unsigned char* touched = calloc((size_t)(n ? n : 1), 1);
  int64_t* touched_list = malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  const int64_t seg = (int64_t)1 << ORC_SEG_LOG2;

  for (int64_t u = 0; u < n; ++u) {
    r[u] = x[u]; /* r^(0) = x */
    out[u] = 0.0;
  }

  for (int32_t i = 0; i <= L; ++i) {
    uint64_t nf = 0, hs = 0, ndet = 0, ncand = 0, nacc = 0, nruns = 0;
    int64_t ntouched = 0;
    for (int64_t u = 0; u < n; ++u) { /* each u with non-zero residue */
      double ru = r[u];
      if (ru == 0.0) continue;
      if (i == stop && stride > 1 && u % stride != 0) continue; /* timing sample: every stride-th node */
      ++nf;
      hs += orc_splitmix64((uint64_t)u);
      /* reserve: pi(u) += (w_i / Y_i) r(u), rescaled by S */
      out[u] = fl_w(out[u] + fl_w(kappa[i] * ru, wp), wp);
      const int64_t du = rp[u + 1] - rp[u]; /* neighbours to push to */
      if (i == L || rho[i] == 0.0 || du == 0) continue;
      const double sgn = ru < 0.0 ? -1.0 : 1.0;
      const double c = (rho[i] * fabs(ru)) * db[deg[u]];
      const int32_t* nb = col_sorted + rp[u];
      /* deterministic pushes to the prefix whose increment reaches theta */
      int64_t j = 0;
      while (j < du) {
        int32_t v = nb[j];
        double inc = c * da[deg[v]];
        if (!(inc >= theta)) break;
        if (!touched[v]) {
          touched[v] = 1;
          touched_list[ntouched++] = v;
        }
        exact_add(acc + (size_t)v * f.words, &f, fl_w(sgn * inc, wp));
        ++j;
      }
      ndet += (uint64_t)j;
      /* subset sampling over the rest, run by run */
      int64_t s = j;
      while (s < du) {
        int64_t e = s + 1;
        while (e < du && (e % seg) != 0 &&
               (a == 0.0 || group_of(deg[nb[e]]) == group_of(deg[nb[s]])))
          ++e;
        ++nruns;
        const double dstart = da[deg[nb[s]]];
        const double pstar = (c * dstart) / theta;
        if (a != 0.0) { /* few expected candidates: the run takes the rest of its window */
          int64_t wend = (s / seg + 1) * seg;
          if (wend > du) wend = du;
          if (pstar * (double)(wend - s) <= ORC_MERGE_CANDIDATES) e = wend;
        }
        int64_t pos = s;
        uint32_t t = 0;
        for (;;) {
          uint32_t ctr[4] = {t, (uint32_t)s, (uint32_t)u, (qid << 8) | (uint32_t)i};
          uint32_t o[4];
          orc_philox4x32_10(ctr, key, o);
          double V = uniform53(o[0], o[1]);
          double V2 = uniform53(o[2], o[3]);
          int64_t cnd = pos + orc_skip(pstar, V);
          if (cnd >= e) break;
          ++ncand;
          int32_t v = nb[cnd];
          double ratio = da[deg[v]] / dstart;
          if (V2 < ratio) {
            ++nacc;
            if (!touched[v]) {
              touched[v] = 1;
              touched_list[ntouched++] = v;
            }
            exact_add(acc + (size_t)v * f.words, &f, fl_w(sgn * theta_w, wp));
          }
          pos = cnd + 1;
          ++t;
        }
        s = e;
      }
    }
    if (cnt) {
      cnt->frontier[i] = nf;
      cnt->hash[i] = hs;
      if (i < L) {
        cnt->det[i] = ndet;
        cnt->cand[i] = ncand;
        cnt->acc[i] = nacc;
        cnt->runs[i] = nruns;
      }
    }
    if (getenv("ORC_PROGRESS")) { /* long runs: one line per level on stderr */
      fprintf(stderr, "[oracle] qid %u level %d: frontier %lld, pushes %llu\n", (unsigned)qid, (int)i,
              (long long)nf, (unsigned long long)(ndet + nacc));
      fflush(stderr);
    }
    if (i == L || i == stop) break;
    /* empty level i; r^(i+1) is the rounded exact sum of what arrived */
    for (int64_t u = 0; u < n; ++u) r[u] = 0.0;
    for (int64_t k = 0; k < ntouched; ++k) {
      int64_t v = touched_list[k];
      r[v] = exact_round(acc + (size_t)v * f.words, &f);
      memset(acc + (size_t)v * f.words, 0, sizeof(uint64_t) * (size_t)f.words);
      touched[v] = 0;
    }
  }
  free(da);
  free(db);
  free(Y);
  free(rho);
  free(kappa);
  free(r);
  free(acc);
  free(touched);
  free(touched_list);
  return 0;
}

/* ------------------------------------------------ many columns, threads */

typedef struct many_job {
  int64_t n;
  const int64_t* rp;
  const int32_t* col;
  const int32_t* deg;
  double a, b;
  const double* w;
  int32_t L;
  int32_t tail;
  const double* x;
  int32_t C;
  double eps;
  uint64_t seed;
  const uint32_t* qids;
  int32_t wp;
  double* out;
  uint64_t* counters;
  int32_t stop;
  int32_t stride;
  int next;
  int status;
  pthread_mutex_t lock;
} many_job;

static void* many_worker(void* arg) {
  many_job* jb = (many_job*)arg;
  const size_t L1 = (size_t)jb->L + 1;
  for (;;) {
    pthread_mutex_lock(&jb->lock);
    int c = jb->next++;
    pthread_mutex_unlock(&jb->lock);
    if (c >= jb->C) break;
    orc_counters cn, *pc = NULL;
    if (jb->counters) {
      uint64_t* base = jb->counters + (size_t)c * ORC_NUM_COUNTERS * L1;
      cn.frontier = base;
      cn.hash = base + L1;
      cn.det = base + 2 * L1;
      cn.cand = base + 3 * L1;
      cn.acc = base + 4 * L1;
      cn.runs = base + 5 * L1;
      memset(base, 0, sizeof(uint64_t) * ORC_NUM_COUNTERS * L1);
      pc = &cn;
    }
    uint32_t qid = jb->qids ? jb->qids[c] : (uint32_t)c;
    int rc = orc_propagate_levels(jb->n, jb->rp, jb->col, jb->deg, jb->a, jb->b, jb->w, jb->L, jb->tail,
                                  jb->x + (size_t)c * (size_t)jb->n, jb->eps, jb->seed, qid, jb->wp,
                                  jb->out + (size_t)c * (size_t)jb->n, pc, jb->stop, jb->stride);
    if (rc) {
      pthread_mutex_lock(&jb->lock);
      jb->status = rc;
      pthread_mutex_unlock(&jb->lock);
    }
  }
  return NULL;
}

int orc_propagate_many(int64_t n, const int64_t* rp, const int32_t* col_sorted,
                       const int32_t* deg, double a, double b, const double* w,
                       int32_t L, int32_t tail, const double* x, int32_t C, double eps,
                       uint64_t seed, const uint32_t* qids, int32_t wp,
                       double* out, uint64_t* counters, int32_t nthreads, int32_t stop, int32_t stride) {
  if (C < 0 || nthreads < 1) return -1;
  many_job jb = {n, rp, col_sorted, deg, a, b, w, L, tail, x, C, eps, seed, qids, wp, out, counters, stop, stride,
                 0, 0};
  pthread_mutex_init(&jb.lock, NULL);
  if (nthreads > C) nthreads = C > 0 ? C : 1;
  pthread_t* th = malloc(sizeof(pthread_t) * (size_t)nthreads);
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, many_worker, &jb);
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(th);
  pthread_mutex_destroy(&jb.lock);
  return jb.status;
}

/* ------------------------------------------------------ clustering sweep */
/* Local clustering sweep (Section 5, the quality of local clusters): nodes
 * sorted by pi(v) / d_v descending, ties by id, nodes without neighbours
 * last; then the prefix S_i = {v_1..v_i}, 1 <= i <= n - 1, of minimum
 * conductance Phi(S) = |cut(S)| / min(vol(S), 2m - vol(S)) (the first such
 * prefix; Phi undefined, and skipped, where the denominator is 0).  cut(S)
 * counts the arcs (u, v), u in S, v outside S, of the symmetric CSR (a loop
 * is never cut); vol(S) sums the row lengths; 2m = rp[n]. */

typedef struct {
  const double* ratio;
  const int64_t* rp;
} sweep_key;

static int cmp_sweep(const void* pa, const void* pb, void* ctx) {
  const sweep_key* k = (const sweep_key*)ctx;
  const int32_t va = *(const int32_t*)pa, vb = *(const int32_t*)pb;
  const int isoa = k->rp[va + 1] == k->rp[va], isob = k->rp[vb + 1] == k->rp[vb];
  if (isoa != isob) return isoa < isob ? -1 : 1;
  const double ra = k->ratio[va], rb = k->ratio[vb];
  if (ra != rb) return ra > rb ? -1 : 1;
  return va < vb ? -1 : (va > vb ? 1 : 0);
}

int orc_sweep(int64_t n, const int64_t* rp, const int32_t* col, const double* pi, int32_t* order,
              int64_t* best_size, double* best_phi) {
  if (n < 0) return -1;
  double* ratio = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  unsigned char* in_s = calloc((size_t)(n > 0 ? n : 1), 1);
  for (int64_t v = 0; v < n; ++v) {
    const int64_t d = rp[v + 1] - rp[v];
    double r = d > 0 ? pi[v] / (double)d : 0.0;
    if (r == 0.0) r = 0.0; /* one zero */
    ratio[v] = r;
    order[v] = (int32_t)v;
  }
  sweep_key key = {ratio, rp};
  qsort_r(order, (size_t)n, sizeof(int32_t), cmp_sweep, &key);
  const int64_t two_m = rp[n];
  int64_t cut = 0, vol = 0;
  *best_size = 0;
  *best_phi = INFINITY;
  for (int64_t i = 0; i + 1 < n; ++i) { /* S_{i+1} = S_i + v */
    const int32_t v = order[i];
    int64_t loops = 0, inside = 0;
    for (int64_t j = rp[v]; j < rp[v + 1]; ++j) {
      if (col[j] == v)
        ++loops;
      else if (in_s[col[j]])
        ++inside;
    }
    const int64_t d = rp[v + 1] - rp[v];
    cut += (d - loops) - 2 * inside; /* v's arcs leave S, except those to S */
    vol += d;
    in_s[v] = 1;
    const int64_t denom = vol < two_m - vol ? vol : two_m - vol;
    if (denom > 0) {
      const double phi = (double)cut / (double)denom;
      if (phi < *best_phi) {
        *best_phi = phi;
        *best_size = i + 1;
      }
    }
  }
  free(ratio);
  free(in_s);
  return 0;
}

/* ---------------------------------------------------------- exact sum */
/* The quantity the method estimates, Eq. 1 truncated at L:
 * pi = sum_{i=0..L} w_i P^i x with P = D^-a A D^-b, in binary64 by Horner's
 * rule: acc = w_L x, then acc = w_i x + P acc for i = L-1 .. 0.  Row v of
 * (rp, col) lists the u with A[v][u] = 1, so (P y)(v) = d_v^-a sum_u d_u^-b y(u),
 * summed in row order.  x and out are n x C row-major.  Rows are shared
 * among nthreads threads; each entry is computed by one thread alone. */

typedef struct {
  int64_t lo, hi;
  const int64_t* rp;
  const int32_t* col;
  const double *fa, *fb;
  const double* x;
  const double* src;
  double* scaled;
  double* dst;
  double wi;
  int32_t C;
  int32_t phase;
} horner_job;

static void* horner_rows(void* arg) {
  const horner_job* jb = (const horner_job*)arg;
  const int32_t C = jb->C;
  if (jb->phase == 0) { /* scaled = D^-b src */
    for (int64_t u = jb->lo; u < jb->hi; ++u)
      for (int32_t c = 0; c < C; ++c) jb->scaled[(size_t)u * C + c] = jb->fb[u] * jb->src[(size_t)u * C + c];
    return NULL;
  }
  double sum[64];
  for (int64_t v = jb->lo; v < jb->hi; ++v) { /* dst = w_i x + D^-a A scaled */
    for (int32_t c = 0; c < C; ++c) sum[c] = 0.0;
    for (int64_t k = jb->rp[v]; k < jb->rp[v + 1]; ++k) {
      const double* y = jb->scaled + (size_t)jb->col[k] * C;
      for (int32_t c = 0; c < C; ++c) sum[c] += y[c];
    }
    for (int32_t c = 0; c < C; ++c)
      jb->dst[(size_t)v * C + c] = jb->wi * jb->x[(size_t)v * C + c] + jb->fa[v] * sum[c];
  }
  return NULL;
}

int orc_exact_sum_horner(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* fdeg, double a, double b,
                         const double* w, int32_t L, const double* x, int32_t C, double* out, int32_t nthreads,
                         int32_t verbose) {
  if (n < 0 || L < 0 || C < 1 || C > 64 || nthreads < 1) return -1;
  const size_t cells = (size_t)(n ? n : 1) * (size_t)C;
  double* fa = malloc(sizeof(double) * (size_t)(n ? n : 1));
  double* fb = malloc(sizeof(double) * (size_t)(n ? n : 1));
  double* tmp = malloc(sizeof(double) * cells);
  double* scaled = malloc(sizeof(double) * cells);
  for (int64_t v = 0; v < n; ++v) {
    int32_t d = fdeg ? fdeg[v] : (int32_t)(rp[v + 1] - rp[v]);
    if (d < 1) d = 1; /* a node without arcs: its factors never meet a non-zero sum */
    fa[v] = deg_pow(d, a);
    fb[v] = deg_pow(d, b);
  }
  /* acc = w_L x, kept in out; each step writes tmp and swaps */
  for (size_t k = 0; k < (size_t)n * (size_t)C; ++k) out[k] = w[L] * x[k];
  double *cur = out, *nxt = tmp;
  if (n < 4096) nthreads = 1;
  pthread_t* th = malloc(sizeof(pthread_t) * (size_t)nthreads);
  horner_job* jobs = malloc(sizeof(horner_job) * (size_t)nthreads);
  int64_t* bounds = malloc(sizeof(int64_t) * ((size_t)nthreads + 1));
  split_rows_by_arcs(n, rp, nthreads, bounds);
  for (int32_t i = L - 1; i >= 0; --i) {
    for (int32_t phase = 0; phase < 2; ++phase) {
      for (int t = 0; t < nthreads; ++t) {
        horner_job jb = {bounds[t], bounds[t + 1], rp, col, fa, fb, x, cur, scaled, nxt, w[i], C, phase};
        jobs[t] = jb;
        pthread_create(&th[t], NULL, horner_rows, &jobs[t]);
      }
      for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    }
    double* sw = cur;
    cur = nxt;
    nxt = sw;
    if (verbose) {
      fprintf(stderr, "[oracle] truncated sum: term %d of %d added\n", (int)(L - i), (int)L);
      fflush(stderr);
    }
  }
  if (cur != out) memcpy(out, cur, sizeof(double) * (size_t)n * (size_t)C);
  free(th);
  free(jobs);
  free(fa);
  free(fb);
  free(tmp);
  free(scaled);
  free(bounds);
  return 0;
}
