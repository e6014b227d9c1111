/*
 * agp_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain sequential CPU reference for randomized graph propagation
 * (Wang, He, Wei, Wang, Yuan, Du, Wen: "Approximate Graph Propagation",
 * KDD'21; Algorithm 2 of Section 4 with the degree-sorted adjacency lists and
 * the degree-group subset sampling described after it).  Only the tests, the
 * package smoke check and the benchmark's CPU-baseline leg may load it; the
 * product library never links or calls it, and it shares no code with the
 * HIP path.
 *
 * Every floating point decision is taken in IEEE binary64 in the operation
 * order written in the comments of agp_oracle.c; this file must be compiled
 * with -ffp-contract=off so that no multiply-add is fused.
 */
#ifndef AGP_ORACLE_H
#define AGP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Subset sampling splits every sampled suffix at multiples of 2^6 positions. */
#define ORC_SEG_LOG2 6
/* A sampling run (a > 0) whose expected candidates over the rest of its
 * window are at most this many takes the rest of the window. */
#define ORC_MERGE_CANDIDATES 4.0

/* Per-level counters of one propagation (one column). Arrays have L + 1
 * entries; det/cand/acc/runs use entries 0..L-1, frontier/hash use 0..L. */
#define ORC_NUM_COUNTERS 6
typedef struct orc_counters {
  uint64_t* frontier; /* |{u : r^(i)(u) != 0}|                        */
  uint64_t* hash;     /* sum of splitmix64(u) over that set, mod 2^64 */
  uint64_t* det;      /* deterministic pushes                         */
  uint64_t* cand;     /* sampled candidates                           */
  uint64_t* acc;      /* accepted sampled pushes                      */
  uint64_t* runs;     /* sampling runs (each starts one skip chain)   */
} orc_counters;

/* Sort every adjacency list ascending by (factor degree of neighbour, id).
 * rp/col: CSR of the push direction; fdeg_in: factor degrees (out-degrees
 * of a directed graph) or NULL for the row lengths.  out_col gets the sorted
 * lists, deg the row lengths, fdeg the factor degrees clamped to >= 1.
 * The rows are sorted by nthreads host threads. */
int orc_degree_sort(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* fdeg_in,
                    int32_t* out_col, int32_t* deg, int32_t* fdeg, int32_t nthreads);

/* S, Y_0..Y_{L+1}, rho_0..rho_L, kappa_0..kappa_L from w_0..w_L; tail != 0
 * takes the paper-literal infinite tail Y_i = 1 - sum_{k<i} w_k (returns -1
 * when w_0 + ... + w_L > 1 + 1e-9). */
int orc_level_tables(const double* w, int32_t L, int32_t tail, double* S, double* Y,
                     double* rho, double* kappa);

/* theta = eps * ||x||_1 with the fixed blocked summation order. */
double orc_theta(const double* x, int64_t n, double eps);

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Geometric skip for success probability p from the uniform V. */
int32_t orc_skip(double p, double V);

/* splitmix64 finaliser of x. */
uint64_t orc_splitmix64(uint64_t x);

/* Exact sum of vals[0..k) rounded once to binary32 (wp = 32) or binary64. */
double orc_exact_sum(const double* vals, int64_t k, int32_t wp);

/* One column of Algorithm 2 (tail as in orc_level_tables). x and out hold n values; with wp = 32 every x
 * must be a binary32 value; deg holds the factor degrees (fdeg of
 * orc_degree_sort), the rows come from rp.  Returns 0, or -1 on invalid
 * arguments. */
int orc_propagate(int64_t n, const int64_t* rp, const int32_t* col_sorted,
                  const int32_t* deg, double a, double b, const double* w,
                  int32_t L, int32_t tail, const double* x, double eps, uint64_t seed,
                  uint32_t qid, int32_t wp, double* out, orc_counters* cnt);

/* orc_propagate that stops after level `stop` (stop < 0: never): out then
 * holds the reserves of levels 0..stop only.  At level `stop` only the nodes
 * u with u % stride == 0 are visited.  Both serve bounded timing samples;
 * stop = -1, stride = 1 is orc_propagate. */
int orc_propagate_levels(int64_t n, const int64_t* rp, const int32_t* col_sorted, const int32_t* deg, double a,
                         double b, const double* w, int32_t L, int32_t tail, const double* x, double eps,
                         uint64_t seed, uint32_t qid, int32_t wp, double* out, orc_counters* cnt, int32_t stop,
                         int32_t stride);

/* Columns c = 0..C-1 of column-major x/out (x + c*n), spread over nthreads
 * host threads; qids may be NULL (qid = c).  counters, if not NULL, is a
 * C x 6 x (L+1) uint64 array (frontier, hash, det, cand, acc, runs per
 * column).  stop and stride as in orc_propagate_levels. */
int orc_propagate_many(int64_t n, const int64_t* rp, const int32_t* col_sorted,
                       const int32_t* deg, double a, double b, const double* w,
                       int32_t L, int32_t tail, const double* x, int32_t C, double eps,
                       uint64_t seed, const uint32_t* qids, int32_t wp,
                       double* out, uint64_t* counters, int32_t nthreads, int32_t stop, int32_t stride);

/* Local clustering sweep of pi (Section 5): order gets the nodes sorted by
 * pi(v)/d_v descending (ties by id, isolated nodes last); best_size is the
 * first prefix size i in [1, n-1] of minimum conductance, best_phi that
 * conductance (best_size 0 and +inf when no prefix has one). */
int orc_sweep(int64_t n, const int64_t* rp, const int32_t* col, const double* pi, int32_t* order,
              int64_t* best_size, double* best_phi);

/* Eq. 1 truncated at L in binary64 by Horner's rule, without sampling or
 * thresholds: out = sum_{i=0..L} w_i (D^-a A D^-b)^i x.  Row v of (rp, col)
 * lists the u with A[v][u] = 1 (the rows that push into v); fdeg: the
 * degrees in the factors, or NULL for the row lengths.  x and out are n x C
 * row-major, 1 <= C <= 64; nthreads host threads share the rows; verbose:
 * a line on stderr after each term (long runs). */
int orc_exact_sum_horner(int64_t n, const int64_t* rp, const int32_t* col, const int32_t* fdeg, double a, double b,
                         const double* w, int32_t L, const double* x, int32_t C, double* out, int32_t nthreads,
                         int32_t verbose);

#ifdef __cplusplus
}
#endif
#endif
