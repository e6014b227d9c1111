/*
 * agp.h -- C ABI of the MI355X (gfx950) randomized graph propagation library.
 *
 * The library estimates, for an undirected graph G with adjacency matrix A and
 * degree matrix D, the graph propagation vector of Eq. (1) of "Approximate
 * Graph Propagation" (Wang et al., KDD'21):
 *
 *     pi = sum_{i=0}^{L} w_i (D^-a A D^-b)^i x,      a, b in [0, 1],
 *
 * with the randomized level-by-level residue push of Algorithm 2 (Section 4):
 * at level i a node u with residue r(u) pushes inc = (Y_{i+1}/Y_i) r(u) /
 * (d_v^a d_u^b) to each neighbour v whose increment reaches the threshold, and
 * samples the remaining neighbours with probability inc/theta, adding theta to
 * each sampled one.  Adjacency lists are kept sorted by neighbour degree
 * (Section 4, pre-sorting) so the exact part is a prefix and the sampled part
 * is visited in degree groups (Section 4, subset sampling).
 *
 * Conventions shared by every entry point:
 *  - Return value: AGP_OK (0) or a positive AGP_E* code; agp_last_error()
 *    returns a thread-local message for the last failure.  No C++ exception
 *    crosses this boundary.
 *  - "device" pointers are HIP device allocations on the current device;
 *    "host" pointers are ordinary host memory.  The library never frees
 *    caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued on it; calls documented as synchronous wait for it.
 *  - Results depend only on (graph, a, b, w, L, x, eps, seed, column query
 *    id), never on launch shapes, tile sizes, batch composition or timing.
 */
#ifndef AGP_H
#define AGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define AGP_OK 0
#define AGP_EINVAL 1   /* invalid argument (sizes, ranges, NaN, asymmetric graph) */
#define AGP_ENOMEM 2   /* device or host allocation failed                       */
#define AGP_EDEVICE 3  /* a HIP runtime call failed                              */
#define AGP_ERANGE 4   /* a residue left the range of the exact accumulators     */
#define AGP_ENOTSUP 5  /* valid but unsupported request                          */
#define AGP_PENDING 6  /* agp_poll: the query has not finished                   */
#define AGP_ENOENT 7   /* agp_poll: unknown ticket                               */
#define AGP_EBUSY 8    /* agp_submit: the submission queue is full               */

/* ---------------------------------------------------- graph creation flags */
#define AGP_HOST_PTRS 1u      /* row_ptr / col_idx are host pointers (else device)   */
#define AGP_VALIDATE 2u       /* also check: no duplicate arcs, symmetric matrix          */
#define AGP_ADD_SELF_LOOPS 4u /* give every node exactly one self-loop (GNN convention) */
#define AGP_DIRECTED 8u       /* row u lists the out-neighbours of u in a directed graph;
                                 pushes follow out-edges (A~ = A^T) */
#define AGP_REVERSE 16u       /* with AGP_DIRECTED: pushes follow in-edges (A~ = A) */

/* Largest supported number of levels L (the level index is 8 bits of the
 * random stream counter). */
#define AGP_MAX_LEVELS 255

typedef struct agp_graph agp_graph_t;

/* Per-call counters (Theorem 3.3 counts one unit of cost per edge push).
 * Entries are summed over all columns of the call; index = level.
 *  frontier[i]  number of (node, column) pairs with non-zero residue at level i
 *  hash[i]      sum over those pairs of splitmix64(node), mod 2^64
 *  det[i]       deterministic pushes made at level i           (i < L)
 *  cand[i]      sampled candidate positions drawn at level i    (i < L)
 *  acc[i]       accepted sampled pushes at level i              (i < L)
 *  runs[i]      sampling runs at level i (a run is a range of one degree
 *               group inside a 64-position window of a sampled suffix; each
 *               starts one geometric-skip chain, so the random draws of the
 *               level number runs[i] + cand[i])                  (i < L)
 * An edge push is det + acc. */
typedef struct agp_stats {
  int32_t levels;  /* L of the call */
  int32_t columns; /* C of the call */
  int32_t tiles;   /* column tiles run one after another: each level launches
                      its level kernel once per tile */
  int32_t dense;   /* 1: node-major dense levels; 0: (node, column) frontier lists */
  uint64_t frontier[AGP_MAX_LEVELS + 1];
  uint64_t hash[AGP_MAX_LEVELS + 1];
  uint64_t det[AGP_MAX_LEVELS + 1];
  uint64_t cand[AGP_MAX_LEVELS + 1];
  uint64_t acc[AGP_MAX_LEVELS + 1];
  uint64_t runs[AGP_MAX_LEVELS + 1];
  double device_ms; /* from the first level kernel's start to the last one's end */
  /* HIP-event time of the level kernel launched for level i and of the
   * launches that make its deferred pushes (ms) */
  double level_ms[AGP_MAX_LEVELS + 1];
  /* HIP-event time of everything level i enqueues (ms): the push estimate,
   * the level kernels, the aggregation of its pushes and the formation of
   * the next frontier */
  double level_total_ms[AGP_MAX_LEVELS + 1];
} agp_stats_t;

/* Thread-local description of the last error raised on this thread. */
const char* agp_last_error(void);

/* ------------------------------------------------------------------ graphs */

/* Build the library's graph from a CSR matrix (Section 2: G = (V, E)
 * undirected; Section 4: adjacency lists pre-sorted by degree; Section 4,
 * propagation on directed graphs).
 *  n        number of nodes, 0 <= n < 2^31
 *  nnz      number of stored arcs, row_ptr[n]; an undirected edge is stored
 *           in both rows
 *  row_ptr  int64[n + 1], non-decreasing, row_ptr[0] = 0
 *  col_idx  int32[nnz], neighbour ids in [0, n)
 *  flags    AGP_HOST_PTRS | AGP_VALIDATE | AGP_ADD_SELF_LOOPS |
 *           AGP_DIRECTED | AGP_REVERSE
 *  stream   stream for the build; the call is synchronous on it
 *  out      receives the graph handle
 * Undirected (default): the matrix must be symmetric; d = row length.
 * AGP_DIRECTED: row u holds the out-neighbours of u; propagation computes
 * sum_i w_i (D^-a A^T D^-b)^i x (PPR, HKPR, Katz on directed graphs), i.e.
 * pushes follow out-edges; D holds the out-degrees.  With AGP_REVERSE the
 * pushes follow in-edges, sum_i w_i (D^-a A D^-b)^i x (single-target
 * proximity); the library transposes the matrix itself.  A node without
 * out-arcs counts as out-degree 1 in D.
 * The library copies the arrays; the caller may free them on return.  Inside
 * the handle every row (in the push direction) is sorted ascending by
 * (degree of neighbour in D, id).  The handle holds 12 bytes of device
 * memory per arc (neighbour id, its degree in D, the end of its degree group
 * within the row) and 16 per node, plus the working memory of later calls.
 * Errors: AGP_EINVAL for bad sizes, ids out of range, unknown flags,
 * AGP_REVERSE without AGP_DIRECTED, or (with AGP_VALIDATE) duplicate arcs or
 * (undirected only) an asymmetric matrix; AGP_ENOMEM; AGP_EDEVICE.
 * Self-loops already in the input are kept (a loop is an ordinary
 * neighbour). */
int agp_graph_create(int64_t n, int64_t nnz, const int64_t* row_ptr,
                     const int32_t* col_idx, uint32_t flags, void* stream,
                     agp_graph_t** out);

/* Sizes of a graph (any pointer may be NULL); max_degree is the longest row
 * in the push direction. */
int agp_graph_info(const agp_graph_t* g, int64_t* n, int64_t* nnz, int32_t* max_degree);

/* Copy the library's CSR to host buffers (any may be NULL):
 * row_ptr int64[n+1], col_sorted int32[nnz] (rows in the push direction,
 * sorted by (degree of neighbour in D, id)), degree int32[n] (row lengths).
 * Synchronous. */
int agp_graph_export(const agp_graph_t* g, int64_t* row_ptr, int32_t* col_sorted,
                     int32_t* degree);

/* Degree group of every stored arc (Section 4, subset sampling: the groups
 * G_k of neighbours with floor(log2 d_v) = k): host uint8[nnz], in the order
 * of agp_graph_export's col_sorted, floor(log2) of the neighbour's degree in
 * D (so non-decreasing along each row).  Synchronous (default stream). */
int agp_graph_groups(const agp_graph_t* g, uint8_t* group_ids);

/* Release a graph and every buffer the library cached for it. */
int agp_graph_destroy(agp_graph_t* g);

/* ------------------------------------------------------------- propagation */

/* Randomized propagation of C signal columns at once (Algorithm 2).
 *  g       graph handle
 *  a, b    exponents of D^-a A D^-b, each in [0, 1]
 *  w       host double[L + 1], w_i >= 0 and finite
 *  L       number of levels, 0 <= L <= AGP_MAX_LEVELS
 *  x       device float[n * C], row-major (x[u * C + c]); finite values
 *  C       number of columns, C >= 1
 *  eps     error parameter, eps > 0.  Column c uses the absolute threshold
 *          theta_c = eps * ||x[:, c]||_1 (Section 3 assumes ||x||_1 = 1)
 *  seed    64-bit key of the random streams
 *  qids    host uint32[C] query id per column, or NULL for qid = column
 *          index; each column's random decisions depend on (seed, qid) only,
 *          qid < 2^24
 *  out     device float[n * C], row-major, written with pi_hat (overwritten)
 *  stream  work is enqueued on this stream; the call waits for it before
 *          returning so that errors can be reported
 *  stats   optional host counters (NULL to skip)
 * Weights are normalised by S = sum w_i and the result rescaled by S
 * (Section 3).  Signed signals are pushed in one pass (decisions on |r|,
 * contributions carry the sign of r).  Each next-level residue is the exact
 * sum of what a node receives in the level, rounded once to binary32.
 * Working memory is kept with the graph for later calls: the column tiles'
 * accumulators, frontier lists and record buffers (within 85% of the free
 * memory), 16 bytes per node of per-call factors and, for a > 0 and when it
 * fits beside them, 8 bytes per arc (reused while a and b stay the same).
 * Errors: AGP_EINVAL (bad sizes/ranges, non-finite x), AGP_ERANGE (a
 * residue outgrew the exact accumulators: contributions larger than about
 * 2^39 theta), AGP_ENOMEM, AGP_EDEVICE.  On AGP_EINVAL nothing is written; on
 * AGP_ERANGE the contents of out are unspecified. */
int agp_propagate(const agp_graph_t* g, double a, double b, const double* w, int32_t L,
                  const float* x, int32_t C, double eps, uint64_t seed,
                  const uint32_t* qids, float* out, void* stream, agp_stats_t* stats);

/* The same in binary64 working precision (x and out are device double[n*C]);
 * each next-level residue is the exact sum rounded once to binary64. */
int agp_propagate_f64(const agp_graph_t* g, double a, double b, const double* w, int32_t L,
                      const double* x, int32_t C, double eps, uint64_t seed,
                      const uint32_t* qids, double* out, void* stream, agp_stats_t* stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * agp_propagate (binary32, same arguments, no stats) that allocates nothing.
 * Its buffers live in one fixed array of AGP_NOALLOC_SCRATCH_BYTES in the
 * library's static device memory, one copy per device, held until the
 * process ends; they take 32 bytes per cell, so n * C is limited to about
 * 2 million cells (AGP_EINVAL beyond, with the sizes in the message).  The
 * degree-power tables of (a, b) must already exist on g: any earlier
 * agp_propagate (or agp_autotune) on g with the same exponents makes them
 * (AGP_EINVAL otherwise).  It runs frontier lists with atomic aggregation
 * in one tile, and its result equals agp_propagate's bit for bit.  Every
 * call on a device shares that device's array, which keeps the last call's
 * contents (each call clears what must start at zero): calls that overlapped
 * on one GPU would race, so the library runs them one at a time per device
 * (each returns only after its work on `stream` has finished).  Errors as
 * agp_propagate. */
#define AGP_NOALLOC_SCRATCH_BYTES (64u << 20)
int agp_propagate_noalloc(const agp_graph_t* g, double a, double b, const double* w, int32_t L,
                          const float* x, int32_t C, double eps, uint64_t seed, const uint32_t* qids,
                          float* out, void* stream);

/* Paper-literal variants of the propagation (agp_propagate_variant). */
#define AGP_VARIANT_INFINITE_TAIL 1u /* Y_i over the infinite weight sequence */
#define AGP_VARIANT_SPLIT_SIGNS 2u   /* x+ and x- propagated separately     */

/* agp_propagate with the paper-literal readings that the default replaces
 * (same arguments and errors, plus `variant`, a set of AGP_VARIANT_* flags;
 * 0 gives exactly agp_propagate):
 *  AGP_VARIANT_INFINITE_TAIL  the weights are the first L + 1 terms of a
 *     sequence whose infinite sum is 1 (Section 3, assumptions on w_i):
 *     Y_i = T + sum_{k=i..L} w_k with T = 1 - (w_0 + ... + w_L) the mass
 *     beyond level L (Definition 3.2), and the last level keeps only
 *     (w_L / Y_L) r^(L) (Algorithm 2, final step); no rescaling.  Needs
 *     w_0 + ... + w_L <= 1 (AGP_EINVAL otherwise).  Residues are larger than
 *     with the default truncated Y_i, so the same eps costs more pushes.
 *  AGP_VARIANT_SPLIT_SIGNS  signed signals as in Section 3 (assumption on
 *     the graph signal): x = x+ + x-, each part propagated as its own signal
 *     with its own threshold eps * ||x+-[:, c]||_1; column c's x+ part draws
 *     from the random stream of query id qid_c, its x- part from that of
 *     qid_c + 2^23 (so qids must be < 2^23); out = pi+ + pi-, rounded once.
 *     Temporary device memory of 4 n C elements (in column tiles that fit a
 *     quarter of the free memory) is allocated for the call.
 * Counters in stats add up both passes of the split. */
int agp_propagate_variant(const agp_graph_t* g, double a, double b, const double* w, int32_t L,
                          const float* x, int32_t C, double eps, uint64_t seed,
                          const uint32_t* qids, uint32_t variant, float* out, void* stream,
                          agp_stats_t* stats);

/* The same in binary64 (x and out are device double[n*C]). */
int agp_propagate_variant_f64(const agp_graph_t* g, double a, double b, const double* w, int32_t L,
                              const double* x, int32_t C, double eps, uint64_t seed,
                              const uint32_t* qids, uint32_t variant, double* out, void* stream,
                              agp_stats_t* stats);

/* ------------------------------------------------------------------ tuning */

/* Execution choices of agp_propagate that never change its results. */
typedef struct agp_tuning {
  int32_t aggregation;  /* 0: integer atomics into the accumulators;
                           1: push records binned by destination, summed in LDS;
                           2: records on dense levels, atomics on sparse ones  */
  int32_t level_blocks; /* workgroups of the level kernel (>= 256)               */
  int32_t dense;        /* node-major levels with one lane per column (binary32):
                           0 never (default), 1 always, 2 when at least a
                           quarter of the signal's entries are non-zero and
                           C >= 16                                             */
  int32_t tile_columns; /* columns per tile; 0: the widest tile that fits       */
  int32_t big_row;      /* deterministic pushes from which an entry's row is
                           deferred to a grid-wide kernel; 0: 4096              */
  int32_t big_items;    /* sampled work items (16 windows each) from which an
                           entry's sampled suffix is deferred; 0: 64            */
  int32_t sparse_shift; /* a level whose frontier holds fewer than n C / 2^k
                           entries appends first contributions directly; 0: 5 */
  int32_t bin_shift;    /* (aggregation 2) a level whose estimated pushes reach
                           n C / 2^k is binned; 0: 3                            */
  int32_t capture;      /* 1: the level loop of each column tile (frontier
                           lists) is captured once into a hipGraph per graph,
                           column count, level count, buffers and modes, and
                           replayed by later calls (per-level times are then
                           not recorded); 0: launched kernel by kernel        */
} agp_tuning_t;

/* Autotuner: runs the propagation of the arguments (as agp_propagate) once
 * with the defaults (untimed), then once per candidate, timing each with HIP
 * events on `stream`: a coordinate descent over dense (0, 1), aggregation
 * (0, 1, 2), level_blocks (1024 .. 8192), tile_columns (all, C/2, C/4) and,
 * unless the dense levels won, big_row, big_items, sparse_shift and
 * bin_shift.  The fastest choice is kept for later agp_propagate calls on g
 * with the same column count and exponents (a, b).  `out` holds the result
 * on return (identical for every candidate).  *best (nullable) receives the
 * choice.  Errors as agp_propagate. */
int agp_autotune(const agp_graph_t* g, double a, double b, const double* w, int32_t L,
                 const float* x, int32_t C, double eps, uint64_t seed, const uint32_t* qids,
                 float* out, void* stream, agp_tuning_t* best);

/* The choice agp_propagate uses for (g, C, a, b): the tuned or set one,
 * else the default (aggregation 2, 4096 workgroups (8192 when n C >= 2^31),
 * dense 0, the other fields at their stated defaults), with the environment
 * overrides below applied. */
int agp_get_tuning(const agp_graph_t* g, int32_t C, double a, double b, agp_tuning_t* out);

/* Pin the choice for later calls on g with C columns and exponents (a, b),
 * replacing an autotuned one (zero fields take their defaults, out-of-range
 * ones are clamped); t == NULL forgets it.  Results never depend on it. */
int agp_set_tuning(const agp_graph_t* g, int32_t C, double a, double b, const agp_tuning_t* t);

/* Environment overrides read by every propagation call (for tuning and
 * tests; none of them changes a result):
 *   AGP_AGGREGATION=atomic|binned|auto   the aggregation of agp_tuning_t;
 *   AGP_DENSE=0|1|auto   the dense field of agp_tuning_t;
 *   AGP_CAPTURE=0|1      the capture field of agp_tuning_t;
 *   AGP_RECORD_CAP=n     at most n push records per binned level (per record
 *                        group on dense levels, split between the two groups
 *                        of frontier-list levels; records beyond it are added
 *                        with atomics);
 *   AGP_RECORD_GROUPS=2  frontier-list levels keep their records in two
 *                        column groups even when n C < 2^31 (they always do
 *                        from n C >= 2^31 on: record cells are 31-bit);
 *   AGP_COLUMN_TILE=n    at most n columns per tile of a call;
 *   AGP_BIG_ROWS=n       at most n entries per level in each list of deferred
 *                        work (0: every entry keeps its pushes in its wave);
 *   AGP_BIG_ITEMS=n      the big_items field;
 *   AGP_FACTOR_VECTORS=0 batched calls read the degree factors through the
 *                        per-exponent tables instead of the per-call node and
 *                        arc factor vectors (and allocate neither);
 *   AGP_DENSE_GROUP_SHIFT=k  dense levels: records grouped by 2^k columns;
 *   AGP_CHECK_ZERO=1     dense levels: after each tile, check on the host
 *                        that the scratch sums and residues are all-zero
 *                        again (AGP_EDEVICE otherwise; slow). */

/* ----------------------------------------------------------------- serving */

/* A proximity query: x = e_source (||x||_1 = 1, so theta = eps), or, with
 * x_nnz > 0, the sparse signal x = sum_k x_val[k] e_{x_idx[k]} (theta = eps
 * ||x||_1, summed as agp_propagate sums a column).  PPR, heat kernel
 * PageRank, Katz and L-hop transition probability are the models of Table 1
 * with x = e_s; a sparse x gives, e.g., a personalised vector over a seed
 * set.  The result equals agp_propagate of the dense x with the same seed
 * and qid = query_id.  Sparse entries must be distinct ids in [0, n), finite,
 * with at least one non-zero, and every non-zero must be a multiple of the
 * column's unit ulp(fl32(theta)) (true for every entry of magnitude at least
 * theta); zeros are ignored.  The arrays are copied by agp_submit. */
typedef struct agp_query {
  int64_t source;    /* node id, 0 <= source < n                                */
  double a, b;       /* exponents in [0, 1]                                     */
  int32_t L;         /* levels, 0 <= L <= AGP_MAX_LEVELS                        */
  const double* w;   /* host double[L + 1], finite, >= 0; copied by agp_submit  */
  double eps;        /* error parameter; 2^-38 <= eps (exact-accumulator range) */
  uint64_t seed;     /* key of the query's random streams                       */
  uint32_t query_id; /* < 2^24; with seed selects the random streams            */
  float* out;        /* device float[n]: receives pi_hat                        */
  int64_t x_nnz;        /* 0: x = e_source; > 0: entries of a sparse x          */
  const int64_t* x_idx; /* host int64[x_nnz]: node ids (source is then unused)  */
  const float* x_val;   /* host float[x_nnz]: values                            */
} agp_query_t;

typedef struct agp_server_config {
  int32_t max_slots;      /* queries advanced together per step (>= 1)          */
  int32_t queue_capacity; /* submitted but not yet admitted queries (>= 1)      */
  double work_budget;     /* admission cap on the summed Theorem 3.3 push
                             estimates of running queries; 0 = no cap          */
  int64_t memory_bytes;   /* device memory of the running queries' residue
                             tables (20 bytes per table entry, two tables of
                             2^k entries per query); 0 = a quarter of the free
                             device memory at creation                        */
} agp_server_config_t;

typedef struct agp_result {
  int32_t status;     /* AGP_OK; AGP_ERANGE if the query's residues outgrew
                         the exact accumulators; AGP_ENOMEM if its tables
                         exceed the whole pool                                 */
  int32_t levels;     /* L                                                     */
  uint64_t frontier;  /* sum over levels of the query's frontier sizes         */
  uint64_t pushes;    /* deterministic + accepted sampled pushes               */
  uint64_t candidates;/* sampled candidate positions                           */
  uint64_t table_entries; /* entries of each of the query's two residue tables  */
  int32_t restarts;   /* runs ended by a full table (the query then ran again
                         with tables twice as large)                           */
  double submit_ms;   /* times in ms on the server's clock (steady, from       */
  double start_ms;    /*   server creation): submission, admission, and the    */
  double end_ms;      /*   end of the step that finished the query             */
} agp_result_t;

typedef struct agp_server agp_server_t;

/* Create a query server over graph g (Section 4's randomized propagation
 * applied to a stream of single-source queries, continuously batched).  A
 * worker thread admits queued queries into free slots, in submission order,
 * while the summed push estimates stay within work_budget, and advances every
 * running query by one level per step in one launch; slots may be at
 * different levels with different a, b, L, w and eps.  A query finishes after
 * its level L; its result is independent of what runs beside it.
 * A query's residues live in two tables (this level's and the next
 * level's).  With a = 0, b = 1 (column-stochastic P) they are
 * open-addressing tables of 2^k entries, at least twice the distinct nodes
 * its busiest level is expected to reach (by Theorem 3.3 the expected
 * pushes of level i are at most (Y_i / S) / eps for x = e_s, and level 1
 * reaches at most the neighbours of the signal's nodes), or, when that
 * would reach n, direct tables of n entries (position = node); with other
 * exponents the residue mass can grow from level to level and the tables
 * are direct from the start;
 * both take one contiguous range of a pool of memory_bytes / 20 entries.  Admission is in submission order, while a
 * slot is free, the work budget allows and the query's range fits in the
 * pool: the running queries never hold more than the pool.  A query whose
 * tables are larger than the whole pool finishes at once with status
 * AGP_ENOMEM.  A table that fills up (a node finds no free position within
 * 128 probes) ends that run: the query is queued again at the head with
 * tables twice as large, and its result is unchanged.  The graph must outlive the server.
 * Errors: AGP_EINVAL, AGP_ENOMEM, AGP_EDEVICE. */
int agp_server_create(const agp_graph_t* g, const agp_server_config_t* cfg, agp_server_t** out);

/* Queue a query; *ticket identifies it for agp_poll.  The descriptor and the
 * weights are copied; the caller keeps ownership of q->out, which the server
 * writes (zero-filled first) only while the query runs.  Returns AGP_EINVAL
 * for an invalid query (nothing is queued), AGP_EBUSY when the queue is full. */
int agp_submit(agp_server_t* s, const agp_query_t* q, uint64_t* ticket);

/* AGP_OK with *res filled once the query has finished (the ticket is then
 * released), AGP_PENDING while it is queued or running, AGP_ENOENT for an
 * unknown or already collected ticket.  Thread-safe. */
int agp_poll(agp_server_t* s, uint64_t ticket, agp_result_t* res);

/* Stop admitting, finish the running queries, drop the queued ones and free
 * the server.  Synchronous. */
int agp_server_destroy(agp_server_t* s);

/* ---------------------------------------------- local clustering sweep */

/* Sweep of a proximity estimate into a local cluster (Section 5, the
 * quality of local clusters, e.g. a heat kernel PageRank estimate): the
 * nodes are ordered by pi(v) / d_v descending (d_v = row length; ties by
 * node id; nodes without arcs last), and the result is the first prefix
 * S_i = {v_1..v_i}, 1 <= i <= n - 1, of minimum conductance
 *   Phi(S) = |cut(S)| / min(vol(S), 2m - vol(S)),
 * cut(S) = arcs from S to the rest (a self-loop is never cut), vol(S) = the
 * sum of the row lengths in S, 2m = nnz.  Prefixes whose denominator is 0
 * are skipped.  Cut and volume are exact integers; Phi is their binary64
 * quotient.
 *  g            an undirected graph (not built with AGP_DIRECTED)
 *  pi, ld       device float: the estimate of node v is pi[v * ld] (ld >= 1;
 *               column c of an n x C agp_propagate result: out + c, ld = C)
 *  stream       work is enqueued on this stream; the call waits for it
 *  best_size    host; receives i (0 when no prefix has a conductance)
 *  best_conductance  host; receives Phi(S_i) (+inf when best_size is 0)
 *  order        optional device int32[n] (NULL to skip): the node order, so
 *               that order[0..best_size) is the cluster
 * Working memory of about 60 n bytes plus the sort's is kept with the graph
 * (released by agp_graph_destroy); calls on one graph are serialised with
 * each other and with agp_propagate.  Synchronous on `stream`.
 * Errors: AGP_EINVAL (NULL argument, ld < 1, directed graph), AGP_ENOMEM,
 * AGP_EDEVICE. */
int agp_sweep(const agp_graph_t* g, const float* pi, int64_t ld, void* stream, int64_t* best_size,
              double* best_conductance, int32_t* order);

/* agp_sweep of C estimates at once: column c is pi[v * ld + c] (1 <= C <=
 * ld; e.g. an n x C agp_propagate result with ld = C).  best_size and
 * best_conductance are host arrays of C entries, each what agp_sweep gives
 * for that column.  Columns are processed in groups of up to 64 (fewer when
 * a group's working memory of about 40 n bytes per column would exceed a
 * quarter of the free memory), each column with its own sort and each group
 * with one pass over the arcs.  Working memory is kept with the graph like
 * agp_sweep's.  Synchronous on `stream`.  Errors: AGP_EINVAL (NULL argument,
 * C < 1 or ld < C, directed graph), AGP_ENOMEM, AGP_EDEVICE. */
int agp_sweep_batch(const agp_graph_t* g, const float* pi, int64_t ld, int32_t C, void* stream,
                    int64_t* best_size, double* best_conductance);

/* ------------------------------------- device random number generators */

/* The device generators that take the propagation's random decisions,
 * evaluated on host inputs (for known-answer checks).  The subset sampling of
 * Section 4 draws its uniforms from Philox4x32-10 (Salmon, Moraes, Dror,
 * Shaw, SC'11: ten rounds of the Philox-4x32 S-box with the published
 * multipliers and Weyl key increments); the per-level frontier hash sums the
 * splitmix64 finaliser (Steele, Lea, Flood, OOPSLA'14) of node ids.
 *  count  number of blocks (>= 0)
 *  ctr    host uint32[4 * count], counter words c0..c3 of each block
 *  key    host uint32[2 * count], key words k0, k1 of each block
 *  out    host uint32[4 * count], receives the four output words
 * Synchronous (default stream); temporary device memory is allocated.
 * Errors: AGP_EINVAL (count < 0 or a NULL array with count > 0),
 * AGP_ENOMEM, AGP_EDEVICE. */
int agp_device_philox4x32_10(int64_t count, const uint32_t* ctr, const uint32_t* key, uint32_t* out);

/* splitmix64 finaliser of in[i] into out[i], i < count (host arrays);
 * as agp_device_philox4x32_10. */
int agp_device_splitmix64(int64_t count, const uint64_t* in, uint64_t* out);

/* ------------------------------------------- weight sequences (Table 1) */

/* w_i = alpha (1 - alpha)^i, i = 0..L (PageRank, PPR, APPNP). */
int agp_weights_ppr(double alpha, int32_t L, double* w);
/* w_i = e^-t t^i / i!, i = 0..L (heat kernel PageRank, GDC). */
int agp_weights_hkpr(double t, int32_t L, double* w);
/* w_i = beta^i, i = 0..L (Katz). */
int agp_weights_katz(double beta, int32_t L, double* w);
/* w_L = 1, w_i = 0 otherwise (L-hop transition probability, SGC). */
int agp_weights_tp(int32_t L, double* w);

#ifdef __cplusplus
}
#endif
#endif
