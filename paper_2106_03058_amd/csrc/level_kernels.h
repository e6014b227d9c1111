// One level of the randomized residue push (Algorithm 2 of "Approximate
// Graph Propagation", Section 4) for many columns at once, shared by the
// batched entry points (agp_propagate*) and the query server.
//
// A column is one signal (a feature column or one query).  Every column
// carries its own level parameters (ColParams), so columns at different
// levels, with different weights, exponents a/b, thresholds and random keys
// advance together in one launch.
//
// Cells: the residue of node u in column c lives at cell u * su + c * sc
// (row-major n x C for agp_propagate; a served query's residues live at
// positions of its own table instead).  Next-level residues are exact
// integers of a per-column unit
// (int64 cells for binary32, 128-bit cells for binary64), so the integer
// atomics that add contributions commute and the result does not depend on
// the order in which pushes land.
//
// A wave takes batches of up to 64 frontier entries (u, c) (from a list, or,
// at level 0 of a mostly non-zero signal, every cell in order): each lane
// converts one entry's residue, updates the reserve (pi(u) += kappa_i r(u)),
// finds the deterministic prefix J of the degree-sorted row (increment >=
// theta, by binary search) and counts the work items of its sampled suffix;
// the wave then makes the batch's deterministic pushes with all lanes (a
// wave-wide scan spreads them) and lanes draw sampled work items (runs of
// 64-position windows) from a per-wave queue, walking their Philox /
// geometric-skip chains.  Rows with long deterministic prefixes and entries
// with many sampled work items are deferred to grid-wide kernels
// (k_det_big, k_samp_big) that run right after the level.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "agp_device.h"

namespace agp {
namespace lvl {

constexpr int kThreads = 256;
constexpr int kLevelBlocks = 4096;
constexpr int kNumCounters = 6;   // frontier, hash, det, cand, acc, runs
constexpr int kThetaRows = 4096;  // rows per partial sum of ||x||_1
constexpr int kServeLdsSlots = 128;  // server columns whose counters a block sums in LDS

enum : int { kLastLevel = 1, kAZero = 2, kDrop = 4 };

// How the next frontier of a level is formed (written by k_level):
enum : int {
  kModeSparse = 0,    // first contributions appended directly
  kModeCompact = 1,   // fire-and-forget atomics, then a compaction scan
  kModeBinned = 2,    // records binned by destination and summed in LDS
  kModeOverflow = 3,  // record buffer overflowed: atomics, then compaction
};

// Binned aggregation: a record is (cell | sign << 31) of a sampled push;
// cells are grouped into at most 1024 buckets of 2^shift cells (shift
// chosen per call from n * C, at least kBinLog2) and every bucket into bins
// of 8192 cells (32-bit counts in 32 KiB of LDS), so n * C must stay below
// 2^31.
constexpr int kBinLog2 = 13;
constexpr int kMaxBinsPerBucket = 1024;
constexpr int kBuckets = 1024;

// Rows with many deterministic pushes (a hub with a large residue) would
// keep one wave busy while the rest of the grid idles; a batched level
// defers rows of at least big_row (default kBigRow) deterministic pushes to a
// list that k_det_big then spreads over the whole grid in chunks of kBigChunk
// pushes.
constexpr uint32_t kBigRow = 4096;
constexpr int kBigChunk = 4096;  // a lane walks from row to row inside its chunk
constexpr int kBigShift = 40;    // list counter: deferred rows << 40 | their pushes (a level's pushes < 2^40)

struct BigRow {
  unsigned long long off;  // deterministic pushes of the rows deferred before this one
  int64_t rp;              // first arc of the row
  double cv;               // c = rho |r| d_u^-b
  uint32_t c, J, neg, pad;
};

// Likewise an entry whose sampled suffix makes samp_items (64 by default)
// or more work items (a hub holding a small residue in some column): its
// items go to a second list that k_samp_big spreads over the whole grid
// (one item per lane).
constexpr long long kBigItems = 64;

struct BigSamp {
  unsigned long long off;  // work items of the entries deferred before this one
  int64_t rp;              // first arc of the row
  double cv;               // c = rho |r| d_u^-b
  double p0;               // a = 0: the sampling probability of every run
  uint32_t u, c, J, d;
  uint32_t neg, items;
};

struct ColParams {
  double theta;          // eps * ||x_c||_1
  double scale;          // 2^-ue (binary32 units)
  double rho;            // Y_{i+1} / Y_i at the column's current level
  double kappa;          // S w_i / Y_i at the column's current level
  long long dtheta;      // fl(theta) in units
  const double* da;      // d^-a, d = 0..max degree
  const double* db;      // d^-b
  void* out;             // reserve of node u at out + u * out_stride
  long long out_stride;
  int ue;                // exponent of the unit
  uint32_t qid;          // query id of the column's random streams
  uint32_t key0, key1;   // 64-bit seed
  int level;
  int flags;             // kLastLevel | kAZero | kDrop
  float theta_w;         // fl(theta) in binary32
};

struct LevelArgs {
  const int64_t* rp;
  const uint32_t* col;
  const uint32_t* nd;
  const uint32_t* gend;  // row-relative end of each arc's degree group
  const int32_t* deg;   // row lengths (neighbours to push to)
  const int32_t* fdeg;  // degrees in the factors d^-a, d^-b
  const ColParams* cp;
  // batched calls (one a and b for every column): per node u, d_u^-b and the
  // d^-a of its first neighbour (2 doubles; 0 for a node without arcs), or
  // null (the setup then reads them through the degree tables)
  const double* nodefac;
  // batched calls: d^-a of every arc's neighbour (arc order), or null
  const double* arcfac;
  long long su, sc;  // cell = u * su + c * sc
  long long xld;     // level 0 of a batched call: x[u * xld + c]
  int level;         // batched calls: counter row
  const uint64_t* fin;
  const unsigned long long* cnt_in;
  uint64_t* fout;
  unsigned long long* cnt_out;
  unsigned long long* counters;  // batched: per level; server: per column
  double* mass;                  // batched: per level; server: per column
  int* err;                      // batched: one flag; server: one per column
  int positive;                  // non-negative signals: sparse levels allowed
  unsigned long long dense_cut;  // frontier size from which a level is dense
  int* mode_out;                 // how the next frontier is formed (kMode*)
  // binned aggregation (binary32 batched calls; rec == nullptr: disabled);
  // records are kept per column group (rec_groups groups of rec_gw columns,
  // 1 group: the whole row), group g's at rec + g * rec_cap
  uint32_t* rec;
  unsigned long long* rec_count;  // this level's record count of each group
  unsigned long long rec_cap;     // records per group
  int rec_groups;
  uint32_t rec_gw;
  unsigned int* bucket_count;    // records per bucket of this level (kBuckets, kBuckets / 2 per group with two)
  int bucket_shift;              // cells per bucket = 2^bucket_shift
  const double* bin_est;         // non-null: bin only if *bin_est >= bin_pushes (estimated pushes)
  double bin_pushes;
  // deferred rows (batched calls; nullptr: every row is pushed by its wave)
  uint32_t big_row;              // deterministic pushes from which an entry's row is deferred
  unsigned long long* big_ctr;   // this level's list counter, zero at the start
  BigRow* big;
  unsigned long long big_cap;
  unsigned long long* samp_ctr;  // the same for deferred sampled suffixes (entries << 40 | items)
  BigSamp* samp;
  long long samp_items;          // work items from which an entry's sampled suffix is deferred
  // binned levels: deterministic pushes mark their destination bin (nullptr:
  // no marks); group g's bins at det_bins + g * det_bins_g
  uint8_t* det_bins;
  unsigned long long det_bins_g;
  // served queries: each query's residues live in an open-addressing table
  // of one pool (query c owns positions tab_off[c] .. tab_off[c] + tab_mask[c];
  // a key is node + 1, 0 when free); frontier entries are (position, c)
  uint32_t* keys_cur;
  uint32_t* keys_nxt;
  const uint32_t* tab_off;   // the next level's tables
  const uint32_t* tab_mask;
  const uint32_t* tab_cur;   // this level's tables
};

// Position of node v in a query's table, claiming it if v is not there yet
// (*first: v was not there); ~0u when the table is too full.  mask == ~0u:
// a direct table of n entries (position base + v); else 2^k = mask + 1
// entries probed linearly from a multiplicative hash of v, at most
// kMaxProbes of them (a table at most half full needs a few; more means
// that the query outgrew its table).
constexpr uint32_t kDirectTable = ~0u;
// mask == kDirectPlain: a direct table of a query whose residues cannot
// cancel (a non-negative signal): no keys (the node is the position's
// offset), plain atomic adds, and the next frontier is formed by a scan of
// the table's non-zero positions after the level
constexpr uint32_t kDirectPlain = ~1u;
constexpr uint32_t kMaxProbes = 128;
__device__ __forceinline__ uint32_t table_find_or_insert(uint32_t* keys, uint32_t base, uint32_t mask, uint32_t v,
                                                         bool* first) {
  // a key changes only once per level (0 -> node + 1), so a coherent read
  // that already shows v spares the compare-and-swap
  if (mask == kDirectTable) {
    const uint32_t pos = base + v;
    uint32_t old = __hip_atomic_load(keys + pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == 0u) old = atomicCAS(keys + pos, 0u, v + 1u);
    *first = old == 0u;
    return pos;
  }
  const uint32_t h = static_cast<uint32_t>((static_cast<unsigned long long>(v) * 0x9E3779B97F4A7C15ull) >> 32);
  const uint32_t probes = mask < kMaxProbes ? mask + 1u : kMaxProbes;
  for (uint32_t k = 0; k < probes; ++k) {
    const uint32_t pos = base + ((h + k) & mask);
    uint32_t old = __hip_atomic_load(keys + pos, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == 0u) old = atomicCAS(keys + pos, 0u, v + 1u);
    if (old == 0u || old == v + 1u) {
      *first = old == 0u;
      return pos;
    }
  }
  *first = false;
  return ~0u;
}
constexpr int kErrTableFull = 2;  // server: a query's table had no free position

// ----------------------------------------------------- working precision
template <typename T>
struct Prec;

__device__ __forceinline__ void atomic_add_relaxed(unsigned long long* p, unsigned long long v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long atomic_add_ret(unsigned long long* p, unsigned long long v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <>
struct Prec<float> {
  using Cell = long long;
  using Delta = long long;
  static constexpr int kWords = 1;
  static __device__ __forceinline__ float take(Cell* acc, size_t cell, const ColParams& p) {
    const long long K = acc[cell];
    acc[cell] = 0;
    return units_to_f32(K, p.ue);
  }
  static __device__ __forceinline__ bool to_units(float v, const ColParams& p, Delta* d) {
    return f32_to_units(v, p.scale, d);
  }
  static __device__ __forceinline__ Delta theta_units(const ColParams& p, bool neg) {
    return neg ? -p.dtheta : p.dtheta;
  }
  static __device__ __forceinline__ double mag_units(float v, const ColParams& p) {
    return fabs(static_cast<double>(v)) * p.scale;
  }
  // true if the cell held zero before (first contribution of the level)
  static __device__ __forceinline__ bool add_ret(Cell* acc, size_t cell, Delta d) {
    return atomic_add_ret(reinterpret_cast<unsigned long long*>(acc + cell),
                          static_cast<unsigned long long>(d)) == 0ull;
  }
  static __device__ __forceinline__ void add(Cell* acc, size_t cell, Delta d) {
    atomic_add_relaxed(reinterpret_cast<unsigned long long*>(acc + cell), static_cast<unsigned long long>(d));
  }
  static __device__ __forceinline__ bool nonzero(const Cell* acc, size_t cell) { return acc[cell] != 0; }
  static __device__ __forceinline__ void set_units(Cell* acc, size_t cell, long long v) { acc[cell] = v; }
};

template <>
struct Prec<double> {
  using Cell = unsigned long long;  // two words per cell
  using Delta = U128;
  static constexpr int kWords = 2;
  static __device__ __forceinline__ double take(Cell* acc, size_t cell, const ColParams& p) {
    U128 K{acc[2 * cell], static_cast<long long>(acc[2 * cell + 1])};
    acc[2 * cell] = 0;
    acc[2 * cell + 1] = 0;
    return units_to_f64(K, p.ue);
  }
  static __device__ __forceinline__ bool to_units(double v, const ColParams& p, Delta* d) {
    return f64_to_units(v, p.ue, d);
  }
  static __device__ __forceinline__ Delta theta_units(const ColParams& p, bool neg) {
    const long long d = neg ? -p.dtheta : p.dtheta;
    return U128{static_cast<unsigned long long>(d), d < 0 ? -1ll : 0ll};
  }
  static __device__ __forceinline__ double mag_units(double v, const ColParams& p) {
    return ldexp(fabs(v), -p.ue);
  }
  // the carry out of the low word needs the old value
  static __device__ __forceinline__ void add(Cell* acc, size_t cell, Delta d) {
    const unsigned long long old = atomic_add_ret(acc + 2 * cell, d.lo);
    const unsigned long long carry = (old + d.lo < old) ? 1ull : 0ull;
    const unsigned long long h = static_cast<unsigned long long>(d.hi) + carry;
    if (h != 0ull) atomic_add_relaxed(acc + 2 * cell + 1, h);
  }
  static __device__ __forceinline__ bool add_ret(Cell* acc, size_t cell, Delta d) {
    add(acc, cell, d);
    return false;  // binary64 calls always compact the next frontier
  }
  static __device__ __forceinline__ bool nonzero(const Cell* acc, size_t cell) {
    return (acc[2 * cell] | acc[2 * cell + 1]) != 0ull;
  }
  static __device__ __forceinline__ void set_units(Cell* acc, size_t cell, long long v) {
    acc[2 * cell] = static_cast<unsigned long long>(v);
    acc[2 * cell + 1] = v < 0 ? ~0ull : 0ull;
  }
};

__device__ __forceinline__ float to_w(double v, float) { return static_cast<float>(v); }
__device__ __forceinline__ double to_w(double v, double) { return v; }

// ------------------------------------------------- record staging
// On binned levels a sampled push becomes a 4-byte record, cell | sign << 31
// (its value is -/+ fl(theta_c) of the cell's column c); deterministic pushes
// still use atomics.  Records go to their group's buffer in chunks (one
// atomic per chunk).  Records beyond the buffer capacity are added to the
// accumulator directly; the level then ends in kModeOverflow (the buffered
// records are applied with atomics too).
//
// The cell of a record is local to a column group, so that it stays below
// 2^31 when n C does not: with one group it is u * su + c * sc; with two
// (row-major cells only) group g = [c >= rec_gw] holds the columns from
// g rec_gw on and the local cell is u * rec_gw + (c - g rec_gw).
constexpr int kRecStage = 2 * kStage;  // 4-byte records per wave stage (both groups)
constexpr uint32_t kRecCellMask = 0x7FFFFFFFu;
constexpr int kMaxRecGroups = 2;

// kG: the groups of the launch (A.rec_groups of a binned level), a template
// argument so that one-group levels keep the plain single-group code.
struct RecCell {
  uint32_t g, cell;
};
template <int kG>
__device__ __forceinline__ RecCell rec_cell(const LevelArgs& A, uint32_t u, uint32_t c) {
  if constexpr (kG > 1) {
    const uint32_t g = c >= A.rec_gw ? 1u : 0u;
    return RecCell{g, u * A.rec_gw + (c - g * A.rec_gw)};
  } else {
    return RecCell{0u, u * static_cast<uint32_t>(A.su) + c * static_cast<uint32_t>(A.sc)};
  }
}

// (kG = 0: the groups of A at run time)
template <int kG>
__device__ __forceinline__ void apply_record(const LevelArgs& A, long long* acc, uint32_t rec, uint32_t g) {
  const uint32_t cell = rec & kRecCellMask;
  uint32_t c;
  size_t at = cell;
  if (kG > 1 || (kG == 0 && A.rec_groups > 1)) {
    const uint32_t u = cell / A.rec_gw;
    c = g * A.rec_gw + (cell - u * A.rec_gw);
    at = static_cast<size_t>(u) * static_cast<size_t>(A.su) + c;
  } else {
    c = A.sc == 1 ? cell % static_cast<uint32_t>(A.su) : cell / static_cast<uint32_t>(A.sc);
  }
  const long long d = (rec >> 31) ? -A.cp[c].dtheta : A.cp[c].dtheta;
  atomic_add_relaxed(reinterpret_cast<unsigned long long*>(acc + at), static_cast<unsigned long long>(d));
}

template <int kG>
__device__ __forceinline__ void apply_record(const LevelArgs&, unsigned long long*, uint32_t, uint32_t) {}

// Staged record counts of a wave: the count (one group), or group 0's in the
// low 16 bits and group 1's in the high 16 bits of one wave-uniform int.
//
// The staged records out: group 0's from the front of the stage, group 1's
// from its back (one atomic on each group's count; records beyond a group's
// buffer are added with atomics).  Wave-uniform.
template <int kG, typename Cell>
__device__ __forceinline__ void stage_flush_records(uint32_t* stage, int& staged, const LevelArgs& A, Cell* acc) {
  if constexpr (kG == 1) {
    if (staged == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(A.rec_count, static_cast<unsigned long long>(staged));
    base = __shfl(base, 0);
    for (int i = lane_id(); i < staged; i += kWave) {
      if (base + i < A.rec_cap)
        A.rec[base + i] = stage[i];
      else
        apply_record<kG>(A, acc, stage[i], 0u);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    staged = 0;
    return;
  }
  const int n0 = staged & 0xFFFF, n1 = staged >> 16;
  const int total = n0 + n1;
  if (total == 0) return;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const int lane = lane_id();
  unsigned long long base = 0;
  if (lane < 2) {
    const int k = lane == 0 ? n0 : n1;
    if (k > 0) base = atomicAdd(A.rec_count + lane, static_cast<unsigned long long>(k));
  }
  const unsigned long long base0 = __shfl(base, 0), base1 = __shfl(base, 1);
  for (int i = lane; i < total; i += kWave) {
    const uint32_t g = i < n0 ? 0u : 1u;
    const int j = i - (g ? n0 : 0);
    const uint32_t r = g ? stage[kRecStage - 1 - j] : stage[j];
    const unsigned long long at = (g ? base1 : base0) + static_cast<unsigned long long>(j);
    if (at < A.rec_cap)
      A.rec[static_cast<size_t>(g) * A.rec_cap + at] = r;
    else
      apply_record<kG>(A, acc, r, g);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  staged = 0;
}

// One sampled push of every lane that emits (a wave-uniform call) as a
// record of its group: its bucket counted in s_hist (kBuckets buckets, or
// kBuckets / 2 per group with two groups), the record staged (group 0 from
// the front of the stage, group 1 from its back); the stage goes out when it
// is nearly full.
template <int kG, typename Cell>
__device__ __forceinline__ void emit_record(const LevelArgs& A, unsigned int* s_hist, uint32_t* stage, int& staged,
                                            bool emit, uint32_t v, uint32_t c, bool neg, Cell* acc) {
  uint32_t rec = 0, g = 0;
  if (emit) {
    const RecCell rc = rec_cell<kG>(A, v, c);
    g = rc.g;
    rec = rc.cell | (neg ? 0x80000000u : 0u);
    atomicAdd(&s_hist[g * (kBuckets / kMaxRecGroups) + (rc.cell >> A.bucket_shift)], 1u);
  }
  const unsigned long long lt = (1ull << lane_id()) - 1ull;
  if constexpr (kG > 1) {
    const int n0 = staged & 0xFFFF, n1 = staged >> 16;
    const unsigned long long m1 = __ballot(emit && g != 0);
    const unsigned long long m0 = __ballot(emit) & ~m1;
    if (emit) stage[g ? kRecStage - 1 - (n1 + __popcll(m1 & lt)) : n0 + __popcll(m0 & lt)] = rec;
    const int k0 = n0 + __popcll(m0), k1 = n1 + __popcll(m1);
    staged = k0 | (k1 << 16);
    if (k0 + k1 > kRecStage - kWave) stage_flush_records<kG>(stage, staged, A, acc);
  } else {
    const unsigned long long m0 = __ballot(emit);
    if (emit) stage[staged + __popcll(m0 & lt)] = rec;
    staged += __popcll(m0);
    if (staged > kRecStage - kWave) stage_flush_records<kG>(stage, staged, A, acc);
  }
}

// The end of a binned launch: the staged records out, then (after a block
// barrier) the block's bucket counts added to the level's.
template <int kG, typename Cell>
__device__ __forceinline__ void finish_records(const LevelArgs& A, unsigned int* s_hist, uint32_t* stage, int& staged,
                                               Cell* acc) {
  stage_flush_records<kG>(stage, staged, A, acc);
  __syncthreads();
  for (int i = threadIdx.x; i < kBuckets; i += blockDim.x)
    if (s_hist[i]) atomicAdd(A.bucket_count + i, s_hist[i]);
}

// a deterministic push's mark on its destination bin (binned levels)
template <int kG>
__device__ __forceinline__ void mark_det_bin(const LevelArgs& A, uint8_t* det_bins, uint32_t v, uint32_t c) {
  const RecCell rc = rec_cell<kG>(A, v, c);
  det_bins[rc.g * A.det_bins_g + (rc.cell >> kBinLog2)] = 1;
}

// Server counters: LDS sums for the first kServeLdsSlots columns, global
// atomics beyond.
__device__ __forceinline__ void serve_count(const LevelArgs& A, unsigned long long (*lds)[kNumCounters],
                                            uint32_t c, int k, unsigned long long v) {
  if (c < kServeLdsSlots)
    atomicAdd(&lds[c][k], v);
  else
    atomicAdd(A.counters + static_cast<size_t>(c) * kNumCounters + k, v);
}

// ------------------------------------------------------------ the level
// Work is organised per wave.  A wave takes batches of up to 64 frontier
// entries (batch b of the level goes to wave b mod #waves); for each batch a lane
// sets up one entry (reserve update, c, the deterministic prefix J, the
// number of sampled work items), the wave then makes the batch's
// deterministic pushes with all lanes, one push per lane and step, and puts
// the sampled work items in a queue that idle lanes draw from.  A sampled
// work item is up to kWinPerItem consecutive 64-position windows of one
// entry's suffix; a lane walks their Philox / geometric-skip chains one draw
// per step and takes the next item from the queue in the step after its last
// draw, so lanes stay busy across entries and batches.  All loops run in
// lockstep per wave so that staging can use wave-wide ballots.
constexpr int kBatch = kWave;
constexpr int kWinPerItem = 16;
constexpr int kItemMap = 128;

struct BatchLds {
  int64_t rp[kBatch];
  double cv[kBatch];
  double p0[kBatch];           // a = 0: sampling probability of every run of the entry;
                               // a > 0: the first arc's factor when the entry has no
                               // deterministic push (its first run starts there), else 0
  long long doff[kBatch + 1];  // deterministic pushes before each entry (exclusive scan)
  long long ioff[kBatch + 1];  // sampled work items before each entry
  // the entry's column parameters that its work items need (theta, the
  // random stream's counter word and key), so that taking an item reads LDS
  double th[kBatch];
  uint32_t ctr3[kBatch], key0[kBatch], key1[kBatch];
  // c: column | kBatchNeg (negative residue) | kBatchAZero (a = 0)
  uint32_t u[kBatch], c[kBatch], d[kBatch], J[kBatch];
  uint8_t item_entry[kItemMap];  // the entry of each of the batch's first kItemMap work items
};
constexpr uint32_t kBatchNeg = 1u << 31, kBatchAZero = 1u << 30, kBatchCol = kBatchAZero - 1u;
// columns of one level launch at most (the column index leaves those two bits free)
constexpr int32_t kMaxTileColumns = static_cast<int32_t>(kBatchCol);

// floor(a / C) and a mod C for a < 2^22, from rc = 1 / C rounded to binary32:
// the product is within one of the quotient, and one correction makes it exact
__device__ __forceinline__ uint32_t div_small(uint32_t a, uint32_t C, float rc, uint32_t* rem) {
  uint32_t q = static_cast<uint32_t>(static_cast<float>(a) * rc);
  int32_t r = static_cast<int32_t>(a) - static_cast<int32_t>(q * C);
  if (r < 0) {
    --q;
    r += static_cast<int32_t>(C);
  } else if (r >= static_cast<int32_t>(C)) {
    ++q;
    r -= static_cast<int32_t>(C);
  }
  *rem = static_cast<uint32_t>(r);
  return q;
}

// Level 0 of a batched call whose signal is mostly non-zero: the frontier is
// every cell in order, entry e = (e / C, e mod C), and no list is formed
// (A.fin == nullptr; C = A.su <= kVirtualMaxC); its zero cells are skipped
// by the level kernel as if they were not listed.
constexpr long long kVirtualMaxC = 1 << 21;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// largest e in [0, 64) with off[e] <= k (off non-decreasing, off[0] <= k)
__device__ __forceinline__ int batch_find(const long long* off, long long k) {
  int e = 0;
#pragma unroll
  for (int step = kBatch / 2; step > 0; step >>= 1)
    if (off[e + step] <= k) e += step;
  return e;
}

// kFirst: the residues are the signal x (level 0 of a batched call).
// kServe: counters and overflow mass are kept per column instead of per level.
// kG: column groups of the records on binned levels (1 or 2).
template <typename T, bool kFirst, bool kServe, int kG = 1>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_level(LevelArgs A, const T* __restrict__ x,
                                                    typename Prec<T>::Cell* __restrict__ acc_cur,
                                                    typename Prec<T>::Cell* __restrict__ acc_next) {
  using P = Prec<T>;
  using Delta = typename P::Delta;
  constexpr int kWaves = kThreads / kWave;
  __shared__ BatchLds s_batch[kWaves];
  __shared__ uint64_t s_stage[kWaves][kStage];
  __shared__ unsigned int s_hist[kBuckets];
  // server: per-column counters summed in LDS, flushed once per block
  __shared__ unsigned long long s_scnt[kServe ? kServeLdsSlots : 1][kNumCounters];
  __shared__ double s_smass[kServe ? kServeLdsSlots : 1];

  const unsigned long long count = *A.cnt_in;
  // Binned levels write (cell, value) records that later kernels group by
  // destination and sum in LDS.  Without binning, sparse levels detect the
  // first contribution to a cell from the atomic's old value and append the
  // cell to the next frontier; dense levels use fire-and-forget atomics and a
  // compaction pass builds the next frontier.
  const bool binned = A.rec != nullptr && (A.bin_est == nullptr || *A.bin_est >= A.bin_pushes);
  const bool sparse = kServe || (!binned && A.positive && count < A.dense_cut);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    *A.mode_out = binned ? kModeBinned : (sparse ? kModeSparse : kModeCompact);
  if (binned) {
    for (int i = threadIdx.x; i < kBuckets; i += blockDim.x) s_hist[i] = 0;
    __syncthreads();
  }
  if (kServe) {
    for (int i = threadIdx.x; i < kServeLdsSlots * kNumCounters; i += blockDim.x) (&s_scnt[0][0])[i] = 0;
    for (int i = threadIdx.x; i < kServeLdsSlots; i += blockDim.x) s_smass[i] = 0.0;
    __syncthreads();
  }
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
  BatchLds& B = s_batch[wave];
  uint64_t* stage = s_stage[wave];
  int staged = 0;  // wave-uniform

  // per-lane and per-wave counts stay far below 2^32 in one launch (at least
  // 1024 waves share at most one candidate per arc and column of the level);
  // the hash wraps mod 2^64
  uint32_t n_det = 0;
  uint32_t w_front = 0, w_cand = 0, w_acc = 0, w_runs = 0;  // wave-uniform (ballot counts)
  unsigned long long n_hash = 0;
  double mass = 0.0;

  // One contribution per lane (or none), in exact units of the next
  // residue.  Wave-uniform calls.  emit_det: a deterministic push (atomics
  // on every level); emit_sampled: a sampled push of -/+ fl(theta) (a
  // 4-byte record on binned levels).
  auto emit_atomic = [&](bool emit, uint32_t v, uint32_t ec, const Delta& delta) {
    bool first = false;
    if constexpr (kServe) {  // the query's table: first touches go to the next frontier
      uint32_t pos = 0;
      if (emit) {
        const uint32_t mask = A.tab_mask[ec];
        if (mask == kDirectPlain) {  // the next frontier comes from a scan of the table
          pos = A.tab_off[ec] + v;
          P::add(acc_next, pos, delta);
        } else {
          pos = table_find_or_insert(A.keys_nxt, A.tab_off[ec], mask, v, &first);
          if (pos == ~0u)
            atomicOr(A.err + ec, kErrTableFull);
          else
            P::add(acc_next, pos, delta);
        }
      }
      stage_push(stage, staged, (static_cast<uint64_t>(pos) << 32) | ec, first, A.fout, A.cnt_out);
      return;
    }
    const size_t vcell = static_cast<size_t>(v) * A.su + static_cast<size_t>(ec) * A.sc;
    if (emit) {
      if (sparse)
        first = P::add_ret(acc_next, vcell, delta);
      else
        P::add(acc_next, vcell, delta);
    }
    if (sparse)  // stage first-touched cells, flush in chunks
      stage_push(stage, staged, (static_cast<uint64_t>(v) << 32) | ec, first, A.fout, A.cnt_out);
  };
  auto emit_sampled = [&](bool emit, uint32_t v, uint32_t ec, const Delta& delta, bool eneg) {
    if (binned) {
      emit_record<kG>(A, s_hist, reinterpret_cast<uint32_t*>(stage), staged, emit, v, ec, eneg, acc_next);
    } else {
      emit_atomic(emit, v, ec, delta);
    }
  };

  // up to 64 entries per batch; fewer when the level has fewer entries than
  // 64 per wave, so that small frontiers still spread over the whole grid
  const unsigned long long nwaves = static_cast<unsigned long long>(gridDim.x) * kWaves;
  const unsigned long long eb_raw = count / nwaves;
  const unsigned long long eb = eb_raw < 1ull ? 1ull : (eb_raw > (unsigned long long)kBatch ? kBatch : eb_raw);
  const unsigned long long nbatch = (count + eb - 1) / eb;
  const unsigned long long bstride = static_cast<unsigned long long>(gridDim.x) * kWaves;
  unsigned long long bnext = static_cast<unsigned long long>(blockIdx.x) * kWaves + wave;
  long long it_next = 0, it_total = 0;  // wave-uniform: queue of the loaded batch
  // the frontier items of this wave's next batch, loaded one batch ahead so
  // that a batch's setup starts from its items
  auto load_items = [&](unsigned long long b) -> uint64_t {
    if (b >= nbatch) return 0ull;
    const unsigned long long e = b * eb;
    const unsigned long long m = (count - e) < eb ? (count - e) : eb;
    if (static_cast<unsigned long long>(lane) >= m) return 0ull;
    if (kFirst && A.fin == nullptr) {  // every cell: (e / C, e mod C)
      const uint32_t C = static_cast<uint32_t>(A.su);
      const unsigned long long u0 = e / C;
      uint32_t c = 0;
      const uint32_t q = div_small(static_cast<uint32_t>(e - u0 * C) + static_cast<uint32_t>(lane), C,
                                   1.0f / static_cast<float>(C), &c);
      return ((u0 + q) << 32) | c;
    }
    return A.fin[e + lane];
  };
  uint64_t next_items = load_items(bnext);

  // lane state: the sampled work item in progress
  bool active = false, need_run = false, neg = false, azero = true;
  uint32_t u = 0, c = 0, s = 0, rend = 0, run_end = 0, pos = 0, t = 0, ctr3 = 0, key0 = 0, key1 = 0;
  uint32_t it_cand = 0, it_acc = 0, it_runs = 0;
  int64_t rpu = 0;
  double cv = 0.0, dstart = 1.0, th = 0.0;
  const ColParams* cpp = A.cp;
  SkipTable tab;

  for (;;) {
    // (a) a lane whose item has no window left becomes idle
    if (active && need_run && s >= rend) {
      active = false;
      if (kServe) {
        if (it_cand) {
          serve_count(A, s_scnt, c, 3, static_cast<unsigned long long>(it_cand));
          if (it_acc) serve_count(A, s_scnt, c, 4, static_cast<unsigned long long>(it_acc));
        }
        if (it_runs) serve_count(A, s_scnt, c, 5, static_cast<unsigned long long>(it_runs));
      }
    }
    // (b) the queue is empty and a lane is idle: set up the next batch
    if (it_next >= it_total && bnext < nbatch && __any(!active)) {
      wave_sync();  // every lane has read the previous batch
      const unsigned long long e0 = bnext * eb;
      bnext += bstride;
      const int ne = static_cast<int>((count - e0) < eb ? (count - e0) : eb);
      const uint64_t batch_item = next_items;
      next_items = load_items(bnext);
      long long dwork = 0, iwork = 0;
      uint32_t eu = 0, ec = 0, ed = 0, eJ = 0, ecw = 0;
      int64_t erp = 0;
      double ecv = 0.0, ep0 = 0.0;
      bool eneg = false;
      bool front_live = false;
      if (lane < ne) {
        const uint64_t item = batch_item;
        eu = static_cast<uint32_t>(item >> 32);
        ec = static_cast<uint32_t>(item);
        size_t cell = static_cast<size_t>(eu) * A.su + static_cast<size_t>(ec) * A.sc;
        if constexpr (kServe) {  // (table position, query): the node is the key (or the offset); free it
          cell = eu;
          if (A.tab_mask[ec] == kDirectPlain) {
            eu = static_cast<uint32_t>(cell) - A.tab_cur[ec];
          } else {
            eu = A.keys_cur[cell] - 1u;
            A.keys_cur[cell] = 0u;
          }
        }
        // The loads that need only the entry go out together (a batched
        // entry always names a node of the graph and a live column: its row
        // bounds and factor degree beside its residue and column parameters),
        // then the ones that need their results (the reserve's old value, the
        // first neighbour's factor degree, d_u^-b).
        uint32_t deg_u = 0;
        int32_t fdeg_u = 0;
        int64_t rp_u = 0;
        const bool pre = !kServe && A.nodefac != nullptr;  // the node's two factors in one load
        const bool pre_arc = !kServe && A.arcfac != nullptr;  // each arc's neighbour factor in one load
        double2 nf = make_double2(0.0, 0.0);
        if (!kServe) {
          deg_u = static_cast<uint32_t>(A.deg[eu]);
          if (pre)
            nf = reinterpret_cast<const double2*>(A.nodefac)[eu];
          else
            fdeg_u = A.fdeg[eu];
          rp_u = A.rp[eu];
        }
        const ColParams& cp = A.cp[ec];
        T r;
        if (kFirst)
          r = x[static_cast<size_t>(eu) * static_cast<size_t>(A.xld) + ec];
        else
          r = P::take(acc_cur, cell, cp);
        // (a served query's table also holds nodes whose sum cancelled to zero,
        // and level 0 over every cell holds the zero cells of x: they are not
        // in the frontier)
        const bool live = !(cp.flags & kDrop) && !((kServe || (kFirst && A.fin == nullptr)) && r == T(0));
        if (kServe && live) {
          deg_u = static_cast<uint32_t>(A.deg[eu]);
          fdeg_u = A.fdeg[eu];
          rp_u = A.rp[eu];
        }
        T* const o = static_cast<T*>(cp.out) + static_cast<size_t>(eu) * static_cast<size_t>(cp.out_stride);
        const T o_old = (live && cp.kappa != 0.0) ? *o : T(0);
        // (a = 0: every factor d^-a is 1, no degree is read)
        const uint32_t nd_first = (!pre && live && deg_u > 0 && !(cp.flags & kAZero)) ? A.nd[rp_u] : 0u;
        const double db_u = live ? (pre ? nf.x : cp.db[fdeg_u]) : 0.0;
        eneg = r < T(0);
        ecw = ec | (eneg ? kBatchNeg : 0u) | ((cp.flags & kAZero) ? kBatchAZero : 0u);
        // (the previous batch is no longer read: these slots are free; the
        // entries past ne get no work items)
        B.th[lane] = cp.theta;
        B.ctr3[lane] = (cp.qid << 8) | static_cast<uint32_t>(cp.level);
        B.key0[lane] = cp.key0;
        B.key1[lane] = cp.key1;
        if (live) {
          if (kServe) {
            serve_count(A, s_scnt, ec, 0, 1ull);
          } else {
            front_live = true;
            n_hash += splitmix64(eu);
          }
          // reserve: pi(u) += (S w_i / Y_i) r(u), rounded to the working precision
          if (cp.kappa != 0.0) {
            const T q = to_w(cp.kappa * static_cast<double>(r), T());
            *o = o_old + q;
          }
          if (!(cp.flags & kLastLevel) && cp.rho != 0.0) {
            ed = deg_u;
            if (ed > 0) {
              const double absr = fabs(static_cast<double>(r));
              const double t0 = cp.rho * absr;
              ecv = t0 * db_u;
              const double eth = cp.theta;
              erp = rp_u;
              double inc0 = ecv;
              if (cp.flags & kAZero) {
                eJ = (ecv >= eth) ? ed : 0u;
                const double num = ecv * 1.0;  // every neighbour's factor d^-0 is 1
                ep0 = num / eth;
              } else {  // increments fall along the degree-sorted row: binary search
                const double da0 = pre ? nf.y : cp.da[nd_first];
                inc0 = ecv * da0;
                uint32_t lo = 0, hi = ed;
                if (!(inc0 >= eth))
                  hi = 0;  // no deterministic push
                else if (ecv * (pre_arc ? A.arcfac[erp + ed - 1] : cp.da[A.nd[erp + ed - 1]]) >= eth)
                  lo = ed;  // every push is deterministic
                while (lo < hi) {
                  const uint32_t mid = (lo + hi) >> 1;
                  const double inc = ecv * (pre_arc ? A.arcfac[erp + mid] : cp.da[A.nd[erp + mid]]);
                  if (inc >= eth)
                    lo = mid + 1;
                  else
                    hi = mid;
                }
                eJ = lo;
                // without deterministic pushes the first sampled run starts at
                // the row's first arc: its factor goes with the entry
                ep0 = eJ == 0 ? da0 : 0.0;
              }
              const long long windows =
                  (eJ < ed) ? static_cast<long long>(((ed - 1) >> kSegLog2) - (eJ >> kSegLog2) + 1) : 0;
              dwork = eJ;
              iwork = (windows + kWinPerItem - 1) / kWinPerItem;
              // a long deterministic prefix goes to the deferred list (the
              // counter is read first so that it never wraps)
              if (!kServe && A.big_ctr != nullptr && eJ >= A.big_row &&
                  (__hip_atomic_load(A.big_ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> kBigShift) <
                      A.big_cap) {
                const unsigned long long old =
                    atomic_add_ret(A.big_ctr, (1ull << kBigShift) | static_cast<unsigned long long>(eJ));
                const unsigned long long slot = old >> kBigShift;
                if (slot < A.big_cap) {
                  BigRow br;
                  br.off = old & ((1ull << kBigShift) - 1ull);
                  br.rp = erp;
                  br.cv = ecv;
                  br.c = ec;
                  br.J = eJ;
                  br.neg = eneg ? 1u : 0u;
                  br.pad = 0;
                  A.big[slot] = br;
                  dwork = 0;
                }
              }
              if (!kServe && A.samp_ctr != nullptr && iwork >= A.samp_items &&
                  (__hip_atomic_load(A.samp_ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> kBigShift) <
                      A.big_cap) {
                const unsigned long long old =
                    atomic_add_ret(A.samp_ctr, (1ull << kBigShift) | static_cast<unsigned long long>(iwork));
                const unsigned long long slot = old >> kBigShift;
                if (slot < A.big_cap) {
                  BigSamp bs;
                  bs.off = old & ((1ull << kBigShift) - 1ull);
                  bs.rp = erp;
                  bs.cv = ecv;
                  bs.p0 = ep0;
                  bs.u = eu;
                  bs.c = ec;
                  bs.J = eJ;
                  bs.d = ed;
                  bs.neg = eneg ? 1u : 0u;
                  bs.items = static_cast<uint32_t>(iwork);
                  A.samp[slot] = bs;
                  iwork = 0;
                }
              }
              // bound on the magnitude this entry can add (every contribution
              // is at most max(inc_0, theta)), for the overflow check
              const T big = to_w(inc0 > eth ? inc0 : eth, T());
              const double m = static_cast<double>(ed) * P::mag_units(big, cp);
              if (kServe) {
                serve_count(A, s_scnt, ec, 2, static_cast<unsigned long long>(eJ));
                if (ec < kServeLdsSlots)
                  atomicAdd(&s_smass[ec], m);
                else
                  atomicAdd(A.mass + ec, m);
              } else {
                n_det += eJ;
                mass += m;
              }
            }
          }
        }
      }
      if (!kServe) w_front += static_cast<uint32_t>(__popcll(__ballot(front_live)));
      long long dinc = dwork, iinc = iwork;
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const long long td = __shfl_up(dinc, off);
        const long long ti = __shfl_up(iinc, off);
        if (lane >= off) {
          dinc += td;
          iinc += ti;
        }
      }
      B.rp[lane] = erp;
      B.cv[lane] = ecv;
      B.p0[lane] = ep0;
      B.doff[lane] = dinc - dwork;
      B.ioff[lane] = iinc - iwork;
      {
        const int j1 = static_cast<int>(iinc < kItemMap ? iinc : kItemMap);
        for (int j = static_cast<int>(iinc - iwork < kItemMap ? iinc - iwork : kItemMap); j < j1; ++j)
          B.item_entry[j] = static_cast<uint8_t>(lane);
      }
      if (lane == kWave - 1) {
        B.doff[kBatch] = dinc;
        B.ioff[kBatch] = iinc;
      }
      B.u[lane] = eu;
      B.c[lane] = ecw;
      B.d[lane] = ed;
      B.J[lane] = eJ;
      wave_sync();
      // deterministic pushes of the batch: the increment reaches theta
      const long long dtot = B.doff[kBatch];
      for (long long kb = 0; kb < dtot; kb += kWave) {
        const long long k = kb + lane;
        bool emit = false;
        uint32_t v = 0, vc = 0;
        Delta delta{};
        if (k < dtot) {
          const int e = batch_find(B.doff, k);
          const int64_t arc = B.rp[e] + (k - B.doff[e]);
          const uint32_t cw = B.c[e];
          vc = cw & kBatchCol;
          const ColParams* cpd = A.cp + vc;
          v = A.col[arc];
          double inc = B.cv[e];
          if (!(cpd->flags & kAZero)) inc = inc * (A.arcfac != nullptr ? A.arcfac[arc] : cpd->da[A.nd[arc]]);
          T val = to_w(inc, T());
          if (cw & kBatchNeg) val = -val;
          emit = P::to_units(val, *cpd, &delta);
          if (!emit) atomicOr(A.err + (kServe ? vc : 0u), 1);
          if (binned && A.det_bins != nullptr) mark_det_bin<kG>(A, A.det_bins, v, vc);
        }
        emit_atomic(emit, v, vc, delta);
      }
      it_next = 0;
      it_total = B.ioff[kBatch];
    }
    // (c) idle lanes take sampled work items from the queue
    {
      const unsigned long long idle = __ballot(!active);
      if (!active) {
        const long long it = it_next + __popcll(idle & lt_mask);
        if (it < it_total) {
          const int e = it < kItemMap ? B.item_entry[it] : batch_find(B.ioff, it);
          const uint32_t il = static_cast<uint32_t>(it - B.ioff[e]);
          u = B.u[e];
          const uint32_t cw = B.c[e];
          c = cw & kBatchCol;
          rpu = B.rp[e];
          cv = B.cv[e];
          neg = (cw & kBatchNeg) != 0;
          const uint32_t J = B.J[e], d = B.d[e];
          cpp = A.cp + c;
          azero = (cw & kBatchAZero) != 0;
          th = B.th[e];
          ctr3 = B.ctr3[e];
          key0 = B.key0[e];
          key1 = B.key1[e];
          const uint32_t nwin = ((d - 1) >> kSegLog2) - (J >> kSegLog2) + 1;
          const uint32_t w0 = il * kWinPerItem;
          const uint32_t w1 = (w0 + kWinPerItem) < nwin ? w0 + kWinPerItem : nwin;
          const uint32_t ws = ((J >> kSegLog2) + w0) << kSegLog2;
          const uint32_t we = ((J >> kSegLog2) + w1) << kSegLog2;
          s = ws > J ? ws : J;
          rend = we < d ? we : d;
          if (azero)
            tab = make_skip_table(B.p0[e]);
          else  // the first run's factor when the entry's setup has it (else 0)
            dstart = il == 0 ? B.p0[e] : 0.0;
          run_end = 0;  // (the item has no run yet)
          active = true;
          need_run = true;
          it_cand = it_acc = it_runs = 0;
        }
      }
      it_next += __popcll(idle);
      if (it_next > it_total) it_next = it_total;
    }
    if (!__any(active)) {
      if (bnext >= nbatch) break;  // queue empty (no idle lane took an item), no batch left
      continue;
    }
    // (d) a run: the rest of the current window, or (a > 0) of its degree
    // group unless few candidates are expected over the rest of the window
    if (!kServe) w_runs += static_cast<uint32_t>(__popcll(__ballot(active && need_run)));
    if (active && need_run) {
      if (kServe) ++it_runs;
      const uint32_t wnext = ((s >> kSegLog2) + 1u) << kSegLog2;
      const uint32_t wend = wnext < rend ? wnext : rend;
      const bool first = run_end == 0;
      run_end = wend;
      if (!azero) {
        // the factor of the run's first arc (for an item's first run at the
        // row start, from the entry's setup); the group end only when the
        // run stops there
        if (!(first && dstart > 0.0))
          dstart = A.arcfac != nullptr ? A.arcfac[rpu + s] : cpp->da[A.nd[rpu + s]];
        const double num = cv * dstart;
        const double pr = num / th;
        if (!(pr * static_cast<double>(wend - s) <= kMergeCandidates)) {
          const uint32_t ge = A.gend[rpu + s];
          if (ge < wend) run_end = ge;
        }
        tab = make_skip_table(pr);
      }
      pos = s;
      t = 0;
      need_run = false;
    }
    // (e) one draw of the run's chain
    bool emit = false, cand_hit = false;
    uint32_t v = 0;
    Delta delta{};
    if (active && !need_run) {
      const U4 o = philox4x32_10(t, s, u, ctr3, key0, key1);
      const double V = unit_double(o.x, o.y);
      const uint32_t cand = pos + static_cast<uint32_t>(geometric_skip(tab, V));
      if (cand >= run_end) {
        s = run_end;
        need_run = true;
      } else {
        cand_hit = true;
        if (kServe) ++it_cand;
        const int64_t arc = rpu + cand;
        // the neighbour is loaded beside its factor degree, before the
        // acceptance test needs it (one round trip instead of two)
        const uint32_t va = A.col[arc];
        bool accept = true;  // a = 0: the ratio is 1 and every uniform is below it
        if (!azero) {
          const double ratio = (A.arcfac != nullptr ? A.arcfac[arc] : cpp->da[A.nd[arc]]) / dstart;
          accept = unit_double(o.z, o.w) < ratio;
        }
        if (accept) {
          if (kServe) ++it_acc;
          v = va;
          emit = true;
          delta = P::theta_units(*cpp, neg);
        }
        pos = cand + 1;
        ++t;
      }
    }
    if (!kServe) {
      w_cand += static_cast<uint32_t>(__popcll(__ballot(cand_hit)));
      w_acc += static_cast<uint32_t>(__popcll(__ballot(emit)));
    }
    emit_sampled(emit, v, c, delta, neg);
  }
  if (sparse) stage_flush(stage, staged, A.fout, A.cnt_out);
  if (binned) finish_records<kG>(A, s_hist, reinterpret_cast<uint32_t*>(stage), staged, acc_next);
  if (kServe) {  // flush the block's per-column sums
    __syncthreads();
    for (int i = threadIdx.x; i < kServeLdsSlots * kNumCounters; i += blockDim.x) {
      const unsigned long long cv2 = (&s_scnt[0][0])[i];
      if (cv2) atomicAdd(A.counters + i, cv2);
    }
    for (int i = threadIdx.x; i < kServeLdsSlots; i += blockDim.x)
      if (s_smass[i] != 0.0) atomicAdd(A.mass + i, s_smass[i]);
  }
  if (!kServe) {  // per-level counters: one atomic per wave
    unsigned long long* cnt = A.counters + static_cast<size_t>(A.level) * kNumCounters;
    const unsigned long long v0 = w_front;
    const unsigned long long v1 = wave_sum_u64(n_hash);
    const unsigned long long v2 = wave_sum_u64(n_det);
    const unsigned long long v3 = w_cand;
    const unsigned long long v4 = w_acc;
    const unsigned long long v5 = w_runs;
    double m = mass;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m += __shfl_down(m, off);
    if (lane == 0) {
      if (v0) atomicAdd(cnt + 0, v0);
      if (v1) atomicAdd(cnt + 1, v1);
      if (v2) atomicAdd(cnt + 2, v2);
      if (v3) atomicAdd(cnt + 3, v3);
      if (v4) atomicAdd(cnt + 4, v4);
      if (v5) atomicAdd(cnt + 5, v5);
      if (m != 0.0) atomicAdd(A.mass + A.level, m);
    }
  }
}

// ------------------------------------------------- deferred rows
// The deterministic pushes of the rows a level deferred, after its k_level
// launch: a wave takes kBigChunk consecutive pushes of the concatenated rows
// (lane l pushes l, l + 64, ...), finds its row once by binary search over
// the rows' offsets and moves to the next row when it crosses its end.  The
// pushes are computed and accumulated as in k_level (first contributions of
// a sparse level appended to the next frontier).
template <typename T, int kG = 1>
__global__ __launch_bounds__(kThreads) void k_det_big(LevelArgs A, typename Prec<T>::Cell* __restrict__ acc_next) {
  using P = Prec<T>;
  using Delta = typename P::Delta;
  constexpr int kWaves = kThreads / kWave;
  __shared__ uint64_t s_stage[kWaves][kStage];
  const unsigned long long ctr = *A.big_ctr;
  unsigned long long nb = ctr >> kBigShift;
  if (nb == 0) return;
  if (nb > A.big_cap) nb = A.big_cap;  // rows beyond the list were pushed by their waves
  const BigRow* R = A.big;
  const unsigned long long total = R[nb - 1].off + R[nb - 1].J;
  const bool sparse = *A.mode_out == kModeSparse;
  uint8_t* const det_bins = *A.mode_out == kModeBinned ? A.det_bins : nullptr;
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  uint64_t* stage = s_stage[wave];
  int staged = 0;  // wave-uniform
  const unsigned long long nchunks = (total + kBigChunk - 1) / kBigChunk;
  for (unsigned long long ch = static_cast<unsigned long long>(blockIdx.x) * kWaves + wave; ch < nchunks;
       ch += static_cast<unsigned long long>(gridDim.x) * kWaves) {
    unsigned long long k = ch * kBigChunk + lane;
    unsigned long long e = 0, hi = nb;  // last row with off <= k
    while (hi - e > 1) {
      const unsigned long long mid = (e + hi) >> 1;
      if (R[mid].off <= k)
        e = mid;
      else
        hi = mid;
    }
    unsigned long long off = R[e].off, next = e + 1 < nb ? R[e + 1].off : total;
    for (int j = 0; j < kBigChunk / kWave; ++j, k += kWave) {
      bool emit = false;
      uint32_t v = 0, vc = 0;
      Delta delta{};
      if (k < total) {
        while (k >= next) {
          ++e;
          off = next;
          next = e + 1 < nb ? R[e + 1].off : total;
        }
        const BigRow& br = R[e];
        vc = br.c;
        const ColParams* cpd = A.cp + vc;
        const int64_t arc = br.rp + static_cast<int64_t>(k - off);
        v = A.col[arc];
        double inc = br.cv;
        if (!(cpd->flags & kAZero)) inc = inc * (A.arcfac != nullptr ? A.arcfac[arc] : cpd->da[A.nd[arc]]);
        T val = to_w(inc, T());
        if (br.neg) val = -val;
        emit = P::to_units(val, *cpd, &delta);
        if (!emit) atomicOr(A.err, 1);
      }
      const size_t vcell = static_cast<size_t>(v) * A.su + static_cast<size_t>(vc) * A.sc;
      if (emit && det_bins != nullptr) mark_det_bin<kG>(A, det_bins, v, vc);
      bool first = false;
      if (emit) {
        if (sparse)
          first = P::add_ret(acc_next, vcell, delta);
        else
          P::add(acc_next, vcell, delta);
      }
      if (sparse) stage_push(stage, staged, (static_cast<uint64_t>(v) << 32) | vc, first, A.fout, A.cnt_out);
    }
  }
  if (sparse) stage_flush(stage, staged, A.fout, A.cnt_out);
}

// The sampled work items of the entries a level deferred, after its k_level
// launch: lane g takes items g, g + G, ... of the concatenated entries (G
// lanes in the grid), finds an item's entry by binary search over the
// entries' item offsets and walks its windows exactly as k_level does (the
// same runs, draws and acceptance tests, so the same pushes); the pushes
// are emitted as in k_level's mode for the level (records, first-touch
// appends or plain atomics), and the level's candidate and acceptance
// counters get this kernel's counts.
template <typename T, int kG = 1>
__global__ __launch_bounds__(kThreads) void k_samp_big(LevelArgs A, typename Prec<T>::Cell* __restrict__ acc_next) {
  using P = Prec<T>;
  using Delta = typename P::Delta;
  constexpr int kWaves = kThreads / kWave;
  __shared__ uint64_t s_stage[kWaves][kStage];
  __shared__ unsigned int s_hist[kBuckets];
  const unsigned long long ctr = *A.samp_ctr;
  unsigned long long nb = ctr >> kBigShift;
  if (nb == 0) return;  // the whole grid
  if (nb > A.big_cap) nb = A.big_cap;  // entries beyond the list kept their items
  const BigSamp* R = A.samp;
  const unsigned long long total = R[nb - 1].off + R[nb - 1].items;
  const int mode = *A.mode_out;
  const bool binned = mode == kModeBinned;
  const bool sparse = mode == kModeSparse;
  if (binned) {
    for (int i = threadIdx.x; i < kBuckets; i += blockDim.x) s_hist[i] = 0;
    __syncthreads();
  }
  const int wave = threadIdx.x / kWave;
  uint64_t* stage = s_stage[wave];
  int staged = 0;  // wave-uniform
  unsigned long long n_cand = 0, n_acc = 0, n_runs = 0;
  const unsigned long long G = static_cast<unsigned long long>(gridDim.x) * blockDim.x;
  unsigned long long next = static_cast<unsigned long long>(blockIdx.x) * blockDim.x + threadIdx.x;

  bool active = false, need_run = false, neg = false, azero = true;
  uint32_t u = 0, c = 0, s = 0, rend = 0, run_end = 0, pos = 0, t = 0, ctr3 = 0, key0 = 0, key1 = 0;
  int64_t rpu = 0;
  double cv = 0.0, dstart = 1.0, th = 0.0;
  const ColParams* cpp = A.cp;
  SkipTable tab;
  for (;;) {
    if (active && need_run && s >= rend) active = false;
    if (!active && next < total) {  // the lane's next item
      unsigned long long e = 0, hi = nb;  // last entry with off <= next
      while (hi - e > 1) {
        const unsigned long long mid = (e + hi) >> 1;
        if (R[mid].off <= next)
          e = mid;
        else
          hi = mid;
      }
      const BigSamp& bs = R[e];
      const uint32_t il = static_cast<uint32_t>(next - bs.off);
      next += G;
      u = bs.u;
      c = bs.c;
      rpu = bs.rp;
      cv = bs.cv;
      neg = bs.neg != 0;
      const uint32_t J = bs.J, d = bs.d;
      cpp = A.cp + c;
      azero = (cpp->flags & kAZero) != 0;
      th = cpp->theta;
      ctr3 = (cpp->qid << 8) | static_cast<uint32_t>(cpp->level);
      key0 = cpp->key0;
      key1 = cpp->key1;
      const uint32_t nwin = ((d - 1) >> kSegLog2) - (J >> kSegLog2) + 1;
      const uint32_t w0 = il * kWinPerItem;
      const uint32_t w1 = (w0 + kWinPerItem) < nwin ? w0 + kWinPerItem : nwin;
      const uint32_t ws = ((J >> kSegLog2) + w0) << kSegLog2;
      const uint32_t we = ((J >> kSegLog2) + w1) << kSegLog2;
      s = ws > J ? ws : J;
      rend = we < d ? we : d;
      if (azero) tab = make_skip_table(bs.p0);
      active = true;
      need_run = true;
    }
    if (!__any(active)) break;
    if (active && need_run) {  // a run, as in k_level
      ++n_runs;
      const uint32_t wnext = ((s >> kSegLog2) + 1u) << kSegLog2;
      const uint32_t wend = wnext < rend ? wnext : rend;
      run_end = wend;
      if (!azero) {
        // the group end is loaded beside the factor degree (one round trip)
        const uint32_t ge = A.gend[rpu + s];
        dstart = A.arcfac != nullptr ? A.arcfac[rpu + s] : cpp->da[A.nd[rpu + s]];
        const double num = cv * dstart;
        const double pr = num / th;
        if (!(pr * static_cast<double>(wend - s) <= kMergeCandidates) && ge < wend) run_end = ge;
        tab = make_skip_table(pr);
      }
      pos = s;
      t = 0;
      need_run = false;
    }
    bool emit = false;
    uint32_t v = 0;
    Delta delta{};
    if (active && !need_run) {  // one draw, as in k_level
      const U4 o = philox4x32_10(t, s, u, ctr3, key0, key1);
      const double V = unit_double(o.x, o.y);
      const uint32_t cand = pos + static_cast<uint32_t>(geometric_skip(tab, V));
      if (cand >= run_end) {
        s = run_end;
        need_run = true;
      } else {
        ++n_cand;
        const int64_t arc = rpu + cand;
        const uint32_t va = A.col[arc];  // beside the factor degree, as in k_level
        bool accept = true;
        if (!azero) {
          const double ratio = (A.arcfac != nullptr ? A.arcfac[arc] : cpp->da[A.nd[arc]]) / dstart;
          accept = unit_double(o.z, o.w) < ratio;
        }
        if (accept) {
          ++n_acc;
          v = va;
          emit = true;
          delta = P::theta_units(*cpp, neg);
        }
        pos = cand + 1;
        ++t;
      }
    }
    if (binned) {
      emit_record<kG>(A, s_hist, reinterpret_cast<uint32_t*>(stage), staged, emit, v, c, neg, acc_next);
    } else {
      const size_t vcell = static_cast<size_t>(v) * A.su + static_cast<size_t>(c) * A.sc;
      bool first = false;
      if (emit) {
        if (sparse)
          first = P::add_ret(acc_next, vcell, delta);
        else
          P::add(acc_next, vcell, delta);
      }
      if (sparse) stage_push(stage, staged, (static_cast<uint64_t>(v) << 32) | c, first, A.fout, A.cnt_out);
    }
  }
  if (sparse) stage_flush(stage, staged, A.fout, A.cnt_out);
  if (binned) finish_records<kG>(A, s_hist, reinterpret_cast<uint32_t*>(stage), staged, acc_next);
  unsigned long long* cnt = A.counters + static_cast<size_t>(A.level) * kNumCounters;
  const unsigned long long v3 = wave_sum_u64(n_cand);
  const unsigned long long v4 = wave_sum_u64(n_acc);
  const unsigned long long v5 = wave_sum_u64(n_runs);
  if (lane_id() == 0) {
    if (v3) atomicAdd(cnt + 3, v3);
    if (v4) atomicAdd(cnt + 4, v4);
    if (v5) atomicAdd(cnt + 5, v5);
  }
}

// ------------------------------------------------- push estimate
// An upper bound on the pushes of a level (deterministic rows count d_u,
// sampled rows their expected d_u c / theta with c = rho |r| d_u^-b), summed
// over the frontier (over a sample of it when it is large): decides whether
// the level is worth binning.
template <typename T, bool kFirst>
__global__ __launch_bounds__(kThreads) void k_estimate(LevelArgs A, const T* __restrict__ x,
                                                       const typename Prec<T>::Cell* __restrict__ acc_cur,
                                                       double* __restrict__ est) {
  __shared__ double s_part[kThreads / kWave];
  const unsigned long long count = *A.cnt_in;
  // large frontiers: an evenly spaced sample of 2^20 to 2^21 entries, scaled
  // up (the estimate only chooses between interchangeable aggregation modes)
  const unsigned long long stride = count >= (1ull << 21) ? count >> 20 : 1ull;
  double sum = 0.0;
  for (unsigned long long j = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; j * stride < count;
       j += (unsigned long long)gridDim.x * blockDim.x) {
    uint32_t u, c;
    if (kFirst && A.fin == nullptr) {  // every cell (see kVirtualMaxC)
      const unsigned long long e = j * stride;
      u = static_cast<uint32_t>(e / static_cast<unsigned long long>(A.su));
      c = static_cast<uint32_t>(e - static_cast<unsigned long long>(u) * static_cast<unsigned long long>(A.su));
    } else {
      const uint64_t item = A.fin[j * stride];
      u = static_cast<uint32_t>(item >> 32);
      c = static_cast<uint32_t>(item);
    }
    const ColParams& cp = A.cp[c];
    if ((cp.flags & (kDrop | kLastLevel)) || cp.rho == 0.0) continue;
    const uint32_t d = static_cast<uint32_t>(A.deg[u]);
    if (d == 0) continue;
    const size_t cell = static_cast<size_t>(u) * A.su + static_cast<size_t>(c) * A.sc;
    double absr;
    if (kFirst) {
      absr = fabs(static_cast<double>(x[static_cast<size_t>(u) * static_cast<size_t>(A.xld) + c]));
    } else if (sizeof(T) == 4) {
      const long long K = reinterpret_cast<const long long*>(acc_cur)[cell];
      absr = fabs(static_cast<double>(K)) / cp.scale;
    } else {
      absr = 0.0;  // binary64 calls are never binned
    }
    const double cv = cp.rho * absr * cp.db[A.fdeg[u]];
    sum += cv >= cp.theta ? static_cast<double>(d) : static_cast<double>(d) * (cv / cp.theta);
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) sum += __shfl_down(sum, off);
  if (lane_id() == 0) s_part[threadIdx.x / kWave] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {  // one atomic per block
    double b = 0.0;
    for (int w = 0; w < kThreads / kWave; ++w) b += s_part[w];
    if (b != 0.0) atomicAdd(est, b * static_cast<double>(stride));
  }
}

// ------------------------------------------------- frontier compaction
// (u << 32 | c) of every cell u * C + c of a row-major n x C array whose
// predicate holds.  Every chunk that goes out costs one atomic on the list
// counter, a round trip to one shared address that all waves contend for,
// so chunks are made large: a wave takes segments of seg consecutive cells
// (a multiple of kCompactUnroll x 64, at most kCompactSeg: large arrays take
// the largest, small ones smaller segments so that every CU has waves),
// issues kCompactUnroll loads of 64 cells together, and stages the passing
// cells as 2-byte offsets into its segment (up to kCompactCap of them, 8 KiB
// of LDS per wave); a chunk goes out when the stage is nearly full and at the
// end of each segment, in cell order.  Rows and columns of the staged cells
// are formed when they go out, from one 64-bit division per segment and a
// float-reciprocal division corrected to the exact quotient per entry.
constexpr int kCompactUnroll = 16;
constexpr int kCompactCap = 4096;
constexpr long long kCompactSeg = 1ll << 16;  // the largest segment: offsets fit in 16 bits
static_assert(kCompactSeg % (kCompactUnroll * kWave) == 0, "segments hold whole load groups");

// The staged offsets of a segment that starts at row u0, column r0: one
// atomic for the chunk, then the items in staging order.  Wave-uniform.
__device__ __forceinline__ void compact_flush(const uint16_t* stage, int& staged, long long u0, uint32_t r0,
                                              uint32_t C, float rc, bool small, uint64_t* __restrict__ F,
                                              unsigned long long* __restrict__ cnt) {
  if (staged == 0) return;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  unsigned long long base = 0;
  if (lane_id() == 0) base = atomicAdd(cnt, static_cast<unsigned long long>(staged));
  base = __shfl(base, 0);
  for (int i = lane_id(); i < staged; i += kWave) {
    const uint32_t a = r0 + stage[i];  // < C + kCompactSeg
    uint32_t c = 0, q = 0;
    if (small) {
      q = div_small(a, C, rc, &c);
    } else {
      q = a / C;
      c = a - q * C;
    }
    F[base + i] = (static_cast<uint64_t>(u0 + q) << 32) | c;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  staged = 0;
}

template <typename Pred>
__global__ __launch_bounds__(kThreads) void k_compact(Pred pred, int64_t n, int C, long long seg,
                                                      uint64_t* __restrict__ F, unsigned long long* __restrict__ cnt,
                                                      const int* __restrict__ mode) {
  if (mode && *mode != kModeCompact && *mode != kModeOverflow) return;  // formed elsewhere
  constexpr int kWaves = kThreads / kWave;
  __shared__ uint16_t s_stage[kWaves][kCompactCap];
  const int lane = lane_id();
  uint16_t* stage = s_stage[threadIdx.x / kWave];
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
  const long long total = static_cast<long long>(n) * C;
  const float rc = 1.0f / static_cast<float>(C);
  const bool small = C <= (1 << 21);  // div_small's range: C + kCompactSeg < 2^22
  const long long wave = static_cast<long long>(blockIdx.x) * kWaves + threadIdx.x / kWave;
  const long long nwaves = static_cast<long long>(gridDim.x) * kWaves;
  for (long long base = wave * seg; base < total; base += nwaves * seg) {
    const long long u0 = base / C;
    const uint32_t r0 = static_cast<uint32_t>(base - u0 * C);
    int staged = 0;  // wave-uniform
    for (int j = 0; j < seg && base + j < total; j += kCompactUnroll * kWave) {
      // the index is clamped instead of guarded, so that the loads carry no
      // branch and go out together
      bool p[kCompactUnroll];
#pragma unroll
      for (int k = 0; k < kCompactUnroll; ++k) {
        const long long i = base + j + k * kWave + lane;
        const bool in = i < total;
        p[k] = pred(0, 0, static_cast<size_t>(in ? i : total - 1)) && in;
      }
#pragma unroll
      for (int k = 0; k < kCompactUnroll; ++k) {
        const unsigned long long m = __ballot(p[k]);
        if (p[k]) stage[staged + __popcll(m & lt_mask)] = static_cast<uint16_t>(j + k * kWave + lane);
        staged += __popcll(m);
        if (staged > kCompactCap - kWave) compact_flush(stage, staged, u0, r0, C, rc, small, F, cnt);
      }
    }
    compact_flush(stage, staged, u0, r0, C, rc, small, F, cnt);
  }
}

template <typename T>
struct NonZeroCell {
  const typename Prec<T>::Cell* acc;
  __device__ bool operator()(int64_t, int64_t, size_t cell) const { return Prec<T>::nonzero(acc, cell); }
};

inline unsigned grid_for(int64_t items, int threads, int64_t cap = 65536) {
  int64_t b = (items + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return static_cast<unsigned>(b);
}

}  // namespace lvl
}  // namespace agp
