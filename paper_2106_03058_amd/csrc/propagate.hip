// Batched randomized propagation (Algorithm 2 of "Approximate Graph
// Propagation", Section 4): C signal columns advance level by level together.
//
// State of a call (row-major n x C, cell = u * C + c):
//   x        the signal, which is also the level-0 residue r^(0)
//   out      the estimate pi_hat, accumulated level by level
//   acc[2]   next-level residues as exact integers of a per-column unit
//            (binary32: int64 cells; binary64: 128-bit cells), ping-ponged
//   F[2]     frontier lists of (u << 32 | c) with non-zero residue
// One k_level launch per level (level_kernels.h); the per-column parameters of
// the level are written by k_set_level.  Non-negative signals append sparse
// frontiers directly; denser frontiers are compacted by a wave-ballot pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <initializer_list>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <type_traits>
#include <vector>

#include "agp_internal.h"
#include "bin_kernels.h"
#include "dense_kernels.h"
#include "level_kernels.h"

namespace agp {
namespace {

// query-id offset of the x- part of a column under the literal sign split
constexpr uint32_t kSplitQid = 1u << 23;

using namespace lvl;

// ---------------------------------------------------------- thresholds
// ||x_c||_1 in binary64: sequential over blocks of 4096 rows, then over the
// block sums.  flags: 1 = non-finite entry, 2 = negative entry.  The same
// pass forms the level-0 frontier (the non-zero cells of x, in any order).
// One wave per (row block, 64 columns); loads are issued 32 rows at a time
// and summed in row order; the frontier goes out in chunks of up to kCap
// entries (one atomic on the shared list counter each).
constexpr int kThetaBatch = 32;
constexpr int kThetaCap = 4096;  // 32 KiB of LDS per wave

__global__ void k_set_u64(unsigned long long* p, unsigned long long v) { *p = v; }

// kList: append the non-zero cells to F (the level-0 frontier); else only
// count them in *cnt (a mostly non-zero signal needs no list).
template <typename T, int kCap, bool kList>
__global__ __launch_bounds__(kWave) void k_theta_partial(const T* __restrict__ x, long long ldx, int64_t n, int C,
                                                         double* __restrict__ partial, int* __restrict__ flags,
                                                         uint64_t* __restrict__ F, unsigned long long* __restrict__ cnt) {
  __shared__ uint64_t s_stage[kList ? kCap : 1];
  const int c = blockIdx.y * blockDim.x + threadIdx.x;
  const bool live = c < C;
  const int64_t lo = (int64_t)blockIdx.x * kThetaRows;
  const int64_t hi = (lo + kThetaRows) < n ? lo + kThetaRows : n;
  double sum = 0.0;
  int f = 0;
  int staged = 0;  // wave-uniform
  for (int64_t i0 = lo; i0 < hi; i0 += kThetaBatch) {
    T v[kThetaBatch];
#pragma unroll
    for (int k = 0; k < kThetaBatch; ++k)
      v[k] = (live && i0 + k < hi) ? x[static_cast<size_t>(i0 + k) * static_cast<size_t>(ldx) + c] : T(0);
#pragma unroll
    for (int k = 0; k < kThetaBatch; ++k) {
      if (i0 + k >= hi) continue;  // wave-uniform
      if (!isfinite(static_cast<double>(v[k]))) f |= 1;
      if (v[k] < T(0)) f |= 2;
      sum = sum + fabs(static_cast<double>(v[k]));
      if constexpr (kList)
        stage_push<kCap>(s_stage, staged, (static_cast<uint64_t>(i0 + k) << 32) | static_cast<uint32_t>(c),
                         v[k] != T(0), F, cnt);
      else
        staged += __popcll(__ballot(v[k] != T(0)));
    }
  }
  if constexpr (kList)
    stage_flush(s_stage, staged, F, cnt);
  else if (staged > 0 && lane_id() == 0)
    atomicAdd(cnt, static_cast<unsigned long long>(staged));
  if (live) partial[(size_t)blockIdx.x * C + c] = sum;
  if (f) atomicOr(flags, f);
}

// Adds the 64 lanes' values of v to sum in lane order (wave-uniform sum).
__device__ __forceinline__ double add_lanes_in_order(double sum, double v) {
  const uint64_t b = static_cast<uint64_t>(__double_as_longlong(v));
  const uint32_t lo = static_cast<uint32_t>(b), hi = static_cast<uint32_t>(b >> 32);
#pragma unroll 16
  for (int j = 0; j < kWave; ++j) {
    const uint64_t bj = (static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readlane(hi, j))) << 32) |
                        static_cast<uint32_t>(__builtin_amdgcn_readlane(lo, j));
    sum = sum + __longlong_as_double(static_cast<long long>(bj));
  }
  return sum;
}

// Exponent of the lowest set bit of a finite a > 0: a is an integer multiple
// of 2^low_exp(a).
__device__ __forceinline__ int low_exp(double a) {
  const uint64_t b = static_cast<uint64_t>(__double_as_longlong(a));
  const int e = static_cast<int>(b >> 52) & 0x7ff;
  uint64_t m = b & ((1ull << 52) - 1);
  if (e) m |= 1ull << 52;
  return (e ? e : 1) - 1075 + __builtin_ctzll(m);
}

// Sum of non-negative values spread over the wave (lane partial sums s, each
// lane's smallest low_exp m, INT_MAX for none), if it is exact.  When every
// value is an integer multiple of 2^m and the exact total is below 2^(m+53),
// every partial sum, in any order, is such a multiple below 2^(m+53) and so a
// binary64 number: each addition is exact and every order of additions, the
// sequential one included, gives the exact total.  An inexact addition would
// round up to at least 2^(m+53), and the additions after it keep the total
// there, so a computed total below that bound proves exactness.  Returns false
// (and the caller adds in order) otherwise, also for non-finite values.
__device__ __forceinline__ bool wave_exact_sum(double s, int m, double& total) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    s = s + __shfl_xor(s, off);
    const int mo = __shfl_xor(m, off);
    m = mo < m ? mo : m;
  }
  const uint64_t sb = static_cast<uint64_t>(__double_as_longlong(s));
  const uint64_t ub = (static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(
                           static_cast<uint32_t>(sb >> 32)))) << 32) |
                      static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(sb)));
  total = __longlong_as_double(static_cast<long long>(ub));
  m = __builtin_amdgcn_readfirstlane(m);
  if (m == INT_MAX) return total == 0.0;
  return total < ldexp(1.0, m + 53);
}

// k_theta_partial for one column (C = 1): the lanes load all 4096 rows of the
// block at once (row lo + 64 k + lane in v[k]); the block's sum is the exact
// one when wave_exact_sum proves it, else the wave adds the rows one by one in
// row order.  Either way it is the sequential sum of k_theta_partial; the
// frontier entries are the same (u << 32).
template <typename T, bool kList>
__global__ __launch_bounds__(kWave) void k_theta_partial_c1(const T* __restrict__ x, long long ldx, int64_t n,
                                                            double* __restrict__ partial, int* __restrict__ flags,
                                                            uint64_t* __restrict__ F,
                                                            unsigned long long* __restrict__ cnt) {
  __shared__ uint64_t s_stage[kList ? kThetaCap : 1];
  constexpr int kLoads = kThetaRows / kWave;
  const int lane = lane_id();
  const int64_t lo = (int64_t)blockIdx.x * kThetaRows;
  const int64_t hi = (lo + kThetaRows) < n ? lo + kThetaRows : n;
  T v[kLoads];
#pragma unroll
  for (int k = 0; k < kLoads; ++k) {
    const int64_t i = lo + k * kWave + lane;
    v[k] = i < hi ? x[static_cast<size_t>(i) * static_cast<size_t>(ldx)] : T(0);  // +0 past the end
  }
  double s = 0.0;
  int m = INT_MAX;
  int f = 0;
  int staged = 0;  // wave-uniform
#pragma unroll
  for (int k = 0; k < kLoads; ++k) {
    if (!isfinite(static_cast<double>(v[k]))) f |= 1;
    if (v[k] < T(0)) f |= 2;
    const double a = fabs(static_cast<double>(v[k]));
    s = s + a;
    if (a != 0.0) {
      const int e = low_exp(a);
      m = e < m ? e : m;
    }
    if constexpr (kList)
      stage_push<kThetaCap>(s_stage, staged, static_cast<uint64_t>(lo + k * kWave + lane) << 32, v[k] != T(0), F,
                            cnt);
    else
      staged += __popcll(__ballot(v[k] != T(0)));
  }
  double sum;
  if (!wave_exact_sum(s, m, sum)) {
    sum = 0.0;
#pragma unroll
    for (int k = 0; k < kLoads; ++k) sum = add_lanes_in_order(sum, fabs(static_cast<double>(v[k])));
  }
  if constexpr (kList)
    stage_flush(s_stage, staged, F, cnt);
  else if (staged > 0 && lane == 0)
    atomicAdd(cnt, static_cast<unsigned long long>(staged));
  if (lane == 0) partial[blockIdx.x] = sum;
  if (f) atomicOr(flags, f);
}

// The same sums as k_theta_partial without forming a frontier; counts the
// non-zero entries of x instead (their share decides the dense path).
template <typename T>
__global__ __launch_bounds__(kWave) void k_theta_scan(const T* __restrict__ x, long long ldx, int64_t n, int C,
                                                      double* __restrict__ partial, int* __restrict__ flags,
                                                      unsigned long long* __restrict__ nnz) {
  const int c = blockIdx.y * blockDim.x + threadIdx.x;
  const bool live = c < C;
  const int64_t lo = (int64_t)blockIdx.x * kThetaRows;
  const int64_t hi = (lo + kThetaRows) < n ? lo + kThetaRows : n;
  double sum = 0.0;
  int f = 0;
  unsigned long long cnt = 0;
  for (int64_t i0 = lo; i0 < hi; i0 += kThetaBatch) {
    T v[kThetaBatch];
#pragma unroll
    for (int k = 0; k < kThetaBatch; ++k)
      v[k] = (live && i0 + k < hi) ? x[static_cast<size_t>(i0 + k) * static_cast<size_t>(ldx) + c] : T(0);
#pragma unroll
    for (int k = 0; k < kThetaBatch; ++k) {
      if (i0 + k >= hi) break;  // wave-uniform
      if (!isfinite(static_cast<double>(v[k]))) f |= 1;
      if (v[k] < T(0)) f |= 2;
      sum = sum + fabs(static_cast<double>(v[k]));
      cnt += v[k] != T(0) ? 1ull : 0ull;
    }
  }
  if (live) partial[(size_t)blockIdx.x * C + c] = sum;
  if (f) atomicOr(flags, f);
  const unsigned long long tot = wave_sum_u64(cnt);
  if (lane_id() == 0 && tot) atomicAdd(nnz, tot);
}

// nnz_out (if not null) receives *nnz_in, so that one copy to the host
// brings the signal flags and the count of non-zero cells together.
template <typename T>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_theta_final(const double* __restrict__ partial, int64_t nblocks, int C, double eps,
                              const uint32_t* __restrict__ qids, uint32_t qid_base, ColParams* __restrict__ cp,
                              const unsigned long long* __restrict__ nnz_in = nullptr,
                              unsigned long long* __restrict__ nnz_out = nullptr) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0 && nnz_out != nullptr) *nnz_out = *nnz_in;
  double total = 0.0;
  if (C == 1) {  // one wave: lane l loads block b0 + 64 k + l
    constexpr int kInFlight = 16;
    double s = 0.0;
    int m = INT_MAX;
    for (int64_t b0 = 0; b0 < nblocks; b0 += kInFlight * kWave) {
      double v[kInFlight];
#pragma unroll
      for (int k = 0; k < kInFlight; ++k) {
        const int64_t b = b0 + k * kWave + threadIdx.x;
        v[k] = b < nblocks ? partial[b] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < kInFlight; ++k) {
        s = s + v[k];
        if (v[k] != 0.0) {
          const int e = low_exp(v[k]);
          m = e < m ? e : m;
        }
      }
    }
    if (!wave_exact_sum(s, m, total)) {  // add in block order
      total = 0.0;
      for (int64_t b0 = 0; b0 < nblocks; b0 += kInFlight * kWave) {
        double v[kInFlight];
#pragma unroll
        for (int k = 0; k < kInFlight; ++k) {
          const int64_t b = b0 + k * kWave + threadIdx.x;
          v[k] = b < nblocks ? partial[b] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kInFlight; ++k) total = add_lanes_in_order(total, v[k]);
      }
    }
  }
  if (c >= C) return;
  if (C > 1) {  // one lane per column, in block order
    constexpr int kInFlight = 64;  // loads issued together
    int64_t b = 0;
    for (; b + kInFlight <= nblocks; b += kInFlight) {
      double v[kInFlight];
#pragma unroll
      for (int k = 0; k < kInFlight; ++k) v[k] = partial[(size_t)(b + k) * C + c];
#pragma unroll
      for (int k = 0; k < kInFlight; ++k) total = total + v[k];
    }
    for (; b < nblocks; ++b) total = total + partial[(size_t)b * C + c];
  }
  ColParams p = cp[c];
  p.theta = eps * total;
  p.qid = qids ? qids[c] : qid_base + static_cast<uint32_t>(c);
  if (sizeof(T) == 4) {
    const float tw = static_cast<float>(p.theta);
    int ue = -149;
    if (tw > 0.0f) {
      const int e = ilog2_f64(static_cast<double>(tw));
      ue = e - 23 < -149 ? -149 : e - 23;
    }
    p.ue = ue;
    p.scale = ldexp(1.0, -ue);
    p.dtheta = static_cast<long long>(static_cast<double>(tw) * p.scale);
    p.theta_w = tw;
  } else {
    int ue = -1074;
    if (p.theta > 0.0) {
      const int e = ilog2_f64(p.theta);
      ue = e - 52 < -1074 ? -1074 : e - 52;
    }
    p.ue = ue;
    p.scale = 0.0;
    U128 d;
    f64_to_units(p.theta, ue, &d);
    p.dtheta = static_cast<long long>(d.lo);  // theta < 2^53 units
    p.theta_w = static_cast<float>(p.theta);
  }
  cp[c] = p;
}

// Level-dependent parameters of every column of a batched call.
// Per-level values of a call, in device memory so that a captured level
// loop serves every call with the same buffers.
struct LevelParams {
  double rho, kappa;
  int flags;
  uint32_t key0, key1;
  int pad;
};

__global__ void k_set_level(ColParams* __restrict__ cp, int C, int level, const LevelParams* __restrict__ lp,
                            const double* da, const double* db, void* out, long long out_stride, size_t elem) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  ColParams& p = cp[c];
  const LevelParams q = lp[level];
  p.level = level;
  p.rho = q.rho;
  p.kappa = q.kappa;
  p.flags = q.flags;
  p.da = da;
  p.db = db;
  p.key0 = q.key0;
  p.key1 = q.key1;
  p.out = static_cast<char*>(out) + static_cast<size_t>(c) * elem;
  p.out_stride = out_stride;
}

// Per node u: d_u^-b (its factor degree's entry) and the d^-a of its first
// neighbour in the degree-sorted row (0 for a node without arcs).
__global__ void k_node_factors(const int64_t* __restrict__ rp, const int32_t* __restrict__ deg,
                               const int32_t* __restrict__ fdeg, const uint32_t* __restrict__ nd,
                               const double* __restrict__ da, const double* __restrict__ db, int64_t n,
                               double2* __restrict__ out) {
  for (int64_t u = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; u < n;
       u += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[u] = make_double2(db[fdeg[u]], deg[u] > 0 ? da[nd[rp[u]]] : 0.0);
}

// Per arc j: d^-a of its neighbour (the factor degree nd[j]).
__global__ void k_arc_factors(const uint32_t* __restrict__ nd, const double* __restrict__ da, int64_t nnz,
                              double* __restrict__ out) {
  for (int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < nnz;
       j += static_cast<int64_t>(gridDim.x) * blockDim.x)
    out[j] = da[nd[j]];
}

// ------------------------------------------------------------ driver
constexpr int kSparseShift = 5;  // sparse levels: frontier below n C / 32
constexpr int kBinShift = 3;     // binned levels: estimated pushes reach n C / 8

agp_tuning_t default_tuning() {
  agp_tuning_t t{};
  t.aggregation = 2;  // records on levels with many pushes, atomics elsewhere
  t.level_blocks = kLevelBlocks;
  t.dense = 0;  // frontier lists: only the active (node, column) entries are visited
  t.tile_columns = 0;
  t.big_row = static_cast<int32_t>(kBigRow);
  t.big_items = static_cast<int32_t>(kBigItems);
  t.sparse_shift = kSparseShift;
  t.bin_shift = kBinShift;
  t.capture = 0;
  return t;
}

// Zero fields of a caller's tuning take the defaults; out-of-range values
// are clamped.
agp_tuning_t normalize_tuning(agp_tuning_t t) {
  const agp_tuning_t d = default_tuning();
  if (t.aggregation < 0 || t.aggregation > 2) t.aggregation = d.aggregation;
  if (t.level_blocks < 256) t.level_blocks = t.level_blocks <= 0 ? d.level_blocks : 256;
  if (t.level_blocks > 65536) t.level_blocks = 65536;
  if (t.dense < 0 || t.dense > 2) t.dense = d.dense;
  if (t.tile_columns < 0) t.tile_columns = 0;
  if (t.big_row <= 0) t.big_row = d.big_row;
  if (t.big_items <= 0) t.big_items = d.big_items;
  if (t.sparse_shift <= 0 || t.sparse_shift > 30) t.sparse_shift = d.sparse_shift;
  if (t.bin_shift <= 0 || t.bin_shift > 30) t.bin_shift = d.bin_shift;
  if (t.capture != 1) t.capture = 0;
  return t;
}

// The tuning in force for a call: an explicit one, else the autotuned one,
// else the default; environment variables (include/agp.h) override single
// fields.
agp_tuning_t tuning_for(agp_graph* g, int32_t C, double a, double b, const agp_tuning_t* force) {
  agp_tuning_t t = default_tuning();
  if (force) {
    t = *force;
  } else {
    auto it = g->tuning.find(agp_tune_key{C, a, b});
    if (it != g->tuning.end()) {
      t = it->second;
    } else if (static_cast<long long>(g->n) * C >= (1ll << 31)) {
      // calls of 2^31 cells and more: twice the level kernel's workgroups
      // (finer batches for the slowest waves; 2% on a 111M x 128 call)
      t.level_blocks = 2 * kLevelBlocks;
    }
  }
  t = normalize_tuning(t);
  if (const char* e = std::getenv("AGP_AGGREGATION")) {
    if (std::strcmp(e, "atomic") == 0) t.aggregation = 0;
    if (std::strcmp(e, "binned") == 0) t.aggregation = 1;
    if (std::strcmp(e, "auto") == 0) t.aggregation = 2;
  }
  if (const char* e = std::getenv("AGP_DENSE")) {
    if (std::strcmp(e, "0") == 0) t.dense = 0;
    if (std::strcmp(e, "1") == 0) t.dense = 1;
    if (std::strcmp(e, "auto") == 0) t.dense = 2;
  }
  if (const char* e = std::getenv("AGP_CAPTURE")) {
    if (std::strcmp(e, "0") == 0) t.capture = 0;
    if (std::strcmp(e, "1") == 0) t.capture = 1;
  }
  if (const char* e = std::getenv("AGP_COLUMN_TILE")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v > 0) t.tile_columns = static_cast<int32_t>(v);
  }
  if (const char* e = std::getenv("AGP_BIG_ITEMS")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v >= 1) t.big_items = static_cast<int32_t>(v);
  }
  return t;
}

// One tile of C columns: x and out point at the tile's first column, rows
// ldc apart; column c of the tile is column qid_base + c of the call (its
// qid when qids is null).  Levels are timed when stats is non-null (the
// tile's counters and times are added to it).  The caller holds g->mu and
// has zeroed out.
template <typename T>
int propagate_tile(agp_graph* g, const char* fn, const agp_tuning_t& tune, double a, double b, const double* rho,
                   const double* kappa, int32_t L, const T* x, long long ldc, int32_t C, double eps, uint64_t seed,
                   const uint32_t* qids, uint32_t qid_base, T* out, hipStream_t s, agp_stats_t* stats, Scratch& sc,
                   bool may_alloc) {
  using Cell = typename Prec<T>::Cell;
  const int64_t n = g->n;
  const size_t cells = static_cast<size_t>(n) * static_cast<size_t>(C);
  int rc;
  const double *da = nullptr, *db = nullptr;
  if ((rc = pow_table(g, a, &da, may_alloc)) || (rc = pow_table(g, b, &db, may_alloc))) return rc;
  const size_t cell_bytes = sizeof(Cell) * (sizeof(T) == 4 ? 1 : 2);
  const int64_t tblocks = (n + kThetaRows - 1) / kThetaRows;
  if ((rc = sc.acc[0].reserve(cells * cell_bytes, true, s)) ||
      (rc = sc.acc[1].reserve(cells * cell_bytes, true, s)) ||
      (rc = sc.frontier[0].reserve(cells * sizeof(uint64_t), false, s)) ||
      (rc = sc.frontier[1].reserve(cells * sizeof(uint64_t), false, s)) ||
      (rc = sc.counts.reserve(sizeof(unsigned long long) * (AGP_MAX_LEVELS + 2), false, s)) ||
      (rc = sc.counters.reserve(sizeof(unsigned long long) * kNumCounters * (AGP_MAX_LEVELS + 1), false, s)) ||
      (rc = sc.colparams.reserve(sizeof(ColParams) * C + sizeof(uint32_t) * C, false, s)) ||
      (rc = sc.partial.reserve(sizeof(double) * (size_t)std::max<int64_t>(tblocks, 1) * C, false, s)) ||
      (rc = sc.flags.reserve(sizeof(int) * 4, false, s)) ||
      (rc = sc.levelinfo.reserve((2 * sizeof(double) + sizeof(int)) * (AGP_MAX_LEVELS + 2) + 256 +
                                     sizeof(LevelParams) * (AGP_MAX_LEVELS + 1),
                                 false, s)))
    return rc;

  ColParams* cp = sc.colparams.as<ColParams>();
  uint32_t* dq = reinterpret_cast<uint32_t*>(cp + C);
  unsigned long long* counts = sc.counts.as<unsigned long long>();
  unsigned long long* counters = sc.counters.as<unsigned long long>();
  int* flags = sc.flags.as<int>();
  double* mass = sc.levelinfo.as<double>();
  double* est = mass + AGP_MAX_LEVELS + 2;  // estimated pushes per level (auto aggregation)
  int* mode = reinterpret_cast<int*>(est + AGP_MAX_LEVELS + 2);
  LevelParams* lpd = reinterpret_cast<LevelParams*>(
      (reinterpret_cast<uintptr_t>(mode + AGP_MAX_LEVELS + 2) + 255) & ~static_cast<uintptr_t>(255));
  AGP_HIP(hipMemsetAsync(sc.levelinfo.ptr, 0, sc.levelinfo.bytes, s));
  AGP_HIP(hipMemsetAsync(counts, 0, sc.counts.bytes, s));
  AGP_HIP(hipMemsetAsync(counters, 0, sc.counters.bytes, s));
  AGP_HIP(hipMemsetAsync(flags, 0, sc.flags.bytes, s));
  if (qids) AGP_HIP(hipMemcpyAsync(dq, qids, sizeof(uint32_t) * C, hipMemcpyHostToDevice, s));

  // thresholds theta_c = eps ||x_c||_1 and signal checks, counting the
  // non-zero cells of x; when at least half of the cells are non-zero,
  // level 0 visits every cell in order (skipping the zeros), else a second
  // pass lists the non-zero cells
  const dim3 tgrid((unsigned)std::max<int64_t>(tblocks, 1), (unsigned)((C + 63) / 64));
  if (tblocks > 0 && C == 1)
    k_theta_partial_c1<T, false><<<tgrid, kWave, 0, s>>>(x, ldc, n, sc.partial.as<double>(), flags + 1, nullptr,
                                                         counts);
  else if (tblocks > 0)
    k_theta_partial<T, kThetaCap, false><<<tgrid, kWave, 0, s>>>(x, ldc, n, C, sc.partial.as<double>(), flags + 1,
                                                                 nullptr, counts);
  // flags[2..3]: the count of non-zero cells of x
  k_theta_final<T><<<grid_for(C, 64), 64, 0, s>>>(sc.partial.as<double>(), tblocks, C, eps,
                                                  qids ? dq : nullptr, qid_base, cp, counts,
                                                  reinterpret_cast<unsigned long long*>(flags + 2));
  AGP_HIP(hipGetLastError());
  int hflags[4] = {0, 0, 0, 0};
  AGP_HIP(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
  AGP_HIP(hipStreamSynchronize(s));
  unsigned long long nnz_x = 0;
  std::memcpy(&nnz_x, hflags + 2, sizeof(nnz_x));
  if (hflags[1] & 1) return fail(AGP_EINVAL, std::string(fn) + ": x holds a non-finite value");
  const bool virtual0 = nnz_x > 0 && 2 * nnz_x >= static_cast<unsigned long long>(cells) &&
                        static_cast<long long>(C) <= kVirtualMaxC;
  if (virtual0) {
    k_set_u64<<<1, 1, 0, s>>>(counts, static_cast<unsigned long long>(cells));  // the level-0 entries
  } else if (tblocks > 0) {
    AGP_HIP(hipMemsetAsync(counts, 0, sizeof(unsigned long long), s));
    if (C == 1)
      k_theta_partial_c1<T, true><<<tgrid, kWave, 0, s>>>(x, ldc, n, sc.partial.as<double>(), flags + 1,
                                                          sc.frontier[0].as<uint64_t>(), counts);
    else
      k_theta_partial<T, kThetaCap, true><<<tgrid, kWave, 0, s>>>(x, ldc, n, C, sc.partial.as<double>(), flags + 1,
                                                                  sc.frontier[0].as<uint64_t>(), counts);
    AGP_HIP(hipGetLastError());
  }
  const bool positive = sizeof(T) == 4 && !(hflags[1] & 2);

  // binned aggregation: binary32, LDS scale table, record cells in 31 bits:
  // one group of all C columns when n C < 2^31, else two column groups of
  // ceil(C / 2) columns (cells local to a group) when n ceil(C / 2) < 2^31
  int ng = static_cast<unsigned long long>(cells) < (1ull << 31) ? 1 : kMaxRecGroups;
  if (const char* e = std::getenv("AGP_RECORD_GROUPS"))  // column groups at any size (tests)
    if (std::strcmp(e, "2") == 0 && C >= 2) ng = kMaxRecGroups;
  const long long gw = ng == 1 ? C : (C + 1) / 2;
  const unsigned long long gcells = static_cast<unsigned long long>(n) * static_cast<unsigned long long>(gw);
  bool binned = (tune.aggregation == 1 || tune.aggregation == 2) && sizeof(T) == 4 && gcells < (1ull << 31) &&
                C <= kMaxBinnedC && cells > 0;
  // buckets of 2^shift group cells: at most 1024 buckets (512 per group with
  // two groups, which share the level kernel's histogram), bins of 8192 cells
  const unsigned long long nbk = static_cast<unsigned long long>(kBuckets / ng);
  int shift = kBinLog2;
  while (shift < 32 && (gcells > 0 ? gcells - 1ull : 0ull) >> shift >= nbk) ++shift;
  const long long nbins = static_cast<long long>(((gcells > 0 ? gcells : 1) - 1) >> kBinLog2) + 1;  // per group
  unsigned long long rec_cap = 0;  // per group
  if (binned) {
    // room for 4 records per cell (1 when the call runs in several tiles,
    // whose width left room for that), within 80% of the free memory (two
    // buffers)
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    const size_t held = sc.rec[0].bytes + sc.rec[1].bytes;
    unsigned long long cap = std::max<unsigned long long>(1ull << 20, (static_cast<long long>(C) < ldc ? 1ull : 4ull) * cells);
    cap = std::min<unsigned long long>(cap, std::max<unsigned long long>(1ull << 20, (free_b + held) / 10));
    if (const char* e = std::getenv("AGP_RECORD_CAP")) {  // smaller record buffer (tuning / tests)
      const unsigned long long v = std::strtoull(e, nullptr, 10);
      if (v > 0 && v < cap) cap = v;
    }
    rec_cap = (cap + ng - 1) / ng;
    if (sc.rec[0].reserve(rec_cap * ng * sizeof(uint32_t), false, s) ||
        sc.rec[1].reserve(rec_cap * ng * sizeof(uint32_t), false, s) ||
        sc.bins.reserve(ng * (sizeof(unsigned int) * kBuckets + sizeof(unsigned long long) * (2 * kBuckets + 1) +
                              sizeof(unsigned long long) * (AGP_MAX_LEVELS + 1) + static_cast<size_t>(nbins)) +
                            sizeof(unsigned long long) * (3 * nbins + 1),
                        true, s)) {
      sc.rec[0].release();  // not enough memory for the record buffers: atomics instead
      sc.rec[1].release();
      binned = false;
      (void)hipGetLastError();
    }
  }
  // bucket counts (group g's kBuckets / ng at g * kBuckets / ng); per group:
  // bucket offsets, partition cursors (kBuckets + 1 and kBuckets), per-level
  // record counts (level i, group g at i * ng + g), deterministic-push flags
  // per bin; shared by the groups in turn: bin counts, offsets, cursors
  unsigned int* bucket_count = binned ? sc.bins.as<unsigned int>() : nullptr;
  unsigned long long* bucket_off = binned ? reinterpret_cast<unsigned long long*>(bucket_count + kBuckets * ng) : nullptr;
  unsigned long long* cursor = binned ? bucket_off + (kBuckets + 1) * ng : nullptr;
  unsigned long long* rec_counts = binned ? cursor + kBuckets * ng : nullptr;
  unsigned long long* bin_count = binned ? rec_counts + (AGP_MAX_LEVELS + 1) * ng : nullptr;
  unsigned long long* bin_off = binned ? bin_count + nbins : nullptr;
  unsigned long long* bin_cur = binned ? bin_off + nbins + 1 : nullptr;
  uint8_t* det_bins = binned ? reinterpret_cast<uint8_t*>(bin_cur + nbins) : nullptr;  // any stale value is safe
  if (binned) {
    AGP_HIP(hipMemsetAsync(rec_counts, 0, sizeof(unsigned long long) * (AGP_MAX_LEVELS + 1) * ng, s));
    AGP_HIP(hipMemsetAsync(bin_count, 0, sizeof(unsigned long long) * nbins, s));
    AGP_HIP(hipMemsetAsync(bucket_count, 0, sizeof(unsigned int) * kBuckets * ng, s));  // the dense path shares the buffer
  }

  hipEvent_t* ev = sc.events;
  if (stats && (rc = sc.ensure_events())) return rc;
  uint64_t* F[2] = {sc.frontier[0].as<uint64_t>(), sc.frontier[1].as<uint64_t>()};
  Cell* acc[2] = {sc.acc[0].as<Cell>(), sc.acc[1].as<Cell>()};
  // compaction: 32 KiB of LDS per block (five per CU); segments of 2^10 to
  // 2^16 cells per wave, as large as leaves about 4096 of them
  long long cseg = kCompactUnroll * kWave;
  while (cseg < kCompactSeg && cseg * 4096 < static_cast<long long>(cells)) cseg <<= 1;
  const unsigned cgrid = grid_for(static_cast<int64_t>((cells + cseg - 1) / cseg), kThreads / kWave, 1280);

  // rows with long deterministic prefixes, deferred per level to k_det_big
  constexpr unsigned long long kBigCap = 1ull << 16;
  unsigned long long big_cap = kBigCap;
  if (const char* e = std::getenv("AGP_BIG_ROWS")) {  // shorter lists (tests); 0: no deferral
    const unsigned long long v = std::strtoull(e, nullptr, 10);
    if (v < big_cap) big_cap = v;
  }
  const long long samp_items = tune.big_items;
  // (and entries with many sampled work items, deferred to k_samp_big):
  // per-level counters of both lists, then the two lists
  unsigned long long* big_ctr = nullptr;
  unsigned long long* samp_ctr = nullptr;
  BigRow* big_rows = nullptr;
  BigSamp* samp_rows = nullptr;
  if (big_cap > 0 && (may_alloc || sc.big.bytes > 0) &&
      sc.big.reserve(sizeof(unsigned long long) * 2 * (AGP_MAX_LEVELS + 1) + sizeof(BigRow) * kBigCap +
                         sizeof(BigSamp) * kBigCap,
                     false, s) == AGP_OK) {
    big_ctr = sc.big.as<unsigned long long>();
    samp_ctr = big_ctr + AGP_MAX_LEVELS + 1;
    big_rows = reinterpret_cast<BigRow*>(samp_ctr + AGP_MAX_LEVELS + 1);
    samp_rows = reinterpret_cast<BigSamp*>(big_rows + kBigCap);
    AGP_HIP(hipMemsetAsync(big_ctr, 0, sizeof(unsigned long long) * 2 * (AGP_MAX_LEVELS + 1), s));
  } else {
    (void)hipGetLastError();  // no room for the list: every row stays with its wave
  }

  LevelArgs A{};
  A.rp = g->row_ptr;
  A.col = g->col;
  A.nd = g->ndeg;
  A.gend = g->gend;
  A.deg = g->degree;
  A.fdeg = g->fdeg;
  A.cp = cp;
  A.su = C;
  A.sc = 1;
  A.xld = ldc;
  A.counters = counters;
  A.mass = mass;
  A.err = flags;
  A.positive = positive ? 1 : 0;
  A.dense_cut = std::max<unsigned long long>(1ull, static_cast<unsigned long long>(cells >> tune.sparse_shift));
  A.big_row = static_cast<uint32_t>(tune.big_row);
  A.rec = nullptr;
  A.rec_count = nullptr;
  A.rec_cap = rec_cap;
  A.rec_groups = ng;
  A.rec_gw = static_cast<uint32_t>(gw);
  A.det_bins_g = static_cast<unsigned long long>(nbins);
  A.bucket_count = bucket_count;
  A.bucket_shift = shift;
  A.bin_est = nullptr;
  // auto: bin levels with n C / 2^k estimated pushes; with two column groups
  // from twice that (on 32-column tiles of a 111M-node graph the record
  // passes cost more than the atomics they replace below about n C / 4)
  A.bin_pushes = std::ldexp(static_cast<double>(cells), -(ng > 1 ? std::max(tune.bin_shift - 1, 1) : tune.bin_shift));
  // per node: d_u^-b and the first neighbour's d^-a, so that a batch setup
  // loads both with the row bounds (kept for later calls with the same a, b)
  A.nodefac = nullptr;
  const char* fv = std::getenv("AGP_FACTOR_VECTORS");  // "0": read the factors through the tables (tests)
  const bool factors = may_alloc && !(fv && std::strcmp(fv, "0") == 0);
  if (factors && n > 0) {
    const void* before = sc.nodefac.ptr;
    if (sc.nodefac.reserve(static_cast<size_t>(n) * sizeof(double2), false, s) == AGP_OK) {
      if (sc.nodefac.ptr != before || sc.nodefac_a != a || sc.nodefac_b != b) {
        k_node_factors<<<grid_for(n, 256), 256, 0, s>>>(g->row_ptr, g->degree, g->fdeg, g->ndeg, da, db, n,
                                                        sc.nodefac.as<double2>());
        sc.nodefac_a = a;
        sc.nodefac_b = b;
      }
      A.nodefac = sc.nodefac.as<double>();
    } else {
      (void)hipGetLastError();  // no room: the setup reads the factors through the degree tables
      sc.nodefac_a = sc.nodefac_b = -1.0;
    }
  }
  // per arc: its neighbour's d^-a (a > 0), so that an acceptance test or a
  // run start loads it beside the neighbour id (kept for later calls with
  // the same a); only when it fits beside the tile's scratch
  A.arcfac = nullptr;
  if (factors && a != 0.0 && g->nnz > 0) {
    const void* before = sc.arcfac.ptr;
    const size_t want = static_cast<size_t>(g->nnz) * sizeof(double);
    size_t free_b = 0, total_b = 0;
    const bool room = sc.arcfac.bytes >= want ||
                      (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > want + (want >> 2) + (1ull << 30));
    if (room && sc.arcfac.reserve(want, false, s) == AGP_OK) {
      if (sc.arcfac.ptr != before || sc.arcfac_a != a) {
        k_arc_factors<<<grid_for(g->nnz, 256), 256, 0, s>>>(g->ndeg, da, g->nnz, sc.arcfac.as<double>());
        sc.arcfac_a = a;
      }
      A.arcfac = sc.arcfac.as<double>();
    } else {
      (void)hipGetLastError();
      sc.arcfac_a = -1.0;
    }
  }
  // per-level values of this call (read by k_set_level from device memory)
  LevelParams lph[AGP_MAX_LEVELS + 1];
  const uint32_t key0 = static_cast<uint32_t>(seed), key1 = static_cast<uint32_t>(seed >> 32);
  for (int32_t i = 0; i <= L; ++i) {
    lph[i].rho = rho[i];
    lph[i].kappa = kappa[i];
    lph[i].flags = (i == L ? kLastLevel : 0) | (a == 0.0 ? kAZero : 0);
    lph[i].key0 = key0;
    lph[i].key1 = key1;
    lph[i].pad = 0;
  }
  AGP_HIP(hipMemcpyAsync(lpd, lph, sizeof(LevelParams) * (L + 1), hipMemcpyHostToDevice, s));

  // the level loop: every decision stays on the device, so it can be
  // captured once and replayed (timed per level only when launched directly)
  auto levels = [&](hipStream_t s, bool timed) {
    for (int32_t i = 0; i <= L; ++i) {
      k_set_level<<<grid_for(C, 64), 64, 0, s>>>(cp, C, i, lpd, da, db, out, ldc, sizeof(T));
      A.level = i;
      A.fin = (i == 0 && virtual0) ? nullptr : F[i & 1];
      A.cnt_in = counts + i;
      A.fout = F[(i + 1) & 1];
      A.cnt_out = counts + i + 1;
      A.mode_out = mode + i + 1;
      const bool bin_level = binned && i < L;
      A.rec = bin_level ? sc.rec[0].as<uint32_t>() : nullptr;
      A.det_bins = bin_level ? det_bins : nullptr;
      A.big_ctr = (big_ctr != nullptr && i < L) ? big_ctr + i : nullptr;
      A.samp_ctr = (samp_ctr != nullptr && i < L) ? samp_ctr + i : nullptr;
      A.big = big_rows;
      A.samp = samp_rows;
      A.samp_items = samp_items;
      A.big_cap = big_cap;
      A.rec_count = bin_level ? rec_counts + static_cast<size_t>(i) * ng : nullptr;
      Cell* cur = acc[i & 1];
      Cell* nxt = acc[(i + 1) & 1];
      A.bin_est = nullptr;
      if (timed) (void)hipEventRecord(ev[4 * i], s);
      if (bin_level && tune.aggregation == 2) {
        A.bin_est = est + i;
        if (i == 0)
          k_estimate<T, true><<<1024, kThreads, 0, s>>>(A, x, cur, est + i);
        else
          k_estimate<T, false><<<1024, kThreads, 0, s>>>(A, x, cur, est + i);
      }
      if (timed) (void)hipEventRecord(ev[4 * i + 1], s);
      bool grouped = false;  // records in two column groups (binary32 only)
      if constexpr (sizeof(T) == 4) {
        grouped = bin_level && ng > 1;
        if (grouped) {
          if (i == 0)
            k_level<T, true, false, 2><<<tune.level_blocks, kThreads, 0, s>>>(A, x, cur, nxt);
          else
            k_level<T, false, false, 2><<<tune.level_blocks, kThreads, 0, s>>>(A, x, cur, nxt);
          if (A.big_ctr != nullptr) k_det_big<T, 2><<<1024, kThreads, 0, s>>>(A, nxt);
          if (A.samp_ctr != nullptr) k_samp_big<T, 2><<<1024, kThreads, 0, s>>>(A, nxt);
        }
      }
      if (!grouped) {
        if (i == 0)
          k_level<T, true, false><<<tune.level_blocks, kThreads, 0, s>>>(A, x, cur, nxt);
        else
          k_level<T, false, false><<<tune.level_blocks, kThreads, 0, s>>>(A, x, cur, nxt);
        if (A.big_ctr != nullptr) k_det_big<T><<<1024, kThreads, 0, s>>>(A, nxt);
        if (A.samp_ctr != nullptr) k_samp_big<T><<<1024, kThreads, 0, s>>>(A, nxt);
      }
      if (timed) (void)hipEventRecord(ev[4 * i + 2], s);
      if (bin_level) {
        uint32_t* r0 = sc.rec[0].as<uint32_t>();
        uint32_t* r1 = sc.rec[1].as<uint32_t>();
        unsigned long long* rc = rec_counts + static_cast<size_t>(i) * ng;
        k_bins_scan<<<ng, kBuckets, 0, s>>>(bucket_count, static_cast<int>(nbk), bucket_off, cursor, rc, rec_cap,
                                            mode + i + 1);
        k_apply_overflow<<<2048, kThreads, 0, s>>>(A, reinterpret_cast<long long*>(nxt), mode + i + 1);
        for (int gi = 0; gi < ng; ++gi) {  // each group's records in turn
          uint32_t* g0 = r0 + static_cast<size_t>(gi) * rec_cap;
          uint32_t* g1 = r1 + static_cast<size_t>(gi) * rec_cap;
          k_partition<<<1024, kReduceThreads, 0, s>>>(g0, rc + gi, cursor + static_cast<size_t>(gi) * kBuckets, g1,
                                                      mode + i + 1, shift);
          k_bin_count<<<2048, kReduceThreads, 0, s>>>(g1, rc + gi, bin_count, mode + i + 1, shift);
          k_bin_scan<<<static_cast<unsigned>(nbins / kScanChunk + 1), 1024, 0, s>>>(bin_count, nbins, bin_off,
                                                                                 bin_cur, mode + i + 1);
          k_bin_scatter<<<2048, kReduceThreads, 0, s>>>(g1, rc + gi, bin_cur, g0, mode + i + 1, shift, bin_count,
                                                        nbins);
          if (ng == 1)
            k_bin_sum<<<static_cast<unsigned>(nbins), kSumThreads, 0, s>>>(
                g0, bin_off, cp, (long long)C, 1ll, static_cast<unsigned long long>(cells),
                reinterpret_cast<long long*>(nxt), F[(i + 1) & 1], counts + i + 1, mode + i + 1, det_bins);
          else
            k_bin_sum<<<static_cast<unsigned>(nbins), kSumThreads, 0, s>>>(
                g0, bin_off, cp, gw, 1ll, gcells, reinterpret_cast<long long*>(nxt), F[(i + 1) & 1], counts + i + 1,
                mode + i + 1, det_bins + static_cast<size_t>(gi) * nbins, (long long)C, static_cast<int>(gi * gw),
                static_cast<int>(std::min<long long>(gw, C - gi * gw)));
        }
      }
      if (i < L)
        k_compact<<<cgrid, kThreads, 0, s>>>(NonZeroCell<T>{nxt}, n, C, cseg, F[(i + 1) & 1], counts + i + 1,
                                             mode + i + 1);
      if (timed) (void)hipEventRecord(ev[4 * i + 3], s);
    }
  };
  if (tune.capture == 1) {
    // key: everything the captured kernels take by value
    char key[512];
    const int kn = std::snprintf(
        key, sizeof(key), "%lld|%d|%d|%lld|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%p|%d|%d|%llu|%d|%llu|%d|%d|%d|%d|%d|%d",
        static_cast<long long>(n), C, L, static_cast<long long>(ldc), static_cast<const void*>(x),
        static_cast<void*>(out), static_cast<void*>(cp), static_cast<void*>(acc[0]), static_cast<void*>(acc[1]),
        static_cast<void*>(F[0]), static_cast<void*>(F[1]), static_cast<void*>(counts), static_cast<void*>(counters),
        static_cast<void*>(sc.levelinfo.ptr), static_cast<void*>(flags), static_cast<const void*>(da),
        static_cast<const void*>(db), static_cast<void*>(sc.rec[0].ptr), static_cast<void*>(sc.bins.ptr),
        positive ? 1 : 0, binned ? ng : 0, rec_cap, shift, big_cap, big_ctr != nullptr ? 1 : 0, tune.aggregation,
        tune.level_blocks, tune.big_row, tune.big_items, (tune.sparse_shift << 8) | tune.bin_shift);
    std::string k(key, kn > 0 ? static_cast<size_t>(kn) : 0);
    k.push_back(virtual0 ? 'v' : 'l');  // level 0 over every cell or over the listed ones
    k.append(reinterpret_cast<const char*>(&big_rows), sizeof(big_rows));
    k.append(reinterpret_cast<const char*>(&samp_rows), sizeof(samp_rows));
    k.append(reinterpret_cast<const char*>(&samp_items), sizeof(samp_items));
    k.append(reinterpret_cast<const char*>(&sc.rec[1].ptr), sizeof(void*));
    k.append(reinterpret_cast<const char*>(&A.nodefac), sizeof(void*));
    k.append(reinterpret_cast<const char*>(&A.arcfac), sizeof(void*));
    hipGraphExec_t exec = nullptr;
    auto it = g->loops.find(k);
    if (it != g->loops.end()) {
      exec = it->second;
    } else {
      if (!g->capture_stream) AGP_HIP(hipStreamCreateWithFlags(&g->capture_stream, hipStreamNonBlocking));
      hipStream_t cs = g->capture_stream;
      AGP_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      levels(cs, false);
      hipGraph_t graph = nullptr;
      const hipError_t le = hipGetLastError();
      const hipError_t ee = hipStreamEndCapture(cs, &graph);
      if (le != hipSuccess || ee != hipSuccess || graph == nullptr) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(AGP_EDEVICE, std::string(fn) + ": capturing the level loop failed: " +
                                     hipGetErrorString(le != hipSuccess ? le : ee));
      }
      const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) return fail(AGP_EDEVICE, std::string(fn) + ": " + hipGetErrorString(ie));
      if (g->loops.size() >= 32) g->drop_loops();  // a bounded cache
      g->loops.emplace(k, exec);
    }
    if (stats) AGP_HIP(hipEventRecord(ev[0], s));
    AGP_HIP(hipGraphLaunch(exec, s));
    if (stats) AGP_HIP(hipEventRecord(ev[4 * L + 3], s));
  } else {
    levels(s, stats != nullptr);
  }
  AGP_HIP(hipGetLastError());
  double hmass[AGP_MAX_LEVELS + 1];
  AGP_HIP(hipMemcpyAsync(hflags, flags, sizeof(int), hipMemcpyDeviceToHost, s));
  AGP_HIP(hipMemcpyAsync(hmass, mass, sizeof(double) * (L + 1), hipMemcpyDeviceToHost, s));
  AGP_HIP(hipStreamSynchronize(s));
  // no partial sum can wrap while a level's total magnitude stays below the cell range
  const double mass_cap = sizeof(T) == 4 ? 0x1p61 : 0x1p125;
  for (int32_t i = 0; i <= L; ++i)
    if (!(hmass[i] < mass_cap)) hflags[0] |= 1;
  if (hflags[0]) {
    // restore the all-zero invariant of the accumulators
    AGP_HIP(hipMemsetAsync(sc.acc[0].ptr, 0, sc.acc[0].bytes, s));
    AGP_HIP(hipMemsetAsync(sc.acc[1].ptr, 0, sc.acc[1].bytes, s));
    AGP_HIP(hipStreamSynchronize(s));
    return fail(AGP_ERANGE, std::string(fn) + ": a residue outgrew the exact accumulator range");
  }
  if (stats) {
    std::vector<unsigned long long> h(static_cast<size_t>(kNumCounters) * (L + 1));
    AGP_HIP(hipMemcpy(h.data(), counters, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    stats->levels = L;
    stats->tiles += 1;
    for (int32_t i = 0; i <= L; ++i) {
      stats->frontier[i] += h[i * kNumCounters + 0];
      stats->hash[i] += h[i * kNumCounters + 1];
      stats->det[i] += h[i * kNumCounters + 2];
      stats->cand[i] += h[i * kNumCounters + 3];
      stats->acc[i] += h[i * kNumCounters + 4];
      stats->runs[i] += h[i * kNumCounters + 5];
    }
    float ms = 0.0f;
    for (int32_t i = 0; i <= L && tune.capture != 1; ++i) {  // a replayed loop is timed as a whole
      AGP_HIP(hipEventElapsedTime(&ms, ev[4 * i + 1], ev[4 * i + 2]));
      stats->level_ms[i] += ms;
      AGP_HIP(hipEventElapsedTime(&ms, ev[4 * i], ev[4 * i + 3]));
      stats->level_total_ms[i] += ms;
    }
    AGP_HIP(hipEventElapsedTime(&ms, ev[0], ev[4 * L + 3]));
    stats->device_ms += ms;
  }
  return AGP_OK;
}


// Tile width: every column at once when the scratch fits in 85% of the free
// memory (plus what the scratch already holds), else the widest tile that
// does; AGP_COLUMN_TILE forces a width (tests).
template <typename T>
int32_t column_tile(agp_graph* g, int32_t C, bool binned, const agp_tuning_t& tune) {
  if (tune.tile_columns > 0) return std::min(tune.tile_columns, C);
  const size_t cell_bytes = sizeof(typename Prec<T>::Cell) * (sizeof(T) == 4 ? 1 : 2);
  // two accumulators and two frontier lists per cell (+ two record buffers
  // of 4 records per cell; of 1 when not every column fits: wider tiles,
  // the records beyond the buffer go to atomics)
  const size_t base_cell = 2 * cell_bytes + 2 * sizeof(uint64_t);
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return C;
  Scratch& sc = g->scratch;
  const size_t held = sc.acc[0].bytes + sc.acc[1].bytes + sc.frontier[0].bytes + sc.frontier[1].bytes +
                      sc.rec[0].bytes + sc.rec[1].bytes + sc.nodefac.bytes + sc.arcfac.bytes;
  const double budget = 0.85 * static_cast<double>(free_b + held);
  for (int recs : {4, 1}) {
    const size_t per_cell = base_cell + (binned ? 2 * static_cast<size_t>(recs) * sizeof(uint32_t) : 0);
    const double per_col = static_cast<double>(g->n > 0 ? g->n : 1) * static_cast<double>(per_cell);
    const double fit = budget / per_col;
    if (fit >= static_cast<double>(C)) return C;
    if (recs == 1) return fit < 1.0 ? 1 : static_cast<int32_t>(fit);
  }
  return 1;
}

// ------------------------------------------------------------ dense levels
// Work items of the dense level kernel, built once per graph on the host
// from the row lengths: runs of up to 64 consecutive nodes holding at most
// dense::kItemArcs arcs, and rows longer than that cut into pieces of 64
// windows (4096 arcs).  The long rows are also listed (their residues are
// cleared after each level).
int dense_items(agp_graph* g, hipStream_t s) {
  Scratch& sc = g->scratch;
  if (sc.dense_nitems >= 0) return AGP_OK;
  const int64_t n = g->n;
  std::vector<int32_t> deg(static_cast<size_t>(n));
  if (n > 0) {
    AGP_HIP(hipMemcpyAsync(deg.data(), g->degree, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    AGP_HIP(hipStreamSynchronize(s));
  }
  std::vector<uint64_t> items;
  std::vector<uint32_t> rows;
  items.reserve(static_cast<size_t>(n / 16 + 16));
  for (int64_t u = 0; u < n;) {
    const int64_t d = deg[u];
    if (d > dense::kItemArcs) {
      const int64_t nwin = (d + kSeg - 1) / kSeg;
      if (nwin >= (1ll << 20)) return fail(AGP_ENOTSUP, "dense levels: a row longer than 2^26 arcs");
      for (int64_t w0 = 0; w0 < nwin; w0 += 64) {
        const uint64_t cnt = static_cast<uint64_t>(std::min<int64_t>(64, nwin - w0));
        items.push_back(dense::kItemLong | (cnt << 52) | (static_cast<uint64_t>(w0) << 32) | static_cast<uint64_t>(u));
      }
      rows.push_back(static_cast<uint32_t>(u));
      ++u;
      continue;
    }
    const int64_t start = u;
    int64_t arcs = 0, cnt = 0;
    while (u < n && cnt < dense::kItemNodes && deg[u] <= dense::kItemArcs && arcs + deg[u] <= dense::kItemArcs) {
      arcs += deg[u];
      ++cnt;
      ++u;
    }
    items.push_back((static_cast<uint64_t>(cnt) << 32) | static_cast<uint64_t>(start));
  }
  int rc;
  if ((rc = sc.dense_items.reserve(sizeof(uint64_t) * std::max<size_t>(items.size(), 1), false, s)) ||
      (rc = sc.dense_rows.reserve(sizeof(uint32_t) * std::max<size_t>(rows.size(), 1), false, s)))
    return rc;
  if (!items.empty())
    AGP_HIP(hipMemcpyAsync(sc.dense_items.ptr, items.data(), sizeof(uint64_t) * items.size(), hipMemcpyHostToDevice, s));
  if (!rows.empty())
    AGP_HIP(hipMemcpyAsync(sc.dense_rows.ptr, rows.data(), sizeof(uint32_t) * rows.size(), hipMemcpyHostToDevice, s));
  AGP_HIP(hipStreamSynchronize(s));
  sc.dense_nitems = static_cast<int64_t>(items.size());
  sc.dense_nrows = static_cast<int64_t>(rows.size());
  return AGP_OK;
}

// Memory plan of a dense call: Ct columns per tile (at most 64, tiles of
// equal width), record groups of 2^gshift columns (n 2^gshift <= 2^31), and
// the record buffers' capacity per group.
struct DensePlan {
  int32_t Ct = 0;
  int gshift = 6;
  int ng = 1;
  unsigned long long rec_cap = 0;  // per group; 0: atomics only
};

DensePlan dense_plan(agp_graph* g, int32_t C, const agp_tuning_t& tune, bool binned) {
  DensePlan p;
  const int64_t n = g->n > 0 ? g->n : 1;
  int32_t want = tune.tile_columns > 0 ? std::min(tune.tile_columns, dense::kMaxCols) : dense::kMaxCols;
  want = std::min(want, C);
  size_t free_b = 0, total_b = 0;
  (void)hipMemGetInfo(&free_b, &total_b);
  Scratch& sc = g->scratch;
  const size_t held = sc.acc[0].bytes + sc.acc[1].bytes + sc.frontier[0].bytes + sc.frontier[1].bytes +
                      sc.rec[0].bytes + sc.rec[1].bytes + sc.nodefac.bytes + sc.arcfac.bytes;
  const double budget = 0.9 * static_cast<double>(free_b + held);
  // 8 B exact sum + 4 B residue per cell, 2 flag bytes per node; records
  // (two buffers of 4 B) take at least a quarter record per cell
  auto fits = [&](int32_t ct, double rpc) {
    return static_cast<double>(n) * (ct * (12.0 + (binned ? 8.0 * rpc : 0.0)) + 2.0) <= budget;
  };
  int32_t ct = want;
  while (ct > 1 && !fits(ct, 0.25)) --ct;
  const int32_t ntiles = (C + ct - 1) / ct;
  p.Ct = (C + ntiles - 1) / ntiles;  // equal tiles
  int gshift = 6;
  while (gshift > 0 && static_cast<double>(n) * static_cast<double>(1 << gshift) > 2147483648.0) --gshift;
  if (const char* e = std::getenv("AGP_DENSE_GROUP_SHIFT")) {  // narrower record groups (tests)
    const long v = std::strtol(e, nullptr, 10);
    if (v >= 0 && v < gshift) gshift = static_cast<int>(v);
  }
  p.gshift = gshift;
  p.ng = (p.Ct + (1 << gshift) - 1) >> gshift;
  if (p.ng > dense::kMaxGroups) p.ng = 0;  // not addressable in 4 groups (n > 2^31 / 16)
  if (binned && p.ng > 0) {
    const double cells = static_cast<double>(n) * p.Ct;
    double room = (budget - static_cast<double>(n) * (12.0 * p.Ct + 2.0)) / 8.0;  // records per buffer
    room = std::min(room, 1.5 * cells);
    if (const char* e = std::getenv("AGP_RECORD_CAP")) {
      const double v = std::strtod(e, nullptr);
      if (v > 0 && v < room * p.ng) room = v * p.ng;
    }
    p.rec_cap = room >= 1024.0 * p.ng ? static_cast<unsigned long long>(room / p.ng) : 0ull;
    // keep record buffers that hold at least 90% of that: the free memory
    // moves a little between calls, and growing them means freeing and
    // allocating tens of GB
    const unsigned long long have = std::min(sc.rec[0].bytes, sc.rec[1].bytes) / (sizeof(uint32_t) * p.ng);
    if (p.rec_cap > 0 && have >= p.rec_cap / 10 * 9) p.rec_cap = std::min<unsigned long long>(have, 2 * p.rec_cap);
  }
  return p;
}

// One dense tile of Ct columns (x, out: the tile's first column, rows ldc
// apart; cpt: the tile's column parameters with theta, units and qids set).
// The caller holds g->mu.
int propagate_dense_tile(agp_graph* g, const char* fn, const agp_tuning_t& tune, const DensePlan& plan, double a,
                         double b, const double* rho, const double* kappa, int32_t L,
                         const float* x, long long ldc, int32_t Ct, const ColParams* cpt, uint64_t seed, float* out,
                         hipStream_t s, agp_stats_t* stats) {
  using namespace dense;
  const int64_t n = g->n;
  const size_t cells = static_cast<size_t>(n) * static_cast<size_t>(Ct);
  int rc;
  const double *da = nullptr, *db = nullptr;
  if ((rc = pow_table(g, a, &da)) || (rc = pow_table(g, b, &db))) return rc;
  if ((rc = dense_items(g, s))) return rc;
  Scratch& sc = g->scratch;
  const int ng = plan.ng;
  const int gw = 1 << plan.gshift;
  const bool binned = plan.rec_cap > 0 && tune.aggregation != 0;
  // group cells: n * width of group 0 (the widest)
  const unsigned long long gcells0 = static_cast<unsigned long long>(n) * static_cast<unsigned long long>(std::min(gw, Ct));
  int shift = kBinLog2;
  while (shift < 32 && (gcells0 > 0 ? gcells0 - 1ull : 0ull) >> shift >= (unsigned long long)kBuckets) ++shift;
  const long long nbins_g = static_cast<long long>(((gcells0 > 0 ? gcells0 : 1) - 1) >> kBinLog2) + 1;
  if ((rc = sc.acc[0].reserve(cells * sizeof(long long), true, s)) ||
      (rc = sc.acc[1].reserve(cells * sizeof(float), true, s)) ||
      (rc = sc.frontier[0].reserve(2 * static_cast<size_t>(n) + 64, false, s)) ||
      (rc = sc.counters.reserve(sizeof(unsigned long long) * kNumCounters * (AGP_MAX_LEVELS + 1), false, s)) ||
      (rc = sc.flags.reserve(sizeof(int) * 4, false, s)) ||
      (rc = sc.levelinfo.reserve((2 * sizeof(double) + sizeof(int)) * (AGP_MAX_LEVELS + 2), false, s)))
    return rc;
  if (binned) {
    const size_t bins_bytes = sizeof(unsigned int) * kBuckets * ng + sizeof(unsigned long long) * (kBuckets + 1) * ng +
                              sizeof(unsigned long long) * kBuckets * ng +
                              sizeof(unsigned long long) * (AGP_MAX_LEVELS + 1) * ng +
                              sizeof(unsigned long long) * (3 * nbins_g + 1) + static_cast<size_t>(nbins_g) * ng;
    if ((rc = sc.rec[0].reserve(plan.rec_cap * ng * sizeof(uint32_t), false, s)) ||
        (rc = sc.rec[1].reserve(plan.rec_cap * ng * sizeof(uint32_t), false, s)) ||
        (rc = sc.bins.reserve(bins_bytes, true, s)))
      return rc;
  }
  long long* acc = sc.acc[0].as<long long>();
  float* r = sc.acc[1].as<float>();
  uint8_t* flags2[2] = {sc.frontier[0].as<uint8_t>(), sc.frontier[0].as<uint8_t>() + n};
  unsigned long long* counters = sc.counters.as<unsigned long long>();
  int* errf = sc.flags.as<int>();
  double* mass = sc.levelinfo.as<double>();
  int* mode = reinterpret_cast<int*>(mass + 2 * (AGP_MAX_LEVELS + 2));
  unsigned int* bucket_count = binned ? sc.bins.as<unsigned int>() : nullptr;
  unsigned long long* bucket_off = binned ? reinterpret_cast<unsigned long long*>(bucket_count + kBuckets * ng) : nullptr;
  unsigned long long* cursor = binned ? bucket_off + (kBuckets + 1) * ng : nullptr;
  unsigned long long* rec_counts = binned ? cursor + kBuckets * ng : nullptr;
  unsigned long long* bin_count = binned ? rec_counts + (AGP_MAX_LEVELS + 1) * ng : nullptr;
  unsigned long long* bin_off = binned ? bin_count + nbins_g : nullptr;
  unsigned long long* bin_cur = binned ? bin_off + nbins_g + 1 : nullptr;
  uint8_t* det_bins = binned ? reinterpret_cast<uint8_t*>(bin_cur + nbins_g) : nullptr;
  AGP_HIP(hipMemsetAsync(sc.levelinfo.ptr, 0, sc.levelinfo.bytes, s));
  AGP_HIP(hipMemsetAsync(counters, 0, sizeof(unsigned long long) * kNumCounters * (L + 1), s));
  AGP_HIP(hipMemsetAsync(errf, 0, sizeof(int), s));
  if (binned) {  // counters that the bin kernels expect at zero (the layout moves with ng and nbins_g)
    AGP_HIP(hipMemsetAsync(rec_counts, 0, sizeof(unsigned long long) * (AGP_MAX_LEVELS + 1) * ng, s));
    AGP_HIP(hipMemsetAsync(bucket_count, 0, sizeof(unsigned int) * kBuckets * ng, s));
    AGP_HIP(hipMemsetAsync(bin_count, 0, sizeof(unsigned long long) * nbins_g, s));
  }
  // every level starts binned (records beyond the buffers switch it to the fallback)
  k_fill_i32<<<1, 256, 0, s>>>(mode, L + 2, binned ? kModeBinned : kModeCompact);
  hipEvent_t* ev = sc.events;
  if (stats && (rc = sc.ensure_events())) return rc;

  DenseArgs D{};
  D.rp = g->row_ptr;
  D.col = g->col;
  D.nd = g->ndeg;
  D.deg = g->degree;
  D.fdeg = g->fdeg;
  D.da = da;
  D.db = db;
  D.items = sc.dense_items.as<uint64_t>();
  D.nitems = sc.dense_nitems;
  D.cp = cpt;
  D.Ct = Ct;
  D.x = x;
  D.xld = ldc;
  D.r = r;
  D.out = out;
  D.old = ldc;
  D.acc = acc;
  D.key0 = static_cast<uint32_t>(seed);
  D.key1 = static_cast<uint32_t>(seed >> 32);
  D.err = errf;
  D.rec_cap = plan.rec_cap;
  D.bucket_shift = shift;
  D.gshift = plan.gshift;
  D.nbins_g = nbins_g;
  const unsigned fgrid = grid_for(n, 256, 4096);
  const unsigned cgrid = grid_for(static_cast<int64_t>(cells), 256, 8192);
  for (int32_t i = 0; i <= L; ++i) {
    uint8_t* fcur = flags2[i & 1];
    uint8_t* fnext = flags2[(i + 1) & 1];
    D.rho = rho[i];
    D.kappa = kappa[i];
    D.level = i;
    D.lflags = (i == L ? kLastLevel : 0) | (a == 0.0 ? kAZero : 0);
    D.counters = counters + static_cast<size_t>(i) * kNumCounters;
    D.mass = mass + i;
    D.flag_in = fcur;
    const bool bin_level = binned && i < L;
    D.rec = bin_level ? sc.rec[0].as<uint32_t>() : nullptr;
    D.rec_count = bin_level ? rec_counts + static_cast<size_t>(i) * ng : nullptr;
    D.bucket_count = bin_level ? bucket_count : nullptr;
    D.det_bins = bin_level ? det_bins : nullptr;
    if (stats) AGP_HIP(hipEventRecord(ev[4 * i], s));
    if (i < L) k_fill_u8<<<fgrid, 256, 0, s>>>(fnext, static_cast<size_t>(n), 0);
    if (stats) AGP_HIP(hipEventRecord(ev[4 * i + 1], s));
    if (i == 0)
      k_dense_level<true><<<tune.level_blocks, dense::kThreads, 0, s>>>(D);
    else
      k_dense_level<false><<<tune.level_blocks, dense::kThreads, 0, s>>>(D);
    if (stats) AGP_HIP(hipEventRecord(ev[4 * i + 2], s));
    if (i > 0 && sc.dense_nrows > 0)
      k_dense_clear_rows<<<grid_for(sc.dense_nrows * Ct, 256, 1024), 256, 0, s>>>(sc.dense_rows.as<uint32_t>(),
                                                                                   sc.dense_nrows, Ct, r);
    if (i < L) {
      if (bin_level) {
        int* md = mode + i;
        k_dense_bins_scan<<<ng, kBuckets, 0, s>>>(bucket_count, bucket_off, cursor, D.rec_count, plan.rec_cap, md);
        for (int gi = 0; gi < ng; ++gi) {
          const int wgi = std::min(gw, Ct - gi * gw);
          const unsigned long long gcells = static_cast<unsigned long long>(n) * static_cast<unsigned long long>(wgi);
          const long long nbins = static_cast<long long>(((gcells > 0 ? gcells : 1) - 1) >> kBinLog2) + 1;
          uint32_t* r0 = sc.rec[0].as<uint32_t>() + static_cast<size_t>(gi) * plan.rec_cap;
          uint32_t* r1 = sc.rec[1].as<uint32_t>() + static_cast<size_t>(gi) * plan.rec_cap;
          const unsigned long long* rc_g = D.rec_count + gi;
          k_partition<<<1024, kReduceThreads, 0, s>>>(r0, rc_g, cursor + static_cast<size_t>(gi) * kBuckets, r1, md,
                                                      shift);
          k_bin_count<<<2048, kReduceThreads, 0, s>>>(r1, rc_g, bin_count, md, shift);
          k_bin_scan<<<static_cast<unsigned>(nbins / kScanChunk + 1), 1024, 0, s>>>(bin_count, nbins, bin_off,
                                                                                 bin_cur, md);
          k_bin_scatter<<<2048, kReduceThreads, 0, s>>>(r1, rc_g, bin_cur, r0, md, shift, bin_count, nbins);
          k_dense_bin_sum<<<static_cast<unsigned>(nbins), dense::kSumThreads, 0, s>>>(
              r0, bin_off, cpt, Ct, gi * gw, wgi, gcells, acc, r, fnext, md, det_bins + static_cast<size_t>(gi) * nbins_g);
        }
        k_dense_apply_overflow<<<2048, 256, 0, s>>>(D, ng, md);
        k_dense_finish<<<cgrid, 256, 0, s>>>(cpt, n, Ct, acc, r, fnext, md);
      } else {
        k_dense_finish<<<cgrid, 256, 0, s>>>(cpt, n, Ct, acc, r, fnext, nullptr);
      }
    }
    if (stats) AGP_HIP(hipEventRecord(ev[4 * i + 3], s));
  }
  AGP_HIP(hipGetLastError());
  int herr = 0;
  double hmass[AGP_MAX_LEVELS + 1];
  AGP_HIP(hipMemcpyAsync(&herr, errf, sizeof(int), hipMemcpyDeviceToHost, s));
  AGP_HIP(hipMemcpyAsync(hmass, mass, sizeof(double) * (L + 1), hipMemcpyDeviceToHost, s));
  AGP_HIP(hipStreamSynchronize(s));
  for (int32_t i = 0; i <= L; ++i)
    if (!(hmass[i] < 0x1p61)) herr |= 1;
  if (herr) {  // restore the all-zero invariant of the sums and residues
    AGP_HIP(hipMemsetAsync(sc.acc[0].ptr, 0, sc.acc[0].bytes, s));
    AGP_HIP(hipMemsetAsync(sc.acc[1].ptr, 0, sc.acc[1].bytes, s));
    AGP_HIP(hipStreamSynchronize(s));
    return fail(AGP_ERANGE, std::string(fn) + ": a residue outgrew the exact accumulator range");
  }
  if (std::getenv("AGP_CHECK_ZERO")) {  // debugging aid: the sums and residues must be all-zero again
    std::vector<long long> ha(cells);
    std::vector<float> hr(cells);
    AGP_HIP(hipMemcpy(ha.data(), acc, cells * sizeof(long long), hipMemcpyDeviceToHost));
    AGP_HIP(hipMemcpy(hr.data(), r, cells * sizeof(float), hipMemcpyDeviceToHost));
    for (size_t k = 0; k < cells; ++k)
      if (ha[k] != 0 || hr[k] != 0.0f)
        return fail(AGP_EDEVICE, std::string(fn) + ": scratch not cleared at cell " + std::to_string(k) +
                                     " (acc " + std::to_string(ha[k]) + ", r " + std::to_string(hr[k]) + ")");
  }
  if (stats) {
    stats->tiles += 1;
    stats->dense = 1;
    std::vector<unsigned long long> h(static_cast<size_t>(kNumCounters) * (L + 1));
    AGP_HIP(hipMemcpy(h.data(), counters, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    for (int32_t i = 0; i <= L; ++i) {
      stats->frontier[i] += h[i * kNumCounters + 0];
      stats->hash[i] += h[i * kNumCounters + 1];
      stats->det[i] += h[i * kNumCounters + 2];
      stats->cand[i] += h[i * kNumCounters + 3];
      stats->acc[i] += h[i * kNumCounters + 4];
      stats->runs[i] += h[i * kNumCounters + 5];
    }
    float ms = 0.0f;
    for (int32_t i = 0; i <= L; ++i) {
      AGP_HIP(hipEventElapsedTime(&ms, ev[4 * i + 1], ev[4 * i + 2]));
      stats->level_ms[i] += ms;
      AGP_HIP(hipEventElapsedTime(&ms, ev[4 * i], ev[4 * i + 3]));
      stats->level_total_ms[i] += ms;
    }
    AGP_HIP(hipEventElapsedTime(&ms, ev[0], ev[4 * L + 3]));
    stats->device_ms += ms;
  }
  return AGP_OK;
}

// Thresholds of all C columns (theta, units, qids) into cp and the number of
// non-zero entries of x; synchronous.  flags_out gets the signal flags
// (1: non-finite entry, 2: negative entry).
template <typename T>
int all_thresholds(agp_graph* g, const T* x, int32_t C, double eps, const uint32_t* qids, ColParams* cp,
                   uint32_t* dq, hipStream_t s, unsigned long long* nnz_out, int* flags_out) {
  Scratch& sc = g->scratch;
  const int64_t n = g->n;
  const int64_t tblocks = (n + kThetaRows - 1) / kThetaRows;
  int rc;
  if ((rc = sc.partial.reserve(sizeof(double) * (size_t)std::max<int64_t>(tblocks, 1) * C, false, s)) ||
      (rc = sc.flags.reserve(sizeof(int) * 4, false, s)) || (rc = sc.counts.reserve(sizeof(unsigned long long) * 4, false, s)))
    return rc;
  int* flags = sc.flags.as<int>();
  unsigned long long* nnz = sc.counts.as<unsigned long long>();
  AGP_HIP(hipMemsetAsync(flags, 0, sc.flags.bytes, s));
  AGP_HIP(hipMemsetAsync(nnz, 0, sizeof(unsigned long long), s));
  if (qids) AGP_HIP(hipMemcpyAsync(dq, qids, sizeof(uint32_t) * C, hipMemcpyHostToDevice, s));
  if (tblocks > 0) {
    dim3 grid((unsigned)tblocks, (unsigned)((C + 63) / 64));
    k_theta_scan<T><<<grid, kWave, 0, s>>>(x, static_cast<long long>(C), n, C, sc.partial.as<double>(), flags + 1, nnz);
  }
  k_theta_final<T><<<grid_for(C, 64), 64, 0, s>>>(sc.partial.as<double>(), tblocks, C, eps, qids ? dq : nullptr, 0u,
                                                  cp);
  AGP_HIP(hipGetLastError());
  int hflags[4] = {0, 0, 0, 0};
  unsigned long long hnnz = 0;
  AGP_HIP(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
  AGP_HIP(hipMemcpyAsync(&hnnz, nnz, sizeof(hnnz), hipMemcpyDeviceToHost, s));
  AGP_HIP(hipStreamSynchronize(s));
  *nnz_out = hnnz;
  *flags_out = hflags[1];
  return AGP_OK;
}

// The dense path of a binary32 call: thresholds of all columns, then (when
// the tuning asks for it, or at least a quarter of x is non-zero) dense
// tiles.  Returns kNotDense to leave the call to the frontier-list path.
constexpr int kNotDense = -1;

int propagate_dense(agp_graph* g, const char* fn, const agp_tuning_t& tune, double a, double b,
                    const double* rho, const double* kappa, int32_t L, const float* x,
                    int32_t C, double eps, uint64_t seed, const uint32_t* qids, float* out, hipStream_t s,
                    agp_stats_t* stats) {
  const int64_t n = g->n;
  if (n == 0) return kNotDense;
  const bool may_bin = tune.aggregation == 1 || tune.aggregation == 2;
  const DensePlan plan = dense_plan(g, C, tune, may_bin);
  if (plan.ng == 0 || plan.Ct < 1) return kNotDense;
  Scratch& sc = g->scratch;
  int rc;
  if ((rc = sc.colparams.reserve(sizeof(ColParams) * C + sizeof(uint32_t) * C, false, s))) return rc;
  ColParams* cp = sc.colparams.as<ColParams>();
  uint32_t* dq = reinterpret_cast<uint32_t*>(cp + C);
  unsigned long long nnz = 0;
  int xflags = 0;
  if ((rc = all_thresholds<float>(g, x, C, eps, qids, cp, dq, s, &nnz, &xflags))) return rc;
  if (xflags & 1) return fail(AGP_EINVAL, std::string(fn) + ": x holds a non-finite value");
  const double cells = static_cast<double>(n) * static_cast<double>(C);
  if (tune.dense == 2 && static_cast<double>(nnz) < 0.25 * cells) return kNotDense;
  for (int32_t c0 = 0; c0 < C; c0 += plan.Ct) {
    const int32_t ct = std::min(plan.Ct, C - c0);
    rc = propagate_dense_tile(g, fn, tune, plan, a, b, rho, kappa, L, x + c0, static_cast<long long>(C), ct, cp + c0,
                              seed, out + c0, s, stats);
    if (rc != AGP_OK) return rc;
  }
  return AGP_OK;
}

// borrowed: a fixed scratch region instead of the graph's (nothing is
// allocated: frontier lists, atomics, one tile of all columns, degree-power
// tables that already exist); name: the entry point named in errors.
template <typename T>
int propagate_impl(agp_graph* g, double a, double b, const double* w, int32_t L, const T* x,
                   int32_t C, double eps, uint64_t seed, const uint32_t* qids, T* out,
                   hipStream_t s, agp_stats_t* stats, const agp_tuning_t* force = nullptr,
                   bool tail = false, Scratch* borrowed = nullptr, const char* name = nullptr) {
  const char* fn = name ? name : (sizeof(T) == 4 ? "agp_propagate" : "agp_propagate_f64");
  if (!g) return fail(AGP_EINVAL, std::string(fn) + ": NULL graph");
  if (!(a >= 0.0 && a <= 1.0) || !(b >= 0.0 && b <= 1.0))
    return fail(AGP_EINVAL, std::string(fn) + ": a and b must lie in [0, 1]");
  if (L < 0 || L > AGP_MAX_LEVELS) return fail(AGP_EINVAL, std::string(fn) + ": need 0 <= L <= 255");
  if (C < 1) return fail(AGP_EINVAL, std::string(fn) + ": need C >= 1");
  if (!w || !x || !out) return fail(AGP_EINVAL, std::string(fn) + ": NULL array");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(AGP_EINVAL, std::string(fn) + ": need eps >= 0");
  if (eps == 0.0)
    return fail(AGP_ENOTSUP, std::string(fn) + ": eps = 0 (Algorithm 1) is not supported on the GPU path");
  for (int32_t i = 0; i <= L; ++i)
    if (!(w[i] >= 0.0) || !std::isfinite(w[i]))
      return fail(AGP_EINVAL, std::string(fn) + ": weights must be finite and >= 0");
  if (qids) {
    for (int32_t c = 0; c < C; ++c)
      if (qids[c] >= (1u << 24)) return fail(AGP_EINVAL, std::string(fn) + ": qid must be < 2^24");
  } else if (C > (1 << 24)) {
    return fail(AGP_EINVAL, std::string(fn) + ": more than 2^24 columns need explicit qids");
  }
  const int64_t n = g->n;
  const size_t cells = static_cast<size_t>(n) * static_cast<size_t>(C);
  if (n > 0 && cells / static_cast<size_t>(n) != static_cast<size_t>(C))
    return fail(AGP_EINVAL, std::string(fn) + ": n * C overflows");

  // level tables in binary64: Y_i = Y_{L+1} + sum_{k=i..L} w_k added from
  // k = L down, S = Y_0, rho_i = Y_{i+1} / Y_i (0 at i = L), kappa_i =
  // (S w_i) / Y_i.  Y_{L+1} = 0 (weights beyond L are 0), or with the
  // infinite tail the mass 1 - (w_0 + ... + w_L) of the terms beyond L
  // (Definition 3.2 for a sequence summing to 1), dropped after level L.
  double tail_mass = 0.0;
  if (tail) {
    double total = 0.0;
    for (int32_t k = 0; k <= L; ++k) total += w[k];
    if (!(total <= 1.0 + 1e-9))
      return fail(AGP_EINVAL, std::string(fn) + ": the infinite tail needs w_0 + ... + w_L <= 1");
    tail_mass = total < 1.0 ? 1.0 - total : 0.0;
  }
  double Y[AGP_MAX_LEVELS + 2], rho[AGP_MAX_LEVELS + 1], kappa[AGP_MAX_LEVELS + 1];
  Y[L + 1] = tail_mass;
  for (int32_t k = L; k >= 0; --k) Y[k] = Y[k + 1] + w[k];
  const double S = Y[0];
  for (int32_t i = 0; i <= L; ++i) {
    rho[i] = (Y[i] == 0.0 || i == L) ? 0.0 : Y[i + 1] / Y[i];
    kappa[i] = (Y[i] == 0.0) ? 0.0 : (S * w[i]) / Y[i];
  }

  std::lock_guard<std::mutex> lk(g->mu);
  agp_tuning_t tune = tuning_for(g, C, a, b, force);
  Scratch& sc = borrowed ? *borrowed : g->scratch;
  const bool may_alloc = borrowed == nullptr;
  if (borrowed) {
    tune.aggregation = 0;
    tune.dense = 0;
    tune.capture = 0;
  }
  auto run = [&]() -> int {
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if constexpr (std::is_same<T, float>::value) {
      if (may_alloc && (tune.dense == 1 || (tune.dense == 2 && C >= 16))) {
        const int rc = propagate_dense(g, fn, tune, a, b, rho, kappa, L, x, C, eps, seed, qids, out, s, stats);
        if (rc != kNotDense) {
          if (rc == AGP_OK && stats) {
            stats->levels = L;
            stats->columns = C;
          }
          return rc;
        }
      }
    }
    const bool may_bin = (tune.aggregation == 1 || tune.aggregation == 2) && sizeof(T) == 4;
    const int32_t tile = std::min(borrowed ? C : column_tile<T>(g, C, may_bin, tune), kMaxTileColumns);
    AGP_HIP(hipMemsetAsync(out, 0, cells * sizeof(T), s));
    for (int32_t c0 = 0; c0 < C; c0 += tile) {
      const int32_t ct = std::min(tile, C - c0);
      const int rc = propagate_tile<T>(g, fn, tune, a, b, rho, kappa, L, x + c0, static_cast<long long>(C), ct,
                                       eps, seed, qids ? qids + c0 : nullptr, static_cast<uint32_t>(c0), out + c0,
                                       s, stats, sc, may_alloc);
      if (rc != AGP_OK) return rc;
    }
    if (stats) {
      stats->levels = L;
      stats->columns = C;
    }
    return AGP_OK;
  };
  int rc = run();
  if (rc == AGP_ENOMEM && may_alloc) {
    // buffers an earlier call shaped differently (another path, tile or
    // mode) may hold the memory this one needs: release them all, once
    (void)hipStreamSynchronize(s);
    g->drop_loops();
    g->scratch.release();
    rc = run();
  }
  return rc;
}

// ------------------------------------------------- literal sign split
// x (n x C, rows ld apart) -> x2 (n x 2C): columns [0, C) hold the positive
// entries, [C, 2C) the negative ones (zeros elsewhere).
template <typename T>
__global__ void k_split_signs(const T* __restrict__ x, long long ld, int64_t n, int C, T* __restrict__ x2) {
  const int64_t total = n * C;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t u = i / C;
    const int c = static_cast<int>(i - u * C);
    const T v = x[u * ld + c];
    T* row = x2 + u * (2 * static_cast<int64_t>(C));
    row[c] = v > T(0) ? v : T(0);
    row[C + c] = v < T(0) ? v : T(0);
  }
}

// out[u, c] = o2[u, c] + o2[u, C + c], rounded once.
template <typename T>
__global__ void k_join_signs(const T* __restrict__ o2, int64_t n, int C, T* __restrict__ out, long long ld) {
  const int64_t total = n * C;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t u = i / C;
    const int c = static_cast<int>(i - u * C);
    const T* row = o2 + u * (2 * static_cast<int64_t>(C));
    out[u * ld + c] = row[c] + row[C + c];
  }
}

void add_stats(agp_stats_t* into, const agp_stats_t& part) {
  for (int i = 0; i <= AGP_MAX_LEVELS; ++i) {
    into->frontier[i] += part.frontier[i];
    into->hash[i] += part.hash[i];
    into->det[i] += part.det[i];
    into->cand[i] += part.cand[i];
    into->acc[i] += part.acc[i];
    into->runs[i] += part.runs[i];
    into->level_ms[i] += part.level_ms[i];
    into->level_total_ms[i] += part.level_total_ms[i];
  }
  into->device_ms += part.device_ms;
  into->tiles += part.tiles;
  into->dense |= part.dense;
}

// The literal treatment of signed signals (Section 3, assumption on the
// graph signal): per tile of columns, x+ and x- as 2 ct columns of one
// batched call (column c's x- part on the stream of query id qid_c + 2^23),
// then pi = pi+ + pi-.
template <typename T>
int propagate_split(agp_graph* g, double a, double b, const double* w, int32_t L, const T* x, int32_t C,
                    double eps, uint64_t seed, const uint32_t* qids, T* out, hipStream_t s, agp_stats_t* stats,
                    bool tail) {
  const char* fn = sizeof(T) == 4 ? "agp_propagate_variant" : "agp_propagate_variant_f64";
  if (!g || !x || !out || !w) return fail(AGP_EINVAL, std::string(fn) + ": NULL argument");
  if (C < 1) return fail(AGP_EINVAL, std::string(fn) + ": need C >= 1");
  if (qids) {
    for (int32_t c = 0; c < C; ++c)
      if (qids[c] >= kSplitQid) return fail(AGP_EINVAL, std::string(fn) + ": the sign split needs qids < 2^23");
  } else if (C > static_cast<int32_t>(kSplitQid)) {
    return fail(AGP_EINVAL, std::string(fn) + ": the sign split needs C <= 2^23 without qids");
  }
  const int64_t n = g->n;
  if (n == 0) return propagate_impl<T>(g, a, b, w, L, x, C, eps, seed, qids, out, s, stats, nullptr, tail);
  // tiles of columns whose doubled signal and result take at most a quarter
  // of the free memory
  size_t free_b = 0, total_b = 0;
  AGP_HIP(hipMemGetInfo(&free_b, &total_b));
  const double per_col = 4.0 * static_cast<double>(n) * sizeof(T);
  int32_t tile = static_cast<int32_t>(std::min<double>(C, std::max(1.0, 0.25 * free_b / per_col)));
  DevBuf x2, o2;
  int rc;
  if ((rc = x2.reserve(static_cast<size_t>(n) * 2 * tile * sizeof(T), false, s)) ||
      (rc = o2.reserve(static_cast<size_t>(n) * 2 * tile * sizeof(T), false, s))) {
    x2.release();
    o2.release();
    return rc;
  }
  if (stats) std::memset(stats, 0, sizeof(*stats));
  std::vector<uint32_t> q2(2 * static_cast<size_t>(tile));
  for (int32_t c0 = 0; c0 < C && rc == AGP_OK; c0 += tile) {
    const int32_t ct = std::min(tile, C - c0);
    for (int32_t c = 0; c < ct; ++c) {
      const uint32_t q = qids ? qids[c0 + c] : static_cast<uint32_t>(c0 + c);
      q2[c] = q;
      q2[ct + c] = q + kSplitQid;
    }
    const unsigned grid = static_cast<unsigned>(std::min<int64_t>((n * ct + 255) / 256, 65536));
    k_split_signs<T><<<grid, 256, 0, s>>>(x + c0, static_cast<long long>(C), n, ct, x2.as<T>());
    agp_stats_t part;
    rc = propagate_impl<T>(g, a, b, w, L, x2.as<T>(), 2 * ct, eps, seed, q2.data(), o2.as<T>(), s,
                           stats ? &part : nullptr, nullptr, tail);
    if (rc != AGP_OK) break;
    k_join_signs<T><<<grid, 256, 0, s>>>(o2.as<T>(), n, ct, out + c0, static_cast<long long>(C));
    if (stats) add_stats(stats, part);
  }
  if (rc == AGP_OK) {
    const hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = fail(AGP_EDEVICE, std::string(fn) + ": " + hipGetErrorString(e));
  }
  x2.release();
  o2.release();
  if (rc == AGP_OK && stats) {
    stats->levels = L;
    stats->columns = C;
  }
  return rc;
}

template <typename T>
int propagate_variant(const agp_graph_t* g, double a, double b, const double* w, int32_t L, const T* x, int32_t C,
                      double eps, uint64_t seed, const uint32_t* qids, uint32_t variant, T* out, void* stream,
                      agp_stats_t* stats) {
  const char* fn = sizeof(T) == 4 ? "agp_propagate_variant" : "agp_propagate_variant_f64";
  if (variant & ~(AGP_VARIANT_INFINITE_TAIL | AGP_VARIANT_SPLIT_SIGNS))
    return fail(AGP_EINVAL, std::string(fn) + ": unknown variant flag");
  const bool tail = (variant & AGP_VARIANT_INFINITE_TAIL) != 0;
  agp_graph* gg = const_cast<agp_graph*>(g);
  if (variant & AGP_VARIANT_SPLIT_SIGNS)
    return propagate_split<T>(gg, a, b, w, L, x, C, eps, seed, qids, out, (hipStream_t)stream, stats, tail);
  return propagate_impl<T>(gg, a, b, w, L, x, C, eps, seed, qids, out, (hipStream_t)stream, stats, nullptr, tail);
}

}  // namespace
}  // namespace agp

namespace agp {
using namespace lvl;
// ------------------------------------------------ allocation-free calls
// One fixed scratch array per device (the library's static device memory),
// for callers that cannot allocate.  In host code `scratch` names a host-side
// stand-in: only the address hipGetSymbolAddress returns for the current
// device may reach a kernel or a copy.
static __device__ __align__(256) unsigned char scratch[AGP_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu[kNoAllocDevices];   // one call at a time per device (they share the array)
void* g_noalloc_base[kNoAllocDevices] = {};  // device address of the array, per device

__global__ void k_zero_words(unsigned long long* p, size_t nwords) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// Successive 256-byte aligned regions of [base, base + cap) as borrowed buffers.
struct Carve {
  char* base;
  size_t cap;
  size_t off = 0;
  bool take(DevBuf& b, size_t bytes) {
    const size_t at = (off + 255) & ~static_cast<size_t>(255);
    const size_t len = bytes > 0 ? bytes : 8;
    if (at > cap || len > cap - at) return false;
    b.ptr = base + at;
    b.bytes = len;
    b.borrowed = true;
    off = at + len;
    return true;
  }
};
}  // namespace

int propagate_noalloc(agp_graph* g, double a, double b, const double* w, int32_t L, const float* x, int32_t C,
                      double eps, uint64_t seed, const uint32_t* qids, float* out, hipStream_t s) {
  const char* fn = "agp_propagate_noalloc";
  if (!g) return fail(AGP_EINVAL, std::string(fn) + ": NULL graph");
  if (C < 1) return fail(AGP_EINVAL, std::string(fn) + ": need C >= 1");
  int dev = 0;
  AGP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocDevices) return fail(AGP_EDEVICE, std::string(fn) + ": device index out of range");
  std::lock_guard<std::mutex> lk(g_noalloc_mu[dev]);
  if (!g_noalloc_base[dev]) {  // first call on this device: the array's address here
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return fail(AGP_EDEVICE, std::string(fn) + ": hipGetSymbolAddress of the scratch array failed: " +
                                   hipGetErrorString(e));
    }
    g_noalloc_base[dev] = p;
  }
  // the buffers of one tile of all C columns (frontier lists, atomics)
  using Cell = Prec<float>::Cell;
  const int64_t n = g->n;
  const size_t cells = static_cast<size_t>(n) * static_cast<size_t>(C);
  if (n > 0 && cells / static_cast<size_t>(n) != static_cast<size_t>(C))
    return fail(AGP_EINVAL, std::string(fn) + ": n * C overflows");
  const int64_t tblocks = (n + kThetaRows - 1) / kThetaRows;
  Scratch v;
  Carve cv{static_cast<char*>(g_noalloc_base[dev]), static_cast<size_t>(AGP_NOALLOC_SCRATCH_BYTES)};
  const bool fits = cells <= (static_cast<size_t>(AGP_NOALLOC_SCRATCH_BYTES) / sizeof(Cell)) &&
                    cv.take(v.acc[0], cells * sizeof(Cell)) && cv.take(v.acc[1], cells * sizeof(Cell)) &&
                    cv.take(v.frontier[0], cells * sizeof(uint64_t)) &&
                    cv.take(v.frontier[1], cells * sizeof(uint64_t)) &&
                    cv.take(v.counts, sizeof(unsigned long long) * (AGP_MAX_LEVELS + 2)) &&
                    cv.take(v.counters, sizeof(unsigned long long) * kNumCounters * (AGP_MAX_LEVELS + 1)) &&
                    cv.take(v.colparams, sizeof(ColParams) * C + sizeof(uint32_t) * C) &&
                    cv.take(v.partial, sizeof(double) * static_cast<size_t>(std::max<int64_t>(tblocks, 1)) * C) &&
                    cv.take(v.flags, sizeof(int) * 4) &&
                    cv.take(v.levelinfo, (2 * sizeof(double) + sizeof(int)) * (AGP_MAX_LEVELS + 2) + 256 +
                                              sizeof(LevelParams) * (AGP_MAX_LEVELS + 1));
  if (!fits)
    return fail(AGP_EINVAL, std::string(fn) + ": n * C = " + std::to_string(cells) + " cells need about " +
                                std::to_string(cells * 2 * (sizeof(Cell) + sizeof(uint64_t))) +
                                " bytes of scratch; the fixed array holds " +
                                std::to_string(static_cast<size_t>(AGP_NOALLOC_SCRATCH_BYTES)));
  // the residue accumulators start at zero (the array keeps the last call's contents)
  const size_t words = 2 * cells * sizeof(Cell) / sizeof(unsigned long long);
  k_zero_words<<<grid_for(static_cast<int64_t>(words > 0 ? words : 1), 256, 4096), 256, 0, s>>>(
      static_cast<unsigned long long*>(v.acc[0].ptr), cells * sizeof(Cell) / sizeof(unsigned long long));
  k_zero_words<<<grid_for(static_cast<int64_t>(words > 0 ? words : 1), 256, 4096), 256, 0, s>>>(
      static_cast<unsigned long long*>(v.acc[1].ptr), cells * sizeof(Cell) / sizeof(unsigned long long));
  AGP_HIP(hipGetLastError());
  return propagate_impl<float>(g, a, b, w, L, x, C, eps, seed, qids, out, s, nullptr, nullptr, false, &v, fn);
}
}  // namespace agp

extern "C" {

int agp_autotune(const agp_graph_t* g, double a, double b, const double* w, int32_t L, const float* x,
                 int32_t C, double eps, uint64_t seed, const uint32_t* qids, float* out, void* stream,
                 agp_tuning_t* best) {
  using namespace agp;
  agp_graph* gg = const_cast<agp_graph*>(g);
  if (!gg) return fail(AGP_EINVAL, "agp_autotune: NULL graph");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  AGP_HIP(hipEventCreate(&e0));
  AGP_HIP(hipEventCreate(&e1));
  // one untimed call with the defaults (allocations, graph work items)
  agp_tuning_t pick = default_tuning();
  int rc = propagate_impl<float>(gg, a, b, w, L, x, C, eps, seed, qids, out, s, nullptr, &pick);
  auto timed = [&](const agp_tuning_t& t, float* ms) {
    (void)hipEventRecord(e0, s);
    const int r = propagate_impl<float>(gg, a, b, w, L, x, C, eps, seed, qids, out, s, nullptr, &t);
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    *ms = 0.0f;
    (void)hipEventElapsedTime(ms, e0, e1);
    return r;
  };
  float best_ms = 0.0f;
  if (rc == AGP_OK) rc = timed(pick, &best_ms);
  // coordinate descent: each field's candidates with the others fixed at the
  // best so far (every candidate gives the same bits)
  auto field = [&](int32_t agp_tuning_t::*f, std::initializer_list<int32_t> vals) {
    for (int32_t v : vals) {
      if (rc != AGP_OK) return;
      agp_tuning_t t = pick;
      if (t.*f == v) continue;
      t.*f = v;
      float ms = 0.0f;
      const int r = timed(t, &ms);
      if (r == AGP_ENOMEM) continue;  // the candidate does not fit: not a choice here
      rc = r;
      if (rc == AGP_OK && ms < best_ms) {
        best_ms = ms;
        pick = t;
      }
    }
  };
  if (C >= 2) field(&agp_tuning_t::dense, {0, 1});
  field(&agp_tuning_t::aggregation, {0, 1, 2});
  field(&agp_tuning_t::level_blocks, {1024, 2048, 4096, 8192});
  if (C >= 4) field(&agp_tuning_t::tile_columns, {0, (C + 1) / 2, (C + 3) / 4});
  if (pick.dense != 1) {  // cut-offs of the frontier-list levels
    field(&agp_tuning_t::big_row, {1024, 4096, 16384});
    field(&agp_tuning_t::big_items, {16, 64, 256});
    field(&agp_tuning_t::sparse_shift, {3, 5, 7});
    if (pick.aggregation == 2) field(&agp_tuning_t::bin_shift, {2, 3, 5});
    field(&agp_tuning_t::capture, {0, 1});
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != AGP_OK) return rc;
  pick = normalize_tuning(pick);
  {
    std::lock_guard<std::mutex> lk(gg->mu);
    gg->tuning[agp_tune_key{C, a, b}] = pick;
  }
  // `out` holds the result of the last candidate (identical for every one)
  if (best) *best = pick;
  return AGP_OK;
}

int agp_get_tuning(const agp_graph_t* g, int32_t C, double a, double b, agp_tuning_t* out) {
  using namespace agp;
  if (!g || !out) return fail(AGP_EINVAL, "agp_get_tuning: NULL argument");
  agp_graph* gg = const_cast<agp_graph*>(g);
  std::lock_guard<std::mutex> lk(gg->mu);
  *out = tuning_for(gg, C, a, b, nullptr);
  return AGP_OK;
}

int agp_set_tuning(const agp_graph_t* g, int32_t C, double a, double b, const agp_tuning_t* t) {
  using namespace agp;
  if (!g) return fail(AGP_EINVAL, "agp_set_tuning: NULL graph");
  agp_graph* gg = const_cast<agp_graph*>(g);
  std::lock_guard<std::mutex> lk(gg->mu);
  if (t)
    gg->tuning[agp_tune_key{C, a, b}] = normalize_tuning(*t);
  else
    gg->tuning.erase(agp_tune_key{C, a, b});
  return AGP_OK;
}

int agp_propagate(const agp_graph_t* g, double a, double b, const double* w, int32_t L, const float* x,
                  int32_t C, double eps, uint64_t seed, const uint32_t* qids, float* out, void* stream,
                  agp_stats_t* stats) {
  return agp::propagate_impl<float>(const_cast<agp_graph_t*>(g), a, b, w, L, x, C, eps, seed, qids, out,
                                    (hipStream_t)stream, stats);
}

int agp_propagate_f64(const agp_graph_t* g, double a, double b, const double* w, int32_t L,
                      const double* x, int32_t C, double eps, uint64_t seed, const uint32_t* qids,
                      double* out, void* stream, agp_stats_t* stats) {
  return agp::propagate_impl<double>(const_cast<agp_graph_t*>(g), a, b, w, L, x, C, eps, seed, qids, out,
                                     (hipStream_t)stream, stats);
}

int agp_propagate_noalloc(const agp_graph_t* g, double a, double b, const double* w, int32_t L, const float* x,
                          int32_t C, double eps, uint64_t seed, const uint32_t* qids, float* out, void* stream) {
  return agp::propagate_noalloc(const_cast<agp_graph_t*>(g), a, b, w, L, x, C, eps, seed, qids, out,
                                (hipStream_t)stream);
}

int agp_propagate_variant(const agp_graph_t* g, double a, double b, const double* w, int32_t L, const float* x,
                          int32_t C, double eps, uint64_t seed, const uint32_t* qids, uint32_t variant, float* out,
                          void* stream, agp_stats_t* stats) {
  return agp::propagate_variant<float>(g, a, b, w, L, x, C, eps, seed, qids, variant, out, stream, stats);
}

int agp_propagate_variant_f64(const agp_graph_t* g, double a, double b, const double* w, int32_t L,
                              const double* x, int32_t C, double eps, uint64_t seed, const uint32_t* qids,
                              uint32_t variant, double* out, void* stream, agp_stats_t* stats) {
  return agp::propagate_variant<double>(g, a, b, w, L, x, C, eps, seed, qids, variant, out, stream, stats);
}

}  // extern "C"
