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
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "agp_internal.h"
#include "level_kernels.h"

namespace agp {
namespace {

using namespace lvl;

// ---------------------------------------------------------- thresholds
// ||x_c||_1 in binary64: sequential over blocks of 4096 rows, then over the
// block sums.  flags: 1 = non-finite entry, 2 = negative entry.
template <typename T>
__global__ void k_theta_partial(const T* __restrict__ x, long long ldx, int64_t n, int C,
                                double* __restrict__ partial, int* __restrict__ flags) {
  const int c = blockIdx.y * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int64_t lo = (int64_t)blockIdx.x * kThetaRows;
  const int64_t hi = (lo + kThetaRows) < n ? lo + kThetaRows : n;
  double sum = 0.0;
  int f = 0;
  for (int64_t i = lo; i < hi; ++i) {
    const T v = x[static_cast<size_t>(i) * static_cast<size_t>(ldx) + c];
    if (!isfinite(static_cast<double>(v))) f |= 1;
    if (v < T(0)) f |= 2;
    sum = sum + fabs(static_cast<double>(v));
  }
  partial[(size_t)blockIdx.x * C + c] = sum;
  if (f) atomicOr(flags, f);
}

template <typename T>
__global__ void k_theta_final(const double* __restrict__ partial, int64_t nblocks, int C, double eps,
                              const uint32_t* __restrict__ qids, uint32_t qid_base, ColParams* __restrict__ cp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  double total = 0.0;
  for (int64_t b = 0; b < nblocks; ++b) total = total + partial[(size_t)b * C + c];
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
__global__ void k_set_level(ColParams* __restrict__ cp, int C, int level, double rho, double kappa,
                            int flags, const double* da, const double* db, uint32_t key0, uint32_t key1,
                            void* out, long long out_stride, size_t elem) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  ColParams& p = cp[c];
  p.level = level;
  p.rho = rho;
  p.kappa = kappa;
  p.flags = flags;
  p.da = da;
  p.db = db;
  p.key0 = key0;
  p.key1 = key1;
  p.out = static_cast<char*>(out) + static_cast<size_t>(c) * elem;
  p.out_stride = out_stride;
}

// ------------------------------------------------ binned aggregation
// After a binned level: bucket offsets (one block), then the records are
// partitioned into buckets, and one block per bucket splits its bucket into
// bins of 8192 cells, counts the signed records of every bin in LDS, adds
// count * fl(theta_c) in units to each cell (the deterministic pushes are
// already there: integer sums, so the order is irrelevant) and appends every
// non-zero cell to the next frontier.
constexpr int kMaxBinnedC = 1024;
constexpr int kReduceThreads = 512;

__global__ __launch_bounds__(1024) void k_bins_scan(unsigned int* __restrict__ bucket_count,
                                                    unsigned long long* __restrict__ bucket_off,
                                                    unsigned long long* __restrict__ cursor,
                                                    const unsigned long long* __restrict__ rec_count,
                                                    unsigned long long cap, int* __restrict__ mode) {
  __shared__ unsigned long long s[kBuckets];
  const int t = threadIdx.x;
  const int m = *mode;
  if (m != kModeBinned) return;
  const unsigned long long v = bucket_count[t];
  bucket_count[t] = 0;  // ready for the next level
  if (*rec_count > cap) {
    if (t == 0) *mode = kModeOverflow;
    return;
  }
  s[t] = v;
  __syncthreads();
  for (int off = 1; off < kBuckets; off <<= 1) {
    const unsigned long long add = t >= off ? s[t - off] : 0ull;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  const unsigned long long excl = s[t] - v;
  bucket_off[t] = excl;
  cursor[t] = excl;
  if (t == kBuckets - 1) bucket_off[kBuckets] = s[t];
}

__global__ __launch_bounds__(kThreads) void k_apply_overflow(LevelArgs A, long long* __restrict__ acc,
                                                             const int* __restrict__ mode) {
  if (*mode != kModeOverflow) return;
  const unsigned long long n = *A.rec_count < A.rec_cap ? *A.rec_count : A.rec_cap;
  for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < n;
       i += (unsigned long long)gridDim.x * blockDim.x)
    apply_record(A, acc, A.rec[i]);
}

constexpr int kBatchLoads = 8;  // records per thread per load batch (memory-level parallelism)

// Exclusive scan of v[0..1024) in LDS by a block of kReduceThreads threads
// (2 slots per thread) into out[0..1024); returns the total.  Ends with a
// block barrier.
__device__ __forceinline__ unsigned int block_scan_1024(const unsigned int* v, unsigned int* out,
                                                        unsigned int* wsum) {
  constexpr int kPer = kBuckets / kReduceThreads;
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  unsigned int x[kPer];
  unsigned int run = 0;
  for (int k = 0; k < kPer; ++k) {
    x[k] = v[threadIdx.x * kPer + k];
    run += x[k];
  }
  unsigned int incl = run;
  for (int off = 1; off < kWave; off <<= 1) {
    const unsigned int t = __shfl_up(incl, off);
    if (lane >= off) incl += t;
  }
  if (lane == kWave - 1) wsum[wave] = incl;
  __syncthreads();
  unsigned int acc0 = 0, total = 0;
  for (int w = 0; w < kReduceThreads / kWave; ++w) {
    if (w < wave) acc0 += wsum[w];
    total += wsum[w];
  }
  acc0 += incl - run;
  for (int k = 0; k < kPer; ++k) {
    out[threadIdx.x * kPer + k] = acc0;
    acc0 += x[k];
  }
  __syncthreads();
  return total;
}

// Partition of the records into buckets: a tile of 16384 records is sorted
// by bucket in LDS, then every bucket's run is written out contiguously.
constexpr int kPartPerThread = 32;
constexpr int kPartTile = kReduceThreads * kPartPerThread;

__global__ __launch_bounds__(kReduceThreads) void k_partition(const uint32_t* __restrict__ rec,
                                                              const unsigned long long* __restrict__ rec_count,
                                                              unsigned long long* __restrict__ cursor,
                                                              uint32_t* __restrict__ out,
                                                              const int* __restrict__ mode, int shift) {
  if (*mode != kModeBinned) return;
  __shared__ uint32_t s_rec[kPartTile];
  __shared__ unsigned int s_hist[kBuckets];
  __shared__ unsigned int s_loc[kBuckets];
  __shared__ unsigned long long s_base[kBuckets];
  __shared__ unsigned int s_wsum[kReduceThreads / kWave];
  const unsigned long long total = *rec_count;
  for (unsigned long long lo = (unsigned long long)blockIdx.x * kPartTile; lo < total;
       lo += (unsigned long long)gridDim.x * kPartTile) {
    const int nt = static_cast<int>(total - lo < (unsigned long long)kPartTile ? total - lo : kPartTile);
    for (int b = threadIdx.x; b < kBuckets; b += blockDim.x) s_hist[b] = 0;
    __syncthreads();
    uint32_t r[kPartPerThread];
    unsigned int rank[kPartPerThread];
#pragma unroll
    for (int k = 0; k < kPartPerThread; ++k) {
      const int i = k * kReduceThreads + threadIdx.x;  // coalesced
      r[k] = i < nt ? rec[lo + i] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kPartPerThread; ++k) {
      const int i = k * kReduceThreads + threadIdx.x;
      rank[k] = i < nt ? atomicAdd(&s_hist[(r[k] & kRecCellMask) >> shift], 1u) : 0u;
    }
    __syncthreads();
    block_scan_1024(s_hist, s_loc, s_wsum);
    for (int b = threadIdx.x; b < kBuckets; b += blockDim.x) {
      const unsigned int h = s_hist[b];
      s_base[b] = h ? atomicAdd(cursor + b, static_cast<unsigned long long>(h)) : 0ull;
    }
#pragma unroll
    for (int k = 0; k < kPartPerThread; ++k) {
      const int i = k * kReduceThreads + threadIdx.x;
      if (i < nt) s_rec[s_loc[(r[k] & kRecCellMask) >> shift] + rank[k]] = r[k];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nt; i += blockDim.x) {  // runs of one bucket are contiguous
      const uint32_t x = s_rec[i];
      const unsigned int b = (x & kRecCellMask) >> shift;
      out[s_base[b] + static_cast<unsigned long long>(i - static_cast<int>(s_loc[b]))] = x;
    }
    __syncthreads();
  }
}

// Reduce tiles: 8192 records (the LDS buffer doubles as one bin's counts).
constexpr int kRedPerThread = 16;
constexpr int kRedTile = kReduceThreads * kRedPerThread;

__global__ __launch_bounds__(kReduceThreads) void k_bin_reduce(const uint32_t* __restrict__ part,
                                                               uint32_t* __restrict__ tmp,
                                                               const unsigned long long* __restrict__ bucket_off,
                                                               const ColParams* __restrict__ cp, int C,
                                                               unsigned long long cells,
                                                               long long* __restrict__ acc, uint64_t* __restrict__ F,
                                                               unsigned long long* __restrict__ cnt,
                                                               const int* __restrict__ mode, int shift) {
  if (*mode != kModeBinned) return;
  constexpr int kBin = 1 << kBinLog2;
  static_assert(kBin <= kRedTile, "bin counts share the tile buffer");
  const int kBinsPer = 1 << (shift - kBinLog2);  // <= kBuckets
  __shared__ uint32_t s_buf[kRedTile];           // a tile of records, or the counts of one bin
  __shared__ unsigned int s_cur[kBuckets];       // per bin: count, then next free slot in tmp
  __shared__ unsigned int s_off[kBuckets + 1];   // per bin: first slot in tmp
  __shared__ unsigned int s_lh[kBuckets];        // per bin: records in the tile
  __shared__ unsigned int s_lo[kBuckets];        // per bin: first slot in the sorted tile
  __shared__ unsigned int s_gb[kBuckets];        // per bin: tile's first slot in tmp
  __shared__ long long s_dth[kMaxBinnedC];
  __shared__ uint64_t s_stage[kReduceThreads / kWave][kStage / 2];
  __shared__ unsigned int s_wsum[kReduceThreads / kWave];
  int* s_cnt = reinterpret_cast<int*>(s_buf);
  uint64_t* stage = s_stage[threadIdx.x / kWave];
  int staged = 0;
  for (int c = threadIdx.x; c < C; c += blockDim.x) s_dth[c] = cp[c].dtheta;
  const unsigned long long nbuckets = ((cells - 1) >> shift) + 1;
  for (unsigned long long b = blockIdx.x; b < nbuckets; b += gridDim.x) {
    const unsigned long long lo = bucket_off[b], hi = bucket_off[b + 1];
    for (int f = threadIdx.x; f < kBuckets; f += blockDim.x) s_cur[f] = 0;
    __syncthreads();
    // bin sizes of the bucket
    for (unsigned long long i0 = lo + (unsigned long long)threadIdx.x * kBatchLoads; i0 < hi;
         i0 += (unsigned long long)blockDim.x * kBatchLoads) {
      uint32_t r[kBatchLoads];
#pragma unroll
      for (int k = 0; k < kBatchLoads; ++k) r[k] = (i0 + k < hi) ? part[i0 + k] : 0u;
#pragma unroll
      for (int k = 0; k < kBatchLoads; ++k)
        if (i0 + k < hi) atomicAdd(&s_cur[((r[k] & kRecCellMask) >> kBinLog2) & (kBinsPer - 1)], 1u);
    }
    __syncthreads();
    const unsigned int nrec = block_scan_1024(s_cur, s_off, s_wsum);
    if (threadIdx.x == 0) s_off[kBuckets] = nrec;
    for (int f = threadIdx.x; f < kBuckets; f += blockDim.x) s_cur[f] = s_off[f];
    __syncthreads();
    // records into bin order in tmp, one LDS-sorted tile at a time
    for (unsigned long long t0 = lo; t0 < hi; t0 += kRedTile) {
      const int nt = static_cast<int>(hi - t0 < (unsigned long long)kRedTile ? hi - t0 : kRedTile);
      for (int f = threadIdx.x; f < kBuckets; f += blockDim.x) s_lh[f] = 0;
      __syncthreads();
      uint32_t r[kRedPerThread];
      unsigned int rank[kRedPerThread];
#pragma unroll
      for (int k = 0; k < kRedPerThread; ++k) {
        const int i = k * kReduceThreads + threadIdx.x;
        r[k] = i < nt ? part[t0 + i] : 0u;
      }
#pragma unroll
      for (int k = 0; k < kRedPerThread; ++k) {
        const int i = k * kReduceThreads + threadIdx.x;
        rank[k] = i < nt ? atomicAdd(&s_lh[((r[k] & kRecCellMask) >> kBinLog2) & (kBinsPer - 1)], 1u) : 0u;
      }
      __syncthreads();
      block_scan_1024(s_lh, s_lo, s_wsum);
      for (int f = threadIdx.x; f < kBuckets; f += blockDim.x) {
        const unsigned int h = s_lh[f];
        s_gb[f] = h ? atomicAdd(&s_cur[f], h) : 0u;
      }
#pragma unroll
      for (int k = 0; k < kRedPerThread; ++k) {
        const int i = k * kReduceThreads + threadIdx.x;
        if (i < nt) s_buf[s_lo[((r[k] & kRecCellMask) >> kBinLog2) & (kBinsPer - 1)] + rank[k]] = r[k];
      }
      __syncthreads();
      for (int i = threadIdx.x; i < nt; i += blockDim.x) {
        const uint32_t x = s_buf[i];
        const unsigned int f = ((x & kRecCellMask) >> kBinLog2) & (kBinsPer - 1);
        tmp[lo + s_gb[f] + static_cast<unsigned int>(i - static_cast<int>(s_lo[f]))] = x;
      }
      __syncthreads();
    }
    // every bin: signed record counts in LDS, then each cell's new value
    for (int f = 0; f < kBinsPer; ++f) {
      const unsigned long long cell0 = (b << shift) | (static_cast<unsigned long long>(f) << kBinLog2);
      if (cell0 >= cells) break;  // uniform per block
      for (int j = threadIdx.x; j < kBin; j += blockDim.x) s_cnt[j] = 0;
      __syncthreads();
      const unsigned long long blo = lo + s_off[f], bhi = lo + s_off[f + 1];
      // loads in flight per thread: 16 records, then 16 cells
      for (unsigned long long i0 = blo + threadIdx.x; i0 < bhi; i0 += (unsigned long long)blockDim.x * 16) {
        uint32_t rr[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const unsigned long long i = i0 + (unsigned long long)k * blockDim.x;
          rr[k] = i < bhi ? tmp[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (i0 + (unsigned long long)k * blockDim.x < bhi)
            atomicAdd(&s_cnt[rr[k] & (kBin - 1)], (rr[k] >> 31) ? -1 : 1);
      }
      __syncthreads();
      constexpr int kCellsPer = kBin / kReduceThreads;
      long long vv[kCellsPer];
#pragma unroll
      for (int k = 0; k < kCellsPer; ++k) {
        const unsigned long long cell = cell0 + static_cast<unsigned long long>(k * kReduceThreads + threadIdx.x);
        vv[k] = cell < cells ? acc[cell] : 0ll;
      }
#pragma unroll
      for (int k = 0; k < kCellsPer; ++k) {  // wave-uniform
        const int j = k * kReduceThreads + threadIdx.x;
        const unsigned long long cell = cell0 + static_cast<unsigned long long>(j);
        const bool valid = cell < cells;
        long long v = vv[k];
        uint32_t u = 0, c = 0;
        if (valid) {
          u = static_cast<uint32_t>(cell / static_cast<unsigned long long>(C));
          c = static_cast<uint32_t>(cell - static_cast<unsigned long long>(u) * C);
          const int kc = s_cnt[j];
          if (kc != 0) {
            v += static_cast<long long>(kc) * s_dth[c];
            acc[cell] = v;
          }
        }
        stage_push<kStage / 2>(stage, staged, (static_cast<uint64_t>(u) << 32) | c, valid && v != 0, F, cnt);
      }
      __syncthreads();
    }
  }
  stage_flush(stage, staged, F, cnt);
}

// ------------------------------------------------------------ driver
agp_tuning_t default_tuning() {
  agp_tuning_t t;
  t.aggregation = 2;  // records on levels with many pushes, atomics elsewhere
  t.level_blocks = kLevelBlocks;
  return t;
}

// The tuning in force for a call: an explicit one, else the autotuned one,
// else the default; AGP_AGGREGATION=atomic|binned|auto overrides the aggregation.
agp_tuning_t tuning_for(agp_graph* g, int32_t C, double a, double b, const agp_tuning_t* force) {
  agp_tuning_t t = default_tuning();
  if (force) {
    t = *force;
  } else {
    auto it = g->tuning.find(agp_tune_key{C, a, b});
    if (it != g->tuning.end()) t = it->second;
  }
  if (const char* e = std::getenv("AGP_AGGREGATION")) {
    if (std::strcmp(e, "atomic") == 0) t.aggregation = 0;
    if (std::strcmp(e, "binned") == 0) t.aggregation = 1;
    if (std::strcmp(e, "auto") == 0) t.aggregation = 2;
  }
  if (t.level_blocks < 256) t.level_blocks = 256;
  return t;
}

// One tile of C columns: x and out point at the tile's first column, rows
// ldc apart; column c of the tile is column qid_base + c of the call (its
// qid when qids is null).  Levels are timed when stats is non-null (the
// tile's counters and times are added to it).  The caller holds g->mu and
// has zeroed out.
template <typename T>
int propagate_tile(agp_graph* g, const char* fn, const agp_tuning_t& tune, double a, double b,
                   const std::vector<double>& rho, const std::vector<double>& kappa, int32_t L, const T* x,
                   long long ldc, int32_t C, double eps, uint64_t seed, const uint32_t* qids, uint32_t qid_base,
                   T* out, hipStream_t s, agp_stats_t* stats) {
  using Cell = typename Prec<T>::Cell;
  const int64_t n = g->n;
  const size_t cells = static_cast<size_t>(n) * static_cast<size_t>(C);
  int rc;
  const double *da = nullptr, *db = nullptr;
  if ((rc = pow_table(g, a, &da)) || (rc = pow_table(g, b, &db))) return rc;
  Scratch& sc = g->scratch;
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
      (rc = sc.levelinfo.reserve((2 * sizeof(double) + sizeof(int)) * (AGP_MAX_LEVELS + 2), false, s)))
    return rc;

  ColParams* cp = sc.colparams.as<ColParams>();
  uint32_t* dq = reinterpret_cast<uint32_t*>(cp + C);
  unsigned long long* counts = sc.counts.as<unsigned long long>();
  unsigned long long* counters = sc.counters.as<unsigned long long>();
  int* flags = sc.flags.as<int>();
  double* mass = sc.levelinfo.as<double>();
  double* est = mass + AGP_MAX_LEVELS + 2;  // estimated pushes per level (auto aggregation)
  int* mode = reinterpret_cast<int*>(est + AGP_MAX_LEVELS + 2);
  AGP_HIP(hipMemsetAsync(sc.levelinfo.ptr, 0, sc.levelinfo.bytes, s));
  AGP_HIP(hipMemsetAsync(counts, 0, sc.counts.bytes, s));
  AGP_HIP(hipMemsetAsync(counters, 0, sc.counters.bytes, s));
  AGP_HIP(hipMemsetAsync(flags, 0, sc.flags.bytes, s));
  if (qids) AGP_HIP(hipMemcpyAsync(dq, qids, sizeof(uint32_t) * C, hipMemcpyHostToDevice, s));

  // thresholds theta_c = eps ||x_c||_1 and signal checks
  if (tblocks > 0) {
    dim3 grid((unsigned)tblocks, (unsigned)((C + 63) / 64));
    k_theta_partial<T><<<grid, 64, 0, s>>>(x, ldc, n, C, sc.partial.as<double>(), flags + 1);
  }
  k_theta_final<T><<<grid_for(C, 64), 64, 0, s>>>(sc.partial.as<double>(), tblocks, C, eps,
                                                  qids ? dq : nullptr, qid_base, cp);
  AGP_HIP(hipGetLastError());
  int hflags[4] = {0, 0, 0, 0};
  AGP_HIP(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
  AGP_HIP(hipStreamSynchronize(s));
  if (hflags[1] & 1) return fail(AGP_EINVAL, std::string(fn) + ": x holds a non-finite value");
  const bool positive = sizeof(T) == 4 && !(hflags[1] & 2);

  // binned aggregation: binary32, cells addressable in 32 bits, LDS scale table
  bool binned = (tune.aggregation == 1 || tune.aggregation == 2) && sizeof(T) == 4 && cells < (1ull << 31) &&
                C <= kMaxBinnedC && cells > 0;
  // buckets of 2^shift cells: at most 1024 buckets, bins of 8192 cells
  int shift = kBinLog2;
  while (shift < 32 && (static_cast<unsigned long long>(cells) - 1ull) >> shift >= (unsigned long long)kBuckets) ++shift;
  const unsigned nbuckets = static_cast<unsigned>(((cells > 0 ? cells : 1) - 1) >> shift) + 1u;
  unsigned long long rec_cap = 0;
  if (binned) {
    // room for 4 records per cell, within an eighth of the free memory (two buffers)
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    rec_cap = std::max<unsigned long long>(1ull << 20, 4ull * cells);
    rec_cap = std::min<unsigned long long>(rec_cap, std::max<unsigned long long>(1ull << 20, free_b / 64));
    if (const char* e = std::getenv("AGP_RECORD_CAP")) {  // smaller record buffer (tuning / tests)
      const unsigned long long v = std::strtoull(e, nullptr, 10);
      if (v > 0 && v < rec_cap) rec_cap = v;
    }
    if (sc.rec[0].reserve(rec_cap * sizeof(uint32_t), false, s) ||
        sc.rec[1].reserve(rec_cap * sizeof(uint32_t), false, s) ||
        sc.bins.reserve(sizeof(unsigned int) * kBuckets + sizeof(unsigned long long) * (2 * kBuckets + 1) +
                            sizeof(unsigned long long) * (AGP_MAX_LEVELS + 1), true, s)) {
      sc.rec[0].release();  // not enough memory for the record buffers: atomics instead
      sc.rec[1].release();
      binned = false;
      (void)hipGetLastError();
    }
  }
  unsigned int* bucket_count = binned ? sc.bins.as<unsigned int>() : nullptr;
  unsigned long long* bucket_off = binned ? reinterpret_cast<unsigned long long*>(bucket_count + kBuckets) : nullptr;
  unsigned long long* cursor = binned ? bucket_off + kBuckets + 1 : nullptr;
  unsigned long long* rec_counts = binned ? cursor + kBuckets : nullptr;
  if (binned) AGP_HIP(hipMemsetAsync(rec_counts, 0, sizeof(unsigned long long) * (AGP_MAX_LEVELS + 1), s));

  hipEvent_t* ev = sc.events;
  if (stats && (rc = sc.ensure_events())) return rc;
  uint64_t* F[2] = {sc.frontier[0].as<uint64_t>(), sc.frontier[1].as<uint64_t>()};
  Cell* acc[2] = {sc.acc[0].as<Cell>(), sc.acc[1].as<Cell>()};
  const unsigned cgrid = grid_for(n * (int64_t)(C >= kWave ? kWave : C), kThreads, 8192);
  k_compact<<<cgrid, kThreads, 0, s>>>(NonZeroValue<T>{x, ldc}, n, C, (long long)C, 1ll, F[0], counts, nullptr);

  LevelArgs A{};
  A.rp = g->row_ptr;
  A.col = g->col;
  A.nd = g->ndeg;
  A.deg = g->degree;
  A.cp = cp;
  A.su = C;
  A.sc = 1;
  A.xld = ldc;
  A.counters = counters;
  A.mass = mass;
  A.err = flags;
  A.positive = positive ? 1 : 0;
  A.dense_cut = std::max<unsigned long long>(1ull, static_cast<unsigned long long>(cells / 32));
  A.rec = nullptr;
  A.rec_count = nullptr;
  A.rec_cap = rec_cap;
  A.bucket_count = bucket_count;
  A.bucket_shift = shift;
  A.bin_est = nullptr;
  A.bin_pushes = static_cast<double>(cells) / 8.0;  // auto: bin levels with at least n C / 8 pushes
  const uint32_t key0 = static_cast<uint32_t>(seed), key1 = static_cast<uint32_t>(seed >> 32);
  for (int32_t i = 0; i <= L; ++i) {
    const int lflags = (i == L ? kLastLevel : 0) | (a == 0.0 ? kAZero : 0);
    k_set_level<<<grid_for(C, 64), 64, 0, s>>>(cp, C, i, rho[i], kappa[i], lflags, da, db, key0, key1, out,
                                              ldc, sizeof(T));
    A.level = i;
    A.fin = F[i & 1];
    A.cnt_in = counts + i;
    A.fout = F[(i + 1) & 1];
    A.cnt_out = counts + i + 1;
    A.mode_out = mode + i + 1;
    const bool bin_level = binned && i < L;
    A.rec = bin_level ? sc.rec[0].as<uint32_t>() : nullptr;
    A.rec_count = bin_level ? rec_counts + i : nullptr;
    Cell* cur = acc[i & 1];
    Cell* nxt = acc[(i + 1) & 1];
    A.bin_est = nullptr;
    if (bin_level && tune.aggregation == 2) {
      A.bin_est = est + i;
      if (i == 0)
        k_estimate<T, true><<<1024, kThreads, 0, s>>>(A, x, cur, est + i);
      else
        k_estimate<T, false><<<1024, kThreads, 0, s>>>(A, x, cur, est + i);
    }
    if (stats) AGP_HIP(hipEventRecord(ev[2 * i], s));
    if (i == 0)
      k_level<T, true, false><<<tune.level_blocks, kThreads, 0, s>>>(A, x, cur, nxt);
    else
      k_level<T, false, false><<<tune.level_blocks, kThreads, 0, s>>>(A, x, cur, nxt);
    if (stats) AGP_HIP(hipEventRecord(ev[2 * i + 1], s));
    if (bin_level) {
      uint32_t* r0 = sc.rec[0].as<uint32_t>();
      uint32_t* r1 = sc.rec[1].as<uint32_t>();
      k_bins_scan<<<1, kBuckets, 0, s>>>(bucket_count, bucket_off, cursor, rec_counts + i, rec_cap, mode + i + 1);
      k_apply_overflow<<<2048, kThreads, 0, s>>>(A, reinterpret_cast<long long*>(nxt), mode + i + 1);
      k_partition<<<1024, kReduceThreads, 0, s>>>(r0, rec_counts + i, cursor, r1, mode + i + 1, shift);
      k_bin_reduce<<<nbuckets, kReduceThreads, 0, s>>>(r1, r0, bucket_off, cp, C, static_cast<unsigned long long>(cells),
                                                       reinterpret_cast<long long*>(nxt), F[(i + 1) & 1],
                                                       counts + i + 1, mode + i + 1, shift);
    }
    if (i < L)
      k_compact<<<cgrid, kThreads, 0, s>>>(NonZeroCell<T>{nxt}, n, C, (long long)C, 1ll, F[(i + 1) & 1],
                                           counts + i + 1, mode + i + 1);
  }
  AGP_HIP(hipGetLastError());
  std::vector<double> hmass(static_cast<size_t>(L) + 1);
  AGP_HIP(hipMemcpyAsync(hflags, flags, sizeof(int), hipMemcpyDeviceToHost, s));
  AGP_HIP(hipMemcpyAsync(hmass.data(), mass, sizeof(double) * (L + 1), hipMemcpyDeviceToHost, s));
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
    for (int32_t i = 0; i <= L; ++i) {
      stats->frontier[i] += h[i * kNumCounters + 0];
      stats->hash[i] += h[i * kNumCounters + 1];
      stats->det[i] += h[i * kNumCounters + 2];
      stats->cand[i] += h[i * kNumCounters + 3];
      stats->acc[i] += h[i * kNumCounters + 4];
    }
    float ms = 0.0f;
    for (int32_t i = 0; i <= L; ++i) {
      AGP_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
      stats->level_ms[i] += ms;
    }
    AGP_HIP(hipEventElapsedTime(&ms, ev[0], ev[2 * L + 1]));
    stats->device_ms += ms;
  }
  return AGP_OK;
}


// Tile width: every column at once when the scratch fits in 85% of the free
// memory (plus what the scratch already holds), else the widest tile that
// does; AGP_COLUMN_TILE forces a width (tests).
template <typename T>
int32_t column_tile(agp_graph* g, int32_t C, bool binned) {
  if (const char* e = std::getenv("AGP_COLUMN_TILE")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v > 0 && v < C) return static_cast<int32_t>(v);
  }
  const size_t cell_bytes = sizeof(typename Prec<T>::Cell) * (sizeof(T) == 4 ? 1 : 2);
  // two accumulators and two frontier lists per cell (+ two record buffers of 4 records)
  const size_t per_cell = 2 * cell_bytes + 2 * sizeof(uint64_t) + (binned ? 2 * 4 * sizeof(uint32_t) : 0);
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return C;
  Scratch& sc = g->scratch;
  const size_t held = sc.acc[0].bytes + sc.acc[1].bytes + sc.frontier[0].bytes + sc.frontier[1].bytes +
                      sc.rec[0].bytes + sc.rec[1].bytes;
  const double budget = 0.85 * static_cast<double>(free_b + held);
  const double per_col = static_cast<double>(g->n > 0 ? g->n : 1) * static_cast<double>(per_cell);
  const double fit = budget / per_col;
  if (fit >= static_cast<double>(C)) return C;
  return fit < 1.0 ? 1 : static_cast<int32_t>(fit);
}

template <typename T>
int propagate_impl(agp_graph* g, double a, double b, const double* w, int32_t L, const T* x,
                   int32_t C, double eps, uint64_t seed, const uint32_t* qids, T* out,
                   hipStream_t s, agp_stats_t* stats, const agp_tuning_t* force = nullptr) {
  const char* fn = sizeof(T) == 4 ? "agp_propagate" : "agp_propagate_f64";
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

  // level tables in binary64: Y_i = sum_{k=i..L} w_k added from k = L down,
  // S = Y_0, rho_i = Y_{i+1} / Y_i, kappa_i = (S w_i) / Y_i
  std::vector<double> Y(static_cast<size_t>(L) + 2, 0.0), rho(static_cast<size_t>(L) + 1),
      kappa(static_cast<size_t>(L) + 1);
  for (int32_t k = L; k >= 0; --k) Y[k] = Y[k + 1] + w[k];
  const double S = Y[0];
  for (int32_t i = 0; i <= L; ++i) {
    rho[i] = (Y[i] == 0.0) ? 0.0 : Y[i + 1] / Y[i];
    kappa[i] = (Y[i] == 0.0) ? 0.0 : (S * w[i]) / Y[i];
  }

  std::lock_guard<std::mutex> lk(g->mu);
  const agp_tuning_t tune = tuning_for(g, C, a, b, force);
  const bool may_bin = (tune.aggregation == 1 || tune.aggregation == 2) && sizeof(T) == 4;
  const int32_t tile = column_tile<T>(g, C, may_bin);
  AGP_HIP(hipMemsetAsync(out, 0, cells * sizeof(T), s));
  if (stats) std::memset(stats, 0, sizeof(*stats));
  for (int32_t c0 = 0; c0 < C; c0 += tile) {
    const int32_t ct = std::min(tile, C - c0);
    const int rc = propagate_tile<T>(g, fn, tune, a, b, rho, kappa, L, x + c0, static_cast<long long>(C), ct, eps,
                                     seed, qids ? qids + c0 : nullptr, static_cast<uint32_t>(c0), out + c0, s, stats);
    if (rc != AGP_OK) return rc;
  }
  if (stats) {
    stats->levels = L;
    stats->columns = C;
  }
  return AGP_OK;
}

}  // namespace
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
  agp_tuning_t cands[6];
  int nc = 0;
  for (int agg = 0; agg < 3; ++agg)
    for (int blocks : {2048, 4096}) cands[nc++] = agp_tuning_t{agg, blocks};
  float best_ms = 0.0f;
  agp_tuning_t pick = default_tuning();
  int rc = AGP_OK;
  for (int k = 0; k < nc && rc == AGP_OK; ++k) {
    (void)hipEventRecord(e0, s);
    rc = propagate_impl<float>(gg, a, b, w, L, x, C, eps, seed, qids, out, s, nullptr, &cands[k]);
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (rc == AGP_OK && (k == 0 || ms < best_ms)) {
      best_ms = ms;
      pick = cands[k];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != AGP_OK) return rc;
  {
    std::lock_guard<std::mutex> lk(gg->mu);
    gg->tuning[agp_tune_key{C, a, b}] = pick;
  }
  // leave `out` with the result (every candidate gives the same bits)
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

}  // extern "C"
