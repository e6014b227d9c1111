// Binned aggregation of a level's sampled pushes (the kernels that run after
// a binned k_level launch), shared by the batched entry points and the query
// server.  Records are (cell | sign << 31); see level_kernels.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "level_kernels.h"

namespace agp {
namespace lvl {
namespace {

// ------------------------------------------------ binned aggregation
// After a binned level: bucket offsets (one block), then the records are
// partitioned into buckets, then into bins of 8192 cells, and one block per
// bin counts the signed records of every cell in LDS, adds count *
// fl(theta_c) in units to each cell (the deterministic pushes are already
// there: integer sums, so the order is irrelevant) and appends every
// non-zero cell to the next frontier.
constexpr int kMaxBinnedC = 1024;
constexpr int kReduceThreads = 512;

// One block per column group of records: the group's nbk bucket counts at
// g * nbk (cleared), its offsets and cursors at g * (kBuckets + 1) and
// g * kBuckets; a group whose records outgrew its buffer switches the level
// to the atomic fallback.
__global__ __launch_bounds__(1024) void k_bins_scan(unsigned int* __restrict__ bucket_count, int nbk,
                                                    unsigned long long* __restrict__ bucket_off,
                                                    unsigned long long* __restrict__ cursor,
                                                    const unsigned long long* __restrict__ rec_count,
                                                    unsigned long long cap, int* __restrict__ mode) {
  __shared__ unsigned long long s[kBuckets];
  const int g = blockIdx.x;
  const int t = threadIdx.x;
  unsigned int* bc = bucket_count + static_cast<size_t>(g) * nbk;
  const unsigned long long v = t < nbk ? bc[t] : 0ull;
  if (t < nbk) bc[t] = 0;  // ready for the next level (zero unless this one was binned)
  if (*mode != kModeBinned) return;  // (or another group overflowed)
  if (rec_count[g] > cap) {
    if (t == 0) atomicExch(mode, kModeOverflow);
    return;
  }
  bucket_off += static_cast<size_t>(g) * (kBuckets + 1);
  cursor += static_cast<size_t>(g) * kBuckets;
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
  const int ng = A.rec_groups > 1 ? A.rec_groups : 1;
  for (int g = 0; g < ng; ++g) {
    const unsigned long long n = A.rec_count[g] < A.rec_cap ? A.rec_count[g] : A.rec_cap;
    const uint32_t* rec = A.rec + static_cast<size_t>(g) * A.rec_cap;
    for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < n;
         i += (unsigned long long)gridDim.x * blockDim.x)
      apply_record<0>(A, acc, rec[i], static_cast<uint32_t>(g));
  }
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

// Partition of the records into buckets: a tile of 32768 records is sorted
// by bucket in LDS, then every bucket's run is written out contiguously.
constexpr int kPartPerThread = 64;
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

// ---------------------------------------------------------- bins
// Second level: the bucket-ordered records are counted per bin (8192 cells),
// scattered into bin order with LDS-sorted tiles, and every bin is summed by
// its own block.  A tile's bins lie in the one or two buckets it overlaps
// (records are bucket-sorted); bins outside that window take a global atomic
// per record, so any record order stays correct.
constexpr int kBinTile = 8192;                    // records per tile
constexpr int kBinPerThread = kBinTile / kReduceThreads;
constexpr int kBinWindow = 2 * kMaxBinsPerBucket;  // bins a tile counts in LDS

__device__ __forceinline__ unsigned long long bin_of(uint32_t rec) {
  return static_cast<unsigned long long>(rec & kRecCellMask) >> kBinLog2;
}

// Counts use tiles of kCountTile records (read kBinPerThread per thread at a
// time): a tile's window of bins is flushed with one global atomic per bin,
// so larger tiles mean fewer atomics on the same counters.
constexpr int kCountTile = 8 * kBinTile;

__global__ __launch_bounds__(kReduceThreads) void k_bin_count(const uint32_t* __restrict__ part,
                                                              const unsigned long long* __restrict__ rec_count,
                                                              unsigned long long* __restrict__ bin_count,
                                                              const int* __restrict__ mode, int shift) {
  if (*mode != kModeBinned) return;
  __shared__ unsigned int s_h[kBinWindow];
  const unsigned long long total = *rec_count;
  const unsigned long long bpb = 1ull << (shift - kBinLog2);  // bins per bucket
  for (unsigned long long t0 = (unsigned long long)blockIdx.x * kCountTile; t0 < total;
       t0 += (unsigned long long)gridDim.x * kCountTile) {
    const unsigned long long w0 = (bin_of(part[t0]) / bpb) * bpb;  // first bin of the tile's first bucket
    const unsigned long long t1 = t0 + kCountTile < total ? t0 + kCountTile : total;
    for (int i = threadIdx.x; i < kBinWindow; i += blockDim.x) s_h[i] = 0;
    __syncthreads();
    for (unsigned long long lo = t0; lo < t1; lo += kBinTile) {
      uint32_t r[kBinPerThread];
#pragma unroll
      for (int k = 0; k < kBinPerThread; ++k) {
        const unsigned long long i = lo + (unsigned long long)(k * kReduceThreads + threadIdx.x);
        r[k] = i < t1 ? part[i] : 0u;
      }
#pragma unroll
      for (int k = 0; k < kBinPerThread; ++k) {
        const unsigned long long i = lo + (unsigned long long)(k * kReduceThreads + threadIdx.x);
        if (i < t1) {
          const unsigned long long gb = bin_of(r[k]);
          if (gb >= w0 && gb - w0 < (unsigned long long)kBinWindow)
            atomicAdd(&s_h[gb - w0], 1u);
          else
            atomicAdd(bin_count + gb, 1ull);
        }
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kBinWindow; i += blockDim.x)
      if (s_h[i]) atomicAdd(bin_count + w0 + i, static_cast<unsigned long long>(s_h[i]));
    __syncthreads();
  }
}

// Exclusive scan of the bin counts: block b takes bins [16384 b, 16384 (b +
// 1)), adds up every count before them itself (coalesced; at most a few
// hundred thousand bins, so the repeated prefix reads stay small), scans its
// own (each k-th load of the 1024 threads is a contiguous run of bins: wave
// scans, then one scan of the 16 x 16 wave totals in LDS) and sets offsets and
// scatter cursors.  Launch nbins / 16384 + 1 blocks: the last one also writes
// bin_off[nbins].  The counts are cleared later, by k_bin_scatter.
constexpr int kScanPer = 16;
constexpr int kScanChunk = 1024 * kScanPer;

__global__ __launch_bounds__(1024) void k_bin_scan(const unsigned long long* __restrict__ bin_count, long long nbins,
                                                   unsigned long long* __restrict__ bin_off,
                                                   unsigned long long* __restrict__ bin_cur,
                                                   const int* __restrict__ mode) {
  if (*mode != kModeBinned) return;
  constexpr int kWaves = 1024 / kWave;
  __shared__ unsigned long long s_pre[kWaves + 1];  // each wave's share of the prefix, then the chunk total
  __shared__ unsigned long long s_w[kScanPer * kWaves];  // (k, wave) totals, then their exclusive prefixes
  const int t = threadIdx.x, lane = lane_id(), wave = t / kWave;
  const long long c0 = static_cast<long long>(blockIdx.x) * kScanChunk;
  unsigned long long pre = 0;
  for (long long b = t; b < c0; b += 1024ll * 8) {  // c0 is a multiple of 8 * 1024
    unsigned long long p[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) p[k] = bin_count[b + 1024ll * k];
#pragma unroll
    for (int k = 0; k < 8; ++k) pre += p[k];
  }
  pre = wave_sum_u64(pre);
  if (lane == 0) s_pre[wave] = pre;
  unsigned long long v[kScanPer], incl[kScanPer];
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const long long i = c0 + 1024ll * k + t;
    v[k] = i < nbins ? bin_count[i] : 0ull;
  }
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    incl[k] = v[k];
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const unsigned long long u = __shfl_up(incl[k], off);
      if (lane >= off) incl[k] += u;
    }
    if (lane == kWave - 1) s_w[k * kWaves + wave] = incl[k];
  }
  __syncthreads();
  if (wave == 0) {  // exclusive scan of the 256 totals in (k, wave) order, 4 per lane
    constexpr int kPer = kScanPer * kWaves / kWave;
    unsigned long long x[kPer], run = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      x[j] = s_w[lane * kPer + j];
      run += x[j];
    }
    unsigned long long sc = run;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const unsigned long long u = __shfl_up(sc, off);
      if (lane >= off) sc += u;
    }
    sc -= run;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
      s_w[lane * kPer + j] = sc;
      sc += x[j];
    }
    if (lane == kWave - 1) s_pre[kWaves] = sc;  // the chunk's total
  }
  __syncthreads();
  unsigned long long base = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) base += s_pre[w];
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    const long long i = c0 + 1024ll * k + t;
    if (i < nbins) {
      const unsigned long long o = base + s_w[k * kWaves + wave] + incl[k] - v[k];
      bin_off[i] = o;
      bin_cur[i] = o;
    }
  }
  if (t == 0 && nbins >= c0 && nbins < c0 + kScanChunk) bin_off[nbins] = base + s_pre[kWaves];
}

// Also clears the nbins bin counts for the next k_bin_count (k_bin_scan has
// read them).
__global__ __launch_bounds__(kReduceThreads) void k_bin_scatter(const uint32_t* __restrict__ part,
                                                                const unsigned long long* __restrict__ rec_count,
                                                                unsigned long long* __restrict__ bin_cur,
                                                                uint32_t* __restrict__ out,
                                                                const int* __restrict__ mode, int shift,
                                                                unsigned long long* __restrict__ bin_count,
                                                                long long nbins) {
  if (*mode != kModeBinned) return;
  for (long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; i < nbins;
       i += static_cast<long long>(gridDim.x) * blockDim.x)
    bin_count[i] = 0;
  __shared__ uint32_t s_rec[kBinTile];
  __shared__ unsigned int s_h[kBinWindow];
  __shared__ unsigned int s_loc[kBinWindow];
  __shared__ unsigned long long s_base[kBinWindow];
  __shared__ unsigned int s_wsum[kReduceThreads / kWave];
  const unsigned long long total = *rec_count;
  const unsigned long long bpb = 1ull << (shift - kBinLog2);
  const int lane = lane_id(), wave = threadIdx.x / kWave;
  for (unsigned long long lo = (unsigned long long)blockIdx.x * kBinTile; lo < total;
       lo += (unsigned long long)gridDim.x * kBinTile) {
    const unsigned long long w0 = (bin_of(part[lo]) / bpb) * bpb;
    for (int i = threadIdx.x; i < kBinWindow; i += blockDim.x) s_h[i] = 0;
    __syncthreads();
    uint32_t r[kBinPerThread];
    unsigned int rank[kBinPerThread];
#pragma unroll
    for (int k = 0; k < kBinPerThread; ++k) {
      const unsigned long long i = lo + (unsigned long long)(k * kReduceThreads + threadIdx.x);
      r[k] = i < total ? part[i] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kBinPerThread; ++k) {
      const unsigned long long i = lo + (unsigned long long)(k * kReduceThreads + threadIdx.x);
      rank[k] = 0xFFFFFFFFu;
      if (i < total) {
        const unsigned long long gb = bin_of(r[k]);
        if (gb >= w0 && gb - w0 < (unsigned long long)kBinWindow)
          rank[k] = atomicAdd(&s_h[gb - w0], 1u);
        else  // outside the window: a slot of its own
          out[atomicAdd(bin_cur + gb, 1ull)] = r[k];
      }
    }
    __syncthreads();
    {  // exclusive scan of the window's counts, 4 per thread
      constexpr int kPer = kBinWindow / kReduceThreads;
      unsigned int x[kPer];
      unsigned int run = 0;
      for (int k = 0; k < kPer; ++k) {
        x[k] = s_h[threadIdx.x * kPer + k];
        run += x[k];
      }
      unsigned int incl = run;
      for (int off = 1; off < kWave; off <<= 1) {
        const unsigned int t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
      }
      if (lane == kWave - 1) s_wsum[wave] = incl;
      __syncthreads();
      unsigned int acc0 = 0;
      for (int w = 0; w < wave; ++w) acc0 += s_wsum[w];
      acc0 += incl - run;
      for (int k = 0; k < kPer; ++k) {
        s_loc[threadIdx.x * kPer + k] = acc0;
        acc0 += x[k];
      }
    }
    for (int i = threadIdx.x; i < kBinWindow; i += blockDim.x) {
      const unsigned int h = s_h[i];
      s_base[i] = h ? atomicAdd(bin_cur + w0 + i, static_cast<unsigned long long>(h)) : 0ull;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kBinPerThread; ++k)
      if (rank[k] != 0xFFFFFFFFu) s_rec[s_loc[bin_of(r[k]) - w0] + rank[k]] = r[k];
    __syncthreads();
    const int nin = static_cast<int>(s_loc[kBinWindow - 1] + s_h[kBinWindow - 1]);  // records in the window
    for (int i = threadIdx.x; i < nin; i += blockDim.x) {  // runs of one bin are contiguous
      const uint32_t x = s_rec[i];
      const unsigned long long j = bin_of(x) - w0;
      out[s_base[j] + static_cast<unsigned long long>(i - static_cast<int>(s_loc[j]))] = x;
    }
    __syncthreads();
  }
}

// One block per bin: signed record counts in LDS, then each cell's new value
// acc += count * fl(theta_c) (its deterministic pushes are already in acc);
// the bin's non-zero cells are gathered in LDS and appended to the next
// frontier with one atomic per bin.  ldacc > 0: the cells are those of a
// column group (local cell u * su + l, l < wg valid, for the accumulator
// cell u * ldacc + c0 + l of column c0 + l; row-major, sc = 1).  With det non-null (a flag per bin that
// the level's deterministic pushes set), a bin whose flag is clear holds
// only zeros before its records: it is not read, and without records it has
// nothing to do.  A set flag is cleared for the next level; a stale set flag
// only costs the reads.
constexpr int kSumThreads = 512;

__global__ __launch_bounds__(kSumThreads) void k_bin_sum(const uint32_t* __restrict__ tmp,
                                                         const unsigned long long* __restrict__ bin_off,
                                                         const ColParams* __restrict__ cp, long long su, long long sc,
                                                         unsigned long long cells, long long* __restrict__ acc,
                                                         uint64_t* __restrict__ F, unsigned long long* __restrict__ cnt,
                                                         const int* __restrict__ mode, uint8_t* __restrict__ det,
                                                         long long ldacc = 0, int c0 = 0, int wg = 0) {
  if (*mode != kModeBinned) return;
  constexpr int kBin = 1 << kBinLog2;
  __shared__ int s_cnt[kBin];
  __shared__ uint16_t s_nz[kBin];  // non-zero cells of the bin, as offsets
  __shared__ unsigned int s_n;
  __shared__ unsigned long long s_base;
  const int lane = lane_id();
  const unsigned long long gb = blockIdx.x;
  const unsigned long long cell0 = gb << kBinLog2;
  const bool read_acc = det == nullptr || det[gb] != 0;
  const unsigned long long lo = bin_off[gb], hi = bin_off[gb + 1];
  if (!read_acc && lo == hi) return;  // the whole block: no record, no deterministic push
  for (int j = threadIdx.x; j < kBin; j += blockDim.x) s_cnt[j] = 0;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  for (unsigned long long i0 = lo + threadIdx.x; i0 < hi; i0 += (unsigned long long)blockDim.x * 8) {
    uint32_t rr[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const unsigned long long i = i0 + (unsigned long long)k * blockDim.x;
      rr[k] = i < hi ? tmp[i] : 0u;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (i0 + (unsigned long long)k * blockDim.x < hi) atomicAdd(&s_cnt[rr[k] & (kBin - 1)], (rr[k] >> 31) ? -1 : 1);
  }
  __syncthreads();
  constexpr int kCellsPer = kBin / kSumThreads;
  // column groups: the bin's first cell as (row u0, local column l0); cells
  // of the bin are u0 + (l0 + j) / su, (l0 + j) mod su (su + kBin < 2^22)
  const bool grouped = ldacc > 0;
  const unsigned long long u0 = grouped ? cell0 / static_cast<unsigned long long>(su) : 0ull;
  const uint32_t l0 = grouped ? static_cast<uint32_t>(cell0 - u0 * static_cast<unsigned long long>(su)) : 0u;
  const float rsu = grouped ? 1.0f / static_cast<float>(su) : 0.0f;
  // accumulator cell of bin cell j and, for a group, its column (false: not
  // a cell of the call)
  auto locate = [&](int j, size_t* at, uint32_t* c) -> bool {
    const unsigned long long cell = cell0 + static_cast<unsigned long long>(j);
    *c = 0u;
    if (cell >= cells) return false;
    if (!grouped) {
      *at = cell;
      return true;
    }
    uint32_t l = 0;
    const uint32_t q = div_small(l0 + static_cast<uint32_t>(j), static_cast<uint32_t>(su), rsu, &l);
    if (l >= static_cast<uint32_t>(wg)) return false;
    *c = static_cast<uint32_t>(c0) + l;
    *at = static_cast<size_t>(u0 + q) * static_cast<size_t>(ldacc) + *c;
    return true;
  };
  for (int k0 = 0; k0 < kCellsPer; k0 += 8) {
    long long vv[8];
    size_t at[8];
    uint32_t col[8];
    bool ok[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      ok[k] = locate((k0 + k) * kSumThreads + threadIdx.x, &at[k], &col[k]);
      vv[k] = (read_acc && ok[k]) ? acc[at[k]] : 0ll;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int j = (k0 + k) * kSumThreads + threadIdx.x;
      long long v = vv[k];
      if (ok[k]) {
        const int kc = s_cnt[j];
        if (kc != 0) {
          const uint32_t c = grouped ? col[k]
                             : sc == 1 ? static_cast<uint32_t>(at[k] % static_cast<unsigned long long>(su))
                                       : static_cast<uint32_t>(at[k] / static_cast<unsigned long long>(sc));
          v += static_cast<long long>(kc) * cp[c].dtheta;
          acc[at[k]] = v;
        }
      }
      const unsigned long long m = __ballot(v != 0);
      unsigned int base = 0;
      if (lane == 0 && m) base = atomicAdd(&s_n, static_cast<unsigned int>(__popcll(m)));
      base = __shfl(base, 0);
      if (v != 0) s_nz[base + __popcll(m & ((1ull << lane) - 1ull))] = static_cast<uint16_t>(j);
    }
  }
  __syncthreads();
  const unsigned int total = s_n;
  if (threadIdx.x == 0 && total) s_base = atomicAdd(cnt, static_cast<unsigned long long>(total));
  if (threadIdx.x == 0 && det != nullptr && read_acc) det[gb] = 0;
  __syncthreads();
  for (unsigned int i = threadIdx.x; i < total; i += blockDim.x) {
    const unsigned long long cell = cell0 + s_nz[i];
    uint32_t u, c;
    if (grouped) {
      uint32_t l = 0;
      u = static_cast<uint32_t>(u0) + div_small(l0 + static_cast<uint32_t>(s_nz[i]), static_cast<uint32_t>(su), rsu, &l);
      c = static_cast<uint32_t>(c0) + l;
    } else if (sc == 1) {  // row-major: cell = u * C + c
      u = static_cast<uint32_t>(cell / static_cast<unsigned long long>(su));
      c = static_cast<uint32_t>(cell - static_cast<unsigned long long>(u) * su);
    } else {  // one n-vector per column: cell = c * n + u
      c = static_cast<uint32_t>(cell / static_cast<unsigned long long>(sc));
      u = static_cast<uint32_t>(cell - static_cast<unsigned long long>(c) * sc);
    }
    F[s_base + i] = (static_cast<uint64_t>(u) << 32) | c;
  }
}

}  // namespace
}  // namespace lvl
}  // namespace agp
