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
                                                               long long su, long long sc, unsigned long long cells,
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
          if (sc == 1) {  // row-major: cell = u * C + c
            u = static_cast<uint32_t>(cell / static_cast<unsigned long long>(su));
            c = static_cast<uint32_t>(cell - static_cast<unsigned long long>(u) * su);
          } else {  // one n-vector per column: cell = c * n + u
            c = static_cast<uint32_t>(cell / static_cast<unsigned long long>(sc));
            u = static_cast<uint32_t>(cell - static_cast<unsigned long long>(c) * sc);
          }
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

}  // namespace
}  // namespace lvl
}  // namespace agp
