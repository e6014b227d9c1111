// Dense levels of feature propagation: one level of the randomized residue
// push (Algorithm 2 of "Approximate Graph Propagation", Section 4) over a
// tile of up to 64 signal columns whose frontiers are dense, as in GNN
// feature propagation (every feature of level 0 is non-zero).
//
// Layout of a tile of Ct columns (row-major n x Ct, cell = u * Ct + c):
//   r     binary32 residues of the current level (level 0 reads x itself)
//   acc   the next level's residues as exact integers of each column's unit
//         (deterministic pushes land here with integer atomics); all-zero
//         between levels
//   flag  one byte per node: some column of the node has a non-zero residue
// A wave handles one node at a time with one lane per column: the node's row
// (row pointer, degree, the degree factors, and per 64-arc window the
// neighbour ids and degree factors) is loaded once and shared by all
// columns, the runs of the subset sampling (degree groups cut at 64-position
// windows) are found with one ballot per window, and every column walks its
// own Philox / geometric-skip chain over the same runs.  No frontier list of
// (node, column) pairs is written or read.
//
// Sampled pushes (each -/+ fl(theta_c) of its column) become 4-byte records
// grouped by column: column c belongs to record group c >> gshift, and a
// record holds the group cell v * wg + (c mod Gw) (wg the group's width) and
// the sign, so a record id stays below 2^31 for any tile width as long as
// n * Gw <= 2^31.  The bin kernels (bin_kernels.h) partition each group's
// records by destination; k_dense_bin_sum then adds each cell's signed
// record count times fl(theta_c) to its deterministic sum and rounds the
// exact total once into r (reading A8 of the oracle: one rounding of the
// exact sum), clearing acc.
//
// Every random decision and every floating point operation that takes one is
// the one of the level kernel in level_kernels.h (same counters, runs and
// operation order), so results are bit-identical to the sparse path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "agp_device.h"
#include "level_kernels.h"

namespace agp {
namespace dense {

using lvl::ColParams;
using lvl::kAZero;
using lvl::kBinLog2;
using lvl::kBuckets;
using lvl::kLastLevel;
using lvl::kNumCounters;

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kMaxCols = 64;       // columns of a tile (one lane each)
constexpr int kMaxGroups = 4;      // record groups of a tile
constexpr int kItemArcs = 4096;    // arcs of a work item (rows above it are cut by windows)
constexpr int kItemNodes = 64;     // nodes of a work item
constexpr int kStageRecs = 1024;   // records staged per wave (split over the groups)

// Work item: bits 0..31 first node; bit 63 set for a piece of one long row
// (bits 32..51 first window, bits 52..58 window count, 1..64), else bits
// 32..39 the number of consecutive nodes (1..64).
constexpr uint64_t kItemLong = 1ull << 63;

struct DenseArgs {
  // graph
  const int64_t* rp;
  const uint32_t* col;
  const uint32_t* nd;    // factor degree of each arc's neighbour
  const int32_t* deg;    // row lengths
  const int32_t* fdeg;   // factor degrees
  const double* da;      // d^-a
  const double* db;      // d^-b
  const uint64_t* items;
  long long nitems;
  // tile
  const ColParams* cp;   // the tile's columns (theta, unit, query id)
  int Ct;
  const float* x;        // level 0: x[u * xld + c]
  long long xld;
  float* r;              // levels >= 1: residues, cleared as they are read
  float* out;            // reserve out[u * old + c]
  long long old;
  long long* acc;        // next level's exact sums
  const uint8_t* flag_in;  // levels >= 1: nodes with a non-zero residue
  // level
  double rho, kappa;
  int level, lflags;
  uint32_t key0, key1;
  unsigned long long* counters;  // this level's 5 counters
  double* mass;                  // this level's contribution mass
  int* err;
  // records (rec == nullptr: sampled pushes are added with atomics)
  uint32_t* rec;                 // group g at rec + g * rec_cap
  unsigned long long* rec_count; // per group
  unsigned long long rec_cap;    // per group
  unsigned int* bucket_count;    // per group, kBuckets each
  int bucket_shift;
  int gshift;                    // columns per record group = 1 << gshift
  uint8_t* det_bins;             // per group, nbins_g flags: bins with deterministic pushes
  long long nbins_g;
};

// Width of record group g of a tile of Ct columns.
__device__ __forceinline__ int group_width(int Ct, int gshift, int g) {
  const int gw = 1 << gshift;
  const int rest = Ct - g * gw;
  return rest < gw ? rest : gw;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const uint32_t o = __shfl_xor(v, off);
    v = o > v ? o : v;
  }
  return v;
}

__device__ __forceinline__ double shfl_f64(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __shfl(static_cast<int>(b & 0xFFFFFFFFll), src);
  const int hi = __shfl(static_cast<int>(b >> 32), src);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Apply one group record with an integer atomic (records beyond the buffer).
__device__ __forceinline__ void apply_group_record(const DenseArgs& D, int g, uint32_t rec) {
  const uint32_t gcell = rec & lvl::kRecCellMask;
  const int wg = group_width(D.Ct, D.gshift, g);
  const uint32_t v = gcell / static_cast<uint32_t>(wg);
  const int c = (g << D.gshift) + static_cast<int>(gcell - v * static_cast<uint32_t>(wg));
  const long long dt = (rec >> 31) ? -D.cp[c].dtheta : D.cp[c].dtheta;
  lvl::atomic_add_relaxed(reinterpret_cast<unsigned long long*>(D.acc + static_cast<size_t>(v) * D.Ct + c),
                          static_cast<unsigned long long>(dt));
}

// Per-wave staging of group records: group g owns kStageRecs / ng slots.
struct GroupStage {
  uint32_t* base;  // the wave's kStageRecs slots
  int per;         // slots per group
  int n[kMaxGroups];
};

__device__ __forceinline__ void group_flush(GroupStage& st, int g, const DenseArgs& D) {
  const int cnt = st.n[g];
  if (cnt == 0) return;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  unsigned long long b0 = 0;
  if (lane_id() == 0) b0 = atomicAdd(D.rec_count + g, static_cast<unsigned long long>(cnt));
  b0 = __shfl(b0, 0);
  const uint32_t* src = st.base + g * st.per;
  uint32_t* dst = D.rec + static_cast<size_t>(g) * D.rec_cap;
  for (int i = lane_id(); i < cnt; i += kWave) {
    if (b0 + i < D.rec_cap)
      dst[b0 + i] = src[i];
    else
      apply_group_record(D, g, src[i]);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  st.n[g] = 0;
}

// ------------------------------------------------------------ the level
// kFirst: level 0 (residues read from x, the reserve written without a read,
// every node visited).  Work items are taken round-robin by the waves of the
// grid; items are balanced by arc count when the graph's items are built.
template <bool kFirst>
__global__ __launch_bounds__(kThreads) void k_dense_level(DenseArgs D) {
  __shared__ uint32_t s_stage[kWaves][kStageRecs];
  __shared__ unsigned int s_hist[kMaxGroups][kBuckets];

  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const bool binned = D.rec != nullptr;
  const int ng = (D.Ct + (1 << D.gshift) - 1) >> D.gshift;
  if (binned) {
    for (int i = threadIdx.x; i < ng * kBuckets; i += blockDim.x) (&s_hist[0][0])[i] = 0;
    __syncthreads();
  }
  GroupStage st;
  st.base = s_stage[wave];
  st.per = kStageRecs / ng;
#pragma unroll
  for (int g = 0; g < kMaxGroups; ++g) st.n[g] = 0;

  // the lane's column
  const int c = lane;
  const bool live = c < D.Ct;
  const int my_g = c >> D.gshift;
  const int my_w = live ? group_width(D.Ct, D.gshift, my_g) : 1;
  const int my_cl = c - (my_g << D.gshift);
  double th = 1.0, scale = 1.0;
  long long dth = 0;
  uint32_t ctr3 = 0;
  if (live) {
    const ColParams& p = D.cp[c];
    th = p.theta;
    scale = p.scale;
    dth = p.dtheta;
    ctr3 = (p.qid << 8) | static_cast<uint32_t>(D.level);
  }
  const bool azero = (D.lflags & kAZero) != 0;
  const bool last = (D.lflags & kLastLevel) != 0;
  const bool pushes = !last && D.rho != 0.0;

  unsigned long long n_front = 0, n_hash = 0, n_det = 0, n_cand = 0, n_acc = 0;
  double mass = 0.0;

  // one sampled push of -/+ fl(theta_c) to (v, c) for the lanes with emit
  auto emit_sampled = [&](bool emit, uint32_t v, bool neg) {
    if (binned) {
      const uint32_t gcell = v * static_cast<uint32_t>(my_w) + static_cast<uint32_t>(my_cl);
      if (emit) atomicAdd(&s_hist[my_g][gcell >> D.bucket_shift], 1u);
      const unsigned long long mask = __ballot(emit);
      if (mask == 0ull) return;
#pragma unroll
      for (int g = 0; g < kMaxGroups; ++g) {
        if (g >= ng) break;
        const int lo = g << D.gshift;
        const unsigned long long gm = (lo >= kWave) ? 0ull : (mask >> lo) << lo;  // lanes >= lo
        const int hi = lo + (1 << D.gshift);
        const unsigned long long inside = gm & (hi >= kWave ? ~0ull : ((1ull << hi) - 1ull));
        if (inside == 0ull) continue;
        if (emit && my_g == g)
          st.base[g * st.per + st.n[g] + __popcll(inside & ((1ull << lane) - 1ull))] =
              gcell | (neg ? 0x80000000u : 0u);
        st.n[g] += __popcll(inside);
        if (st.n[g] > st.per - kWave) group_flush(st, g, D);
      }
    } else if (emit) {
      const long long dt = neg ? -dth : dth;
      lvl::atomic_add_relaxed(reinterpret_cast<unsigned long long*>(D.acc + static_cast<size_t>(v) * D.Ct + c),
                              static_cast<unsigned long long>(dt));
    }
  };

  const long long nwaves = static_cast<long long>(gridDim.x) * kWaves;
  for (long long item = static_cast<long long>(blockIdx.x) * kWaves + wave; item < D.nitems; item += nwaves) {
    const uint64_t it = D.items[item];
    const bool longrow = (it & kItemLong) != 0;
    const uint32_t u0 = static_cast<uint32_t>(it);
    int nodes;
    uint32_t wlo = 0, whi = 0xFFFFFFFFu;
    if (longrow) {
      nodes = 1;
      wlo = static_cast<uint32_t>((it >> 32) & 0xFFFFFull);
      whi = wlo + static_cast<uint32_t>((it >> 52) & 0x7Full);
    } else {
      nodes = static_cast<int>((it >> 32) & 0xFFull);
    }
    unsigned long long todo;
    if (kFirst) {
      todo = nodes >= kWave ? ~0ull : ((1ull << nodes) - 1ull);
    } else {
      const bool f = lane < nodes && D.flag_in[u0 + lane] != 0;
      todo = __ballot(f);
    }
    // the first piece of a long row owns the row's per-node work (reserve,
    // frontier counters, mass); the row's residues are cleared after the
    // level (every piece reads them)
    const bool owner = !longrow || wlo == 0;
    while (todo) {
      const int b = __ffsll(static_cast<long long>(todo)) - 1;
      todo &= todo - 1ull;
      const uint32_t u = u0 + static_cast<uint32_t>(b);
      const size_t ucell = static_cast<size_t>(u) * static_cast<size_t>(D.Ct) + c;
      float r = 0.0f;
      if (live) r = kFirst ? D.x[static_cast<size_t>(u) * static_cast<size_t>(D.xld) + c] : D.r[ucell];
      const bool nz = live && r != 0.0f;
      if (!kFirst && !longrow && nz) D.r[ucell] = 0.0f;
      if (owner) {
        if (nz) {
          ++n_front;
          n_hash += splitmix64(u);
        }
        float* o = D.out + static_cast<size_t>(u) * static_cast<size_t>(D.old) + c;
        if (kFirst) {  // pi starts at +0: pi = +0 + fl(kappa r)
          if (live) *o = nz ? 0.0f + static_cast<float>(D.kappa * static_cast<double>(r)) : 0.0f;
        } else if (nz && D.kappa != 0.0) {
          *o = *o + static_cast<float>(D.kappa * static_cast<double>(r));
        }
      }
      if (!pushes || !__any(nz)) continue;
      const uint32_t d = static_cast<uint32_t>(D.deg[u]);
      if (d == 0) continue;
      const int64_t rp = D.rp[u];
      const bool neg = r < 0.0f;
      // c = (rho |r|) d_u^-b and the deterministic prefix J (increment >= theta)
      const double absr = fabs(static_cast<double>(r));
      const double t0 = D.rho * absr;
      const double cv = t0 * D.db[D.fdeg[u]];
      uint32_t J = 0;
      double inc0 = cv, p0 = 0.0;
      if (azero) {
        J = (nz && cv >= th) ? d : 0u;
        const double num = cv * 1.0;
        p0 = num / th;
      } else {
        inc0 = cv * D.da[D.nd[rp]];
        uint32_t lo = 0, hi = d;
        if (!nz || !(inc0 >= th))
          hi = 0;
        else if (cv * D.da[D.nd[rp + d - 1]] >= th)
          lo = d;
        while (lo < hi) {
          const uint32_t mid = (lo + hi) >> 1;
          if (cv * D.da[D.nd[rp + mid]] >= th)
            lo = mid + 1;
          else
            hi = mid;
        }
        J = lo;
      }
      if (nz && owner) {
        const float big = static_cast<float>(inc0 > th ? inc0 : th);
        mass += static_cast<double>(d) * (fabs(static_cast<double>(big)) * scale);
      }
      const uint32_t nwin = ((d - 1) >> kSegLog2) + 1;
      const uint32_t w1 = whi < nwin ? whi : nwin;
      if (nz) {  // deterministic pushes of this piece: positions [jlo, min(J, jhi))
        const uint32_t jlo = wlo << kSegLog2, jhi = (w1 << kSegLog2) < d ? (w1 << kSegLog2) : d;
        n_det += (J > jlo ? (J < jhi ? J : jhi) - jlo : 0u);
      }
      const uint32_t Jmax = wave_max_u32(nz ? J : 0u);
      SkipTable tab0;
      if (azero) tab0 = make_skip_table(p0);
      for (uint32_t w = wlo; w < w1; ++w) {
        const uint32_t ws = w << kSegLog2;
        const uint32_t we = (ws + kSeg) < d ? ws + kSeg : d;
        const bool need_samp = __any(nz && J < we);
        const bool need_det = Jmax > ws;
        if (!need_samp && !need_det) continue;
        // the window's arcs, one per lane
        const uint32_t j = ws + static_cast<uint32_t>(lane);
        const bool valid = j < we;
        const uint32_t colw = valid ? D.col[rp + j] : 0u;
        double daw = 1.0;
        int gw = 0;
        if (!azero && valid) {
          const uint32_t ndw = D.nd[rp + j];
          daw = D.da[ndw];
          gw = 31 - __clz(ndw);
        }
        // deterministic pushes at positions [ws, min(Jmax, we))
        if (need_det) {
          const uint32_t jd = Jmax < we ? Jmax : we;
          for (uint32_t q = ws; q < jd; ++q) {
            const int src = static_cast<int>(q - ws);
            const uint32_t v = static_cast<uint32_t>(__shfl(static_cast<int>(colw), src));
            const double dav = azero ? 1.0 : shfl_f64(daw, src);
            if (nz && q < J) {
              double inc = cv;
              if (!azero) inc = inc * dav;
              float val = static_cast<float>(inc);
              if (neg) val = -val;
              long long units;
              if (f32_to_units(val, scale, &units)) {
                lvl::atomic_add_relaxed(
                    reinterpret_cast<unsigned long long*>(D.acc + static_cast<size_t>(v) * D.Ct + c),
                    static_cast<unsigned long long>(units));
                if (D.det_bins) {
                  const uint32_t gcell = v * static_cast<uint32_t>(my_w) + static_cast<uint32_t>(my_cl);
                  D.det_bins[static_cast<size_t>(my_g) * D.nbins_g + (gcell >> kBinLog2)] = 1;
                }
              } else {
                atomicOr(D.err, 1);
              }
            }
          }
        }
        if (!need_samp) continue;
        // runs: the window start and every change of degree group (a > 0)
        unsigned long long runs;
        if (azero) {
          runs = 1ull;
        } else {
          const int gprev = __shfl(gw, lane > 0 ? lane - 1 : 0);
          runs = __ballot(valid && (lane == 0 || gw != gprev));
        }
        const int wlen = static_cast<int>(we - ws);
        while (runs) {
          const int s0 = __ffsll(static_cast<long long>(runs)) - 1;
          runs &= runs - 1ull;
          const int e0 = runs ? __ffsll(static_cast<long long>(runs)) - 1 : wlen;
          // the lane's run: from max(s0, J) to e0 (only if it is non-empty)
          const int jrel = J > ws ? static_cast<int>(J - ws) : 0;
          bool active = nz && jrel < e0;
          const int sl = jrel > s0 ? jrel : s0;
          const int slc = sl < kWave ? sl : kWave - 1;
          double dstart = 1.0;
          SkipTable tab;
          if (azero) {
            tab = tab0;
          } else {
            dstart = shfl_f64(daw, slc);
            const double num = cv * dstart;
            tab = make_skip_table(num / th);
          }
          const uint32_t s_abs = ws + static_cast<uint32_t>(sl);
          int pos = sl;
          uint32_t t = 0;
          while (__any(active)) {
            const U4 o = philox4x32_10(t, s_abs, u, ctr3, D.key0, D.key1);
            const double V = unit_double(o.x, o.y);
            const int cand = pos + geometric_skip(tab, V);
            const bool hit = active && cand < e0;
            if (active && !hit) active = false;
            const int cidx = hit ? cand : 0;
            const uint32_t vcand = static_cast<uint32_t>(__shfl(static_cast<int>(colw), cidx));
            const double dcand = azero ? 1.0 : shfl_f64(daw, cidx);
            bool emit = false;
            if (hit) {
              ++n_cand;
              bool accept = true;
              if (!azero) {
                const double ratio = dcand / dstart;
                accept = unit_double(o.z, o.w) < ratio;
              }
              if (accept) {
                ++n_acc;
                emit = true;
              }
              pos = cand + 1;
              ++t;
            }
            emit_sampled(emit, vcand, neg);
          }
        }
      }
    }
  }
  if (binned) {
    for (int g = 0; g < kMaxGroups; ++g) {
      if (g >= ng) break;
      group_flush(st, g, D);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ng * kBuckets; i += blockDim.x) {
      const unsigned int h = (&s_hist[0][0])[i];
      if (h) atomicAdd(D.bucket_count + i, h);
    }
  }
  const unsigned long long v0 = wave_sum_u64(n_front);
  const unsigned long long v1 = wave_sum_u64(n_hash);
  const unsigned long long v2 = wave_sum_u64(n_det);
  const unsigned long long v3 = wave_sum_u64(n_cand);
  const unsigned long long v4 = wave_sum_u64(n_acc);
  double m = mass;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) m += __shfl_down(m, off);
  if (lane == 0) {
    if (v0) atomicAdd(D.counters + 0, v0);
    if (v1) atomicAdd(D.counters + 1, v1);
    if (v2) atomicAdd(D.counters + 2, v2);
    if (v3) atomicAdd(D.counters + 3, v3);
    if (v4) atomicAdd(D.counters + 4, v4);
    if (m != 0.0) atomicAdd(D.mass, m);
  }
}

// Residues of long rows (read by every piece of the row) are cleared after
// the level kernel.
__global__ void k_dense_clear_rows(const uint32_t* __restrict__ rows, long long nrows, int Ct,
                                   float* __restrict__ r) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nrows * Ct;
       i += (long long)gridDim.x * blockDim.x) {
    const long long k = i / Ct;
    r[static_cast<size_t>(rows[k]) * Ct + static_cast<size_t>(i - k * Ct)] = 0.0f;
  }
}

// ------------------------------------------------- aggregation
// Per group: bucket offsets and partition cursors from the level's bucket
// counts (clearing them); a group whose records outgrew its buffer switches
// the level to the atomic fallback.
__global__ __launch_bounds__(1024) void k_dense_bins_scan(unsigned int* __restrict__ bucket_count,
                                                          unsigned long long* __restrict__ bucket_off,
                                                          unsigned long long* __restrict__ cursor,
                                                          const unsigned long long* __restrict__ rec_count,
                                                          unsigned long long cap, int* __restrict__ mode) {
  __shared__ unsigned long long s[kBuckets];
  const int g = blockIdx.x;
  const int t = threadIdx.x;
  unsigned int* bc = bucket_count + static_cast<size_t>(g) * kBuckets;
  const unsigned long long v = bc[t];
  bc[t] = 0;
  if (rec_count[g] > cap) {
    if (t == 0) atomicExch(mode, lvl::kModeOverflow);
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
  bucket_off[static_cast<size_t>(g) * (kBuckets + 1) + t] = excl;
  cursor[static_cast<size_t>(g) * kBuckets + t] = excl;
  if (t == kBuckets - 1) bucket_off[static_cast<size_t>(g) * (kBuckets + 1) + kBuckets] = s[t];
}

// One block per bin of group cells: signed record counts in LDS; each cell's
// exact total (its deterministic sum in acc, read only for bins that the
// level's deterministic pushes flagged, plus count * fl(theta_c)) is rounded
// once into r, acc is cleared, and the node is flagged for the next level.
constexpr int kSumThreads = 512;

__global__ __launch_bounds__(kSumThreads) void k_dense_bin_sum(const uint32_t* __restrict__ rec,
                                                               const unsigned long long* __restrict__ bin_off,
                                                               const ColParams* __restrict__ cp, int Ct, int cbase,
                                                               int wg, unsigned long long gcells,
                                                               long long* __restrict__ acc, float* __restrict__ r,
                                                               uint8_t* __restrict__ flag_out,
                                                               const int* __restrict__ mode, uint8_t* __restrict__ det) {
  if (*mode != lvl::kModeBinned) return;
  constexpr int kBin = 1 << kBinLog2;
  __shared__ int s_cnt[kBin];
  const unsigned long long gb = blockIdx.x;
  const unsigned long long cell0 = gb << kBinLog2;
  const bool read_acc = det[gb] != 0;
  const unsigned long long lo = bin_off[gb], hi = bin_off[gb + 1];
  if (!read_acc && lo == hi) return;
  for (int j = threadIdx.x; j < kBin; j += blockDim.x) s_cnt[j] = 0;
  __syncthreads();
  for (unsigned long long i0 = lo + threadIdx.x; i0 < hi; i0 += (unsigned long long)blockDim.x * 8) {
    uint32_t rr[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const unsigned long long i = i0 + (unsigned long long)k * blockDim.x;
      rr[k] = i < hi ? rec[i] : 0u;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (i0 + (unsigned long long)k * blockDim.x < hi) atomicAdd(&s_cnt[rr[k] & (kBin - 1)], (rr[k] >> 31) ? -1 : 1);
  }
  __syncthreads();
  constexpr int kCellsPer = kBin / kSumThreads;
#pragma unroll 4
  for (int k = 0; k < kCellsPer; ++k) {
    const int j = k * kSumThreads + threadIdx.x;
    const unsigned long long gcell = cell0 + static_cast<unsigned long long>(j);
    if (gcell >= gcells) continue;
    const int kc = s_cnt[j];
    if (!read_acc && kc == 0) continue;
    const unsigned long long u = gcell / static_cast<unsigned long long>(wg);
    const int c = cbase + static_cast<int>(gcell - u * static_cast<unsigned long long>(wg));
    const size_t idx = static_cast<size_t>(u) * static_cast<size_t>(Ct) + static_cast<size_t>(c);
    long long a = 0;
    if (read_acc) a = acc[idx];
    const long long v = a + static_cast<long long>(kc) * cp[c].dtheta;
    if (a != 0) acc[idx] = 0;
    if (v != 0) {
      r[idx] = units_to_f32(v, cp[c].ue);
      flag_out[u] = 1;
    }
  }
  if (threadIdx.x == 0 && read_acc) det[gb] = 0;
}

// Records of the groups' buffers added with atomics (level in the fallback).
__global__ void k_dense_apply_overflow(DenseArgs D, int ng, const int* __restrict__ mode) {
  if (*mode != lvl::kModeOverflow) return;
  for (int g = 0; g < ng; ++g) {
    const unsigned long long cnt = D.rec_count[g] < D.rec_cap ? D.rec_count[g] : D.rec_cap;
    const uint32_t* rg = D.rec + static_cast<size_t>(g) * D.rec_cap;
    for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < cnt;
         i += (unsigned long long)gridDim.x * blockDim.x)
      apply_group_record(D, g, rg[i]);
  }
}

// Every cell of the tile (levels aggregated with atomics only): the exact
// sums rounded into r, acc cleared, nodes flagged.  mode == nullptr: always.
__global__ void k_dense_finish(const ColParams* __restrict__ cp, int64_t n, int Ct, long long* __restrict__ acc,
                               float* __restrict__ r, uint8_t* __restrict__ flag_out, const int* __restrict__ mode) {
  if (mode && *mode != lvl::kModeOverflow && *mode != lvl::kModeCompact) return;
  const size_t total = static_cast<size_t>(n) * static_cast<size_t>(Ct);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const long long v = acc[i];
    if (v == 0) continue;
    const size_t u = i / static_cast<size_t>(Ct);
    const int c = static_cast<int>(i - u * static_cast<size_t>(Ct));
    acc[i] = 0;
    r[i] = units_to_f32(v, cp[c].ue);
    flag_out[u] = 1;
  }
}

// Fills (used instead of memset nodes so that the level loop can be
// captured in a graph).
__global__ void k_fill_u8(uint8_t* __restrict__ p, size_t n, uint8_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_i32(int* __restrict__ p, int n, int v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

}  // namespace dense
}  // namespace agp
