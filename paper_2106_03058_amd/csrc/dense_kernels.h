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
using lvl::wave_sync;

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kMaxCols = 64;       // columns of a tile (one lane each)
constexpr int kMaxGroups = 4;      // record groups of a tile
constexpr int kItemArcs = 4096;    // arcs of a work item (rows above it are cut by windows)
constexpr int kItemNodes = 64;     // nodes of a work item
constexpr int kStageRecs = 512;    // records staged per wave (split over the groups)

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
  unsigned long long* counters;  // this level's counters (frontier, hash, det, cand, acc, runs)
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

// ------------------------------------------------------------ the level
// Per work item (a run of consecutive nodes, or a piece of one long row) the
// wave first loads the row pointer, degree and d_u^-b of every node (one lane
// per node).  Each node with a non-zero residue is then set up with one lane
// per column (residue, reserve, c = rho |r| d_u^-b, the deterministic prefix
// J) and its row is taken 64 arcs (one window) at a time: the window's
// neighbour ids, degree factors and run boundaries (degree groups cut at the
// window) go to LDS, and the (column, run) pairs of the window -- every run
// after each column's deterministic prefix -- are numbered column by column
// and handed out to the lanes: a lane builds the skip table of its pair's
// run and walks the run's Philox / geometric-skip chain one draw per step,
// reading candidates' neighbours from LDS, and takes the next pair of the
// window as soon as its chain ends.  So lanes stay busy whether a node has
// one active column or 64, however many degree groups its row holds and
// however long each chain runs.  The next node's residues and first window
// are loaded while the current node draws.
struct WaveLds {
  int64_t rp[kItemNodes];       // the item's nodes: first arc
  uint32_t d[kItemNodes];       //   degree
  double db[kItemNodes];        //   d_u^-b
  uint32_t col[kWave];          // the window's neighbour ids
  double da[kWave];             //   their factors d^-a (1 when a = 0)
  uint32_t rs[kWave + 1];       //   run starts (window-relative); rs[R] = window length
  uint32_t meta[kWave];         // per sampling column, by rank: column | k0 << 8 | jr << 16 |
                                // whole << 23 | sign << 31 (k0 its first run, jr its deterministic
                                // prefix in the window, whole: run k0 takes the rest of the window)
  double cv[kWave];             // per sampling column, by rank: c = rho |r| d_u^-b
  uint8_t more[kWave];          // ranks of the sampling columns whose run k0 ends with its group
  int nst[kMaxGroups];          // records staged per group
  uint32_t stage[kStageRecs];   // staged records, kStageRecs / ng per group
};

template <bool kFirst>
__global__ __launch_bounds__(kThreads, 4) void k_dense_level(DenseArgs D) {
  __shared__ WaveLds s_w[kWaves];
  __shared__ unsigned int s_hist[kMaxGroups][kBuckets];
  __shared__ double s_theta[kMaxCols];
  __shared__ long long s_dth[kMaxCols];
  __shared__ uint32_t s_ctr3[kMaxCols];
  __shared__ uint32_t s_magic[kWave + 1];  // ceil(2^32 / R) for R = 2..64 (R = 1: 2^32 - 1)

  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const unsigned long long lt_mask = (1ull << lane) - 1ull;
  const bool binned = D.rec != nullptr;
  const int ng = (D.Ct + (1 << D.gshift) - 1) >> D.gshift;
  const int per = kStageRecs / ng;
  WaveLds& W = s_w[wave];
  for (int i = threadIdx.x; i <= kWave; i += blockDim.x)
    s_magic[i] = i <= 1 ? 0xFFFFFFFFu
                        : static_cast<uint32_t>((0x100000000ull + static_cast<unsigned long long>(i) - 1ull) /
                                                static_cast<unsigned long long>(i));
  for (int i = threadIdx.x; i < D.Ct; i += blockDim.x) {
    const ColParams& p = D.cp[i];
    s_theta[i] = p.theta;
    s_dth[i] = p.dtheta;
    s_ctr3[i] = (p.qid << 8) | static_cast<uint32_t>(D.level);
  }
  if (binned)
    for (int i = threadIdx.x; i < ng * kBuckets; i += blockDim.x) (&s_hist[0][0])[i] = 0;
  if (lane < kMaxGroups) W.nst[lane] = 0;
  __syncthreads();

  // the lane's column during the per-node setup
  const int c = lane;
  const bool live = c < D.Ct;
  const int my_g = c >> D.gshift;
  const int my_w = live ? group_width(D.Ct, D.gshift, my_g) : 1;
  const int my_cl = c - (my_g << D.gshift);
  double th = 1.0, scale = 1.0;
  if (live) {
    th = D.cp[c].theta;
    scale = D.cp[c].scale;
  }
  const bool azero = (D.lflags & kAZero) != 0;
  const bool last = (D.lflags & kLastLevel) != 0;
  const bool pushes = !last && D.rho != 0.0;

  unsigned long long n_front = 0, n_hash = 0, n_det = 0, n_cand = 0, n_acc = 0, n_runs = 0;
  double mass = 0.0;

  // records of group g to the level's buffer (all lanes together)
  auto flush = [&](int g) {
    const int cnt = W.nst[g];
    if (cnt == 0) return;
    unsigned long long b0 = 0;
    if (lane == 0) b0 = atomicAdd(D.rec_count + g, static_cast<unsigned long long>(cnt));
    b0 = __shfl(b0, 0);
    const uint32_t* src = W.stage + g * per;
    uint32_t* dst = D.rec + static_cast<size_t>(g) * D.rec_cap;
    for (int i = lane; i < cnt; i += kWave) {
      if (b0 + i < D.rec_cap)
        dst[b0 + i] = src[i];
      else
        apply_group_record(D, g, src[i]);
    }
    wave_sync();
    if (lane == 0) W.nst[g] = 0;
    wave_sync();
  };
  // a sampled push of -/+ fl(theta_ec) to (v, ec) for the lanes with e (all
  // lanes together): a staged record, or an integer atomic without records
  auto emit = [&](bool e, uint32_t v, int ec, bool neg) {
    if (__ballot(e) == 0ull) return;
    if (binned) {
      if (e) {
        const int eg = ec >> D.gshift;
        const int ew = group_width(D.Ct, D.gshift, eg);
        const uint32_t gcell = v * static_cast<uint32_t>(ew) + static_cast<uint32_t>(ec - (eg << D.gshift));
        atomicAdd(&s_hist[eg][gcell >> D.bucket_shift], 1u);
        const int slot = atomicAdd(&W.nst[eg], 1);
        W.stage[eg * per + slot] = gcell | (neg ? 0x80000000u : 0u);
      }
      wave_sync();
      for (int g = 0; g < ng; ++g)
        if (W.nst[g] > per - kWave) flush(g);
    } else if (e) {
      const long long dt = neg ? -s_dth[ec] : s_dth[ec];
      lvl::atomic_add_relaxed(reinterpret_cast<unsigned long long*>(D.acc + static_cast<size_t>(v) * D.Ct + ec),
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
    // the item's nodes (lane = node)
    bool f = false;
    if (lane < nodes) {
      const uint32_t uu = u0 + static_cast<uint32_t>(lane);
      f = kFirst || D.flag_in[uu] != 0;
      if (f) {
        W.rp[lane] = D.rp[uu];
        W.d[lane] = static_cast<uint32_t>(D.deg[uu]);
        W.db[lane] = pushes ? D.db[D.fdeg[uu]] : 0.0;
      }
    }
    unsigned long long todo = __ballot(f);
    wave_sync();
    // the first piece of a long row owns the row's per-node work (reserve,
    // frontier counters, mass); the row's residues are cleared after the
    // level (every piece reads them)
    const bool owner = !longrow || wlo == 0;
    const uint32_t ws0 = wlo << kSegLog2;
    // loads of a node's residues (lane = column) and first window (lane = arc)
    float r_n = 0.0f;
    uint32_t col_n = 0, nd_n = 0;
    auto prefetch = [&](int bb) {
      const uint32_t uu = u0 + static_cast<uint32_t>(bb);
      r_n = 0.0f;
      if (live) r_n = kFirst ? D.x[static_cast<size_t>(uu) * static_cast<size_t>(D.xld) + c]
                             : D.r[static_cast<size_t>(uu) * static_cast<size_t>(D.Ct) + c];
      col_n = nd_n = 0;
      if (pushes) {
        const uint32_t j = ws0 + static_cast<uint32_t>(lane);
        if (j < W.d[bb]) {
          const int64_t a = W.rp[bb] + j;
          col_n = D.col[a];
          nd_n = D.nd[a];
        }
      }
    };
    if (todo) prefetch(__ffsll(static_cast<long long>(todo)) - 1);
    while (todo) {
      const int b = __ffsll(static_cast<long long>(todo)) - 1;
      todo &= todo - 1ull;
      const uint32_t u = u0 + static_cast<uint32_t>(b);
      const float r = r_n;
      const uint32_t colw0 = col_n, ndw0 = nd_n;
      const uint32_t d = W.d[b];
      const int64_t rp = W.rp[b];
      const bool nz = live && r != 0.0f;
      // dependent loads of this node before the next node's prefetch
      const bool valid0 = ws0 + static_cast<uint32_t>(lane) < d;
      double daw0 = 1.0;
      if (pushes && !azero && valid0) daw0 = D.da[ndw0];
      float* o = D.out + static_cast<size_t>(u) * static_cast<size_t>(D.old) + c;
      float o_old = 0.0f;
      if (!kFirst && owner && nz && D.kappa != 0.0) o_old = *o;
      if (todo) prefetch(__ffsll(static_cast<long long>(todo)) - 1);
      // ---- per-column setup (lane = column)
      if (!kFirst && !longrow && nz) D.r[static_cast<size_t>(u) * static_cast<size_t>(D.Ct) + c] = 0.0f;
      if (owner) {
        // frontier counters: (node, column) pairs with a non-zero residue and
        // their hash, counted once per node (lane 0)
        const unsigned long long nzm = __ballot(nz);
        if (lane == 0 && nzm) {
          const unsigned long long kk = static_cast<unsigned long long>(__popcll(nzm));
          n_front += kk;
          n_hash += kk * splitmix64(u);
        }
        if (kFirst) {  // pi starts at +0: pi = +0 + fl(kappa r)
          if (live) *o = nz ? 0.0f + static_cast<float>(D.kappa * static_cast<double>(r)) : 0.0f;
        } else if (nz && D.kappa != 0.0) {
          *o = o_old + static_cast<float>(D.kappa * static_cast<double>(r));
        }
      }
      if (!pushes || d == 0 || !__any(nz)) continue;
      const bool neg = r < 0.0f;
      // c = (rho |r|) d_u^-b and the deterministic prefix J (increment >= theta):
      // the increments fall along the degree-sorted row
      const double absr = fabs(static_cast<double>(r));
      const double t0 = D.rho * absr;
      const double cv = t0 * W.db[b];
      uint32_t J = 0;
      double inc0 = cv;
      const bool onewin = d - ws0 <= static_cast<uint32_t>(kWave);  // the piece's first window ends the row
      if (azero) {
        J = (nz && cv >= th) ? d : 0u;
      } else {
        const double da_first = wlo == 0 ? shfl_f64(daw0, 0) : D.da[D.nd[rp]];
        inc0 = cv * da_first;
        double da_last;
        if (wlo == 0 && onewin)
          da_last = shfl_f64(daw0, static_cast<int>(d - 1));
        else
          da_last = D.da[D.nd[rp + d - 1]];
        uint32_t lo = 0, hi = d;
        if (!nz || !(inc0 >= th))
          hi = 0;
        else if (cv * da_last >= th)
          lo = d;
        if (__any(lo < hi)) {
          if (wlo == 0 && onewin) {  // the row is in registers: search by lane exchanges
            for (int step = 0; step < 7; ++step) {
              const uint32_t mid = (lo + hi) >> 1;
              const double dm = shfl_f64(daw0, static_cast<int>(mid < d ? mid : 0u));
              if (lo < hi) {
                if (cv * dm >= th)
                  lo = mid + 1;
                else
                  hi = mid;
              }
            }
          } else {
            while (lo < hi) {
              const uint32_t mid = (lo + hi) >> 1;
              if (cv * D.da[D.nd[rp + mid]] >= th)
                lo = mid + 1;
              else
                hi = mid;
            }
          }
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
        const uint32_t jlo = ws0, jhi = (w1 << kSegLog2) < d ? (w1 << kSegLog2) : d;
        n_det += (J > jlo ? (J < jhi ? J : jhi) - jlo : 0u);
      }
      const uint32_t Jmax = wave_max_u32(nz ? J : 0u);
      for (uint32_t w = wlo; w < w1; ++w) {
        const uint32_t ws = w << kSegLog2;
        const uint32_t we = (ws + kSeg) < d ? ws + kSeg : d;
        const bool has = nz && J < we;  // the column samples in this window
        const bool need_samp = __any(has);
        const bool need_det = Jmax > ws;
        if (!need_samp && !need_det) continue;
        // ---- the window's arcs (lane = arc)
        const bool valid = ws + static_cast<uint32_t>(lane) < we;
        uint32_t colw = colw0;
        double daw = daw0;
        if (w != wlo) {
          colw = 0u;
          daw = 1.0;
          if (valid) {
            const int64_t a = rp + ws + static_cast<uint32_t>(lane);
            colw = D.col[a];
            if (!azero) daw = D.da[D.nd[a]];
          }
        }
        // deterministic pushes at positions [ws, min(Jmax, we)) (lane = column)
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
        // runs: the window start and every change of degree group (a > 0);
        // floor(log2) of d^-a's degree is read back from the factor's bits
        unsigned long long runs;
        if (azero) {
          runs = 1ull;
        } else {
          const uint32_t ndv = valid ? (w == wlo ? ndw0 : D.nd[rp + ws + static_cast<uint32_t>(lane)]) : 1u;
          const int gw = 31 - __clz(ndv);
          const int gprev = __shfl(gw, lane > 0 ? lane - 1 : 0);
          runs = __ballot(valid && (lane == 0 || gw != gprev));
        }
        const int R = __popcll(runs);
        // per sampling column: its first run (runs ending at or before its
        // prefix are deterministic), its prefix inside the window, and
        // whether that run takes the rest of the window (few expected
        // candidates); the run contains position jr, so it starts there
        const uint32_t jr = J > ws ? J - ws : 0u;
        const uint32_t wlen = we - ws;
        int k0 = 0;
        bool whole = true;
        if (has) {
          const unsigned long long upto = jr >= 63u ? ~0ull : ((2ull << jr) - 1ull);
          k0 = __popcll(runs & upto & ~1ull);
        }
        const double da_jr = shfl_f64(daw, static_cast<int>(jr < 63u ? jr : 63u));
        if (has && !azero && k0 + 1 < R) {
          const double pr = (cv * da_jr) / s_theta[c];
          whole = pr * static_cast<double>(wlen - jr) <= kMergeCandidates;
        }
        const unsigned long long hasm = __ballot(has);
        const unsigned long long morem = __ballot(has && !whole);
        // pairs: one per sampling column for its run k0, then (column, run
        // 1..R-1) for the columns whose run k0 ends with its degree group
        const uint32_t H = static_cast<uint32_t>(__popcll(hasm));
        const uint32_t R2 = static_cast<uint32_t>(R > 1 ? R - 1 : 1);
        const uint32_t total = H + static_cast<uint32_t>(__popcll(morem)) * R2;
        const uint32_t magic = s_magic[R2];
        wave_sync();  // the previous window's pairs have been read
        W.col[lane] = colw;
        W.da[lane] = daw;
        if ((runs >> lane) & 1ull) W.rs[__popcll(runs & lt_mask)] = static_cast<uint32_t>(lane);
        if (lane == 0) W.rs[R] = wlen;
        if (has) {
          const int rk = __popcll(hasm & lt_mask);
          W.meta[rk] = static_cast<uint32_t>(c) | (static_cast<uint32_t>(k0) << 8) | (jr << 16) |
                       (whole ? 0x800000u : 0u) | (neg ? 0x80000000u : 0u);
          W.cv[rk] = cv;
          if (!whole) W.more[__popcll(morem & lt_mask)] = static_cast<uint8_t>(rk);
        }
        wave_sync();
        // ---- the window's pairs; a lane takes the next pair as soon as its
        // chain has ended (lane = pair)
        uint32_t next = 0;
        bool active = false;
        int pc = 0;
        bool pneg = false;
        uint32_t ctr3 = 0, s_abs = 0, pos = 0, e = 0, t = 0;
        double dstart = 1.0;
        SkipTable tab;
        for (;;) {
          const unsigned long long idle = __ballot(!active);
          if (idle != 0ull && next < total) {
            const uint32_t idx = next + static_cast<uint32_t>(__popcll(idle & lt_mask));
            next += static_cast<uint32_t>(__popcll(idle));
            if (!active && idx < total) {
              uint32_t cr = idx, k = 0;
              const bool first = idx < H;
              if (!first) {
                const uint32_t i2 = idx - H;
                uint32_t r2 = __umulhi(i2, magic);
                k = i2 - r2 * R2;
                if (k >= R2) {
                  k -= R2;
                  ++r2;
                }
                ++k;
                cr = W.more[r2];
              }
              const uint32_t meta = W.meta[cr];
              const uint32_t k0c = (meta >> 8) & 0xFFu;
              const int q = static_cast<int>(meta & 0xFFu);
              const double cvr = W.cv[cr];
              const double thq = s_theta[q];
              bool live = true;
              uint32_t s0 = (meta >> 16) & 0x7Fu;  // run k0 starts at the prefix
              if (first) {
                k = k0c;
                e = (meta & 0x800000u) ? wlen : W.rs[k + 1];
              } else {
                // runs up to k0 are taken; a run after one that took the rest
                // of the window is covered by it (p* (wlen - s) does not grow
                // along the sorted row, and run k0 did not)
                live = k > k0c;
                if (live && k > k0c + 1) {
                  const uint32_t sp = W.rs[k - 1];
                  const double pp = (cvr * W.da[sp]) / thq;
                  live = !(pp * static_cast<double>(wlen - sp) <= kMergeCandidates);
                }
                if (live) s0 = W.rs[k];
              }
              if (live) {
                ++n_runs;
                dstart = azero ? 1.0 : W.da[s0];
                const double num = cvr * dstart;
                const double pr = num / thq;
                if (!first) e = pr * static_cast<double>(wlen - s0) <= kMergeCandidates ? wlen : W.rs[k + 1];
                tab = make_skip_table(pr);
                pneg = (meta >> 31) != 0;
                ctr3 = s_ctr3[q];
                s_abs = ws + s0;
                pos = s0;
                t = 0;
                pc = q;
                active = true;
              }
            }
          }
          if (!__any(active)) {
            if (next >= total) break;
            continue;
          }
          bool e_push = false;
          uint32_t vcand = 0;
          if (active) {
            const U4 o = philox4x32_10_skey(t, s_abs, u, ctr3, D.key0, D.key1);
            const double V = unit_double(o.x, o.y);
            const uint32_t cand = pos + static_cast<uint32_t>(geometric_skip(tab, V));
            if (cand < e) {
              ++n_cand;
              bool accept = true;
              if (!azero) {
                const double ratio = W.da[cand] / dstart;
                accept = unit_double(o.z, o.w) < ratio;
              }
              if (accept) {
                ++n_acc;
                e_push = true;
                vcand = W.col[cand];
              }
              pos = cand + 1;
              ++t;
            } else {
              active = false;
            }
          }
          emit(e_push, vcand, pc, pneg);
        }
      }
    }
  }
  if (binned) {
    for (int g = 0; g < ng; ++g) flush(g);
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
  const unsigned long long v5 = wave_sum_u64(n_runs);
  double m = mass;
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) m += __shfl_down(m, off);
  if (lane == 0) {
    if (v0) atomicAdd(D.counters + 0, v0);
    if (v1) atomicAdd(D.counters + 1, v1);
    if (v2) atomicAdd(D.counters + 2, v2);
    if (v3) atomicAdd(D.counters + 3, v3);
    if (v4) atomicAdd(D.counters + 4, v4);
    if (v5) atomicAdd(D.counters + 5, v5);
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
  const uint32_t uwg = static_cast<uint32_t>(wg);
#pragma unroll 4
  for (int k = 0; k < kCellsPer; ++k) {
    const int j = k * kSumThreads + threadIdx.x;
    const unsigned long long gcell = cell0 + static_cast<unsigned long long>(j);
    if (gcell >= gcells) continue;
    const int kc = s_cnt[j];
    if (!read_acc && kc == 0) continue;
    const uint32_t g32 = static_cast<uint32_t>(gcell);  // group cells stay below 2^31
    const uint32_t u = g32 / uwg;
    const int c = cbase + static_cast<int>(g32 - u * uwg);
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
