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
// (row-major n x C for agp_propagate, one contiguous n-vector per slot for
// the server).  Next-level residues are exact integers of a per-column unit
// (int64 cells for binary32, 128-bit cells for binary64), so the integer
// atomics that add contributions commute and the result does not depend on
// the order in which pushes land.
//
// Per tile of up to 256 frontier entries a block converts each residue,
// updates the reserve (pi(u) += kappa_i r(u)), finds the deterministic prefix
// J of the degree-sorted row by binary search (increment >= theta) and counts
// the 64-position windows of the sampled suffix; a block-wide scan spreads
// single pushes and windows over the lanes, which walk the Philox /
// geometric-skip chains in lockstep per wave.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "agp_device.h"

namespace agp {
namespace lvl {

constexpr int kThreads = 256;
constexpr int kTile = 256;  // frontier entries per block tile
constexpr int kLevelBlocks = 2048;
constexpr int kNumCounters = 5;   // frontier, hash, det, cand, acc
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

// Binned aggregation: a record is (cell << 32 | fp32 bits of the
// contribution); cells are grouped into 1024 buckets of 1024 bins of 4096
// cells (an LDS accumulator of 32 KiB), so n * C must stay below 2^32.
constexpr int kBinLog2 = 12;
constexpr int kBinsPerBucketLog2 = 10;
constexpr int kBucketShift = kBinLog2 + kBinsPerBucketLog2;
constexpr int kBuckets = 1024;

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
  const int32_t* deg;
  const ColParams* cp;
  long long su, sc;  // cell = u * su + c * sc
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
  // binned aggregation (binary32 batched calls; rec == nullptr: disabled)
  uint64_t* rec;
  unsigned long long* rec_count;
  unsigned long long rec_cap;
  unsigned int* bucket_count;    // records per bucket of this level
};

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
// Records go to A.rec in chunks (one atomic per chunk).  Records beyond the
// buffer capacity are added to the accumulator directly; the level then ends
// in kModeOverflow (the buffered records are applied with atomics too).
template <typename Cell>
__device__ __forceinline__ void apply_record(const LevelArgs& A, Cell* acc, uint64_t rec);

template <>
__device__ __forceinline__ void apply_record<long long>(const LevelArgs& A, long long* acc, uint64_t rec) {
  const uint32_t cell = static_cast<uint32_t>(rec >> 32);
  const float val = __uint_as_float(static_cast<uint32_t>(rec));
  const uint32_t c = cell % static_cast<uint32_t>(A.su);
  long long d;
  if (f32_to_units(val, A.cp[c].scale, &d))
    atomic_add_relaxed(reinterpret_cast<unsigned long long*>(acc + cell), static_cast<unsigned long long>(d));
  else
    atomicOr(A.err, 1);
}

template <>
__device__ __forceinline__ void apply_record<unsigned long long>(const LevelArgs&, unsigned long long*, uint64_t) {}

template <typename Cell>
__device__ __forceinline__ void stage_flush_records(uint64_t* stage, int& staged, const LevelArgs& A, Cell* acc) {
  if (staged == 0) return;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  unsigned long long base = 0;
  if (lane_id() == 0) base = atomicAdd(A.rec_count, static_cast<unsigned long long>(staged));
  base = __shfl(base, 0);
  for (int i = lane_id(); i < staged; i += kWave) {
    if (base + i < A.rec_cap)
      A.rec[base + i] = stage[i];
    else
      apply_record(A, acc, stage[i]);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  staged = 0;
}

template <typename Cell>
__device__ __forceinline__ void stage_push_records(uint64_t* stage, int& staged, uint64_t rec, bool pred,
                                                   const LevelArgs& A, Cell* acc) {
  const unsigned long long mask = __ballot(pred);
  if (pred) stage[staged + __popcll(mask & ((1ull << lane_id()) - 1ull))] = rec;
  staged += __popcll(mask);
  if (staged > kStage - kWave) stage_flush_records(stage, staged, A, acc);
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
// kFirst: the residues are the signal x (level 0 of a batched call).
// kServe: counters and overflow mass are kept per column instead of per level.
template <typename T, bool kFirst, bool kServe>
__global__ __launch_bounds__(kThreads) void k_level(LevelArgs A, const T* __restrict__ x,
                                                    typename Prec<T>::Cell* __restrict__ acc_cur,
                                                    typename Prec<T>::Cell* __restrict__ acc_next) {
  using P = Prec<T>;
  using Delta = typename P::Delta;
  __shared__ long long s_off[kTile + 1];
  __shared__ int64_t s_rp[kTile];
  __shared__ double s_cv[kTile];
  __shared__ double s_p0[kTile];  // a = 0: the sampling probability of every run
  __shared__ uint32_t s_u[kTile];
  __shared__ uint32_t s_c[kTile];
  __shared__ uint32_t s_d[kTile];
  __shared__ uint32_t s_J[kTile];
  __shared__ uint32_t s_neg[kTile];
  __shared__ long long s_wave[kThreads / kWave];
  __shared__ uint64_t s_stage[kThreads / kWave][kStage];
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
  const bool binned = A.rec != nullptr;
  const bool sparse = !binned && A.positive && count < A.dense_cut;
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
  unsigned long long te = (count + gridDim.x - 1) / gridDim.x;
  te = te < 1 ? 1 : (te > (unsigned long long)kTile ? (unsigned long long)kTile : te);
  const unsigned long long ntiles = (count + te - 1) / te;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = tid / kWave;
  uint64_t* stage = s_stage[wave];
  int staged = 0;  // wave-uniform

  unsigned long long n_front = 0, n_hash = 0, n_det = 0, n_cand = 0, n_acc = 0;
  double mass = 0.0;

  for (unsigned long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const unsigned long long e0 = tile * te;
    const int ne = static_cast<int>((count - e0) < te ? (count - e0) : te);
    long long work = 0;
    if (tid < ne) {
      const uint64_t item = A.fin[e0 + tid];
      const uint32_t u = static_cast<uint32_t>(item >> 32);
      const uint32_t c = static_cast<uint32_t>(item);
      const size_t cell = static_cast<size_t>(u) * A.su + static_cast<size_t>(c) * A.sc;
      const ColParams& cp = A.cp[c];
      T r;
      if (kFirst)
        r = x[cell];
      else
        r = P::take(acc_cur, cell, cp);
      uint32_t d = 0, J = 0;
      double cv = 0.0;
      if (!(cp.flags & kDrop)) {
        if (kServe) {
          serve_count(A, s_scnt, c, 0, 1ull);
        } else {
          ++n_front;
          n_hash += splitmix64(u);
        }
        // reserve: pi(u) += (S w_i / Y_i) r(u), rounded to the working precision
        if (cp.kappa != 0.0) {
          T* o = static_cast<T*>(cp.out) + static_cast<size_t>(u) * static_cast<size_t>(cp.out_stride);
          const T q = to_w(cp.kappa * static_cast<double>(r), T());
          *o = *o + q;
        }
        if (!(cp.flags & kLastLevel) && cp.rho != 0.0) {
          d = static_cast<uint32_t>(A.deg[u]);
          if (d > 0) {
            const double absr = fabs(static_cast<double>(r));
            const double t0 = cp.rho * absr;
            cv = t0 * cp.db[d];
            const double th = cp.theta;
            const int64_t rpu = A.rp[u];
            const bool azero = (cp.flags & kAZero) != 0;
            double inc0 = cv;
            if (azero) {
              J = (cv >= th) ? d : 0u;
              const double num = cv * 1.0;  // every neighbour's factor d^-0 is 1
              s_p0[tid] = num / th;
            } else {  // increments fall along the degree-sorted row: binary search
              inc0 = cv * cp.da[A.nd[rpu]];
              uint32_t lo = 0, hi = d;
              while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                const double inc = cv * cp.da[A.nd[rpu + mid]];
                if (inc >= th)
                  lo = mid + 1;
                else
                  hi = mid;
              }
              J = lo;
            }
            const long long windows =
                (J < d) ? static_cast<long long>(((d - 1) >> kSegLog2) - (J >> kSegLog2) + 1) : 0;
            work = static_cast<long long>(J) + windows;
            // bound on the magnitude this entry can add (every contribution
            // is at most max(inc_0, theta)), for the overflow check
            const T big = to_w(inc0 > th ? inc0 : th, T());
            const double m = static_cast<double>(d) * P::mag_units(big, cp);
            if (kServe) {
              serve_count(A, s_scnt, c, 2, static_cast<unsigned long long>(J));
              if (c < kServeLdsSlots)
                atomicAdd(&s_smass[c], m);
              else
                atomicAdd(A.mass + c, m);
            } else {
              n_det += J;
              mass += m;
            }
            s_rp[tid] = rpu;
          }
        }
      }
      s_u[tid] = u;
      s_c[tid] = c;
      s_d[tid] = d;
      s_J[tid] = J;
      s_cv[tid] = cv;
      s_neg[tid] = (r < T(0)) ? 1u : 0u;
    }
    // block exclusive scan of the work counts
    long long incl = work;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const long long t = __shfl_up(incl, off);
      if (lane >= off) incl += t;
    }
    if (lane == kWave - 1) s_wave[wave] = incl;
    __syncthreads();
    long long wbase = 0;
    for (int w = 0; w < wave; ++w) wbase += s_wave[w];
    s_off[tid] = wbase + incl - work;
    if (tid == kThreads - 1) s_off[kThreads] = wbase + incl;
    __syncthreads();
    const long long total = s_off[kThreads];

    // Every lane pulls work items k = tid, tid + 256, ...: a single push of
    // the deterministic prefix, or a 64-position window of the sampled suffix
    // walked one random draw per step.  The loop runs in lockstep per wave so
    // that frontier staging can use wave-wide ballots.
    long long k = tid;
    int ttype = 0;  // 0 idle, 1 single push, 2 window
    bool need_run = false, neg = false, azero = true;
    uint32_t u = 0, c = 0, s = 0, wend = 0, run_end = 0, pos = 0, t = 0, ctr3 = 0;
    uint32_t win_cand = 0, win_acc = 0;
    int64_t rpu = 0;
    double cv = 0.0, dstart = 1.0, th = 0.0, p0 = 0.0;
    long long local = 0;
    const ColParams* cpp = nullptr;
    SkipTable tab;
    for (;;) {
      if (ttype == 0 && k < total) {
        int lo = 0, hi = ne - 1;  // largest e with s_off[e] <= k
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_off[mid] <= k)
            lo = mid;
          else
            hi = mid - 1;
        }
        const int e = lo;
        local = k - s_off[e];
        k += kThreads;
        const uint32_t J = s_J[e];
        u = s_u[e];
        c = s_c[e];
        rpu = s_rp[e];
        cv = s_cv[e];
        neg = s_neg[e] != 0;
        cpp = A.cp + c;
        azero = (cpp->flags & kAZero) != 0;
        if (azero) p0 = s_p0[e];
        if (local < static_cast<long long>(J)) {
          ttype = 1;
        } else {
          ttype = 2;
          const uint32_t d = s_d[e];
          const uint32_t wstart = ((J >> kSegLog2) + static_cast<uint32_t>(local - J)) << kSegLog2;
          s = wstart > J ? wstart : J;
          wend = (wstart + static_cast<uint32_t>(kSeg)) < d ? wstart + static_cast<uint32_t>(kSeg) : d;
          need_run = true;
          th = cpp->theta;
          ctr3 = (cpp->qid << 8) | static_cast<uint32_t>(cpp->level);
          win_cand = win_acc = 0;
        }
      }
      if (!__any(ttype != 0)) break;

      bool emit = false;
      bool ttype_val_det = false;
      T det_val = T(0);
      Delta delta{};
      uint32_t v = 0;
      if (ttype == 1) {
        // deterministic push: the increment reaches theta
        const int64_t arc = rpu + local;
        v = A.col[arc];
        double inc = cv;
        if (!azero) inc = cv * cpp->da[A.nd[arc]];
        T val = to_w(inc, T());
        if (neg) val = -val;
        emit = P::to_units(val, *cpp, &delta);
        if (!emit) atomicOr(A.err + (kServe ? c : 0u), 1);
        ttype_val_det = true;
        det_val = val;
        ttype = 0;
      } else if (ttype == 2) {
        if (need_run) {
          if (s >= wend) {
            ttype = 0;
            if (kServe && win_cand) {
              serve_count(A, s_scnt, c, 3, static_cast<unsigned long long>(win_cand));
              if (win_acc) serve_count(A, s_scnt, c, 4, static_cast<unsigned long long>(win_acc));
            }
          } else {  // a run: same degree group (a > 0) inside the window
            run_end = wend;
            dstart = 1.0;
            if (!azero) {
              const uint32_t ds = A.nd[rpu + s];
              dstart = cpp->da[ds];
              const int g = 31 - __clz(ds);
              if (g < 31) {
                const uint32_t lim = 1u << (g + 1);
                uint32_t blo = s + 1, bhi = wend;
                while (blo < bhi) {
                  const uint32_t mid = (blo + bhi) >> 1;
                  if (A.nd[rpu + mid] < lim)
                    blo = mid + 1;
                  else
                    bhi = mid;
                }
                run_end = blo;
              }
            }
            double pstar = p0;  // a = 0: computed once per entry, (cv * 1) / theta
            if (!azero) {
              const double num = cv * dstart;
              pstar = num / th;
            }
            tab = make_skip_table(pstar);
            pos = s;
            t = 0;
            need_run = false;
          }
        }
        if (ttype == 2 && !need_run) {
          const U4 o = philox4x32_10(t, s, u, ctr3, cpp->key0, cpp->key1);
          const double V = unit_double(o.x, o.y);
          const uint32_t cand = pos + static_cast<uint32_t>(geometric_skip(tab, V));
          if (cand >= run_end) {
            s = run_end;
            need_run = true;
          } else {
            ++n_cand;
            ++win_cand;
            const int64_t arc = rpu + cand;
            bool accept = true;  // a = 0: the ratio is 1 and every uniform is below it
            if (!azero) {
              const double ratio = cpp->da[A.nd[arc]] / dstart;
              accept = unit_double(o.z, o.w) < ratio;
            }
            if (accept) {
              ++n_acc;
              ++win_acc;
              v = A.col[arc];
              emit = true;
              delta = P::theta_units(*cpp, neg);
            }
            pos = cand + 1;
            ++t;
          }
        }
      }
      bool first = false;
      const size_t vcell = static_cast<size_t>(v) * A.su + static_cast<size_t>(c) * A.sc;
      if (binned) {  // wave-uniform: stage records, flush in chunks
        uint64_t rec = 0;
        if (emit) {
          T val = T(0);
          if (ttype_val_det) {
            val = det_val;
          } else {
            val = neg ? -static_cast<T>(cpp->theta_w) : static_cast<T>(cpp->theta_w);
          }
          rec = (static_cast<uint64_t>(vcell) << 32) | static_cast<uint64_t>(__float_as_uint(static_cast<float>(val)));
          atomicAdd(&s_hist[vcell >> kBucketShift], 1u);
        }
        stage_push_records(stage, staged, rec, emit, A, acc_next);
      } else {
        if (emit) {
          if (sparse)
            first = P::add_ret(acc_next, vcell, delta);
          else
            P::add(acc_next, vcell, delta);
        }
        if (sparse)  // wave-uniform: stage first-touched cells, flush in chunks
          stage_push(stage, staged, (static_cast<uint64_t>(v) << 32) | c, first, A.fout, A.cnt_out);
      }
    }
    __syncthreads();
  }
  if (sparse) stage_flush(stage, staged, A.fout, A.cnt_out);
  if (binned) {
    stage_flush_records(stage, staged, A, acc_next);
    __syncthreads();
    for (int i = threadIdx.x; i < kBuckets; i += blockDim.x)
      if (s_hist[i]) atomicAdd(A.bucket_count + i, s_hist[i]);
  }
  if (kServe) {  // flush the block's per-column sums
    __syncthreads();
    for (int i = threadIdx.x; i < kServeLdsSlots * kNumCounters; i += blockDim.x) {
      const unsigned long long v = (&s_scnt[0][0])[i];
      if (v) atomicAdd(A.counters + i, v);
    }
    for (int i = threadIdx.x; i < kServeLdsSlots; i += blockDim.x)
      if (s_smass[i] != 0.0) atomicAdd(A.mass + i, s_smass[i]);
  }
  if (!kServe) {  // per-level counters: one atomic per wave
    unsigned long long* cnt = A.counters + static_cast<size_t>(A.level) * kNumCounters;
    const unsigned long long v0 = wave_sum_u64(n_front);
    const unsigned long long v1 = wave_sum_u64(n_hash);
    const unsigned long long v2 = wave_sum_u64(n_det);
    const unsigned long long v3 = wave_sum_u64(n_cand);
    const unsigned long long v4 = wave_sum_u64(n_acc);
    double m = mass;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) m += __shfl_down(m, off);
    if (lane == 0) {
      if (v0) atomicAdd(cnt + 0, v0);
      if (v1) atomicAdd(cnt + 1, v1);
      if (v2) atomicAdd(cnt + 2, v2);
      if (v3) atomicAdd(cnt + 3, v3);
      if (v4) atomicAdd(cnt + 4, v4);
      if (m != 0.0) atomicAdd(A.mass + A.level, m);
    }
  }
}

// ------------------------------------------------- frontier compaction
// (u << 32 | c) of every cell whose predicate holds, staged per wave in LDS
// and appended with one atomic per chunk.  Cells are u * su + c * sc:
// row-major (su = C, sc = 1) or one n-vector per column (su = 1, sc = n).
template <typename Pred>
__global__ __launch_bounds__(kThreads) void k_compact(Pred pred, int64_t n, int C, long long su, long long sc,
                                                      uint64_t* __restrict__ F,
                                                      unsigned long long* __restrict__ cnt,
                                                      const int* __restrict__ mode) {
  if (mode && *mode != kModeCompact && *mode != kModeOverflow) return;  // formed elsewhere
  __shared__ uint64_t s_stage[kThreads / kWave][kStage];
  const int lane = lane_id();
  uint64_t* stage = s_stage[threadIdx.x / kWave];
  int staged = 0;
  if (su == C && sc == 1 && C >= kWave) {  // row-major, wide rows: a wave per row
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t u = wave; u < n; u += nwaves) {
      for (int c0 = 0; c0 < C; c0 += kWave) {
        const int c = c0 + lane;
        const bool p = (c < C) && pred(static_cast<size_t>(u) * C + c);
        stage_push(stage, staged, (static_cast<uint64_t>(u) << 32) | static_cast<uint32_t>(c), p, F, cnt);
      }
    }
  } else {
    const int64_t total = n * C;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // every lane of a wave runs the same number of iterations
    const int64_t first = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t iters = (total + stride - 1) / stride;
    const bool rowmajor = (sc == 1);
    for (int64_t it = 0; it < iters; ++it) {
      const int64_t i = first + it * stride;
      bool p = false;
      uint64_t item = 0;
      if (i < total) {
        int64_t u, c;
        if (rowmajor) {
          u = i / C;
          c = i - u * C;
        } else {
          c = i / n;
          u = i - c * n;
        }
        p = pred(static_cast<size_t>(i));
        item = (static_cast<uint64_t>(u) << 32) | static_cast<uint32_t>(c);
      }
      stage_push(stage, staged, item, p, F, cnt);
    }
  }
  stage_flush(stage, staged, F, cnt);
}

template <typename T>
struct NonZeroValue {
  const T* x;
  __device__ bool operator()(size_t i) const { return x[i] != T(0); }
};

template <typename T>
struct NonZeroCell {
  const typename Prec<T>::Cell* acc;
  __device__ bool operator()(size_t i) const { return Prec<T>::nonzero(acc, i); }
};

inline unsigned grid_for(int64_t items, int threads, int64_t cap = 65536) {
  int64_t b = (items + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return static_cast<unsigned>(b);
}

}  // namespace lvl
}  // namespace agp
