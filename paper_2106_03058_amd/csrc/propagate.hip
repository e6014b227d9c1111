// Randomized level-by-level residue push (Algorithm 2 of "Approximate Graph
// Propagation", Section 4) for C signal columns at once on gfx950.
//
// State of a call (row-major n x C, cell = u * C + c):
//   x        the signal, which is also the level-0 residue r^(0)
//   out      the estimate pi_hat, accumulated level by level
//   acc[2]   next-level residues as exact integers of a per-column unit
//            (binary32: int64 cells; binary64: 128-bit cells), ping-ponged
//   F[2]     frontier lists of (u << 32 | c) with non-zero residue
//
// One kernel launch per level.  A block takes tiles of up to 256 frontier
// entries; per entry it converts the residue, updates the reserve
// (pi(u) += kappa_i r(u)), finds the deterministic prefix J of the
// degree-sorted row by binary search (increment >= theta) and counts the
// 64-position windows of the sampled suffix.  A block-wide scan of these work
// counts then spreads single pushes and windows evenly over the 256 threads,
// so a hub's row is shared by the whole block.  Windows run Philox-driven
// geometric-skip chains per degree-group run (the paper's subset sampling).
// Contributions are added with integer atomics, so the result does not
// depend on their order.  For non-negative signals the first atomic that
// finds a zero cell appends it to the next frontier (wave-aggregated); for
// signed signals the next frontier is compacted from the accumulators by a
// wave-ballot pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "agp_device.h"
#include "agp_internal.h"

namespace agp {
namespace {

constexpr int kThreads = 256;
constexpr int kTile = 256;  // frontier entries per block tile
constexpr int kLevelBlocks = 2048;
constexpr int kNumCounters = 5;  // frontier, hash, det, cand, acc
constexpr int kThetaRows = 4096; // rows per partial sum of ||x||_1

struct ColParams {
  double theta;       // eps * ||x_c||_1
  double scale;       // 2^-ue (binary32 path)
  long long dtheta;   // fl(theta) in units (binary32) / low word (binary64)
  int ue;             // exponent of the unit
  uint32_t qid;       // query id of the column's random streams
};

struct LevelArgs {
  const int64_t* rp;
  const uint32_t* col;
  const uint32_t* nd;
  const int32_t* deg;
  const double* da;
  const double* db;
  const ColParams* cp;
  int C;
  int a_zero;
  uint32_t key0, key1;
  int level;
  double rho;
  double kappa;
  const uint64_t* fin;
  const unsigned long long* cnt_in;
  uint64_t* fout;
  unsigned long long* cnt_out;
  unsigned long long* counters;
  int* err;
  int positive;                   // non-negative signal: sparse levels allowed
  unsigned long long dense_cut;   // frontier size from which a level is dense
  int* mode;                      // mode[i] = 1: level i's frontier is compacted
  double* mass;                   // per level: sum of |contribution| in units
};

// ----------------------------------------------------- working precision
// Binary32: int64 cells.  Binary64: 128-bit cells (lo, hi) stored adjacently.
// `mass` collects the magnitude of every contribution in units: while a
// level's total stays below the cell range no partial sum can wrap.
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
  static __device__ __forceinline__ float take(Cell* acc, size_t cell, const ColParams& p) {
    const long long K = acc[cell];
    acc[cell] = 0;
    return units_to_f32(K, p.ue);
  }
  static __device__ __forceinline__ bool to_units(float v, const ColParams& p, Delta* d, double* mass) {
    if (!f32_to_units(v, p.scale, d)) return false;
    *mass += fabs(static_cast<double>(*d));
    return true;
  }
  static __device__ __forceinline__ Delta theta_units(const ColParams& p, bool neg, double* mass) {
    *mass += static_cast<double>(p.dtheta);
    return neg ? -p.dtheta : p.dtheta;
  }
  // returns true if the cell held zero before (first contribution)
  static __device__ __forceinline__ bool add_ret(Cell* acc, size_t cell, Delta d) {
    return atomic_add_ret(reinterpret_cast<unsigned long long*>(acc + cell),
                          static_cast<unsigned long long>(d)) == 0ull;
  }
  static __device__ __forceinline__ void add(Cell* acc, size_t cell, Delta d) {
    atomic_add_relaxed(reinterpret_cast<unsigned long long*>(acc + cell), static_cast<unsigned long long>(d));
  }
  static __device__ __forceinline__ bool nonzero(const Cell* acc, size_t cell) { return acc[cell] != 0; }
};

template <>
struct Prec<double> {
  using Cell = unsigned long long;  // two words per cell
  using Delta = U128;
  static __device__ __forceinline__ double take(Cell* acc, size_t cell, const ColParams& p) {
    U128 K{acc[2 * cell], static_cast<long long>(acc[2 * cell + 1])};
    acc[2 * cell] = 0;
    acc[2 * cell + 1] = 0;
    return units_to_f64(K, p.ue);
  }
  static __device__ __forceinline__ bool to_units(double v, const ColParams& p, Delta* d, double* mass) {
    if (!f64_to_units(v, p.ue, d)) return false;
    *mass += ldexp(fabs(v), -p.ue);
    return true;
  }
  static __device__ __forceinline__ Delta theta_units(const ColParams& p, bool neg, double* mass) {
    *mass += static_cast<double>(p.dtheta);
    const long long d = neg ? -p.dtheta : p.dtheta;
    return U128{static_cast<unsigned long long>(d), d < 0 ? -1ll : 0ll};
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
};

__device__ __forceinline__ float to_w(double v, float) { return static_cast<float>(v); }
__device__ __forceinline__ double to_w(double v, double) { return v; }

// ------------------------------------------------------------ the level
template <typename T, bool kFirst, bool kLast>
__global__ __launch_bounds__(kThreads) void k_level(LevelArgs A, const T* __restrict__ x,
                                                    typename Prec<T>::Cell* __restrict__ acc_cur,
                                                    typename Prec<T>::Cell* __restrict__ acc_next,
                                                    T* __restrict__ out) {
  using P = Prec<T>;
  using Delta = typename P::Delta;
  __shared__ long long s_off[kTile + 1];
  __shared__ int64_t s_rp[kTile];
  __shared__ double s_cv[kTile];
  __shared__ uint32_t s_u[kTile];
  __shared__ uint32_t s_c[kTile];
  __shared__ uint32_t s_d[kTile];
  __shared__ uint32_t s_J[kTile];
  __shared__ uint32_t s_neg[kTile];
  __shared__ long long s_wave[kThreads / kWave];
  __shared__ uint64_t s_stage[kThreads / kWave][kStage];

  const unsigned long long count = *A.cnt_in;
  // Sparse levels detect the first contribution to a cell from the atomic's
  // old value and append the cell to the next frontier; dense levels use
  // fire-and-forget atomics and a compaction pass builds the next frontier.
  const bool sparse = !kLast && A.positive && count < A.dense_cut;
  if (!kLast && blockIdx.x == 0 && threadIdx.x == 0) A.mode[A.level + 1] = sparse ? 0 : 1;
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
      const size_t cell = static_cast<size_t>(u) * static_cast<size_t>(A.C) + c;
      const ColParams& cp = A.cp[c];
      T r;
      if (kFirst)
        r = x[cell];
      else
        r = P::take(acc_cur, cell, cp);
      ++n_front;
      n_hash += splitmix64(u);
      // reserve: pi(u) += (S w_i / Y_i) r(u), rounded to the working precision
      if (A.kappa != 0.0) {
        const T q = to_w(A.kappa * static_cast<double>(r), T());
        out[cell] = out[cell] + q;
      }
      uint32_t d = 0, J = 0;
      double cv = 0.0;
      if (!kLast && A.rho != 0.0) {
        d = static_cast<uint32_t>(A.deg[u]);
        if (d > 0) {
          const double absr = fabs(static_cast<double>(r));
          const double t0 = A.rho * absr;
          cv = t0 * A.db[d];
          const double th = cp.theta;
          const int64_t rpu = A.rp[u];
          if (A.a_zero) {
            J = (cv >= th) ? d : 0u;
          } else {  // increments fall along the degree-sorted row: binary search
            uint32_t lo = 0, hi = d;
            while (lo < hi) {
              const uint32_t mid = (lo + hi) >> 1;
              const double inc = cv * A.da[A.nd[rpu + mid]];
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
          n_det += J;
          s_rp[tid] = rpu;
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
    bool need_run = false;
    uint32_t u = 0, c = 0, s = 0, wend = 0, run_end = 0, pos = 0, t = 0, ctr3 = 0;
    int64_t rpu = 0;
    double cv = 0.0, dstart = 1.0, th = 0.0;
    bool neg = false;
    long long local = 0;
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
        if (local < static_cast<long long>(J)) {
          ttype = 1;
        } else {
          ttype = 2;
          const uint32_t d = s_d[e];
          const uint32_t wstart = ((J >> kSegLog2) + static_cast<uint32_t>(local - J)) << kSegLog2;
          s = wstart > J ? wstart : J;
          wend = (wstart + static_cast<uint32_t>(kSeg)) < d ? wstart + static_cast<uint32_t>(kSeg) : d;
          need_run = true;
          const ColParams& cp = A.cp[c];
          th = cp.theta;
          ctr3 = (cp.qid << 8) | static_cast<uint32_t>(A.level);
        }
      }
      if (!__any(ttype != 0)) break;

      bool emit = false;
      size_t vcell = 0;
      Delta delta{};
      uint32_t v = 0;
      if (ttype == 1) {
        // deterministic push: the increment reaches theta
        const int64_t arc = rpu + local;
        v = A.col[arc];
        double inc = cv;
        if (!A.a_zero) inc = cv * A.da[A.nd[arc]];
        T val = to_w(inc, T());
        if (neg) val = -val;
        emit = true;
        if (!P::to_units(val, A.cp[c], &delta, &mass)) {
          atomicOr(A.err, 1);
          emit = false;
        }
        ttype = 0;
      } else if (ttype == 2) {
        if (need_run) {
          if (s >= wend) {
            ttype = 0;
          } else {  // a run: same degree group (a > 0) inside the window
            run_end = wend;
            dstart = 1.0;
            if (!A.a_zero) {
              const uint32_t ds = A.nd[rpu + s];
              dstart = A.da[ds];
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
            const double num = cv * dstart;
            const double pstar = num / th;
            tab = make_skip_table(pstar);
            pos = s;
            t = 0;
            need_run = false;
          }
        }
        if (ttype == 2 && !need_run) {
          const U4 o = philox4x32_10(t, s, u, ctr3, A.key0, A.key1);
          const double V = unit_double(o.x, o.y);
          const double V2 = unit_double(o.z, o.w);
          const uint32_t cand = pos + static_cast<uint32_t>(geometric_skip(tab, V));
          if (cand >= run_end) {
            s = run_end;
            need_run = true;
          } else {
            ++n_cand;
            const int64_t arc = rpu + cand;
            double ratio = 1.0;
            if (!A.a_zero) ratio = A.da[A.nd[arc]] / dstart;
            if (V2 < ratio) {
              ++n_acc;
              v = A.col[arc];
              emit = true;
              delta = P::theta_units(A.cp[c], neg, &mass);
            }
            pos = cand + 1;
            ++t;
          }
        }
      }
      bool first = false;
      if (emit) {
        vcell = static_cast<size_t>(v) * static_cast<size_t>(A.C) + c;
        if (sparse)
          first = P::add_ret(acc_next, vcell, delta);
        else
          P::add(acc_next, vcell, delta);
      }
      if (sparse)  // wave-uniform: stage first-touched cells, flush in chunks
        stage_push(stage, staged, (static_cast<uint64_t>(v) << 32) | c, first, A.fout, A.cnt_out);
    }
    __syncthreads();
  }
  if (sparse) stage_flush(stage, staged, A.fout, A.cnt_out);
  // per-level counters: one atomic per wave
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

// ------------------------------------------------- frontier compaction
// (u << 32 | c) of every cell whose predicate holds, appended with one
// atomic per wave.  Wide rows: a wave per row; narrow rows: flat cells.
template <typename Pred>
__global__ __launch_bounds__(kThreads) void k_compact(Pred pred, int64_t n, int C,
                                                      uint64_t* __restrict__ F,
                                                      unsigned long long* __restrict__ cnt,
                                                      const int* __restrict__ mode) {
  if (mode && *mode == 0) return;  // this level's frontier was appended directly
  __shared__ uint64_t s_stage[kThreads / kWave][kStage];
  const int lane = lane_id();
  uint64_t* stage = s_stage[threadIdx.x / kWave];
  int staged = 0;
  if (C >= kWave) {
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
    for (int64_t it = 0; it < iters; ++it) {
      const int64_t i = first + it * stride;
      bool p = false;
      uint64_t item = 0;
      if (i < total) {
        const int64_t u = i / C;
        const int c = static_cast<int>(i - u * C);
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

// ---------------------------------------------------------- thresholds
// ||x_c||_1 in binary64: sequential over blocks of 4096 rows, then over the
// block sums.  flags: 1 = non-finite entry, 2 = negative entry.
template <typename T>
__global__ void k_theta_partial(const T* __restrict__ x, int64_t n, int C, double* __restrict__ partial,
                                int* __restrict__ flags) {
  const int c = blockIdx.y * blockDim.x + threadIdx.x;
  if (c >= C) return;
  const int64_t lo = (int64_t)blockIdx.x * kThetaRows;
  const int64_t hi = (lo + kThetaRows) < n ? lo + kThetaRows : n;
  double sum = 0.0;
  int f = 0;
  for (int64_t i = lo; i < hi; ++i) {
    const T v = x[static_cast<size_t>(i) * C + c];
    if (!isfinite(static_cast<double>(v))) f |= 1;
    if (v < T(0)) f |= 2;
    sum = sum + fabs(static_cast<double>(v));
  }
  partial[(size_t)blockIdx.x * C + c] = sum;
  if (f) atomicOr(flags, f);
}

template <typename T>
__global__ void k_theta_final(const double* __restrict__ partial, int64_t nblocks, int C, double eps,
                              const uint32_t* __restrict__ qids, ColParams* __restrict__ cp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  double total = 0.0;
  for (int64_t b = 0; b < nblocks; ++b) total = total + partial[(size_t)b * C + c];
  ColParams p;
  p.theta = eps * total;
  p.qid = qids ? qids[c] : static_cast<uint32_t>(c);
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
  }
  cp[c] = p;
}

unsigned grid_for(int64_t items, int threads, int64_t cap = 65536) {
  int64_t b = (items + threads - 1) / threads;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

// ------------------------------------------------------------ driver
template <typename T>
int propagate_impl(agp_graph* g, double a, double b, const double* w, int32_t L, const T* x,
                   int32_t C, double eps, uint64_t seed, const uint32_t* qids, T* out,
                   hipStream_t s, agp_stats_t* stats) {
  using Cell = typename Prec<T>::Cell;
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
  if (qids)
    for (int32_t c = 0; c < C; ++c)
      if (qids[c] >= (1u << 24)) return fail(AGP_EINVAL, std::string(fn) + ": qid must be < 2^24");
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
      (rc = sc.levelinfo.reserve((sizeof(double) + sizeof(int)) * (AGP_MAX_LEVELS + 2), false, s)))
    return rc;

  ColParams* cp = sc.colparams.as<ColParams>();
  uint32_t* dq = reinterpret_cast<uint32_t*>(cp + C);
  unsigned long long* counts = sc.counts.as<unsigned long long>();
  unsigned long long* counters = sc.counters.as<unsigned long long>();
  int* flags = sc.flags.as<int>();
  double* mass = sc.levelinfo.as<double>();
  int* mode = reinterpret_cast<int*>(mass + AGP_MAX_LEVELS + 2);
  AGP_HIP(hipMemsetAsync(sc.levelinfo.ptr, 0, sc.levelinfo.bytes, s));
  AGP_HIP(hipMemsetAsync(counts, 0, sc.counts.bytes, s));
  AGP_HIP(hipMemsetAsync(counters, 0, sc.counters.bytes, s));
  AGP_HIP(hipMemsetAsync(flags, 0, sc.flags.bytes, s));
  if (qids) AGP_HIP(hipMemcpyAsync(dq, qids, sizeof(uint32_t) * C, hipMemcpyHostToDevice, s));

  // thresholds theta_c = eps ||x_c||_1 and signal checks
  if (tblocks > 0) {
    dim3 grid((unsigned)tblocks, (unsigned)((C + 63) / 64));
    k_theta_partial<T><<<grid, 64, 0, s>>>(x, n, C, sc.partial.as<double>(), flags + 1);
  }
  k_theta_final<T><<<grid_for(C, 64), 64, 0, s>>>(sc.partial.as<double>(), tblocks, C, eps,
                                                  qids ? dq : nullptr, cp);
  AGP_HIP(hipGetLastError());
  int hflags[4] = {0, 0, 0, 0};
  AGP_HIP(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
  AGP_HIP(hipStreamSynchronize(s));
  if (hflags[1] & 1) return fail(AGP_EINVAL, std::string(fn) + ": x holds a non-finite value");
  const bool positive = sizeof(T) == 4 && !(hflags[1] & 2);

  AGP_HIP(hipMemsetAsync(out, 0, cells * sizeof(T), s));
  hipEvent_t* ev = sc.events;
  if (stats && (rc = sc.ensure_events())) return rc;
  uint64_t* F[2] = {sc.frontier[0].as<uint64_t>(), sc.frontier[1].as<uint64_t>()};
  Cell* acc[2] = {sc.acc[0].as<Cell>(), sc.acc[1].as<Cell>()};
  const unsigned cgrid = grid_for(n * (int64_t)(C >= kWave ? kWave : C), kThreads, 8192);
  k_compact<<<cgrid, kThreads, 0, s>>>(NonZeroValue<T>{x}, n, C, F[0], counts, nullptr);

  LevelArgs A;
  A.rp = g->row_ptr;
  A.col = g->col;
  A.nd = g->ndeg;
  A.deg = g->degree;
  A.da = da;
  A.db = db;
  A.cp = cp;
  A.C = C;
  A.a_zero = (a == 0.0) ? 1 : 0;
  A.key0 = static_cast<uint32_t>(seed);
  A.key1 = static_cast<uint32_t>(seed >> 32);
  A.counters = counters;
  A.err = flags;
  A.positive = positive ? 1 : 0;
  A.dense_cut = std::max<unsigned long long>(1ull, static_cast<unsigned long long>(cells / 32));
  A.mode = mode;
  A.mass = mass;
  for (int32_t i = 0; i <= L; ++i) {
    A.level = i;
    A.rho = rho[i];
    A.kappa = kappa[i];
    A.fin = F[i & 1];
    A.cnt_in = counts + i;
    A.fout = F[(i + 1) & 1];
    A.cnt_out = counts + i + 1;
    Cell* cur = acc[i & 1];
    Cell* nxt = acc[(i + 1) & 1];
    const bool first = i == 0, last = i == L;
    if (stats) AGP_HIP(hipEventRecord(ev[2 * i], s));
    if (first && last)
      k_level<T, true, true><<<kLevelBlocks, kThreads, 0, s>>>(A, x, cur, nxt, out);
    else if (first)
      k_level<T, true, false><<<kLevelBlocks, kThreads, 0, s>>>(A, x, cur, nxt, out);
    else if (last)
      k_level<T, false, true><<<kLevelBlocks, kThreads, 0, s>>>(A, x, cur, nxt, out);
    else
      k_level<T, false, false><<<kLevelBlocks, kThreads, 0, s>>>(A, x, cur, nxt, out);
    if (stats) AGP_HIP(hipEventRecord(ev[2 * i + 1], s));
    if (!last)
      k_compact<<<cgrid, kThreads, 0, s>>>(NonZeroCell<T>{nxt}, n, C, F[(i + 1) & 1], counts + i + 1,
                                           mode + i + 1);
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
    std::memset(stats, 0, sizeof(*stats));
    stats->levels = L;
    stats->columns = C;
    for (int32_t i = 0; i <= L; ++i) {
      stats->frontier[i] = h[i * kNumCounters + 0];
      stats->hash[i] = h[i * kNumCounters + 1];
      stats->det[i] = h[i * kNumCounters + 2];
      stats->cand[i] = h[i * kNumCounters + 3];
      stats->acc[i] = h[i * kNumCounters + 4];
    }
    float ms = 0.0f;
    for (int32_t i = 0; i <= L; ++i) {
      AGP_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
      stats->level_ms[i] = ms;
    }
    AGP_HIP(hipEventElapsedTime(&ms, ev[0], ev[2 * L + 1]));
    stats->device_ms = ms;
  }
  return AGP_OK;
}

}  // namespace
}  // namespace agp

extern "C" {

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
