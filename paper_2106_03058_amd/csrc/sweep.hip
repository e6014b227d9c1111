// Local clustering sweep (Section 5, the quality of local clusters): the
// nodes sorted by pi(v) / d_v descending (ties by id, nodes without
// neighbours last), then the prefix S_i = {v_1..v_i}, 1 <= i <= n - 1, of
// minimum conductance Phi(S) = |cut(S)| / min(vol(S), 2m - vol(S)).
//
// On the device: 64-bit order keys and a radix sort (rocPRIM) give the
// order; every node's rank, then per node the number of its neighbours
// ranked before it gives the change of the cut when it joins
// (d_v - loops - 2 * earlier neighbours); two integer prefix sums give
// cut(S_i) and vol(S_i) exactly, and a min-reduction over (Phi_i, i) the
// first prefix of minimum conductance.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/counting_iterator.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <vector>

#include "agp_internal.h"

namespace agp {
namespace {

constexpr int kSweepThreads = 256;
constexpr int kSweepBlocks = 1024;
constexpr int kDeltaUnroll = 8;  // arcs per lane per pass of the delta kernel
constexpr long long kItemArcs = 4096;  // arcs per work item of the delta kernel

// Descending order of pi(v)/d_v as an ascending unsigned key; isolated nodes
// get the largest key.  The double is mapped to an order-preserving integer
// (sign bit flipped for >= 0, all bits flipped for < 0) and inverted.
__device__ __forceinline__ uint64_t sweep_key(float p, int d) {
  if (d <= 0) return ~0ull;
  double r = static_cast<double>(p) / static_cast<double>(d);
  if (r == 0.0) r = 0.0;  // one zero
  const uint64_t b = static_cast<uint64_t>(__double_as_longlong(r));
  const uint64_t mono = (b >> 63) ? ~b : (b | 0x8000000000000000ull);
  const uint64_t key = ~mono;
  return key == ~0ull ? ~0ull - 1 : key;  // stays before the isolated nodes
}

__global__ void k_sweep_keys(const float* __restrict__ pi, int64_t ld, const int32_t* __restrict__ deg, int64_t n,
                             uint64_t* __restrict__ keys, int32_t* __restrict__ ids) {
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    keys[v] = sweep_key(pi[v * ld], deg[v]);
    ids[v] = static_cast<int32_t>(v);
  }
}

// rank[v] = position of v in the order; coarse[v] = rank >> shift, a byte
// per node (n >> shift < 256) so that most comparisons of the delta kernel
// read an array small enough to stay in the L2 cache.  Position i starts
// with vol term d_v and cut change d_v (the delta kernel subtracts loops and
// twice the earlier neighbours).
__global__ void k_sweep_rank(const int32_t* __restrict__ order, const int32_t* __restrict__ deg, int64_t n, int shift,
                             int32_t* __restrict__ rank, uint8_t* __restrict__ coarse, long long* __restrict__ dvol,
                             long long* __restrict__ dcut) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = order[i];
    rank[v] = static_cast<int32_t>(i);
    coarse[v] = static_cast<uint8_t>(i >> shift);
    const long long d = deg[v];
    dvol[i] = d;
    dcut[i] = d;
  }
}

// Work items of the delta kernel: the nodes in chunks of 64 consecutive ids
// (their rows form one run of arcs), each chunk's run cut into pieces of at
// most kItemArcs arcs, so that the hubs' chunks are shared by many waves.
// first[c] = index of chunk c's first item (exclusive scan of the counts).
__global__ void k_items_count(const int64_t* __restrict__ rp, int64_t n, int64_t nchunks,
                              long long* __restrict__ count) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c <= nchunks; c += (int64_t)gridDim.x * blockDim.x) {
    long long k = 0;
    if (c < nchunks) {
      const int64_t v0 = c * 64, v1 = v0 + 64 < n ? v0 + 64 : n;
      k = (rp[v1] - rp[v0] + kItemArcs - 1) / kItemArcs;
    }
    count[c] = k;
  }
}

__global__ void k_items_fill(const long long* __restrict__ first, int64_t nchunks, int32_t* __restrict__ items) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nchunks; c += (int64_t)gridDim.x * blockDim.x)
    for (long long t = first[c]; t < first[c + 1]; ++t) items[t] = static_cast<int32_t>(c);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per node v at sorted position i = rank[v]: subtracts loops + 2 * |{u in
// N(v) : rank(u) < i}| from the cut change at position i.  A wave takes one
// work item, a piece of the arc run of 64 consecutive node ids, and walks it
// with all 64 lanes (arc k of the run belongs to the row whose offset range
// holds k): the column reads are coalesced, short rows leave no lane idle,
// and every lane keeps kDeltaUnroll loads in flight.  A neighbour's byte rank
// decides the comparison unless it equals the node's own, then the full rank
// does.  Each lane counts in registers while it stays in one row and adds to
// the row's LDS counter when it moves on; the item's per-row totals go to
// the cut changes with integer atomics (rows cut into several items get
// several, in any order, with the same sum).
__global__ __launch_bounds__(kSweepThreads) void k_sweep_delta(const int64_t* __restrict__ rp,
                                                               const uint32_t* __restrict__ col,
                                                               const int32_t* __restrict__ rank,
                                                               const uint8_t* __restrict__ coarse, int shift,
                                                               int64_t n, const int32_t* __restrict__ items,
                                                               const long long* __restrict__ first, int64_t nitems,
                                                               long long* __restrict__ dcut) {
  constexpr int kW = kSweepThreads / 64;
  __shared__ long long s_off[kW][65];
  __shared__ int32_t s_rank[kW][64];
  __shared__ unsigned int s_earlier[kW][64];
  __shared__ unsigned int s_loops[kW][64];
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  for (int64_t t = blockIdx.x * (int64_t)kW + w; t < nitems; t += (int64_t)gridDim.x * kW) {
    const int64_t c = items[t];
    const long long kb = (t - first[c]) * kItemArcs;
    const int64_t v0 = c * 64;
    const int64_t v = v0 + lane;
    const int64_t vend = v0 + 64 < n ? v0 + 64 : n;
    const long long base_arc = rp[v0];
    const long long total = rp[vend] - base_arc;
    const long long ke = kb + kItemArcs < total ? kb + kItemArcs : total;
    long long off = total;
    int32_t r = 0;
    if (v < n) {
      off = rp[v] - base_arc;
      r = rank[v];
    }
    s_off[w][lane] = off;
    if (lane == 0) s_off[w][64] = total;
    s_rank[w][lane] = r;
    s_earlier[w][lane] = 0;
    s_loops[w][lane] = 0;
    wave_sync();
    int cur = 0;
    unsigned int earlier = 0, loops = 0;
    for (long long base = kb; base < ke; base += 64 * kDeltaUnroll) {
      uint32_t u[kDeltaUnroll];
      int own[kDeltaUnroll];
      int from = cur;
#pragma unroll
      for (int j = 0; j < kDeltaUnroll; ++j) {
        // past the end: the item's last arc is read again and ignored, so
        // that no load sits under a branch and all of them are in flight
        const long long kk = base + lane + 64ll * j;
        const long long k = kk < ke ? kk : ke - 1;
        // s_off[lo] <= k < s_off[hi]; the row of k is the last lo with s_off[lo] <= k
        int lo = from, hi = 64;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_off[w][mid] <= k)
            lo = mid;
          else
            hi = mid;
        }
        own[j] = kk < ke ? lo : -1;
        from = lo;
        u[j] = __builtin_nontemporal_load(&col[base_arc + k]);
      }
      unsigned int cu[kDeltaUnroll];
#pragma unroll
      for (int j = 0; j < kDeltaUnroll; ++j) cu[j] = coarse[u[j]];
#pragma unroll
      for (int j = 0; j < kDeltaUnroll; ++j) {
        const int o = own[j];
        if (o < 0) break;
        if (o != cur) {
          if (earlier) atomicAdd(&s_earlier[w][cur], earlier);
          if (loops) atomicAdd(&s_loops[w][cur], loops);
          earlier = loops = 0;
          cur = o;
        }
        const int32_t iv = s_rank[w][o];
        const unsigned int cv = static_cast<unsigned int>(iv >> shift);
        if (u[j] == static_cast<uint32_t>(v0 + o))
          ++loops;
        else if (cu[j] < cv || (cu[j] == cv && rank[u[j]] < iv))
          ++earlier;
      }
    }
    if (earlier) atomicAdd(&s_earlier[w][cur], earlier);
    if (loops) atomicAdd(&s_loops[w][cur], loops);
    wave_sync();
    if (v < n) {
      const long long sub = static_cast<long long>(s_loops[w][lane]) + 2 * static_cast<long long>(s_earlier[w][lane]);
      if (sub)
        atomicAdd(reinterpret_cast<unsigned long long*>(&dcut[r]), static_cast<unsigned long long>(-sub));
    }
    wave_sync();  // the next item rewrites the LDS rows
  }
}

struct PhiIdx {
  double phi;
  long long idx;
};

__device__ __forceinline__ PhiIdx better(PhiIdx a, PhiIdx b) {
  if (b.phi < a.phi || (b.phi == a.phi && b.idx < a.idx)) return b;
  return a;
}

// Phi of the prefixes of sizes 1..n-1 from the inclusive sums; per block the
// first minimum.
__global__ __launch_bounds__(kSweepThreads) void k_sweep_phi(const long long* __restrict__ vol,
                                                             const long long* __restrict__ cut, int64_t n,
                                                             long long two_m, PhiIdx* __restrict__ part) {
  __shared__ PhiIdx s[kSweepThreads / 64];
  PhiIdx best{INFINITY, 0x7FFFFFFFFFFFFFFFll};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i + 1 < n; i += (int64_t)gridDim.x * blockDim.x) {
    const long long vv = vol[i];
    const long long denom = vv < two_m - vv ? vv : two_m - vv;
    if (denom > 0) {
      const PhiIdx c{static_cast<double>(cut[i]) / static_cast<double>(denom), static_cast<long long>(i)};
      best = better(best, c);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    PhiIdx o{__shfl_down(best.phi, off), __shfl_down(best.idx, off)};
    best = better(best, o);
  }
  if (threadIdx.x % 64 == 0) s[threadIdx.x / 64] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kSweepThreads / 64; ++w) best = better(best, s[w]);
    part[blockIdx.x] = best;
  }
}

__global__ __launch_bounds__(kSweepThreads) void k_sweep_final(const PhiIdx* __restrict__ part, int nparts,
                                                               PhiIdx* __restrict__ out) {
  __shared__ PhiIdx s[kSweepThreads / 64];
  PhiIdx best{INFINITY, 0x7FFFFFFFFFFFFFFFll};
  for (int b = threadIdx.x; b < nparts; b += kSweepThreads) best = better(best, part[b]);
  for (int off = 32; off > 0; off >>= 1) {
    PhiIdx o{__shfl_down(best.phi, off), __shfl_down(best.idx, off)};
    best = better(best, o);
  }
  if (threadIdx.x % 64 == 0) s[threadIdx.x / 64] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kSweepThreads / 64; ++w) best = better(best, s[w]);
    *out = best;
  }
}

}  // namespace
}  // namespace agp

namespace agp {
namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// The graph's work items of the delta kernels (built once per graph; the
// caller holds g->mu).
int ensure_items(agp_graph* gg, hipStream_t s) {
  if (gg->scratch.sweep_nitems >= 0) return AGP_OK;
  const int64_t n = gg->n;
  const int64_t nchunks = (n + 63) / 64;
  const int64_t max_items = nchunks + gg->nnz / kItemArcs + 1;
  const size_t first_bytes = align256(sizeof(long long) * (size_t)(nchunks + 1));
  if (int rc = gg->scratch.sweep_items.reserve(first_bytes + sizeof(int32_t) * (size_t)max_items, false, s))
    return rc;
  long long* first = gg->scratch.sweep_items.as<long long>();
  int32_t* items = reinterpret_cast<int32_t*>(gg->scratch.sweep_items.as<char>() + first_bytes);
  DevBuf count, temp;
  size_t eb = 0;
  int rc = count.reserve(sizeof(long long) * (size_t)(nchunks + 1), false, s);
  if (rc == AGP_OK) {
    const hipError_t e = rocprim::exclusive_scan(nullptr, eb, count.as<long long>(), first, 0ll,
                                                 (size_t)(nchunks + 1), rocprim::plus<long long>(), s);
    if (e != hipSuccess) rc = fail(AGP_EDEVICE, std::string("agp_sweep: ") + hipGetErrorString(e));
  }
  if (rc == AGP_OK) rc = temp.reserve(eb, false, s);
  long long nit = 0;
  if (rc == AGP_OK) {
    const unsigned cgrid = static_cast<unsigned>(std::min<int64_t>((nchunks + 256) / 256, 65536));
    k_items_count<<<cgrid, 256, 0, s>>>(gg->row_ptr, n, nchunks, count.as<long long>());
    hipError_t e = rocprim::exclusive_scan(temp.ptr, eb, count.as<long long>(), first, 0ll, (size_t)(nchunks + 1),
                                           rocprim::plus<long long>(), s);
    if (e == hipSuccess) {
      k_items_fill<<<cgrid, 256, 0, s>>>(first, nchunks, items);
      e = hipMemcpyAsync(&nit, first + nchunks, sizeof(long long), hipMemcpyDeviceToHost, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = fail(AGP_EDEVICE, std::string("agp_sweep: ") + hipGetErrorString(e));
  }
  count.release();
  temp.release();
  if (rc != AGP_OK) return rc;
  if (nit > max_items) return fail(AGP_EDEVICE, "agp_sweep: work item count");
  gg->scratch.sweep_nitems = nit;
  return AGP_OK;
}

void items_of(agp_graph* gg, const long long** first, const int32_t** items) {
  const int64_t nchunks = (gg->n + 63) / 64;
  const size_t first_bytes = align256(sizeof(long long) * (size_t)(nchunks + 1));
  *first = gg->scratch.sweep_items.as<long long>();
  *items = reinterpret_cast<const int32_t*>(gg->scratch.sweep_items.as<char>() + first_bytes);
}

}  // namespace
}  // namespace agp

extern "C" int agp_sweep(const agp_graph_t* g, const float* pi, int64_t ld, void* stream, int64_t* best_size,
                         double* best_conductance, int32_t* order) {
  using namespace agp;
  if (!g || !pi || !best_size || !best_conductance) return fail(AGP_EINVAL, "agp_sweep: NULL argument");
  if (ld < 1) return fail(AGP_EINVAL, "agp_sweep: ld must be >= 1");
  if (g->directed) return fail(AGP_EINVAL, "agp_sweep: conductance is defined on undirected graphs");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = g->n;
  *best_size = 0;
  *best_conductance = INFINITY;
  if (n < 2) {
    if (n == 1 && order) AGP_HIP(hipMemsetAsync(order, 0, sizeof(int32_t), s));
    if (n == 1) AGP_HIP(hipStreamSynchronize(s));
    return AGP_OK;
  }
  const size_t N = static_cast<size_t>(n);
  size_t sort_bytes = 0, scan_bytes = 0;
  AGP_HIP(rocprim::radix_sort_pairs(nullptr, sort_bytes, static_cast<uint64_t*>(nullptr),
                                    static_cast<uint64_t*>(nullptr), static_cast<int32_t*>(nullptr),
                                    static_cast<int32_t*>(nullptr), N, 0, 64, s));
  AGP_HIP(rocprim::inclusive_scan(nullptr, scan_bytes, static_cast<long long*>(nullptr),
                                  static_cast<long long*>(nullptr), N, rocprim::plus<long long>(), s));
  const size_t temp_bytes = align256(std::max(sort_bytes, scan_bytes));
  // layout: keys[2] (8N), ids[2] (4N), rank (4N), dvol, dcut, vol, cut (8N each), coarse (N),
  // block minima, sort/scan space
  const size_t b8 = align256(N * 8), b4 = align256(N * 4);
  const size_t part_bytes = align256(sizeof(PhiIdx) * (kSweepBlocks + 1));
  const size_t b1 = align256(N);
  const size_t total = 6 * b8 + 3 * b4 + b1 + part_bytes + temp_bytes;
  agp_graph* gg = const_cast<agp_graph*>(g);
  std::lock_guard<std::mutex> lk(gg->mu);
  DevBuf& buf = gg->scratch.sweep;
  if (int rc = buf.reserve(total, false, s)) return rc;
  char* p = buf.as<char>();
  uint64_t* keys_in = reinterpret_cast<uint64_t*>(p);
  uint64_t* keys_out = reinterpret_cast<uint64_t*>(p + b8);
  long long* dvol = reinterpret_cast<long long*>(p + 2 * b8);
  long long* dcut = reinterpret_cast<long long*>(p + 3 * b8);
  long long* vol = reinterpret_cast<long long*>(p + 4 * b8);
  long long* cut = reinterpret_cast<long long*>(p + 5 * b8);
  int32_t* ids_in = reinterpret_cast<int32_t*>(p + 6 * b8);
  int32_t* ids_out = reinterpret_cast<int32_t*>(p + 6 * b8 + b4);
  int32_t* rank = reinterpret_cast<int32_t*>(p + 6 * b8 + 2 * b4);
  uint8_t* coarse = reinterpret_cast<uint8_t*>(p + 6 * b8 + 3 * b4);
  PhiIdx* parts = reinterpret_cast<PhiIdx*>(p + 6 * b8 + 3 * b4 + b1);
  void* temp = p + 6 * b8 + 3 * b4 + b1 + part_bytes;
  int shift = 0;
  while ((n - 1) >> shift >= 256) ++shift;

  const unsigned grid = static_cast<unsigned>(std::min<int64_t>((n + 255) / 256, 65536));
  k_sweep_keys<<<grid, 256, 0, s>>>(pi, ld, g->degree, n, keys_in, ids_in);
  size_t tb = temp_bytes;
  AGP_HIP(rocprim::radix_sort_pairs(temp, tb, keys_in, keys_out, ids_in, ids_out, N, 0, 64, s));
  k_sweep_rank<<<grid, 256, 0, s>>>(ids_out, g->degree, n, shift, rank, coarse, dvol, dcut);
  if (int rc = ensure_items(gg, s)) return rc;
  {
    const long long* first = nullptr;
    const int32_t* items = nullptr;
    items_of(gg, &first, &items);
    const int64_t nitems = gg->scratch.sweep_nitems;
    const unsigned dgrid = static_cast<unsigned>(
        std::max<int64_t>(1, std::min<int64_t>((nitems + kSweepThreads / 64 - 1) / (kSweepThreads / 64), 65536)));
    k_sweep_delta<<<dgrid, kSweepThreads, 0, s>>>(g->row_ptr, g->col, rank, coarse, shift, n, items, first, nitems,
                                                 dcut);
  }
  tb = temp_bytes;
  AGP_HIP(rocprim::inclusive_scan(temp, tb, dvol, vol, N, rocprim::plus<long long>(), s));
  tb = temp_bytes;
  AGP_HIP(rocprim::inclusive_scan(temp, tb, dcut, cut, N, rocprim::plus<long long>(), s));
  k_sweep_phi<<<kSweepBlocks, kSweepThreads, 0, s>>>(vol, cut, n, static_cast<long long>(g->nnz), parts);
  k_sweep_final<<<1, kSweepThreads, 0, s>>>(parts, kSweepBlocks, parts + kSweepBlocks);
  AGP_HIP(hipGetLastError());
  PhiIdx h{};
  AGP_HIP(hipMemcpyAsync(&h, parts + kSweepBlocks, sizeof(PhiIdx), hipMemcpyDeviceToHost, s));
  if (order) AGP_HIP(hipMemcpyAsync(order, ids_out, N * 4, hipMemcpyDeviceToDevice, s));
  AGP_HIP(hipStreamSynchronize(s));
  if (std::isfinite(h.phi)) {
    *best_size = h.idx + 1;
    *best_conductance = h.phi;
  }
  return AGP_OK;
}

// ------------------------------------------------------------ batched sweep
// The sweeps of many columns at once.  Per group of up to 64 columns: the
// keys of all columns, a radix sort per column, the ranks, and one pass over
// the arcs in which a wave's lanes are the columns:
// an arc's neighbour costs one coalesced gather of its 64 byte ranks instead
// of 64 single-byte gathers.  The per-(node, column) cut terms are node-major;
// one scan over the group (read through the order of each column) gives every
// column's prefix sums, from which each column's first minimum of Phi is
// taken.
namespace agp {
namespace {

constexpr int kBatchCols = 64;    // columns per group (one per lane)
constexpr int kBatchUnroll = 8;   // arcs per lane with their gathers in flight
constexpr int kBatchPhiBlocks = 256;

__global__ void k_sweepb_keys(const float* __restrict__ pi, int64_t ld, int64_t c0, int G,
                              const int32_t* __restrict__ deg, int64_t n, uint64_t* __restrict__ keys,
                              int32_t* __restrict__ ids) {
  const int64_t total = n * G;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = t / G;
    const int64_t g = t - v * G;
    keys[g * n + v] = sweep_key(pi[v * ld + c0 + g], deg[v]);  // reads of a node's columns coalesce
    ids[g * n + v] = static_cast<int32_t>(v);
  }
}

// rank (column-major) and byte rank (node-major: a node's 64 columns are 64
// consecutive bytes) of every column
__global__ void k_sweepb_rank(const int32_t* __restrict__ ids, int64_t n, int G, int shift,
                              int32_t* __restrict__ rank, uint8_t* __restrict__ coarse) {
  const int64_t total = n * G;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = t / n;
    const int64_t i = t - g * n;
    const int32_t v = ids[t];
    rank[g * n + v] = static_cast<int32_t>(i);
    coarse[static_cast<int64_t>(v) * G + g] = static_cast<uint8_t>(i >> shift);
  }
}

// cut terms (node-major) start at d_v
__global__ void k_sweepb_init(const int32_t* __restrict__ deg, int64_t n, int G, long long* __restrict__ dcut) {
  const int64_t total = n * G;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x)
    dcut[t] = deg[t / G];
}

// One wave per work item (a piece of the arc run of 64 consecutive node ids),
// lane g = column g: for each arc (v, u) of the piece, in order, the column's
// count of earlier neighbours of v grows when u ranks before v; a row's total
// (plus its loops, shared by all columns) is subtracted from the cut term of
// (v, g) with one integer atomic per column when the row ends in the piece.
__global__ __launch_bounds__(kSweepThreads) void k_sweepb_delta(
    const int64_t* __restrict__ rp, const uint32_t* __restrict__ col, const int32_t* __restrict__ rank,
    const uint8_t* __restrict__ coarse, int shift, int64_t n, int G, const int32_t* __restrict__ items,
    const long long* __restrict__ first, int64_t nitems, long long* __restrict__ dcut) {
  constexpr int kW = kSweepThreads / 64;
  __shared__ long long s_off[kW][65];
  __shared__ uint8_t s_cv[kW][64 * kBatchCols];  // byte ranks of the chunk's 64 nodes
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  const bool col_lane = lane < G;
  for (int64_t t = blockIdx.x * (int64_t)kW + w; t < nitems; t += (int64_t)gridDim.x * kW) {
    const int64_t c = items[t];
    const long long kb = (t - first[c]) * kItemArcs;
    const int64_t v0 = c * 64;
    const int64_t vend = v0 + 64 < n ? v0 + 64 : n;
    const long long base_arc = rp[v0];
    const long long total = rp[vend] - base_arc;
    const long long ke = kb + kItemArcs < total ? kb + kItemArcs : total;
    s_off[w][lane] = v0 + lane < n ? rp[v0 + lane] - base_arc : total;
    if (lane == 0) s_off[w][64] = total;
    for (int r = 0; r < 64; ++r)
      s_cv[w][r * kBatchCols + lane] = (col_lane && v0 + r < n) ? coarse[(v0 + r) * G + lane] : 0;
    wave_sync();
    int cur = 0;  // wave-uniform: the row of the arc in hand
    while (s_off[w][cur + 1] <= kb) ++cur;
    unsigned int earlier = 0, loops = 0;
    int32_t rv = -1;  // the row's full rank in this column, read on the first tie
    auto flush = [&]() {
      const long long sub = static_cast<long long>(loops) + 2ll * static_cast<long long>(earlier);
      if (col_lane && sub)
        atomicAdd(reinterpret_cast<unsigned long long*>(&dcut[(v0 + cur) * G + lane]),
                  static_cast<unsigned long long>(-sub));
      earlier = loops = 0;
      rv = -1;
    };
    for (long long k0 = kb; k0 < ke; k0 += 64) {
      const int m = ke - k0 < 64 ? static_cast<int>(ke - k0) : 64;
      const uint32_t uvec = lane < m ? col[base_arc + k0 + lane] : 0u;
      for (int j0 = 0; j0 < m; j0 += kBatchUnroll) {
        uint32_t u[kBatchUnroll];
        unsigned int cu[kBatchUnroll];
#pragma unroll
        for (int jj = 0; jj < kBatchUnroll; ++jj) {
          u[jj] = __shfl(uvec, j0 + jj);  // arcs past m read u = 0 and are not used
          cu[jj] = col_lane ? coarse[static_cast<int64_t>(u[jj]) * G + lane] : 0u;
        }
#pragma unroll
        for (int jj = 0; jj < kBatchUnroll; ++jj) {
          if (j0 + jj >= m) break;
          const long long k = k0 + j0 + jj;
          while (k >= s_off[w][cur + 1]) {  // the row ends: its totals go out
            flush();
            ++cur;
          }
          const int64_t v = v0 + cur;
          if (u[jj] == static_cast<uint32_t>(v)) {
            ++loops;
          } else if (col_lane) {
            const unsigned int cv = s_cv[w][cur * kBatchCols + lane];
            if (cu[jj] < cv) {
              ++earlier;
            } else if (cu[jj] == cv) {
              if (rv < 0) rv = rank[static_cast<int64_t>(lane) * n + v];
              if (rank[static_cast<int64_t>(lane) * n + u[jj]] < rv) ++earlier;
            }
          }
        }
      }
    }
    flush();
    wave_sync();  // the next item rewrites the LDS rows
  }
}

struct VolCut {
  long long vol, cut;
};

struct VolCutPlus {
  __device__ __host__ VolCut operator()(const VolCut& a, const VolCut& b) const {
    return VolCut{a.vol + b.vol, a.cut + b.cut};
  }
};

// position t = g n + i of the group: (d_v, cut term of (v, g)), v = order_g[i]
struct VolCutAt {
  const int32_t* ids;
  const int32_t* deg;
  const long long* dcut;
  int64_t n;
  int G;
  __device__ VolCut operator()(size_t t) const {
    const int64_t g = static_cast<int64_t>(t) / n;
    const int32_t v = ids[t];
    return VolCut{deg[v], dcut[static_cast<int64_t>(v) * G + g]};
  }
};

// Phi of column g's prefixes from the group's running sums (minus the sums
// before the column); per block the first minimum.
__global__ __launch_bounds__(kSweepThreads) void k_sweepb_phi(const VolCut* __restrict__ P, int64_t n,
                                                              long long two_m, PhiIdx* __restrict__ part) {
  __shared__ PhiIdx s[kSweepThreads / 64];
  const int64_t g = blockIdx.y;
  const VolCut base = g > 0 ? P[g * n - 1] : VolCut{0, 0};
  PhiIdx best{INFINITY, 0x7FFFFFFFFFFFFFFFll};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i + 1 < n; i += (int64_t)gridDim.x * blockDim.x) {
    const VolCut x = P[g * n + i];
    const long long vv = x.vol - base.vol;
    const long long cc = x.cut - base.cut;
    const long long denom = vv < two_m - vv ? vv : two_m - vv;
    if (denom > 0) best = better(best, PhiIdx{static_cast<double>(cc) / static_cast<double>(denom), i});
  }
  for (int off = 32; off > 0; off >>= 1) {
    PhiIdx o{__shfl_down(best.phi, off), __shfl_down(best.idx, off)};
    best = better(best, o);
  }
  if (threadIdx.x % 64 == 0) s[threadIdx.x / 64] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kSweepThreads / 64; ++w) best = better(best, s[w]);
    part[g * gridDim.x + blockIdx.x] = best;
  }
}

__global__ void k_sweepb_final(const PhiIdx* __restrict__ part, int nparts, PhiIdx* __restrict__ out) {
  const int g = blockIdx.x;
  if (threadIdx.x != 0) return;
  PhiIdx best{INFINITY, 0x7FFFFFFFFFFFFFFFll};
  for (int b = 0; b < nparts; ++b) best = better(best, part[g * nparts + b]);
  out[g] = best;
}

}  // namespace
}  // namespace agp

extern "C" int agp_sweep_batch(const agp_graph_t* g, const float* pi, int64_t ld, int32_t C, void* stream,
                               int64_t* best_size, double* best_conductance) {
  using namespace agp;
  if (!g || !pi || !best_size || !best_conductance) return fail(AGP_EINVAL, "agp_sweep_batch: NULL argument");
  if (C < 1 || ld < C) return fail(AGP_EINVAL, "agp_sweep_batch: need C >= 1 and ld >= C");
  if (g->directed) return fail(AGP_EINVAL, "agp_sweep_batch: conductance is defined on undirected graphs");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = g->n;
  for (int32_t c = 0; c < C; ++c) {
    best_size[c] = 0;
    best_conductance[c] = INFINITY;
  }
  if (n < 2) return AGP_OK;
  agp_graph* gg = const_cast<agp_graph*>(g);
  std::lock_guard<std::mutex> lk(gg->mu);
  if (int rc = ensure_items(gg, s)) return rc;
  // columns per group: at most 64, and the group's buffers (37 bytes per
  // node and column plus the sort space) within a quarter of the free memory
  size_t free_b = 0, total_b = 0;
  AGP_HIP(hipMemGetInfo(&free_b, &total_b));
  const double per_col = 40.0 * static_cast<double>(n) + 4096.0;
  int G = static_cast<int>(std::min<double>(std::min<int32_t>(C, kBatchCols), 0.25 * free_b / per_col));
  if (G < 1) G = 1;
  if (static_cast<double>(n) * G >= 4294967295.0) G = static_cast<int>(4294967294.0 / static_cast<double>(n));
  if (G < 1) return fail(AGP_EINVAL, "agp_sweep_batch: graph too large");
  const size_t GN = static_cast<size_t>(n) * G;
  size_t sort_bytes = 0, scan_bytes = 0;
  AGP_HIP(rocprim::radix_sort_pairs(nullptr, sort_bytes, static_cast<uint64_t*>(nullptr),
                                    static_cast<uint64_t*>(nullptr), static_cast<int32_t*>(nullptr),
                                    static_cast<int32_t*>(nullptr), static_cast<size_t>(n), 0, 64, s));
  const VolCutAt at0{nullptr, nullptr, nullptr, n, G};
  AGP_HIP(rocprim::inclusive_scan(nullptr, scan_bytes,
                                  rocprim::make_transform_iterator(rocprim::make_counting_iterator<size_t>(0), at0),
                                  static_cast<VolCut*>(nullptr), GN, VolCutPlus(), s));
  const size_t temp_bytes = align256(std::max(sort_bytes, scan_bytes));
  // layout: keys[2] (8 GN each; then the running sums, 16 GN), ids[2] and rank
  // (4 GN each), cut terms (8 GN), byte ranks (GN), block minima, sort/scan space
  const size_t b8 = align256(GN * 8), b4 = align256(GN * 4), b1 = align256(GN);
  const size_t bpart = align256(sizeof(PhiIdx) * (kBatchCols * (kBatchPhiBlocks + 1)));
  const size_t total = 3 * b8 + 3 * b4 + b1 + bpart + temp_bytes;
  DevBuf& buf = gg->scratch.sweep;
  if (int rc = buf.reserve(total, false, s)) return rc;
  char* p = buf.as<char>();
  uint64_t* keys_in = reinterpret_cast<uint64_t*>(p);
  uint64_t* keys_out = reinterpret_cast<uint64_t*>(p + b8);
  VolCut* P = reinterpret_cast<VolCut*>(p);  // over both key arrays once the sort is done
  long long* dcut = reinterpret_cast<long long*>(p + 2 * b8);
  int32_t* ids_in = reinterpret_cast<int32_t*>(p + 3 * b8);
  int32_t* ids_out = reinterpret_cast<int32_t*>(p + 3 * b8 + b4);
  int32_t* rank = reinterpret_cast<int32_t*>(p + 3 * b8 + 2 * b4);
  uint8_t* coarse = reinterpret_cast<uint8_t*>(p + 3 * b8 + 3 * b4);
  PhiIdx* parts = reinterpret_cast<PhiIdx*>(p + 3 * b8 + 3 * b4 + b1);
  PhiIdx* fin = parts + static_cast<size_t>(kBatchCols) * kBatchPhiBlocks;
  void* temp = p + 3 * b8 + 3 * b4 + b1 + bpart;
  static_assert(sizeof(VolCut) == 16, "running sums take the two key arrays");
  int shift = 0;
  while ((n - 1) >> shift >= 256) ++shift;
  const long long* first = nullptr;
  const int32_t* items = nullptr;
  items_of(gg, &first, &items);
  const int64_t nitems = gg->scratch.sweep_nitems;
  std::vector<PhiIdx> h(kBatchCols);
  for (int32_t c0 = 0; c0 < C; c0 += G) {
    const int Gc = std::min<int32_t>(G, C - c0);
    const size_t gn = static_cast<size_t>(n) * Gc;
    const unsigned grid = static_cast<unsigned>(std::min<int64_t>((static_cast<int64_t>(gn) + 255) / 256, 65536));
    k_sweepb_keys<<<grid, 256, 0, s>>>(pi, ld, c0, Gc, g->degree, n, keys_in, ids_in);
    size_t tb = temp_bytes;
    for (int gi = 0; gi < Gc; ++gi) {  // one device-wide sort per column (a segmented sort takes a
      tb = temp_bytes;                 // block per segment, far slower on segments of millions)
      const size_t o = static_cast<size_t>(gi) * static_cast<size_t>(n);
      AGP_HIP(rocprim::radix_sort_pairs(temp, tb, keys_in + o, keys_out + o, ids_in + o, ids_out + o,
                                        static_cast<size_t>(n), 0, 64, s));
    }
    k_sweepb_rank<<<grid, 256, 0, s>>>(ids_out, n, Gc, shift, rank, coarse);
    k_sweepb_init<<<grid, 256, 0, s>>>(g->degree, n, Gc, dcut);
    const unsigned dgrid = static_cast<unsigned>(
        std::max<int64_t>(1, std::min<int64_t>((nitems + kSweepThreads / 64 - 1) / (kSweepThreads / 64), 65536)));
    k_sweepb_delta<<<dgrid, kSweepThreads, 0, s>>>(g->row_ptr, g->col, rank, coarse, shift, n, Gc, items, first,
                                                  nitems, dcut);
    tb = temp_bytes;
    const VolCutAt at{ids_out, g->degree, dcut, n, Gc};
    AGP_HIP(rocprim::inclusive_scan(temp, tb,
                                    rocprim::make_transform_iterator(rocprim::make_counting_iterator<size_t>(0), at),
                                    P, gn, VolCutPlus(), s));
    k_sweepb_phi<<<dim3(kBatchPhiBlocks, Gc), kSweepThreads, 0, s>>>(P, n, static_cast<long long>(g->nnz), parts);
    k_sweepb_final<<<Gc, 64, 0, s>>>(parts, kBatchPhiBlocks, fin);
    AGP_HIP(hipGetLastError());
    AGP_HIP(hipMemcpyAsync(h.data(), fin, sizeof(PhiIdx) * Gc, hipMemcpyDeviceToHost, s));
    AGP_HIP(hipStreamSynchronize(s));
    for (int gi = 0; gi < Gc; ++gi)
      if (std::isfinite(h[gi].phi)) {
        best_size[c0 + gi] = h[gi].idx + 1;
        best_conductance[c0 + gi] = h[gi].phi;
      }
  }
  return AGP_OK;
}
