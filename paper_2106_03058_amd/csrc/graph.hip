// Graph construction: device copy of the CSR, optional self-loops, and the
// degree-sorted adjacency lists of Section 4 ("pre-sorting adjacency list by
// degrees"): every row N_u is ordered ascending by (d_v, v), so the neighbours
// whose increment reaches the threshold form a prefix and each degree group
// [2^k, 2^(k+1)) is a contiguous range.  Rows are sorted by a segmented sort
// keyed on (d_v << 32 | v): LDS bitonic sorts for rows of up to 4096 entries
// and an LDS-chunked merge sort for longer rows.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "agp_device.h"
#include "agp_internal.h"

namespace agp {
namespace {

constexpr int kSortTile = 4096;  // keys per LDS tile (32 KiB)
constexpr int kSortThreads = 256;

__global__ void k_check_row_ptr(const int64_t* __restrict__ rp, int64_t n, int64_t nnz,
                                int* __restrict__ flag) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    if (rp[u] > rp[u + 1]) atomicOr(flag, 1);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (rp[0] != 0 || rp[n] != nnz)) atomicOr(flag, 1);
}

__global__ void k_check_ids(const int32_t* __restrict__ col, int64_t nnz, int64_t n,
                            int* __restrict__ flag) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nnz;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = col[j];
    if (v < 0 || v >= n) atomicOr(flag, 2);
  }
}

// new_deg[u] = d_u + 1 if row u has no self-loop, else d_u.
__global__ void k_loop_degree(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                              int64_t n, int64_t* __restrict__ new_deg) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    bool has = false;
    for (int64_t j = rp[u]; j < rp[u + 1] && !has; ++j) has = (col[j] == (int32_t)u);
    new_deg[u] = (rp[u + 1] - rp[u]) + (has ? 0 : 1);
  }
}

__global__ void k_copy_add_loop(const int64_t* __restrict__ rp, const int32_t* __restrict__ col,
                                const int64_t* __restrict__ nrp, int64_t n,
                                int32_t* __restrict__ ncol) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    int64_t o = nrp[u];
    for (int64_t j = rp[u]; j < rp[u + 1]; ++j) ncol[o++] = col[j];
    if (o < nrp[u + 1]) ncol[o] = (int32_t)u;
  }
}

// --- exclusive scan of int64 counts: out[0] = 0, out[i+1] = sum(in[0..i]).
constexpr int kScanItems = 4;  // per thread
constexpr int kScanBlock = 256 * kScanItems;

__global__ void k_scan_local(const int64_t* __restrict__ in, int64_t n, int64_t* __restrict__ out,
                             int64_t* __restrict__ block_sums) {
  __shared__ int64_t s[256];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t run = 0;
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    run += v[k];
  }
  s[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int64_t t = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  int64_t acc = s[threadIdx.x] - run;  // exclusive prefix of this thread
  for (int k = 0; k < kScanItems; ++k) {
    acc += v[k];
    if (base + k < n) out[base + k + 1] = acc;  // inclusive, shifted by one
  }
  if (threadIdx.x == 255) block_sums[blockIdx.x] = s[255];
}

__global__ void k_scan_block_sums(int64_t* __restrict__ sums, int64_t nb) {
  // single thread: the number of blocks is small (n / 1024)
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int64_t run = 0;
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t t = sums[b];
      sums[b] = run;
      run += t;
    }
  }
}

__global__ void k_scan_add(int64_t* __restrict__ out, int64_t n, const int64_t* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  const int64_t add = sums[blockIdx.x];
  for (int k = threadIdx.x; k < kScanBlock; k += blockDim.x) {
    const int64_t i = base + k;
    if (i < n) out[i + 1] += add;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = 0;
}

int exclusive_scan(const int64_t* in, int64_t n, int64_t* out, hipStream_t s) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  DevBuf sums;
  int rc = sums.reserve(sizeof(int64_t) * (size_t)std::max<int64_t>(nb, 1), false, s);
  if (rc) return rc;
  if (nb > 0) {
    k_scan_local<<<(unsigned)nb, 256, 0, s>>>(in, n, out, sums.as<int64_t>());
    k_scan_block_sums<<<1, 1, 0, s>>>(sums.as<int64_t>(), nb);
    k_scan_add<<<(unsigned)nb, 256, 0, s>>>(out, n, sums.as<int64_t>());
  } else {
    AGP_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), s));
  }
  AGP_HIP(hipGetLastError());
  AGP_HIP(hipStreamSynchronize(s));
  sums.release();
  return AGP_OK;
}

__global__ void k_degree(const int64_t* __restrict__ rp, int64_t n, int32_t* __restrict__ deg,
                         int* __restrict__ max_deg) {
  int local = 0;
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int d = (int)(rp[u + 1] - rp[u]);
    deg[u] = d;
    local = max(local, d);
  }
  atomicMax(max_deg, local);
}

// Degree in the factors d^-a, d^-b: the row length of the given matrix
// (out-degree of a directed graph), a node without arcs counting as 1.
__global__ void k_factor_degree(const int64_t* __restrict__ rp, int64_t n, int32_t* __restrict__ fdeg,
                                int* __restrict__ max_f) {
  int local = 0;
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int d = (int)(rp[u + 1] - rp[u]);
    const int f = d < 1 ? 1 : d;
    fdeg[u] = f;
    local = max(local, f);
  }
  atomicMax(max_f, local);
}

// Transpose of a CSR: in-degree counts, then every arc u -> v placed in row v
// (order inside a row is fixed later by the row sort).
__global__ void k_in_count(const int32_t* __restrict__ col, int64_t nnz, unsigned long long* __restrict__ cnt) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nnz;
       j += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(cnt + col[j], 1ull);
}

__global__ void k_transpose_scatter(const int64_t* __restrict__ rp, const int32_t* __restrict__ col, int64_t n,
                                    unsigned long long* __restrict__ cursor, int32_t* __restrict__ tcol) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x)
    for (int64_t j = rp[u]; j < rp[u + 1]; ++j) tcol[atomicAdd(cursor + col[j], 1ull)] = (int32_t)u;
}

__global__ void k_make_keys(const int32_t* __restrict__ col, const int32_t* __restrict__ deg,
                            int64_t nnz, uint64_t* __restrict__ keys) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nnz;
       j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t v = (uint32_t)col[j];
    keys[j] = ((uint64_t)(uint32_t)deg[v] << 32) | v;
  }
}

// Bitonic sort of s[0..P), P a power of two <= kSortTile, by the whole block.
__device__ void lds_bitonic(uint64_t* s, int P) {
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint64_t a = s[i], b = s[ixj];
          const bool up = (i & k) == 0;
          if ((a > b) == up) {
            s[i] = b;
            s[ixj] = a;
          }
        }
      }
      __syncthreads();
    }
  }
}

// One block per row of at most kSortTile entries.
__global__ __launch_bounds__(kSortThreads) void k_sort_small_rows(const int64_t* __restrict__ rp,
                                                                  int64_t n,
                                                                  uint64_t* __restrict__ keys) {
  __shared__ uint64_t s[kSortTile];
  for (int64_t u = blockIdx.x; u < n; u += gridDim.x) {
    const int64_t beg = rp[u];
    const int d = (int)(rp[u + 1] - beg);
    if (d <= 1 || d > kSortTile) continue;  // uniform per block
    int P = 2;
    while (P < d) P <<= 1;
    for (int i = threadIdx.x; i < P; i += blockDim.x) s[i] = (i < d) ? keys[beg + i] : ~0ull;
    __syncthreads();
    lds_bitonic(s, P);
    for (int i = threadIdx.x; i < d; i += blockDim.x) keys[beg + i] = s[i];
    __syncthreads();
  }
}

__global__ void k_collect_large(const int64_t* __restrict__ rp, int64_t n, int64_t* __restrict__ list,
                                unsigned long long* __restrict__ cnt) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    if (rp[u + 1] - rp[u] > kSortTile) list[atomicAdd(cnt, 1ull)] = u;
  }
}

// Position in the merge of a[0..na) and b[0..nb) where diagonal k splits:
// returns i such that the first k outputs are a[0..i) and b[0..k-i).
__device__ int64_t merge_path(const uint64_t* a, int64_t na, const uint64_t* b, int64_t nb,
                              int64_t k) {
  int64_t lo = k > nb ? k - nb : 0;
  int64_t hi = k < na ? k : na;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    // take a[mid] before b[k-mid-1] iff a[mid] <= b[k-mid-1]
    if (a[mid] <= b[k - mid - 1])
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// One block per long row: sort 4096-key tiles in LDS, then merge runs of
// doubling width through a scratch copy of the row.
__global__ __launch_bounds__(kSortThreads) void k_sort_large_rows(
    const int64_t* __restrict__ rp, const int64_t* __restrict__ list, uint64_t* __restrict__ keys,
    uint64_t* __restrict__ tmp) {
  __shared__ uint64_t s[kSortTile];
  const int64_t u = list[blockIdx.x];
  const int64_t beg = rp[u];
  const int64_t d = rp[u + 1] - beg;
  for (int64_t t0 = 0; t0 < d; t0 += kSortTile) {
    const int len = (int)((d - t0) < kSortTile ? (d - t0) : kSortTile);
    for (int i = threadIdx.x; i < kSortTile; i += blockDim.x)
      s[i] = (i < len) ? keys[beg + t0 + i] : ~0ull;
    __syncthreads();
    lds_bitonic(s, kSortTile);
    for (int i = threadIdx.x; i < len; i += blockDim.x) keys[beg + t0 + i] = s[i];
    __syncthreads();
  }
  uint64_t* src = keys + beg;
  uint64_t* dst = tmp + beg;
  constexpr int kPer = 8;
  for (int64_t width = kSortTile; width < d; width <<= 1) {
    for (int64_t lo = 0; lo < d; lo += 2 * width) {
      const int64_t mid = (lo + width) < d ? lo + width : d;
      const int64_t hi = (lo + 2 * width) < d ? lo + 2 * width : d;
      const uint64_t* a = src + lo;
      const uint64_t* b = src + mid;
      const int64_t na = mid - lo, nb = hi - mid;
      for (int64_t k0 = (int64_t)threadIdx.x * kPer; k0 < na + nb; k0 += (int64_t)blockDim.x * kPer) {
        int64_t i = merge_path(a, na, b, nb, k0);
        int64_t j = k0 - i;
        const int64_t kend = (k0 + kPer) < (na + nb) ? k0 + kPer : na + nb;
        for (int64_t k = k0; k < kend; ++k) {
          const bool take_a = (j >= nb) || (i < na && a[i] <= b[j]);
          dst[lo + k] = take_a ? a[i++] : b[j++];
        }
      }
    }
    __syncthreads();
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  if (src != keys + beg) {
    for (int64_t i = threadIdx.x; i < d; i += blockDim.x) keys[beg + i] = src[i];
  }
}

// Duplicate arcs (equal adjacent keys) and symmetry: (u, v) needs (v, u).
__global__ void k_validate_sorted(const int64_t* __restrict__ rp, const uint64_t* __restrict__ keys,
                                  const int32_t* __restrict__ deg, int64_t n, int* __restrict__ flag) {
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n;
       u += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t want = ((uint64_t)(uint32_t)deg[u] << 32) | (uint64_t)u;
    for (int64_t j = rp[u]; j < rp[u + 1]; ++j) {
      if (j > rp[u] && keys[j] == keys[j - 1]) atomicOr(flag, 4);
      const int64_t v = (int64_t)(uint32_t)keys[j];
      int64_t lo = rp[v], hi = rp[v + 1];
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < want)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (lo >= rp[v + 1] || keys[lo] != want) atomicOr(flag, 8);
    }
  }
}

__global__ void k_split_keys(const uint64_t* __restrict__ keys, int64_t nnz, uint32_t* __restrict__ col,
                             uint32_t* __restrict__ nd) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nnz;
       j += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[j];
    col[j] = (uint32_t)k;
    nd[j] = (uint32_t)(k >> 32);
  }
}

// End of each arc's degree group inside its row (row-relative, exclusive):
// the first later position whose factor degree reaches the next power of
// two, else the row length.  Rows ascend in the factor degree, so a run of
// sampled pushes that starts at position s of a row stays in one group up to
// gend[s].  One wave per row; each lane binary-searches for its arcs.
__global__ void k_group_ends(const int64_t* __restrict__ rp, const uint32_t* __restrict__ nd, int64_t n,
                             uint32_t* __restrict__ gend) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t u = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; u < n; u += nw) {
    const int64_t r0 = rp[u], r1 = rp[u + 1];
    for (int64_t j = r0 + lane; j < r1; j += 64) {
      const int g = 31 - __clz(nd[j]);
      int64_t lo = r1;
      if (g < 31) {
        const uint32_t lim = 1u << (g + 1);
        lo = j + 1;
        int64_t hi = r1;
        while (lo < hi) {
          const int64_t mid = (lo + hi) >> 1;
          if (nd[mid] < lim)
            lo = mid + 1;
          else
            hi = mid;
        }
      }
      gend[j] = (uint32_t)(lo - r0);
    }
  }
}

unsigned grid_for(int64_t items, int threads) {
  int64_t b = (items + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

// RAII list of device allocations made during a build.
struct Allocs {
  std::vector<void*> ptrs;
  ~Allocs() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  int get(T** out, size_t count) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(AGP_ENOMEM, "hipMalloc failed during graph build");
    }
    ptrs.push_back(p);
    *out = static_cast<T*>(p);
    return AGP_OK;
  }
  void keep(void* p) { ptrs.erase(std::remove(ptrs.begin(), ptrs.end(), p), ptrs.end()); }
};

int build_graph(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                uint32_t flags, hipStream_t s, agp_graph* g) {
  Allocs al;
  int rc;
  int64_t* rp = nullptr;
  int32_t* col = nullptr;
  int* dflag = nullptr;
  if ((rc = al.get(&rp, (size_t)n + 1)) || (rc = al.get(&col, (size_t)nnz)) ||
      (rc = al.get(&dflag, 2)))
    return rc;
  const hipMemcpyKind kind = (flags & AGP_HOST_PTRS) ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  AGP_HIP(hipMemcpyAsync(rp, row_ptr, sizeof(int64_t) * ((size_t)n + 1), kind, s));
  if (nnz) AGP_HIP(hipMemcpyAsync(col, col_idx, sizeof(int32_t) * (size_t)nnz, kind, s));
  AGP_HIP(hipMemsetAsync(dflag, 0, 2 * sizeof(int), s));
  k_check_row_ptr<<<grid_for(n, 256), 256, 0, s>>>(rp, n, nnz, dflag);
  k_check_ids<<<grid_for(nnz, 256), 256, 0, s>>>(col, nnz, n, dflag);
  int hflag = 0;
  AGP_HIP(hipMemcpyAsync(&hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
  AGP_HIP(hipStreamSynchronize(s));
  if (hflag & 1) return fail(AGP_EINVAL, "row_ptr must start at 0, be non-decreasing and end at nnz");
  if (hflag & 2) return fail(AGP_EINVAL, "col_idx holds an id outside [0, n)");

  if (flags & AGP_ADD_SELF_LOOPS) {
    int64_t *nd = nullptr, *nrp = nullptr;
    if ((rc = al.get(&nd, (size_t)n)) || (rc = al.get(&nrp, (size_t)n + 1))) return rc;
    k_loop_degree<<<grid_for(n, 256), 256, 0, s>>>(rp, col, n, nd);
    if ((rc = exclusive_scan(nd, n, nrp, s))) return rc;
    int64_t new_nnz = 0;
    AGP_HIP(hipMemcpy(&new_nnz, nrp + n, sizeof(int64_t), hipMemcpyDeviceToHost));
    int32_t* ncol = nullptr;
    if ((rc = al.get(&ncol, (size_t)new_nnz))) return rc;
    k_copy_add_loop<<<grid_for(n, 256), 256, 0, s>>>(rp, col, nrp, n, ncol);
    rp = nrp;
    col = ncol;
    nnz = new_nnz;
  }
  if (nnz >= ((int64_t)1 << 40)) return fail(AGP_EINVAL, "too many arcs");

  // factor degrees from the given rows (out-degrees when directed)
  int32_t* fdeg = nullptr;
  int* fmax = nullptr;
  if ((rc = al.get(&fdeg, (size_t)n)) || (rc = al.get(&fmax, 1))) return rc;
  AGP_HIP(hipMemsetAsync(fmax, 0, sizeof(int), s));
  k_factor_degree<<<grid_for(n, 256), 256, 0, s>>>(rp, n, fdeg, fmax);
  if (flags & AGP_REVERSE) {  // pushes follow in-edges: rows of the transpose
    unsigned long long* cnt = nullptr;
    int64_t* trp = nullptr;
    int32_t* tcol = nullptr;
    if ((rc = al.get(&cnt, (size_t)n)) || (rc = al.get(&trp, (size_t)n + 1)) || (rc = al.get(&tcol, (size_t)nnz)))
      return rc;
    AGP_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long) * (size_t)n, s));
    k_in_count<<<grid_for(nnz, 256), 256, 0, s>>>(col, nnz, cnt);
    if ((rc = exclusive_scan(reinterpret_cast<const int64_t*>(cnt), n, trp, s))) return rc;
    AGP_HIP(hipMemcpyAsync(cnt, trp, sizeof(int64_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    k_transpose_scatter<<<grid_for(n, 256), 256, 0, s>>>(rp, col, n, cnt, tcol);
    rp = trp;
    col = tcol;
  }

  int32_t* deg = nullptr;
  int* dmax = nullptr;
  uint64_t* keys = nullptr;
  if ((rc = al.get(&deg, (size_t)n)) || (rc = al.get(&dmax, 1)) || (rc = al.get(&keys, (size_t)nnz)))
    return rc;
  AGP_HIP(hipMemsetAsync(dmax, 0, sizeof(int), s));
  k_degree<<<grid_for(n, 256), 256, 0, s>>>(rp, n, deg, dmax);
  k_make_keys<<<grid_for(nnz, 256), 256, 0, s>>>(col, fdeg, nnz, keys);
  if (n > 0) {
    const unsigned rows_grid = (unsigned)std::min<int64_t>(n, 1 << 20);
    k_sort_small_rows<<<rows_grid, kSortThreads, 0, s>>>(rp, n, keys);
  }
  int64_t* large = nullptr;
  unsigned long long* dcnt = nullptr;
  if ((rc = al.get(&large, (size_t)n)) || (rc = al.get(&dcnt, 1))) return rc;
  AGP_HIP(hipMemsetAsync(dcnt, 0, sizeof(unsigned long long), s));
  k_collect_large<<<grid_for(n, 256), 256, 0, s>>>(rp, n, large, dcnt);
  unsigned long long nlarge = 0;
  AGP_HIP(hipMemcpyAsync(&nlarge, dcnt, sizeof(nlarge), hipMemcpyDeviceToHost, s));
  AGP_HIP(hipStreamSynchronize(s));
  if (nlarge > 0) {
    uint64_t* tmp = nullptr;
    if ((rc = al.get(&tmp, (size_t)nnz))) return rc;
    k_sort_large_rows<<<(unsigned)nlarge, kSortThreads, 0, s>>>(rp, large, keys, tmp);
  }
  if (flags & AGP_VALIDATE) {
    AGP_HIP(hipMemsetAsync(dflag, 0, sizeof(int), s));
    k_validate_sorted<<<grid_for(n, 256), 256, 0, s>>>(rp, keys, fdeg, n, dflag);
    AGP_HIP(hipMemcpyAsync(&hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    AGP_HIP(hipStreamSynchronize(s));
    if (hflag & 4) return fail(AGP_EINVAL, "duplicate arcs in a row");
    if ((hflag & 8) && !(flags & AGP_DIRECTED)) return fail(AGP_EINVAL, "the matrix is not symmetric");
  }
  uint32_t *scol = nullptr, *snd = nullptr, *gend = nullptr;
  if ((rc = al.get(&scol, (size_t)nnz)) || (rc = al.get(&snd, (size_t)nnz)) || (rc = al.get(&gend, (size_t)nnz)))
    return rc;
  k_split_keys<<<grid_for(nnz, 256), 256, 0, s>>>(keys, nnz, scol, snd);
  if (n > 0) k_group_ends<<<(unsigned)std::min<int64_t>((n + 3) / 4, 1 << 16), 256, 0, s>>>(rp, snd, n, gend);
  int maxd = 0, maxf = 0;
  AGP_HIP(hipMemcpyAsync(&maxd, dmax, sizeof(int), hipMemcpyDeviceToHost, s));
  AGP_HIP(hipMemcpyAsync(&maxf, fmax, sizeof(int), hipMemcpyDeviceToHost, s));
  AGP_HIP(hipGetLastError());
  AGP_HIP(hipStreamSynchronize(s));

  g->n = n;
  g->nnz = nnz;
  g->max_degree = maxd;
  g->max_fdeg = maxf;
  g->row_ptr = rp;
  g->col = scol;
  g->ndeg = snd;
  g->gend = gend;
  g->degree = deg;
  g->fdeg = fdeg;
  al.keep(rp);
  al.keep(scol);
  al.keep(snd);
  al.keep(gend);
  al.keep(deg);
  al.keep(fdeg);
  return AGP_OK;
}

// degree group of every arc's neighbour: floor(log2 d) of its factor degree
__global__ void k_groups(const uint32_t* __restrict__ nd, int64_t nnz, uint8_t* __restrict__ out) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nnz; j += (int64_t)gridDim.x * blockDim.x)
    out[j] = static_cast<uint8_t>(31 - __clz(nd[j]));
}

}  // namespace
}  // namespace agp

extern "C" {

int agp_graph_create(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                     uint32_t flags, void* stream, agp_graph_t** out) {
  if (!out) return agp::fail(AGP_EINVAL, "agp_graph_create: out is NULL");
  *out = nullptr;
  if (n < 0 || n >= ((int64_t)1 << 31) - 1 || nnz < 0 || !row_ptr || (nnz > 0 && !col_idx))
    return agp::fail(AGP_EINVAL, "agp_graph_create: need 0 <= n < 2^31 - 1, nnz >= 0, non-NULL arrays");
  if (flags & ~(AGP_HOST_PTRS | AGP_VALIDATE | AGP_ADD_SELF_LOOPS | AGP_DIRECTED | AGP_REVERSE))
    return agp::fail(AGP_EINVAL, "agp_graph_create: unknown flag");
  if ((flags & AGP_REVERSE) && !(flags & AGP_DIRECTED))
    return agp::fail(AGP_EINVAL, "agp_graph_create: AGP_REVERSE needs AGP_DIRECTED");
  if ((flags & AGP_HOST_PTRS) && (row_ptr[0] != 0 || row_ptr[n] != nnz))
    return agp::fail(AGP_EINVAL, "agp_graph_create: row_ptr[0] must be 0 and row_ptr[n] = nnz");
  agp_graph* g = new (std::nothrow) agp_graph();
  if (!g) return agp::fail(AGP_ENOMEM, "agp_graph_create: host allocation failed");
  hipError_t e = hipGetDevice(&g->device);
  if (e != hipSuccess) {
    delete g;
    return agp::fail(AGP_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  }
  g->directed = (flags & AGP_DIRECTED) != 0;
  const int rc = agp::build_graph(n, nnz, row_ptr, col_idx, flags, (hipStream_t)stream, g);
  if (rc != AGP_OK) {
    delete g;
    return rc;
  }
  *out = g;
  return AGP_OK;
}

int agp_graph_info(const agp_graph_t* g, int64_t* n, int64_t* nnz, int32_t* max_degree) {
  if (!g) return agp::fail(AGP_EINVAL, "agp_graph_info: NULL graph");
  if (n) *n = g->n;
  if (nnz) *nnz = g->nnz;
  if (max_degree) *max_degree = g->max_degree;
  return AGP_OK;
}

int agp_graph_export(const agp_graph_t* g, int64_t* row_ptr, int32_t* col_sorted, int32_t* degree) {
  if (!g) return agp::fail(AGP_EINVAL, "agp_graph_export: NULL graph");
  if (row_ptr)
    AGP_HIP(hipMemcpy(row_ptr, g->row_ptr, sizeof(int64_t) * ((size_t)g->n + 1), hipMemcpyDeviceToHost));
  if (col_sorted && g->nnz)
    AGP_HIP(hipMemcpy(col_sorted, g->col, sizeof(int32_t) * (size_t)g->nnz, hipMemcpyDeviceToHost));
  if (degree && g->n)
    AGP_HIP(hipMemcpy(degree, g->degree, sizeof(int32_t) * (size_t)g->n, hipMemcpyDeviceToHost));
  return AGP_OK;
}

int agp_graph_groups(const agp_graph_t* g, uint8_t* group_ids) {
  if (!g || !group_ids) return agp::fail(AGP_EINVAL, "agp_graph_groups: NULL argument");
  if (g->nnz == 0) return AGP_OK;
  uint8_t* d = nullptr;
  AGP_HIP(hipMalloc(&d, static_cast<size_t>(g->nnz)));
  agp::k_groups<<<agp::grid_for(g->nnz, 256), 256>>>(g->ndeg, g->nnz, d);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpy(group_ids, d, static_cast<size_t>(g->nnz), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return agp::fail(AGP_EDEVICE, std::string("agp_graph_groups: ") + hipGetErrorString(e));
  return AGP_OK;
}

int agp_graph_destroy(agp_graph_t* g) {
  if (!g) return AGP_OK;
  {
    std::lock_guard<std::mutex> lk(g->mu);
    (void)hipDeviceSynchronize();
    g->drop_loops();
    if (g->capture_stream) (void)hipStreamDestroy(g->capture_stream);
    g->scratch.release();
    for (auto& kv : g->pow_tables) (void)hipFree(kv.second);
    (void)hipFree(g->row_ptr);
    (void)hipFree(g->col);
    (void)hipFree(g->ndeg);
    (void)hipFree(g->gend);
    (void)hipFree(g->degree);
    (void)hipFree(g->fdeg);
  }
  delete g;
  return AGP_OK;
}

}  // extern "C"
