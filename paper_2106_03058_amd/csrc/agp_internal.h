// Host-side internals shared by the translation units of libagp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>

#include "../../include/agp.h"

namespace agp {

// Thread-local error text behind agp_last_error().
int fail(int code, const std::string& msg);

#define AGP_HIP(call)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return ::agp::fail(e_ == hipErrorOutOfMemory ? AGP_ENOMEM : AGP_EDEVICE,             \
                         std::string(#call) + ": " + hipGetErrorString(e_));               \
  } while (0)

// A device buffer that only grows.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  bool borrowed = false;  // a view of memory the library does not own: never freed or grown
  int reserve(size_t want, bool zero, hipStream_t s);
  void release();
  template <typename T>
  T* as() const {
    return static_cast<T*>(ptr);
  }
};

// Scratch reused across propagation calls on one graph (guarded by the
// graph's mutex).  acc[] are kept all-zero between calls.
struct Scratch {
  DevBuf acc[2];
  DevBuf frontier[2];
  DevBuf counts;     // frontier sizes per level
  DevBuf counters;   // 5 x (L + 1) uint64
  DevBuf colparams;  // per-column theta / unit / qid
  DevBuf partial;    // per-block partial norms
  DevBuf flags;      // error and signal flags
  DevBuf levelinfo;  // per level: contribution mass (double), frontier mode (int)
  DevBuf rec[2];     // binned aggregation: push records, partitioned records
  DevBuf bins;       // bucket counts, offsets, cursors, per-level record counts
  DevBuf big;        // deferred long deterministic rows: per-level counters, then the row list
  DevBuf nodefac;    // batched calls: per node d_u^-b and the d^-a of its first neighbour
  double nodefac_a = -1.0, nodefac_b = -1.0;  // the exponents it holds (-1: none)
  DevBuf arcfac;     // batched calls: d^-a of every arc's neighbour (arc order)
  double arcfac_a = -1.0;                      // the exponent it holds (-1: none)
  DevBuf sweep;      // clustering sweep: keys, order, ranks, prefix sums, sort space
  DevBuf sweep_items;        // clustering sweep: arc-balanced work items of the graph
  int64_t sweep_nitems = -1; // their number (-1: not built yet)
  DevBuf dense_items;        // dense levels: arc-balanced work items (node ranges, long-row pieces)
  DevBuf dense_rows;         // dense levels: the long rows (cut into pieces)
  int64_t dense_nitems = -1; // number of items (-1: not built yet)
  int64_t dense_nrows = 0;   // number of long rows
  // level timing, created on demand: per level its start, the level kernel's
  // start and end, and the end of the level's next frontier
  hipEvent_t events[4 * (AGP_MAX_LEVELS + 1)] = {};
  int ensure_events();
  void release();
};

}  // namespace agp

struct agp_tune_key {
  int32_t C;
  double a, b;
  bool operator<(const agp_tune_key& o) const {
    if (C != o.C) return C < o.C;
    if (a != o.a) return a < o.a;
    return b < o.b;
  }
};

struct agp_graph {
  int64_t n = 0;
  int64_t nnz = 0;
  int32_t max_degree = 0;       // longest row
  int32_t max_fdeg = 0;         // largest factor degree
  int device = 0;
  bool directed = false;        // built with AGP_DIRECTED
  int64_t* row_ptr = nullptr;   // device int64[n + 1], rows in the push direction
  uint32_t* col = nullptr;      // device uint32[nnz], rows sorted by (factor degree, id)
  uint32_t* ndeg = nullptr;     // device uint32[nnz], factor degree of col[j]
  uint32_t* gend = nullptr;     // device uint32[nnz], row-relative end of arc j's degree group
  int32_t* degree = nullptr;    // device int32[n], row lengths
  int32_t* fdeg = nullptr;      // device int32[n], degree in the factors d^-a, d^-b (>= 1)
  std::map<double, double*> pow_tables;  // exponent e -> device d^-e, d = 0..max_fdeg
  std::map<agp_tune_key, agp_tuning_t> tuning;  // autotuned execution choices
  std::mutex mu;
  agp::Scratch scratch;
  // captured level loops (tuning field `capture`), keyed by everything their
  // kernels take by value: sizes, pointers, exponents, modes
  std::map<std::string, hipGraphExec_t> loops;
  hipStream_t capture_stream = nullptr;  // private stream the loops are captured on
  void drop_loops();
};

namespace agp {
// Device table d^-e for d = 0..max_fdeg (0 at d = 0), made on first use (may_alloc) and
// kept with the graph; without may_alloc a missing table is AGP_EINVAL.
int pow_table(agp_graph* g, double e, const double** out, bool may_alloc = true);
}  // namespace agp
