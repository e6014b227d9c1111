// Continuous-batching query server: single-source proximity queries (PPR,
// heat kernel PageRank, Katz, L-hop transition probability) arrive at any
// time; each is admitted into a free slot (a column of the level kernel) and
// advances one level per step together with every other running query,
// whatever their levels, weights, exponents and thresholds.  The random
// streams are keyed by (seed, query_id) and the level sums are exact, so a
// query's result is the same alone, in a batch or in any mix.
//
// A query's residues live in two open-addressing tables (this level's and
// the next one's) that take a contiguous range of one pool of table entries,
// sized from the query's push estimate (Theorem 3.3); a query is admitted
// when a slot is free and its range fits in the pool, so the device memory
// of the running queries never exceeds the pool.  A table that fills up
// ends the query's run: it is dropped for one step, then queued again at
// the head with tables twice as large (its result does not depend on the
// table size).  The reserve goes straight to the query's output buffer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>
#include <vector>

#include "agp_internal.h"
#include "bin_kernels.h"
#include "level_kernels.h"
#include "server_admission.h"

namespace agp {
namespace srv {
struct AdmitItem {
  long long units;  // an initial residue (x value) in the column's units
  uint32_t node;
  uint32_t slot;
};
struct PlainTable {
  uint32_t off;  // the next level's table of a query with a plain direct table
  uint32_t slot;
};
}  // namespace srv

namespace {

using namespace lvl;
using srv::AdmitItem;

// New slots: seed the residues of the signal's entries in the slot's table
// and append them to the frontier, clear the slots' counters (every item of a
// slot clears them).
__global__ void k_admit(const AdmitItem* __restrict__ items, int k, uint32_t* __restrict__ keys,
                        long long* __restrict__ vals, const uint32_t* __restrict__ tab_off,
                        const uint32_t* __restrict__ tab_mask, uint64_t* __restrict__ F,
                        unsigned long long* __restrict__ cnt, unsigned long long* __restrict__ counters,
                        double* __restrict__ mass, int* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const AdmitItem it = items[i];
  for (int j = 0; j < kNumCounters; ++j) counters[static_cast<size_t>(it.slot) * kNumCounters + j] = 0;
  mass[it.slot] = 0.0;
  bool first = false;
  const uint32_t mask = tab_mask[it.slot];
  const uint32_t pos = mask == kDirectPlain ? tab_off[it.slot] + it.node
                                            : table_find_or_insert(keys, tab_off[it.slot], mask, it.node, &first);
  if (pos == ~0u) {
    atomicOr(err + it.slot, kErrTableFull);
    return;
  }
  vals[pos] = it.units;  // the signal's ids are distinct
  const unsigned long long at = atomicAdd(cnt, 1ull);
  F[at] = (static_cast<uint64_t>(pos) << 32) | it.slot;
}

__global__ void k_zero_count(unsigned long long* c) { *c = 0; }

// The next frontier of the queries with plain direct tables: the non-zero
// positions of their next tables (row y of the grid scans table t[y]; the
// other queries append first touches in the level kernel).
__global__ __launch_bounds__(kThreads) void k_scan_plain(const srv::PlainTable* __restrict__ t, int64_t n,
                                                         const long long* __restrict__ vals, uint64_t* __restrict__ F,
                                                         unsigned long long* __restrict__ cnt) {
  __shared__ uint64_t s_stage[kThreads / kWave][kStage];
  uint64_t* stage = s_stage[threadIdx.x / kWave];
  int staged = 0;
  const srv::PlainTable pt = t[blockIdx.y];
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t first = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t iters = (n + stride - 1) / stride;  // the same for every wave (wave-wide staging)
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t v = first + it * stride;
    bool p = false;
    uint64_t item = 0;
    if (v < n) {
      const uint32_t pos = pt.off + static_cast<uint32_t>(v);
      p = vals[pos] != 0;
      item = (static_cast<uint64_t>(pos) << 32) | pt.slot;
    }
    stage_push(stage, staged, item, p, F, cnt);
  }
  stage_flush(stage, staged, F, cnt);
}

__global__ void k_clear_err(const AdmitItem* __restrict__ items, int k, int* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) err[items[i].slot] = 0;
}

double now_ms(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace
}  // namespace agp

using agp::lvl::ColParams;

struct QueryRec {
  agp_query_t q;
  std::vector<double> w;
  std::vector<double> rho, kappa;
  double theta = 0.0;                // eps ||x||_1
  std::vector<uint32_t> xi;          // sparse signal: ascending node ids
  std::vector<long long> xu;         //   and values in units of ulp(fl32(theta))
  double estimate = 0.0;
  uint64_t entries = 0;   // table entries (per table; two tables)
  bool signed_x = false;  // some signal entry is negative (residues may cancel)
  uint64_t offset = 0;    // the tables' range in the pool
  int restarts = 0;       // runs ended by a full table
  bool restart = false;   // its table filled up: drop this step, then queue again
  int slot = -1;
  int level = 0;
  bool fresh = false;  // admitted; its source residue is seeded in the next step
  bool done = false;
  bool failed = false;
  agp_result_t res{};
};

struct agp_server {
  agp_graph* g = nullptr;
  agp_server_config_t cfg{};
  int64_t n = 0;
  int S = 0;
  hipStream_t stream = nullptr;
  std::chrono::steady_clock::time_point t0;
  // device state: the table pool (keys and values of this step's and the
  // next step's tables, frontier lists of pool positions) and per-slot data
  agp::DevBuf keys, vals, F[2], counts, counters, mass, err, cp, admit, mode, tabs;
  int cur = 0;
  uint64_t pool_entries = 0;
  agp::srv::RangePool pool;  // guarded by mu
  // host state (guarded by mu)
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, QueryRec> recs;
  std::vector<uint64_t> slot_ticket;  // 0 = free
  double running_estimate = 0.0;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  // pinned staging
  ColParams* h_cp = nullptr;
  uint32_t* h_tabs = nullptr;  // per slot: this step's table offset, the mask, the next step's offset (3 S)
  std::vector<int32_t> h_degree;  // row lengths (table sizes of new queries)
  agp::srv::PlainTable* h_plain = nullptr;  // this step's plain direct tables (pinned, S)
  agp::DevBuf plain;
  std::vector<agp::srv::AdmitItem> h_admit;  // the step's admissions (kept until the step syncs)
  unsigned long long* h_counters = nullptr;
  double* h_mass = nullptr;
  int* h_err = nullptr;
  int worker_error = AGP_OK;
};

namespace agp {
namespace {

// unit of a column with threshold theta (binary32): ulp of fl(theta)
void unit_of(double theta, int* ue, double* scale, long long* dtheta) {
  const float tw = static_cast<float>(theta);
  int e = -149;
  if (tw > 0.0f) {
    int ex;
    std::frexp(static_cast<double>(tw), &ex);
    e = (ex - 1) - 23 < -149 ? -149 : (ex - 1) - 23;
  }
  *ue = e;
  *scale = std::ldexp(1.0, -e);
  *dtheta = static_cast<long long>(static_cast<double>(tw) * *scale);
}

int validate(const agp_server* s, const agp_query_t* q) {
  if (!q) return fail(AGP_EINVAL, "agp_submit: NULL query");
  if (q->x_nnz < 0) return fail(AGP_EINVAL, "agp_submit: x_nnz < 0");
  if (q->x_nnz == 0 && (q->source < 0 || q->source >= s->n))
    return fail(AGP_EINVAL, "agp_submit: source out of range");
  if (q->x_nnz > 0) {
    if (!q->x_idx || !q->x_val) return fail(AGP_EINVAL, "agp_submit: NULL sparse signal");
    if (q->x_nnz > s->n) return fail(AGP_EINVAL, "agp_submit: more entries than nodes");
    for (int64_t k = 0; k < q->x_nnz; ++k) {
      if (q->x_idx[k] < 0 || q->x_idx[k] >= s->n) return fail(AGP_EINVAL, "agp_submit: signal id out of range");
      if (!std::isfinite(q->x_val[k])) return fail(AGP_EINVAL, "agp_submit: non-finite signal value");
    }
  }
  if (!(q->a >= 0.0 && q->a <= 1.0) || !(q->b >= 0.0 && q->b <= 1.0))
    return fail(AGP_EINVAL, "agp_submit: a and b must lie in [0, 1]");
  if (q->L < 0 || q->L > AGP_MAX_LEVELS) return fail(AGP_EINVAL, "agp_submit: need 0 <= L <= 255");
  if (!q->w || !q->out) return fail(AGP_EINVAL, "agp_submit: NULL weights or output");
  if (!(q->eps > 0.0) || !std::isfinite(q->eps)) return fail(AGP_EINVAL, "agp_submit: need eps > 0");
  if (q->query_id >= (1u << 24)) return fail(AGP_EINVAL, "agp_submit: query_id must be < 2^24");
  for (int32_t i = 0; i <= q->L; ++i)
    if (!(q->w[i] >= 0.0) || !std::isfinite(q->w[i]))
      return fail(AGP_EINVAL, "agp_submit: weights must be finite and >= 0");
  return AGP_OK;
}

// theta = eps ||x||_1 summed as the batched path sums a column (ascending
// rows, in blocks of kThetaRows, then over the blocks), and the signal in
// units of ulp(fl32(theta)).
int signal_of(const agp_query_t* q, QueryRec* r) {
  int ue;
  double scale;
  long long dth;
  if (q->x_nnz == 0) {
    r->theta = q->eps;  // ||e_s||_1 = 1
    unit_of(r->theta, &ue, &scale, &dth);
    if (-ue > 61) return fail(AGP_EINVAL, "agp_submit: eps below the exact-accumulator range (2^-38)");
    r->xi.assign(1, static_cast<uint32_t>(q->source));
    r->xu.assign(1, static_cast<long long>(std::ldexp(1.0, -ue)));
    return AGP_OK;
  }
  std::vector<std::pair<int64_t, float>> e;
  e.reserve(static_cast<size_t>(q->x_nnz));
  for (int64_t k = 0; k < q->x_nnz; ++k) e.emplace_back(q->x_idx[k], q->x_val[k]);
  std::sort(e.begin(), e.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
  for (size_t k = 1; k < e.size(); ++k)
    if (e[k].first == e[k - 1].first) return fail(AGP_EINVAL, "agp_submit: repeated signal id");
  double total = 0.0, part = 0.0;
  int64_t block = e.front().first / lvl::kThetaRows;
  for (const auto& x : e) {
    if (x.first / lvl::kThetaRows != block) {
      total = total + part;
      part = 0.0;
      block = x.first / lvl::kThetaRows;
    }
    part = part + std::fabs(static_cast<double>(x.second));
  }
  total = total + part;
  if (!(total > 0.0)) return fail(AGP_EINVAL, "agp_submit: the signal has no non-zero entry");
  r->theta = q->eps * total;
  unit_of(r->theta, &ue, &scale, &dth);
  if (-ue > 61) return fail(AGP_EINVAL, "agp_submit: eps ||x||_1 below the exact-accumulator range (2^-38)");
  r->xi.clear();
  r->xu.clear();
  for (const auto& x : e) {
    if (x.second == 0.0f) continue;
    const double u = std::ldexp(static_cast<double>(x.second), -ue);
    if (u != std::nearbyint(u) || !(std::fabs(u) < 4.0e18))
      return fail(AGP_EINVAL, "agp_submit: a signal value is not a multiple of the unit ulp(fl32(eps ||x||_1))");
    r->xi.push_back(static_cast<uint32_t>(x.first));
    r->xu.push_back(static_cast<long long>(u));
    if (x.second < 0.0f) r->signed_x = true;
  }
  return AGP_OK;
}

// One step: admit, advance every running query by one level, retire.
int step(agp_server* s) {
  hipStream_t st = s->stream;
  int nplain = 0;
  std::vector<uint64_t> admitted;
  s->h_admit.clear();
  {
    std::unique_lock<std::mutex> lk(s->mu);
    // admission in submission order: a free slot, the work budget, and the
    // query's tables in the pool
    int free_slots = 0;
    for (int c = 0; c < s->S; ++c) free_slots += s->slot_ticket[c] == 0 ? 1 : 0;
    int next_slot = 0;
    srv::admit_fifo(
        s->pending, free_slots, s->pool,
        [&](uint64_t t) -> uint64_t { return 2 * s->recs[t].entries; },  // this level's and the next level's table
        [&](uint64_t t) {
          const bool idle = s->running_estimate == 0.0;
          return !(s->cfg.work_budget > 0.0 && !idle && s->running_estimate + s->recs[t].estimate > s->cfg.work_budget);
        },
        [&](uint64_t t, uint64_t off) {
          QueryRec& r = s->recs[t];
          while (s->slot_ticket[next_slot]) ++next_slot;
          r.slot = next_slot;
          r.offset = off;
          r.level = 0;
          r.fresh = true;
          r.res.start_ms = now_ms(s->t0);
          s->slot_ticket[next_slot] = t;
          s->running_estimate += r.estimate;
          admitted.push_back(t);
        },
        [&](uint64_t t) {
          QueryRec& r = s->recs[t];  // its tables exceed the whole pool
          r.res.status = AGP_ENOMEM;
          r.res.levels = r.q.L;
          r.res.end_ms = now_ms(s->t0);
          r.done = true;
        });
    // per-slot parameters of this step
    nplain = 0;
    for (int c = 0; c < s->S; ++c) {
      ColParams& p = s->h_cp[c];
      const uint64_t t = s->slot_ticket[c];
      if (!t) {
        p.flags = kDrop;
        s->h_tabs[c] = 0;
        s->h_tabs[s->S + c] = 0;
        s->h_tabs[2 * s->S + c] = 0;
        continue;
      }
      QueryRec& r = s->recs[t];
      const int i = r.level;
      p.theta = r.theta;
      unit_of(p.theta, &p.ue, &p.scale, &p.dtheta);
      p.theta_w = static_cast<float>(p.theta);
      p.rho = r.rho[i];
      p.kappa = r.kappa[i];
      p.out = r.q.out;
      p.out_stride = 1;
      p.qid = r.q.query_id;
      p.key0 = static_cast<uint32_t>(r.q.seed);
      p.key1 = static_cast<uint32_t>(r.q.seed >> 32);
      p.level = i;
      p.flags = (i == r.q.L ? kLastLevel : 0) | (r.q.a == 0.0 ? kAZero : 0) | (r.failed || r.restart ? kDrop : 0);
      // the query's two tables, [offset, offset + entries) and the range
      // after it, take turns with the step parity
      s->h_tabs[c] = static_cast<uint32_t>(r.offset + (s->cur == 0 ? 0 : r.entries));
      s->h_tabs[s->S + c] = r.entries >= static_cast<uint64_t>(s->n)
                                ? (r.signed_x ? kDirectTable : kDirectPlain)  // position = offset + node
                                : static_cast<uint32_t>(r.entries - 1);
      s->h_tabs[2 * s->S + c] = static_cast<uint32_t>(r.offset + (s->cur == 0 ? r.entries : 0));
      if (s->h_tabs[s->S + c] == kDirectPlain && !(r.failed || r.restart) && i < r.q.L)
        s->h_plain[nplain++] = srv::PlainTable{s->h_tabs[2 * s->S + c], static_cast<uint32_t>(c)};
      if (r.fresh) {
        r.fresh = false;
        for (size_t k = 0; k < r.xi.size(); ++k)
          s->h_admit.push_back(srv::AdmitItem{r.xu[k], r.xi[k], static_cast<uint32_t>(c)});
      }
    }
  }
  // degree tables (created under the graph's lock) and output zero-fill
  for (uint64_t t : admitted) {
    QueryRec* r;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      r = &s->recs[t];
    }
    const double *da, *db;
    {
      std::lock_guard<std::mutex> lk(s->g->mu);
      int rc;
      if ((rc = pow_table(s->g, r->q.a, &da)) || (rc = pow_table(s->g, r->q.b, &db))) return rc;
    }
    s->h_cp[r->slot].da = da;
    s->h_cp[r->slot].db = db;
    AGP_HIP(hipMemsetAsync(r->q.out, 0, sizeof(float) * static_cast<size_t>(s->n), st));
  }
  const int cur = s->cur, nxt = 1 - s->cur;
  unsigned long long* counts = s->counts.as<unsigned long long>();
  uint32_t* tab_off = s->tabs.as<uint32_t>();  // this step's tables
  uint32_t* tab_mask = tab_off + s->S;
  uint32_t* tab_next = tab_off + 2 * s->S;      // the next step's tables
  uint64_t* F[2] = {s->F[0].as<uint64_t>(), s->F[1].as<uint64_t>()};
  AGP_HIP(hipMemcpyAsync(s->cp.ptr, s->h_cp, sizeof(ColParams) * s->S, hipMemcpyHostToDevice, st));
  AGP_HIP(hipMemcpyAsync(s->tabs.ptr, s->h_tabs, sizeof(uint32_t) * 3 * s->S, hipMemcpyHostToDevice, st));
  const int nadmit = static_cast<int>(s->h_admit.size());
  if (nadmit) {
    if (int rc = s->admit.reserve(sizeof(srv::AdmitItem) * static_cast<size_t>(nadmit), false, st)) return rc;
    AGP_HIP(hipMemcpyAsync(s->admit.ptr, s->h_admit.data(), sizeof(srv::AdmitItem) * nadmit, hipMemcpyHostToDevice,
                           st));
    k_clear_err<<<grid_for(nadmit, 64), 64, 0, st>>>(s->admit.as<srv::AdmitItem>(), nadmit, s->err.as<int>());
    k_admit<<<grid_for(nadmit, 64), 64, 0, st>>>(s->admit.as<srv::AdmitItem>(), nadmit, s->keys.as<uint32_t>(),
                                                  s->vals.as<long long>(), tab_off, tab_mask, F[cur],
                                                  counts + cur, s->counters.as<unsigned long long>(),
                                                  s->mass.as<double>(), s->err.as<int>());
  }
  k_zero_count<<<1, 1, 0, st>>>(counts + nxt);
  LevelArgs A{};
  A.rp = s->g->row_ptr;
  A.col = s->g->col;
  A.nd = s->g->ndeg;
  A.gend = s->g->gend;
  A.deg = s->g->degree;
  A.fdeg = s->g->fdeg;
  A.cp = s->cp.as<ColParams>();
  A.su = 1;
  A.sc = 1;
  A.level = 0;
  A.fin = F[cur];
  A.cnt_in = counts + cur;
  A.fout = F[nxt];
  A.cnt_out = counts + nxt;
  A.counters = s->counters.as<unsigned long long>();
  A.mass = s->mass.as<double>();
  A.err = s->err.as<int>();
  A.positive = 0;
  A.dense_cut = ~0ull;
  A.mode_out = s->mode.as<int>();
  // frontier entries are positions of this step's tables; pushes go to the
  // next step's tables (both in the one pool)
  A.keys_cur = s->keys.as<uint32_t>();
  A.keys_nxt = s->keys.as<uint32_t>();
  A.tab_off = tab_next;
  A.tab_mask = tab_mask;
  A.tab_cur = tab_off;
  k_level<float, false, true><<<kLevelBlocks, kThreads, 0, st>>>(A, nullptr, s->vals.as<long long>(),
                                                                 s->vals.as<long long>());
  if (nplain > 0) {
    AGP_HIP(hipMemcpyAsync(s->plain.ptr, s->h_plain, sizeof(srv::PlainTable) * nplain, hipMemcpyHostToDevice, st));
    const unsigned gx = std::max(1u, std::min(grid_for(s->n, kThreads, 65536), 8192u / static_cast<unsigned>(nplain)));
    k_scan_plain<<<dim3(gx, static_cast<unsigned>(nplain)), kThreads, 0, st>>>(
        s->plain.as<srv::PlainTable>(), s->n, s->vals.as<long long>(), F[nxt], counts + nxt);
  }
  AGP_HIP(hipGetLastError());
  AGP_HIP(hipMemcpyAsync(s->h_counters, s->counters.ptr, sizeof(unsigned long long) * kNumCounters * s->S,
                         hipMemcpyDeviceToHost, st));
  AGP_HIP(hipMemcpyAsync(s->h_mass, s->mass.ptr, sizeof(double) * s->S, hipMemcpyDeviceToHost, st));
  AGP_HIP(hipMemcpyAsync(s->h_err, s->err.ptr, sizeof(int) * s->S, hipMemcpyDeviceToHost, st));
  AGP_HIP(hipStreamSynchronize(st));
  s->cur = nxt;
  // retire
  std::lock_guard<std::mutex> lk(s->mu);
  const double t_end = now_ms(s->t0);
  std::vector<uint64_t> again;
  for (int c = 0; c < s->S; ++c) {
    const uint64_t t = s->slot_ticket[c];
    if (!t) continue;
    QueryRec& r = s->recs[t];
    const bool full = (s->h_err[c] & kErrTableFull) != 0;
    const bool overflow = (s->h_err[c] & ~kErrTableFull) != 0 || !(s->h_mass[c] < 0x1p61);
    bool finish = false, requeue = false;
    if (r.restart) {
      requeue = true;  // its residues were dropped in this step: run it again with larger tables
    } else if (r.failed) {
      finish = true;  // its residues were dropped in this step
    } else if (full) {
      r.restart = true;  // drop its residues in the next step, then queue it again
    } else if (overflow) {
      r.failed = true;  // drop its remaining residues in the next step
    } else if (r.level == r.q.L) {
      finish = true;
    } else {
      ++r.level;
    }
    if (finish || requeue) {
      s->pool.release(r.offset, 2 * r.entries);
      s->slot_ticket[c] = 0;
      s->running_estimate -= r.estimate;
      if (s->running_estimate < 1e-9) s->running_estimate = 0.0;
    }
    if (requeue) {
      r.restart = false;
      r.restarts += 1;
      r.entries = std::min<uint64_t>(2 * r.entries, static_cast<uint64_t>(s->n));  // n: a direct table
      r.slot = -1;
      again.push_back(t);
    }
    if (finish) {
      const unsigned long long* k = s->h_counters + static_cast<size_t>(c) * kNumCounters;
      r.res.status = r.failed ? AGP_ERANGE : AGP_OK;
      r.res.levels = r.q.L;
      r.res.frontier = k[0];
      r.res.pushes = k[2] + k[4];
      r.res.candidates = k[3];
      r.res.table_entries = r.entries;
      r.res.restarts = r.restarts;
      r.res.end_ms = t_end;
      r.done = true;
    }
  }
  for (auto it = again.rbegin(); it != again.rend(); ++it) s->pending.push_front(*it);  // at the head, in order
  s->cv.notify_all();
  return AGP_OK;
}

void worker_main(agp_server* s) {
  (void)hipSetDevice(s->g->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv.wait(lk, [s] {
        bool active = false;
        for (uint64_t t : s->slot_ticket) active |= (t != 0);
        return s->stop || active || !s->pending.empty();
      });
      bool active = false;
      for (uint64_t t : s->slot_ticket) active |= (t != 0);
      if (s->stop && !active) break;
      if (s->stop) s->pending.clear();
    }
    const int rc = step(s);
    if (rc != AGP_OK) {
      // a device failure ends every running and queued query
      std::lock_guard<std::mutex> lk(s->mu);
      s->worker_error = rc;
      for (auto& kv : s->recs) {
        if (!kv.second.done) {
          kv.second.done = true;
          kv.second.res.status = rc;
        }
      }
      s->pending.clear();
      std::fill(s->slot_ticket.begin(), s->slot_ticket.end(), 0);
      s->cv.notify_all();
      break;
    }
  }
}

}  // namespace
}  // namespace agp

extern "C" {

int agp_server_create(const agp_graph_t* g, const agp_server_config_t* cfg, agp_server_t** out) {
  using namespace agp;
  if (!out) return fail(AGP_EINVAL, "agp_server_create: out is NULL");
  *out = nullptr;
  if (!g || !cfg || cfg->max_slots < 1 || cfg->queue_capacity < 1 || !(cfg->work_budget >= 0.0) ||
      cfg->memory_bytes < 0)
    return fail(AGP_EINVAL, "agp_server_create: need a graph, max_slots >= 1, queue_capacity >= 1, budgets >= 0");
  agp_server* s = new (std::nothrow) agp_server();
  if (!s) return fail(AGP_ENOMEM, "agp_server_create: host allocation failed");
  s->g = const_cast<agp_graph*>(g);
  s->cfg = *cfg;
  s->n = g->n;
  s->S = cfg->max_slots;
  s->t0 = std::chrono::steady_clock::now();
  s->slot_ticket.assign(s->S, 0);
  // the pool: per entry a key (4 B) and a value (8 B), and half a frontier
  // entry in each of the two lists (a step's frontier holds at most one
  // entry per position of the current tables, half the pool)
  constexpr uint64_t kEntryBytes = 4 + 8 + 8;
  uint64_t budget = static_cast<uint64_t>(cfg->memory_bytes);
  if (budget == 0) {  // a quarter of the free device memory
    size_t free_b = 0, total_b = 0;
    (void)hipMemGetInfo(&free_b, &total_b);
    budget = free_b / 4;
  }
  s->pool_entries = std::min<uint64_t>(budget / kEntryBytes, 0xFFFFFFF0ull) & ~1ull;
  s->pool.reset(s->pool_entries);
  int rc = AGP_OK;
  if (s->pool_entries < 512) rc = fail(AGP_EINVAL, "agp_server_create: memory_bytes leaves no room for a query");
  hipError_t e = hipSuccess;
  if (!rc) {
    e = hipStreamCreate(&s->stream);
    if (e != hipSuccess) rc = fail(AGP_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
  }
  if (!rc) {
    const uint64_t P = s->pool_entries;
    if ((rc = s->keys.reserve(P * sizeof(uint32_t), true, s->stream)) ||
        (rc = s->vals.reserve(P * sizeof(long long), true, s->stream)) ||
        (rc = s->F[0].reserve(P / 2 * sizeof(uint64_t), false, s->stream)) ||
        (rc = s->F[1].reserve(P / 2 * sizeof(uint64_t), false, s->stream)) ||
        (rc = s->counts.reserve(2 * sizeof(unsigned long long), true, s->stream)) ||
        (rc = s->counters.reserve(sizeof(unsigned long long) * lvl::kNumCounters * s->S, true, s->stream)) ||
        (rc = s->mass.reserve(sizeof(double) * s->S, true, s->stream)) ||
        (rc = s->err.reserve(sizeof(int) * s->S, true, s->stream)) ||
        (rc = s->cp.reserve(sizeof(ColParams) * s->S, false, s->stream)) ||
        (rc = s->admit.reserve(sizeof(srv::AdmitItem) * s->S, false, s->stream)) ||
        (rc = s->mode.reserve(sizeof(int), true, s->stream)) ||
        (rc = s->tabs.reserve(sizeof(uint32_t) * 3 * s->S, true, s->stream)) ||
        (rc = s->plain.reserve(sizeof(srv::PlainTable) * s->S, false, s->stream))) {
    }
  }
  if (!rc) {
    if (hipHostMalloc(reinterpret_cast<void**>(&s->h_cp), sizeof(ColParams) * s->S) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&s->h_tabs), sizeof(uint32_t) * 3 * s->S) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&s->h_plain), sizeof(srv::PlainTable) * s->S) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&s->h_counters),
                      sizeof(unsigned long long) * lvl::kNumCounters * s->S) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&s->h_mass), sizeof(double) * s->S) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&s->h_err), sizeof(int) * s->S) != hipSuccess)
      rc = fail(AGP_ENOMEM, "agp_server_create: pinned host allocation failed");
  }
  if (!rc) {
    s->h_degree.resize(static_cast<size_t>(s->n));
    if (s->n > 0 && hipMemcpyAsync(s->h_degree.data(), g->degree, sizeof(int32_t) * s->n, hipMemcpyDeviceToHost,
                                   s->stream) != hipSuccess)
      rc = fail(AGP_EDEVICE, "agp_server_create: degree copy");
  }
  if (!rc && hipStreamSynchronize(s->stream) != hipSuccess) rc = fail(AGP_EDEVICE, "agp_server_create: sync");
  if (rc) {
    agp_server_destroy(s);
    return rc;
  }
  std::memset(static_cast<void*>(s->h_cp), 0, sizeof(ColParams) * s->S);
  s->worker = std::thread(agp::worker_main, s);
  *out = s;
  return AGP_OK;
}

int agp_submit(agp_server_t* s, const agp_query_t* q, uint64_t* ticket) {
  using namespace agp;
  if (!s || !ticket) return fail(AGP_EINVAL, "agp_submit: NULL server or ticket");
  int rc = validate(s, q);
  if (rc) return rc;
  QueryRec r;
  r.q = *q;
  rc = signal_of(q, &r);
  if (rc) return rc;
  r.q.x_idx = nullptr;  // copied into r.xi / r.xu
  r.q.x_val = nullptr;
  r.w.assign(q->w, q->w + q->L + 1);
  r.q.w = r.w.data();
  // level tables: Y_i = sum_{k=i..L} w_k from k = L down; rho, kappa as in
  // the batched path
  const int32_t L = q->L;
  std::vector<double> Y(static_cast<size_t>(L) + 2, 0.0);
  for (int32_t k = L; k >= 0; --k) Y[k] = Y[k + 1] + r.w[k];
  const double S = Y[0];
  r.rho.resize(L + 1);
  r.kappa.resize(L + 1);
  double est = 0.0, busiest = static_cast<double>(r.xi.size());
  for (int32_t i = 0; i <= L; ++i) {
    r.rho[i] = (Y[i] == 0.0) ? 0.0 : Y[i + 1] / Y[i];
    r.kappa[i] = (Y[i] == 0.0) ? 0.0 : (S * r.w[i]) / Y[i];
    if (i >= 1 && S > 0.0) {
      const double level = std::min((Y[i] / S) / q->eps, static_cast<double>(s->g->nnz));
      est += level;
      busiest = std::max(busiest, level);
    }
  }
  r.estimate = est;  // Theorem 3.3: E[pushes] <= (1/eps) sum_{i>=1} ||Y_i P^i x||_1
  // the first level touches at most the signal's neighbours (the estimate
  // above assumes ||P^i x||_1 <= ||x||_1, which D^-a A D^-b need not keep)
  double nb = 0.0;
  for (uint32_t u : r.xi) nb += static_cast<double>(s->h_degree[u]);
  busiest = std::max(busiest, std::min(nb, static_cast<double>(s->n)));
  // tables for the distinct nodes of the busiest level (a level touches at
  // most as many nodes as it pushes to), or direct tables of n entries;
  // AGP_SERVE_TABLE_ENTRIES forces a starting size (tests: tables that fill up)
  r.entries = srv::table_entries(busiest, s->n);
  // the bound holds for a column-stochastic P (a = 0, b = 1: PPR, heat
  // kernel, transition probabilities); other exponents (Katz's A, the
  // normalised GNN matrices) can grow the residue mass from level to level,
  // so their queries start with direct tables
  if (!(q->a == 0.0 && q->b == 1.0)) r.entries = static_cast<uint64_t>(s->n > 0 ? s->n : 1);
  if (const char* e = std::getenv("AGP_SERVE_TABLE_ENTRIES")) {
    const unsigned long long v = std::strtoull(e, nullptr, 10);
    if (v >= 1 && (v & (v - 1)) == 0) r.entries = std::min<uint64_t>(v, static_cast<uint64_t>(s->n));
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->worker_error) return fail(s->worker_error, "agp_submit: the server stopped after a device error");
  if (s->stop) return fail(AGP_EINVAL, "agp_submit: the server is shutting down");
  if (static_cast<int32_t>(s->pending.size()) >= s->cfg.queue_capacity)
    return fail(AGP_EBUSY, "agp_submit: queue full");
  const uint64_t t = s->next_ticket++;
  r.res.submit_ms = now_ms(s->t0);
  s->recs.emplace(t, std::move(r));
  s->recs[t].q.w = s->recs[t].w.data();
  s->pending.push_back(t);
  *ticket = t;
  s->cv.notify_all();
  return AGP_OK;
}

int agp_poll(agp_server_t* s, uint64_t ticket, agp_result_t* res) {
  using namespace agp;
  if (!s) return fail(AGP_EINVAL, "agp_poll: NULL server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->recs.find(ticket);
  if (it == s->recs.end()) return fail(AGP_ENOENT, "agp_poll: unknown ticket");
  if (!it->second.done) return AGP_PENDING;
  if (res) *res = it->second.res;
  s->recs.erase(it);
  return AGP_OK;
}

int agp_server_destroy(agp_server_t* s) {
  if (!s) return AGP_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (auto* b : {&s->keys, &s->vals, &s->F[0], &s->F[1], &s->counts, &s->counters, &s->mass, &s->err, &s->cp,
                  &s->admit, &s->mode, &s->tabs, &s->plain})
    b->release();
  if (s->h_cp) (void)hipHostFree(s->h_cp);
  if (s->h_tabs) (void)hipHostFree(s->h_tabs);
  if (s->h_plain) (void)hipHostFree(s->h_plain);
  if (s->h_counters) (void)hipHostFree(s->h_counters);
  if (s->h_mass) (void)hipHostFree(s->h_mass);
  if (s->h_err) (void)hipHostFree(s->h_err);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
  return AGP_OK;
}

}  // extern "C"
