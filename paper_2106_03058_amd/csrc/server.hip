// Continuous-batching query server: single-source proximity queries (PPR,
// heat kernel PageRank, Katz, L-hop transition probability) arrive at any
// time; each is admitted into a free slot (a column of the level kernel) and
// advances one level per step together with every other running query,
// whatever their levels, weights, exponents and thresholds.  The random
// streams are keyed by (seed, query_id) and the level sums are exact, so a
// query's result is the same alone, in a batch or in any mix.
//
// Slot c owns the n-vector cells c * n .. c * n + n - 1 of two accumulator
// arrays; the reserve goes straight to the query's output buffer.
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

namespace agp {
namespace srv {
struct AdmitItem {
  long long units;  // an initial residue (x value) in the column's units
  uint32_t node;
  uint32_t slot;
};
}  // namespace srv

namespace {

using namespace lvl;
using srv::AdmitItem;

// New slots: seed the residues of the signal's entries, append them to the
// frontier, clear the slots' counters (every item of a slot clears them).
__global__ void k_admit(const AdmitItem* __restrict__ items, int k, long long* __restrict__ acc, int64_t n,
                        uint64_t* __restrict__ F, unsigned long long* __restrict__ cnt,
                        unsigned long long* __restrict__ counters, double* __restrict__ mass,
                        int* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const AdmitItem it = items[i];
  acc[static_cast<size_t>(it.slot) * static_cast<size_t>(n) + it.node] = it.units;
  const unsigned long long pos = atomicAdd(cnt, 1ull);
  F[pos] = (static_cast<uint64_t>(it.node) << 32) | it.slot;
  for (int j = 0; j < kNumCounters; ++j) counters[static_cast<size_t>(it.slot) * kNumCounters + j] = 0;
  mass[it.slot] = 0.0;
  err[it.slot] = 0;
}

__global__ void k_zero_count(unsigned long long* c) { *c = 0; }

// binned steps: clear the record count and the push estimate of the step
__global__ void k_bin_reset(unsigned long long* rec_count, double* est) {
  *rec_count = 0;
  *est = 0.0;
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
  bool signed_x = false;             // some entry is negative
  double estimate = 0.0;
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
  // device state
  agp::DevBuf acc[2], F[2], counts, counters, mass, err, cp, admit, mode;
  int cur = 0;
  // binned aggregation of steps with many pushes (records, bucket state)
  bool binned = false;
  double bin_pushes = 0.0;  // estimated pushes from which a step is binned
  int bucket_shift = 0;
  long long nbins = 0;
  unsigned long long rec_cap = 0;
  agp::DevBuf rec[2], bins;
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
  std::vector<uint64_t> admitted;
  s->h_admit.clear();
  bool positive = true;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    for (int c = 0; c < s->S && !s->pending.empty(); ++c) {
      if (s->slot_ticket[c]) continue;
      QueryRec& r = s->recs[s->pending.front()];
      const bool idle = s->running_estimate == 0.0;
      if (s->cfg.work_budget > 0.0 && !idle && s->running_estimate + r.estimate > s->cfg.work_budget) break;
      const uint64_t t = s->pending.front();
      s->pending.pop_front();
      r.slot = c;
      r.level = 0;
      r.fresh = true;
      r.res.start_ms = now_ms(s->t0);
      s->slot_ticket[c] = t;
      s->running_estimate += r.estimate;
      admitted.push_back(t);
    }
    // per-slot parameters of this step
    for (int c = 0; c < s->S; ++c) {
      ColParams& p = s->h_cp[c];
      const uint64_t t = s->slot_ticket[c];
      if (!t) {
        p.flags = kDrop;
        continue;
      }
      QueryRec& r = s->recs[t];
      const int i = r.level;
      if (r.signed_x) positive = false;
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
      p.flags = (i == r.q.L ? kLastLevel : 0) | (r.q.a == 0.0 ? kAZero : 0) | (r.failed ? kDrop : 0);
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
  long long* acc[2] = {s->acc[0].as<long long>(), s->acc[1].as<long long>()};
  uint64_t* F[2] = {s->F[0].as<uint64_t>(), s->F[1].as<uint64_t>()};
  AGP_HIP(hipMemcpyAsync(s->cp.ptr, s->h_cp, sizeof(ColParams) * s->S, hipMemcpyHostToDevice, st));
  const int nadmit = static_cast<int>(s->h_admit.size());
  if (nadmit) {
    if (int rc = s->admit.reserve(sizeof(srv::AdmitItem) * static_cast<size_t>(nadmit), false, st)) return rc;
    AGP_HIP(hipMemcpyAsync(s->admit.ptr, s->h_admit.data(), sizeof(srv::AdmitItem) * nadmit, hipMemcpyHostToDevice,
                           st));
    k_admit<<<grid_for(nadmit, 64), 64, 0, st>>>(s->admit.as<srv::AdmitItem>(), nadmit, acc[cur], s->n, F[cur],
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
  A.sc = s->n;
  A.level = 0;
  A.fin = F[cur];
  A.cnt_in = counts + cur;
  A.fout = F[nxt];
  A.cnt_out = counts + nxt;
  A.counters = s->counters.as<unsigned long long>();
  A.mass = s->mass.as<double>();
  A.err = s->err.as<int>();
  A.positive = positive ? 1 : 0;  // first-touch appends need residues that cannot cancel
  A.dense_cut = std::max<unsigned long long>(1ull, static_cast<unsigned long long>(s->n) * s->S / 32);
  A.mode_out = s->mode.as<int>();
  A.rec = nullptr;
  A.rec_count = nullptr;
  A.rec_cap = 0;
  A.bucket_count = nullptr;
  A.bin_est = nullptr;
  unsigned int* bucket_count = nullptr;
  unsigned long long *bucket_off = nullptr, *cursor = nullptr, *rec_count = nullptr;
  unsigned long long *bin_count = nullptr, *bin_off = nullptr, *bin_cur = nullptr;
  if (s->binned) {  // records when the step's estimated pushes reach bin_pushes
    bucket_count = s->bins.as<unsigned int>();
    bucket_off = reinterpret_cast<unsigned long long*>(bucket_count + kBuckets);
    cursor = bucket_off + kBuckets + 1;
    rec_count = cursor + kBuckets;
    double* est = reinterpret_cast<double*>(rec_count + 1);
    bin_count = reinterpret_cast<unsigned long long*>(est + 1);
    bin_off = bin_count + s->nbins;
    bin_cur = bin_off + s->nbins + 1;
    A.det_bins = reinterpret_cast<uint8_t*>(bin_cur + s->nbins);  // any stale value is safe
    A.rec = s->rec[0].as<uint32_t>();
    A.rec_count = rec_count;
    A.rec_cap = s->rec_cap;
    A.bucket_count = bucket_count;
    A.bucket_shift = s->bucket_shift;
    A.bin_est = est;
    A.bin_pushes = s->bin_pushes;
    k_bin_reset<<<1, 1, 0, st>>>(rec_count, est);
    k_estimate<float, false><<<1024, kThreads, 0, st>>>(A, nullptr, acc[cur], est);
  }
  k_level<float, false, true><<<kLevelBlocks, kThreads, 0, st>>>(A, nullptr, acc[cur], acc[nxt]);
  if (s->binned) {
    uint32_t* r0 = s->rec[0].as<uint32_t>();
    uint32_t* r1 = s->rec[1].as<uint32_t>();
    int* mode = s->mode.as<int>();
    k_bins_scan<<<1, kBuckets, 0, st>>>(bucket_count, bucket_off, cursor, rec_count, s->rec_cap, mode);
    k_apply_overflow<<<2048, kThreads, 0, st>>>(A, acc[nxt], mode);
    k_partition<<<1024, kReduceThreads, 0, st>>>(r0, rec_count, cursor, r1, mode, s->bucket_shift);
    k_bin_count<<<2048, kReduceThreads, 0, st>>>(r1, rec_count, bin_count, mode, s->bucket_shift);
    k_bin_scan<<<1, 1024, 0, st>>>(bin_count, s->nbins, bin_off, bin_cur, mode);
    k_bin_scatter<<<2048, kReduceThreads, 0, st>>>(r1, rec_count, bin_cur, r0, mode, s->bucket_shift);
    k_bin_sum<<<static_cast<unsigned>(s->nbins), kSumThreads, 0, st>>>(
        r0, bin_off, A.cp, 1ll, (long long)s->n, static_cast<unsigned long long>(s->n) * s->S, acc[nxt], F[nxt],
        counts + nxt, mode, A.det_bins);
  }
  k_compact<<<grid_for(s->n * (int64_t)s->S, kThreads, 8192), kThreads, 0, st>>>(
      NonZeroCell<float>{acc[nxt]}, s->n, s->S, 1ll, (long long)s->n, F[nxt], counts + nxt, s->mode.as<int>());
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
  for (int c = 0; c < s->S; ++c) {
    const uint64_t t = s->slot_ticket[c];
    if (!t) continue;
    QueryRec& r = s->recs[t];
    const bool overflow = s->h_err[c] != 0 || !(s->h_mass[c] < 0x1p61);
    bool finish = false;
    if (r.failed) {
      finish = true;  // its residues were dropped in this step
    } else if (overflow) {
      r.failed = true;  // drop its remaining residues in the next step
    } else if (r.level == r.q.L) {
      finish = true;
    } else {
      ++r.level;
    }
    if (finish) {
      const unsigned long long* k = s->h_counters + static_cast<size_t>(c) * kNumCounters;
      r.res.status = r.failed ? AGP_ERANGE : AGP_OK;
      r.res.levels = r.q.L;
      r.res.frontier = k[0];
      r.res.pushes = k[2] + k[4];
      r.res.candidates = k[3];
      r.res.end_ms = t_end;
      r.done = true;
      s->slot_ticket[c] = 0;
      s->running_estimate -= r.estimate;
      if (s->running_estimate < 1e-9) s->running_estimate = 0.0;
    }
  }
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
  if (!g || !cfg || cfg->max_slots < 1 || cfg->queue_capacity < 1 || !(cfg->work_budget >= 0.0))
    return fail(AGP_EINVAL, "agp_server_create: need a graph, max_slots >= 1, queue_capacity >= 1");
  agp_server* s = new (std::nothrow) agp_server();
  if (!s) return fail(AGP_ENOMEM, "agp_server_create: host allocation failed");
  s->g = const_cast<agp_graph*>(g);
  s->cfg = *cfg;
  s->n = g->n;
  s->S = cfg->max_slots;
  s->t0 = std::chrono::steady_clock::now();
  s->slot_ticket.assign(s->S, 0);
  const size_t cells = static_cast<size_t>(s->n) * static_cast<size_t>(s->S);
  int rc = AGP_OK;
  hipError_t e = hipStreamCreate(&s->stream);
  if (e != hipSuccess) rc = fail(AGP_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
  if (!rc) {
    if ((rc = s->acc[0].reserve(cells * sizeof(long long), true, s->stream)) ||
        (rc = s->acc[1].reserve(cells * sizeof(long long), true, s->stream)) ||
        (rc = s->F[0].reserve(cells * sizeof(uint64_t), false, s->stream)) ||
        (rc = s->F[1].reserve(cells * sizeof(uint64_t), false, s->stream)) ||
        (rc = s->counts.reserve(2 * sizeof(unsigned long long), true, s->stream)) ||
        (rc = s->counters.reserve(sizeof(unsigned long long) * lvl::kNumCounters * s->S, true, s->stream)) ||
        (rc = s->mass.reserve(sizeof(double) * s->S, true, s->stream)) ||
        (rc = s->err.reserve(sizeof(int) * s->S, true, s->stream)) ||
        (rc = s->cp.reserve(sizeof(ColParams) * s->S, false, s->stream)) ||
        (rc = s->admit.reserve(sizeof(srv::AdmitItem) * s->S, false, s->stream)) ||
        (rc = s->mode.reserve(sizeof(int), true, s->stream))) {
    }
  }
  // Binned aggregation for steps with many pushes (cells addressable in 31
  // bits); AGP_AGGREGATION=atomic turns it off, =binned bins every step.
  if (!rc && cells > 0 && cells < (1ull << 31) && s->S <= lvl::kMaxBinnedC) {
    const char* agg = std::getenv("AGP_AGGREGATION");
    if (!(agg && std::strcmp(agg, "atomic") == 0)) {
      // a binned step costs about one pass over the cells; the server's
      // sparse steps run returning atomics, so records pay off from n S / 64
      s->bin_pushes = (agg && std::strcmp(agg, "binned") == 0) ? 0.0 : static_cast<double>(cells) / 64.0;
      int shift = lvl::kBinLog2;
      while ((static_cast<unsigned long long>(cells) - 1ull) >> shift >= (unsigned long long)lvl::kBuckets) ++shift;
      s->bucket_shift = shift;
      s->nbins = static_cast<long long>((static_cast<unsigned long long>(cells) - 1ull) >> lvl::kBinLog2) + 1;
      size_t free_b = 0, total_b = 0;
      (void)hipMemGetInfo(&free_b, &total_b);
      s->rec_cap = std::max<unsigned long long>(1ull << 20, 4ull * cells);
      s->rec_cap = std::min<unsigned long long>(s->rec_cap, std::max<unsigned long long>(1ull << 20, free_b / 64));
      if (s->rec[0].reserve(s->rec_cap * sizeof(uint32_t), false, s->stream) ||
          s->rec[1].reserve(s->rec_cap * sizeof(uint32_t), false, s->stream) ||
          s->bins.reserve(sizeof(unsigned int) * lvl::kBuckets + sizeof(unsigned long long) * (2 * lvl::kBuckets + 2) +
                              sizeof(double) + sizeof(unsigned long long) * (3 * s->nbins + 1) +
                              static_cast<size_t>(s->nbins), true, s->stream)) {
        s->rec[0].release();  // not enough memory for the records: atomics only
        s->rec[1].release();
        s->bins.release();
        (void)hipGetLastError();
      } else {
        s->binned = true;
      }
    }
  }
  if (!rc) {
    if (hipHostMalloc(reinterpret_cast<void**>(&s->h_cp), sizeof(ColParams) * s->S) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&s->h_counters),
                      sizeof(unsigned long long) * lvl::kNumCounters * s->S) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&s->h_mass), sizeof(double) * s->S) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&s->h_err), sizeof(int) * s->S) != hipSuccess)
      rc = fail(AGP_ENOMEM, "agp_server_create: pinned host allocation failed");
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
  double est = 0.0;
  for (int32_t i = 0; i <= L; ++i) {
    r.rho[i] = (Y[i] == 0.0) ? 0.0 : Y[i + 1] / Y[i];
    r.kappa[i] = (Y[i] == 0.0) ? 0.0 : (S * r.w[i]) / Y[i];
    if (i >= 1 && S > 0.0) est += std::min((Y[i] / S) / q->eps, static_cast<double>(s->g->nnz));
  }
  r.estimate = est;  // Theorem 3.3: E[pushes] <= (1/eps) sum_{i>=1} ||Y_i P^i x||_1
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
  for (auto* b : {&s->acc[0], &s->acc[1], &s->F[0], &s->F[1], &s->counts, &s->counters, &s->mass, &s->err,
                  &s->cp, &s->admit, &s->mode, &s->rec[0], &s->rec[1], &s->bins})
    b->release();
  if (s->h_cp) (void)hipHostFree(s->h_cp);
  if (s->h_counters) (void)hipHostFree(s->h_counters);
  if (s->h_mass) (void)hipHostFree(s->h_mass);
  if (s->h_err) (void)hipHostFree(s->h_err);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
  return AGP_OK;
}

}  // extern "C"
