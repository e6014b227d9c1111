// Error reporting, device buffers and weight sequences of libagp.
#include <cmath>
#include <cstring>
#include <vector>

#include "agp_internal.h"

namespace agp {

static thread_local std::string t_last_error;

int fail(int code, const std::string& msg) {
  t_last_error = msg;
  return code;
}

int DevBuf::reserve(size_t want, bool zero, hipStream_t s) {
  if (want <= bytes && ptr) return AGP_OK;
  if (borrowed)  // a fixed region: it cannot grow
    return fail(AGP_ENOMEM, "scratch region of " + std::to_string(bytes) + " bytes, " + std::to_string(want) +
                                " needed");
  release();
  if (want == 0) want = 8;
  hipError_t e = hipMalloc(&ptr, want);
  if (e != hipSuccess) {
    ptr = nullptr;
    bytes = 0;
    (void)hipGetLastError();
    return fail(AGP_ENOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
  }
  bytes = want;
  if (zero) AGP_HIP(hipMemsetAsync(ptr, 0, want, s));
  return AGP_OK;
}

void DevBuf::release() {
  if (ptr && !borrowed) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

int Scratch::ensure_events() {
  for (auto& e : events)
    if (!e) AGP_HIP(hipEventCreate(&e));
  return AGP_OK;
}

void Scratch::release() {
  for (auto& e : events)
    if (e) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
  for (auto& b : acc) b.release();
  for (auto& b : frontier) b.release();
  counts.release();
  counters.release();
  colparams.release();
  partial.release();
  flags.release();
  levelinfo.release();
  rec[0].release();
  rec[1].release();
  big.release();
  nodefac.release();
  nodefac_a = nodefac_b = -1.0;
  arcfac.release();
  arcfac_a = -1.0;
  sweep.release();
  sweep_items.release();
  sweep_nitems = -1;
  dense_items.release();
  dense_rows.release();
  dense_nitems = -1;
  dense_nrows = 0;
  bins.release();
}

// d^-e on the host in binary64: exact IEEE forms 1, 1/sqrt(d), 1/d for the
// exponents 0, 1/2 and 1 (correctly rounded sqrt and division), pow otherwise.
static double degree_power(int64_t d, double e) {
  if (d <= 0) return 0.0;
  if (e == 0.0) return 1.0;
  if (e == 0.5) return 1.0 / std::sqrt(static_cast<double>(d));
  if (e == 1.0) return 1.0 / static_cast<double>(d);
  return std::pow(static_cast<double>(d), -e);
}

int pow_table(agp_graph* g, double e, const double** out, bool may_alloc) {
  auto it = g->pow_tables.find(e);
  if (it != g->pow_tables.end()) {
    *out = it->second;
    return AGP_OK;
  }
  if (!may_alloc)
    return fail(AGP_EINVAL, "no degree-power table for exponent " + std::to_string(e) +
                                " on this graph yet: an allocating call with it makes one");
  const size_t cnt = static_cast<size_t>(g->max_fdeg) + 1;
  std::vector<double> host(cnt);
  for (size_t d = 0; d < cnt; ++d) host[d] = degree_power(static_cast<int64_t>(d), e);
  double* dev = nullptr;
  AGP_HIP(hipMalloc(&dev, cnt * sizeof(double)));
  hipError_t err = hipMemcpy(dev, host.data(), cnt * sizeof(double), hipMemcpyHostToDevice);
  if (err != hipSuccess) {
    (void)hipFree(dev);
    return fail(AGP_EDEVICE, std::string("table upload: ") + hipGetErrorString(err));
  }
  g->pow_tables[e] = dev;
  *out = dev;
  return AGP_OK;
}

}  // namespace agp

void agp_graph::drop_loops() {
  for (auto& kv : loops) (void)hipGraphExecDestroy(kv.second);
  loops.clear();
}

extern "C" {

const char* agp_last_error(void) { return agp::t_last_error.c_str(); }

int agp_weights_ppr(double alpha, int32_t L, double* w) {
  if (!w || L < 0 || L > AGP_MAX_LEVELS || !(alpha > 0.0 && alpha <= 1.0))
    return agp::fail(AGP_EINVAL, "agp_weights_ppr: need 0 < alpha <= 1, 0 <= L <= 255");
  double v = alpha;
  for (int32_t i = 0; i <= L; ++i) {
    w[i] = v;
    v *= 1.0 - alpha;
  }
  return AGP_OK;
}

int agp_weights_hkpr(double t, int32_t L, double* w) {
  if (!w || L < 0 || L > AGP_MAX_LEVELS || !(t >= 0.0 && std::isfinite(t)))
    return agp::fail(AGP_EINVAL, "agp_weights_hkpr: need t >= 0, 0 <= L <= 255");
  double v = std::exp(-t);
  for (int32_t i = 0; i <= L; ++i) {
    w[i] = v;
    v = v * t / static_cast<double>(i + 1);
  }
  return AGP_OK;
}

int agp_weights_katz(double beta, int32_t L, double* w) {
  if (!w || L < 0 || L > AGP_MAX_LEVELS || !(beta >= 0.0 && std::isfinite(beta)))
    return agp::fail(AGP_EINVAL, "agp_weights_katz: need beta >= 0, 0 <= L <= 255");
  double v = 1.0;
  for (int32_t i = 0; i <= L; ++i) {
    w[i] = v;
    v *= beta;
  }
  return AGP_OK;
}

int agp_weights_tp(int32_t L, double* w) {
  if (!w || L < 0 || L > AGP_MAX_LEVELS)
    return agp::fail(AGP_EINVAL, "agp_weights_tp: need 0 <= L <= 255");
  for (int32_t i = 0; i < L; ++i) w[i] = 0.0;
  w[L] = 1.0;
  return AGP_OK;
}

}  // extern "C"
