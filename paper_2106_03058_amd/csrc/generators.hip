// The device random number generators evaluated on caller-supplied inputs,
// so that known-answer vectors pin exactly the functions the level kernels
// use (agp_device.h): Philox4x32-10 (Salmon et al., SC'11), which draws every
// random decision of the subset sampling, and the splitmix64 finaliser behind
// the per-level frontier hash.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>

#include "agp_device.h"
#include "agp_internal.h"

namespace agp {
namespace {

__global__ void k_philox_blocks(int64_t count, const uint32_t* __restrict__ ctr, const uint32_t* __restrict__ key,
                                uint32_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= count) return;
  const U4 o = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], key[2 * i], key[2 * i + 1]);
  out[4 * i] = o.x;
  out[4 * i + 1] = o.y;
  out[4 * i + 2] = o.z;
  out[4 * i + 3] = o.w;
}

__global__ void k_splitmix(int64_t count, const uint64_t* __restrict__ in, uint64_t* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) out[i] = splitmix64(in[i]);
}

// Copies `bytes_in` host bytes to a temporary device buffer, runs `launch`
// on it and copies `bytes_out` bytes back (synchronous, default stream).
template <typename F>
int run_on_device(const char* fn, const void* in, size_t bytes_in, void* out, size_t bytes_out, F launch) {
  DevBuf din, dout;
  int rc;
  if ((rc = din.reserve(bytes_in, false, nullptr)) || (rc = dout.reserve(bytes_out, false, nullptr))) {
    din.release();
    dout.release();
    return rc;
  }
  hipError_t e = hipMemcpy(din.ptr, in, bytes_in, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    launch(din.ptr, dout.ptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(out, dout.ptr, bytes_out, hipMemcpyDeviceToHost);
  din.release();
  dout.release();
  if (e != hipSuccess) return fail(AGP_EDEVICE, std::string(fn) + ": " + hipGetErrorString(e));
  return AGP_OK;
}

}  // namespace
}  // namespace agp

extern "C" {

int agp_device_philox4x32_10(int64_t count, const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  using namespace agp;
  if (count < 0 || (count > 0 && (!ctr || !key || !out)))
    return fail(AGP_EINVAL, "agp_device_philox4x32_10: bad count or NULL array");
  if (count == 0) return AGP_OK;
  // inputs packed as [ctr (4 words) x count | key (2 words) x count]
  std::string packed(static_cast<size_t>(count) * 24, '\0');
  std::memcpy(&packed[0], ctr, static_cast<size_t>(count) * 16);
  std::memcpy(&packed[static_cast<size_t>(count) * 16], key, static_cast<size_t>(count) * 8);
  return run_on_device("agp_device_philox4x32_10", packed.data(), packed.size(), out,
                       static_cast<size_t>(count) * 16, [count](void* din, void* dout) {
                         const uint32_t* dc = static_cast<const uint32_t*>(din);
                         k_philox_blocks<<<static_cast<unsigned>((count + 255) / 256), 256>>>(
                             count, dc, dc + 4 * count, static_cast<uint32_t*>(dout));
                       });
}

int agp_device_splitmix64(int64_t count, const uint64_t* in, uint64_t* out) {
  using namespace agp;
  if (count < 0 || (count > 0 && (!in || !out)))
    return fail(AGP_EINVAL, "agp_device_splitmix64: bad count or NULL array");
  if (count == 0) return AGP_OK;
  return run_on_device("agp_device_splitmix64", in, static_cast<size_t>(count) * 8, out,
                       static_cast<size_t>(count) * 8, [count](void* din, void* dout) {
                         k_splitmix<<<static_cast<unsigned>((count + 255) / 256), 256>>>(
                             count, static_cast<const uint64_t*>(din), static_cast<uint64_t*>(dout));
                       });
}

}  // extern "C"
