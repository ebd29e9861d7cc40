// rrt_relight without caller memory: the workspace of the relight (source
// map and staging buffer) lives in a file-scope device array, for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).  Nothing here allocates:
// the array is part of the code object and each GPU holds its own copy from
// module load until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rrt_internal.h"

namespace rrt {
namespace {

constexpr size_t kScratchBytes = size_t(RRT_NOALLOC_SCRATCH_BYTES);

// The host name of this array is a stand-in, not a device address: host
// code only ever uses the per-device address from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current.
int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(RRT_ERR_DEVICE, "relight_noalloc: hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(RRT_ERR_UNSUPPORTED, "relight_noalloc: device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(RRT_ERR_DEVICE, "relight_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
    if (reinterpret_cast<uintptr_t>(p) & 255u)
      return fail(RRT_ERR_DEVICE, "relight_noalloc: scratch not 256-byte aligned");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return RRT_OK;
}

}  // namespace
}  // namespace rrt

using namespace rrt;

extern "C" int rrt_relight_noalloc(const rrt_light* L, const rrt_rotations* R,
                                   const rrt_transport* T, float* radiance, unsigned flags,
                                   void* stream) {
  // every argument check before the first HIP call
  int st = validate_relight(L, R, T);
  if (st) return st;
  st = check_relight_flags(L, flags, T);
  if (st) return st;
  const size_t need = relight_ws(L->n).total;
  if (need > kScratchBytes)
    return fail(RRT_ERR_UNSUPPORTED,
                "relight_noalloc: n=%d needs %zu bytes of scratch, more than the %zu held "
                "(n <= 256)", L->n, need, kScratchBytes);
  if (T->nvert > 0 && !radiance) return fail(RRT_ERR_INVALID, "relight_noalloc: null radiance");
  void* ws = nullptr;
  st = scratch_address(&ws);
  if (st) return st;
  // the staging part is cleared by a fill kernel inside, the source map is
  // written whole: nothing depends on what an earlier call left behind
  return rrt_relight(L, R, T, radiance, flags, ws, kScratchBytes, stream);
}
