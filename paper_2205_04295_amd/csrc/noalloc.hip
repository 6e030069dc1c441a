// mrpie_rpie_noalloc: the sweep of mrpie_rpie with its workspace in a
// static device array of this file, for callers that cannot allocate device
// memory (code under graph capture, serving loops, harnesses that forbid
// hipMalloc).  The kernels are mrpie_rpie's; only where the scratch comes
// from differs.
#include <mutex>

#include "sweep.hpp"

namespace mrpie {
namespace {

// Largest workspace the static array serves: the plain sweep of a 256^2
// probe with up to 8 modes for up to 100 iterations per call (or 3 modes
// for up to ~550), and small refining problems.  Every GPU the library runs
// on holds one copy until the process ends.
constexpr size_t kScratchBytes = MRPIE_NOALLOC_MAX_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

// Host code sees `scratch` only as a host-side stand-in: its device address
// (a different one on every GPU) comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that address is passed on.
constexpr int kMaxDevices = 16;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

int scratch_ptr(void** out) {
  int dev = 0;
  MRPIE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MRPIE_EDEVICE, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(MRPIE_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return MRPIE_OK;
}

}  // namespace
}  // namespace mrpie

using namespace mrpie;

extern "C" {

int mrpie_rpie_noalloc(const mrpie_problem* pb, const mrpie_params* pr, void* obj, void* probe, float* pos,
                       float* adam, const float* intens, float* err_out, int32_t* status, void* stream) {
  int rc = mrpie_validate(pb, pr);
  if (rc) return rc;
  if (!obj || !probe || !pos || !intens) return fail(MRPIE_EINVAL, "null array pointer");
  if (pr->refine && !adam) return fail(MRPIE_EINVAL, "adam state is NULL with refine = 1");
  const size_t need = rpie_ws_total(pb, pr);
  if (need > kScratchBytes)
    return fail(MRPIE_EWORKSPACE, "problem needs %zu bytes of scratch, above the static maximum of %zu "
                                  "(use mrpie_rpie with a workspace)", need, kScratchBytes);
  void* ws = nullptr;
  rc = scratch_ptr(&ws);
  if (rc) return rc;
  return mrpie_rpie(pb, pr, obj, probe, pos, adam, intens, err_out, status, ws, kScratchBytes, stream);
}

}  // extern "C"
