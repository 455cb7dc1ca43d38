// rts_solve_static: the forward solve for callers that cannot allocate device
// memory (code under stream capture, serving loops, harnesses that forbid
// hipMalloc).  Its workspace is `scratch`, a fixed device array of this
// library; each GPU the library runs on holds one copy until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/rts.h"

namespace rts {
int static_solve_check(void* plan, int nbox, const rts_inputs* in, const rts_outputs* out,
                       size_t cap);
int static_solve(void* plan, int nbox, const rts_inputs* in, const rts_outputs* out, void* ws,
                 size_t cap, void* stream);
int static_fail(hipError_t e, const char* where);
int static_scratch(void** out);
}  // namespace rts

// The workspace of rts_solve_static.  In host code this name is only a
// stand-in for the device array: host code uses the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[RTS_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

}  // namespace

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
int rts::static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return rts::static_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return RTS_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return rts::static_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return RTS_E_HIP;
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  return RTS_OK;
}

extern "C" int rts_solve_static(void* plan, int32_t nbox, const rts_inputs* in,
                                const rts_outputs* out, void* hip_stream) {
  // a plan whose workspace exceeds the array is refused before any device call
  int rc = rts::static_solve_check(plan, nbox, in, out, RTS_STATIC_SCRATCH_BYTES);
  if (rc) return rc;
  void* ws = nullptr;
  if ((rc = rts::static_scratch(&ws))) return rc;
  return rts::static_solve(plan, nbox, in, out, ws, RTS_STATIC_SCRATCH_BYTES, hip_stream);
}
