// Allocation-free solve: opdhg_solve on a static device scratch.
//
// The scratch is a file-scope __device__ array; each device that loads the
// library holds its own copy for the life of the process. In host code the
// array's name stands for a host-side shadow, not a device address, so its
// device address is looked up once per device (hipGetSymbolAddress, with the
// device current) and only that address is ever handed to the kernels. The
// solve runs its launch group in direct mode: no graph, no streams, events
// or pinned memory of its own, so nothing is allocated during the call.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "opdhg.h"
#include "opdhg_host.h"

namespace opdhg {
namespace {

constexpr size_t kScratchBytes = OPDHG_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

struct DeviceScratch {
  std::mutex call;      // held for a whole call: calls on one device run one at a time
  void* ptr = nullptr;  // the device address of `scratch` on this device
};

std::mutex g_setup;
DeviceScratch g_dev[kMaxDevices];

// The current device's scratch, looked up on the first call on the device.
int scratch_for_current_device(DeviceScratch** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(OPDHG_ERR_DEVICE, "device index " + std::to_string(dev) + " out of range");
  std::lock_guard<std::mutex> lock(g_setup);
  DeviceScratch& d = g_dev[dev];
  if (!d.ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(OPDHG_ERR_DEVICE, "hipGetSymbolAddress(scratch) gave a null address");
    d.ptr = p;
  }
  *out = &d;
  return OPDHG_OK;
}

}  // namespace
}  // namespace opdhg

using namespace opdhg;

extern "C" int opdhg_solve_noalloc(const opdhg_lp* lp, const opdhg_params* p, void* hip_stream,
                                   double* x_out, double* y_out, opdhg_result* res) {
  DeviceScratch* d = nullptr;
  int rc = scratch_for_current_device(&d);
  if (rc) return rc;
  std::lock_guard<std::mutex> lock(d->call);
  opdhg_session* s = nullptr;
  size_t need = 0;
  rc = session_create(lp, p, d->ptr, kScratchBytes, hip_stream, true, &s, &need);
  if (rc == OPDHG_ERR_WORKSPACE_TOO_SMALL)
    return fail(rc, "opdhg_solve_noalloc: the LP needs " + std::to_string(need) +
                        " bytes of device memory; the static scratch holds " +
                        std::to_string(kScratchBytes) +
                        " (opdhg_solve takes a workspace of any size)");
  if (rc) return rc;
  rc = opdhg_session_run(s, -1);
  if (!rc) rc = opdhg_session_result(s, x_out, y_out, res);
  opdhg_session_destroy(s);
  return rc;
}
