// btdf_noalloc.hip -- the entry point that allocates nothing: the corrected
// marker velocity of btdf_marker_velocity (eqs 11, 12; at rest markers its
// root mean square is the boundary error of eq 45), with its only scratch,
// the per-marker results staged on the device before they are copied to the
// caller's host arrays, in a fixed array of device memory.

#include <hip/hip_runtime.h>

#include <mutex>

#include "btdf_internal.h"

using namespace btdf;
using namespace btdf::host;

namespace {

// The staging array: ux of every marker, then uy. One copy per GPU, at its
// own device address, held until the process ends. Host code never passes
// its name to a kernel or a copy (on the host it is a stand-in, not a device
// address); it uses the address hipGetSymbolAddress returns for the current
// device.
static __device__ __align__(256) double scratch[2 * BTDF_NOALLOC_MAX_MARKERS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// the current device's address of the staging array, looked up on its first
// use on that device
int scratch_ptr(double **out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(BTDF_EDEVICE, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(BTDF_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double *>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return ok();
}

}  // namespace

extern "C" {

int btdf_marker_velocity_noalloc(btdf_t *h, double *ux, double *uy) {
  return guard([&]() -> int {
    if (!h || !ux || !uy) return fail(BTDF_EINVAL, "NULL argument");
    if (h->owner) return fail(BTDF_ESTATE, "this handle is a case of a batch");
    const int nm = h->nm();
    if (nm > BTDF_NOALLOC_MAX_MARKERS)
      return fail(BTDF_EINVAL, "%d markers: btdf_marker_velocity_noalloc takes at most %d", nm,
                  BTDF_NOALLOC_MAX_MARKERS);
    // the marker arrays and tile lists on the device must be those of the
    // last step, in the current layout
    if (!h->stepped || !h->layout_ok || !h->device_ok || !h->ws)
      return fail(BTDF_ESTATE, "no step since the state, the bodies or the layout last changed");
    if (nm == 0) return ok();
    if (h->any_moving())
      return fail(BTDF_ESTATE, "moving bodies: the markers have moved on since the last step's forces");
    double *buf = nullptr;
    int rc = scratch_ptr(&buf);
    if (rc) return rc;
    const LbmParams p = make_params(h);
    const IbParams ib = make_ib(h);
    hipError_t e = launch_marker_velocity_tiles(h->prec, h->ws + h->off_pop[h->cur], p, ib, h->tile_x, h->tile_y,
                                                buf, buf + nm, h->stream);
    const size_t bytes = (size_t)nm * sizeof(double);
    if (e == hipSuccess) e = hipMemcpyAsync(ux, buf, bytes, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(uy, buf + nm, bytes, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(BTDF_EDEVICE, "marker velocity: %s", hipGetErrorString(e));
    return ok();
  });
}

}  // extern "C"
