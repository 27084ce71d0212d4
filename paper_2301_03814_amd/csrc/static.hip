// swkb_propagate_static: a plan and a propagation in one call, with the
// plan's workspace in a static device array instead of caller memory, for
// callers that cannot allocate device memory.  Host code only; every kernel
// is the one swkb_propagate launches.
#include <mutex>
#include <string>
#include <vector>

#include "swkb_internal.h"

namespace {

// The workspace of one call (every call on a device shares its device's
// copy).  In host code `scratch` names a host-side stand-in: its device
// address comes from hipGetSymbolAddress, per device.
constexpr size_t kStaticBytes = (size_t)SWKB_STATIC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

struct DeviceScratch {
  bool ready = false;
  void* ptr = nullptr;       // device address of this device's scratch
  hipEvent_t done = nullptr; // end of the last call's work on this device
};

std::mutex g_mu;                   // one call at a time enqueues work into scratch
std::vector<DeviceScratch> g_dev;  // by device ordinal

// Address of the current device's array and its ordering event, looked up
// (with that device current) on the first call there.
swkb_status device_scratch(DeviceScratch** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    swkb::set_error(std::string("swkb_propagate_static: hipGetDevice: ") + hipGetErrorString(e));
    return SWKB_ERR_DEVICE;
  }
  if ((int)g_dev.size() <= dev) g_dev.resize(dev + 1);
  DeviceScratch& d = g_dev[dev];
  if (!d.ready) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      swkb::set_error(std::string("swkb_propagate_static: hipGetSymbolAddress: ") + hipGetErrorString(e));
      return SWKB_ERR_DEVICE;
    }
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      swkb::set_error(std::string("swkb_propagate_static: hipEventCreate: ") + hipGetErrorString(e));
      return SWKB_ERR_DEVICE;
    }
    d.ptr = ptr;
    d.done = ev;
    d.ready = true;
  }
  *out = &d;
  return SWKB_OK;
}

}  // namespace

extern "C" {

swkb_status swkb_propagate_static(const swkb_params* p, const void* u_in, int32_t q_begin, int32_t q_end,
                                  void* history, void* u_out, void* hip_stream) {
  if (!p || !u_in) {
    swkb::set_error("swkb_propagate_static: params or u_in is NULL");
    return SWKB_ERR_ARG;
  }
  const size_t need = swkb_workspace_bytes(p);
  if (need == 0) {
    // the message of the failed validation, as swkb_plan gives it
    swkb_plan_t none = nullptr;
    return swkb::plan_impl(p, nullptr, 0, nullptr, false, &none);
  }
  if (need > kStaticBytes) {
    swkb::set_error("swkb_propagate_static: the problem needs " + std::to_string(need) +
                    " bytes of workspace, more than the static workspace of " + std::to_string(kStaticBytes) +
                    " bytes (SWKB_STATIC_WORKSPACE_BYTES); use swkb_plan with a workspace of that size");
    return SWKB_ERR_NOMEM;
  }
  if (q_begin < 0 || q_end <= q_begin || q_end > p->n_screens) {
    swkb::set_error("swkb_propagate_static: need 0 <= q_begin < q_end <= n_screens");
    return SWKB_ERR_ARG;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceScratch* d = nullptr;
  swkb_status s = device_scratch(&d);
  if (s != SWKB_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  // the previous call's kernels may still read the array: start after them
  hipError_t e = hipStreamWaitEvent(st, d->done, 0);
  if (e != hipSuccess) {
    swkb::set_error(std::string("swkb_propagate_static: stream wait: ") + hipGetErrorString(e));
    return SWKB_ERR_DEVICE;
  }
  swkb_plan_t pl = nullptr;
  s = swkb::plan_impl(p, d->ptr, kStaticBytes, st, false, &pl);
  if (s == SWKB_OK) s = swkb::propagate_impl(pl, u_in, q_begin, q_end, history, st);
  if (s == SWKB_OK && u_out) {
    e = hipMemcpyAsync(u_out, pl->u, sizeof(double2) * (size_t)p->n_z, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) {
      swkb::set_error(std::string("swkb_propagate_static: field copy: ") + hipGetErrorString(e));
      s = SWKB_ERR_DEVICE;
    }
  }
  // the next call waits for this one's kernels (also after a failure here)
  e = hipEventRecord(d->done, st);
  if (pl) swkb_destroy(pl);  // host handle only: no device memory is freed
  if (s == SWKB_OK && e != hipSuccess) {
    swkb::set_error(std::string("swkb_propagate_static: event record: ") + hipGetErrorString(e));
    s = SWKB_ERR_DEVICE;
  }
  return s;
}

}  // extern "C"
