// wvl_apply_local_ham_static: the local-H apply on a workspace the library
// holds in a static device array, for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc).  The array lives in this file's code object: each GPU the
// library runs on holds its own copy, at its own address, until the process
// ends.  In host code the array's name is only a stand-in for the symbol;
// its device address comes from hipGetSymbolAddress, taken once per device
// with that device current, and only that address reaches a kernel.
#include <hip/hip_runtime.h>

#include <mutex>

#include "wvl_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[WVL_STATIC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device

// the device the plan's stream runs on (the current one for the NULL stream)
hipError_t stream_device(void* stream, int* dev) {
  if (stream) return hipStreamGetDevice((hipStream_t)stream, dev);
  return hipGetDevice(dev);
}

// device address of the array on `dev`, looked up on the first call there
hipError_t scratch_on(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    // the kernels' code objects are loaded here, never inside a capture
    int pe = wvl::preload_kernels();
    if (pe == 0) pe = wvl::preload_fused_kernels();
    void* p = nullptr;
    e = pe != 0 ? (hipError_t)pe : hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const hipError_t r = hipSetDevice(cur);
      if (e == hipSuccess) e = r;
    }
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" wvl_status wvl_apply_local_ham_static(wvl_plan* plan, wvl_dtype dt, uint32_t terms,
                                                 const void* psi_c, const void* pot,
                                                 void* hpsi_c, double* e_kin, double* e_pot) {
  static const char* who = "wvl_apply_local_ham_static";
  if (!plan) return wvl::plan_error(nullptr, WVL_EINVAL, "wvl_apply_local_ham_static: null plan");
  int dev = -1;
  hipError_t e = stream_device(wvl::plan_stream(plan), &dev);
  if (e != hipSuccess) {
    char msg[256];
    snprintf(msg, sizeof msg, "%s: device of the context's stream: %s", who,
             hipGetErrorString(e));
    return wvl::plan_error(plan, WVL_EDEVICE, msg);
  }
  if (dev < 0 || dev >= kMaxDevices)
    return wvl::plan_error(plan, WVL_EUNSUPPORTED, "wvl_apply_local_ham_static: device index");
  void* ws = nullptr;
  if ((e = scratch_on(dev, &ws)) != hipSuccess) {
    char msg[256];
    snprintf(msg, sizeof msg, "%s: hipGetSymbolAddress(scratch) on device %d: %s", who, dev,
             hipGetErrorString(e));
    return wvl::plan_error(plan, WVL_EDEVICE, msg);
  }
  return wvl::apply_in_workspace(plan, dt, terms, psi_c, pot, hpsi_c, e_kin, e_pot, ws,
                                 WVL_STATIC_WORKSPACE_BYTES, who);
}
