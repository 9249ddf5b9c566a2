// moa_inner_split_static: the split (+,*) product with no allocation at all.
//
// moa_inner_split takes its scratch (row/column scales and the slices of A
// and B) from a caller-supplied workspace. This variant runs the same kernels
// on a file-scope device array instead, so callers that cannot allocate (code
// being captured into a HIP graph, tight serving loops, harnesses that forbid
// hipMalloc) need to pass only their inputs and output.
//
// In host code `scratch` is a host-side stand-in, not a device address: the
// device address of each GPU's copy comes from hipGetSymbolAddress, called
// once per device with that device current, and only that address is handed
// to the kernels.
#include <stdio.h>

#include <mutex>

#include "common.hpp"
#include "internal.hpp"

namespace moa {
moa_status set_error(moa_status st, const char *msg);
}  // namespace moa

namespace {

static_assert(MOA_SPLIT_STATIC_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");

static __device__ __align__(256) unsigned char scratch[MOA_SPLIT_STATIC_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch` per device, once resolved

// Device address of this device's copy of `scratch` (resolved on the first
// call on the device), or an error status.
moa_status scratch_of_current_device(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return moa::set_error(MOA_ERR_HIP, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return moa::set_error(MOA_ERR_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      char buf[160];
      snprintf(buf, sizeof buf, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      return moa::set_error(MOA_ERR_HIP, buf);
    }
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return MOA_OK;
}

}  // namespace

extern "C" moa_status moa_inner_split_static(moa_shape sa, const double *A, moa_shape sb, const double *B, double *D,
                                             int32_t fmt, int32_t nslices, void *stream) {
  // Shape, format and slice-count errors are reported by moa_inner_split
  // below; a problem whose scratch exceeds the static array is refused here.
  const size_t need = moa_inner_split_workspace(sa, sb, fmt, nslices);
  if (need > (size_t)MOA_SPLIT_STATIC_BYTES) {
    char buf[200];
    snprintf(buf, sizeof buf,
             "the problem needs %zu bytes of split scratch; the static scratch holds %zu "
             "(MOA_SPLIT_STATIC_BYTES): use moa_inner_split with a workspace",
             need, (size_t)MOA_SPLIT_STATIC_BYTES);
    return moa::set_error(MOA_ERR_WORKSPACE, buf);
  }
  void *ws = nullptr;
  moa_status st = scratch_of_current_device(&ws);
  if (st != MOA_OK) return st;
  return moa_inner_split(sa, A, sb, B, D, fmt, nslices, ws, (size_t)MOA_SPLIT_STATIC_BYTES, stream);
}
