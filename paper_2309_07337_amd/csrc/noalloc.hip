// Entry point that allocates nothing: the backward of a request with its
// launch table in a fixed per-device buffer (for callers that cannot
// allocate device memory during the call).
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.h"
#include "internal.h"

namespace {

// Launch-table area of hx_backward_noalloc.  Each GPU holds its own copy
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (the name itself is a
// host-side stand-in, not a device address).
static __device__ __align__(256) unsigned char scratch[HX_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of the area, looked up once
// per device with that device current.
int scratch_address(void** out) {
  int dev = 0;
  HX_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return hx::fail(HX_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    HX_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) return hx::fail(HX_ERR_HIP, "no device address for the launch-table area");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return HX_SUCCESS;
}

}  // namespace

extern "C" int hx_backward_noalloc(hx_req* r, const void* g_send, void* g_x, void* stream) {
  if (!r) return hx::fail(HX_ERR_ARG, "null request");
  HX_TRY(hx::req_usable(r));
  if (r->E1 > 0 && !g_send) return hx::fail(HX_ERR_ARG, "null g_send");
  if (r->n_local > 0 && !g_x) return hx::fail(HX_ERR_ARG, "null g_x");
  if (r->n_local == 0) return HX_SUCCESS;
  void* area = nullptr;
  HX_TRY(scratch_address(&area));
  // the job of hx_backward, with these buffers instead of the bound ones
  hx::SegSumJob job{static_cast<const char*>(g_send), static_cast<char*>(g_x), r->bt_ptr.as<int32_t>(),
                    r->bt_perm.as<int32_t>(), r->n_local};
  job.win_rows = r->E1;  // the terms are the request's own send-slot gradients
  const hx::Sched sc = hx::default_sched(hx::KIND_SEGSUM, (int)r->row_bytes);
  return hx::launch_segsum_in_area(job, r->dtype, (int)r->row_bytes, sc, area, HX_NOALLOC_SCRATCH_BYTES,
                                   (hipStream_t)stream);
}
