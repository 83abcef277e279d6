// xs_lookup_batch_noalloc: xs_lookup_batch with its sort scratch taken from
// a fixed device-side array instead of a caller workspace, so the call
// allocates nothing.
//
// The array is a file-scope device variable: every GPU the library runs on
// holds its own copy (XS_NOALLOC_SCRATCH_BYTES) from the module load until
// the process ends.  Host code never uses the array's name as an address
// (in host code it names a host-side stand-in); the device address comes
// from hipGetSymbolAddress, taken once per device with that device current
// and cached here.
#include <mutex>

#include "xs_internal.h"

namespace xs {

namespace {

static __device__ __align__(256) unsigned char scratch[XS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device`, or null (after xs::fail) when it
// could not be found.
void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) {
    fail(XS_EHIP, "device %d is beyond the %d devices the fixed scratch "
         "supports", device, kMaxDevices);
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      fail(XS_EHIP, "hipGetSymbolAddress of the fixed scratch on device %d "
           "failed: %s", device, hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

}  // namespace

xs_status scratch_setup(int device) {
  return scratch_ptr(device) ? XS_OK : XS_EHIP;
}

}  // namespace xs

using namespace xs;

extern "C" {

xs_status xs_lookup_batch_noalloc(xs_tables_t h, int64_t n, const double* d_E,
                                  const int32_t* d_mat, void* d_out,
                                  const xs_params* params, void* stream) {
  clear_error();
  if (!h) return fail(XS_EINVAL, "table handle is NULL");
  if (n < 0 || n > 0x7fffffffLL) return fail(XS_EINVAL, "n out of range");
  xs_params p;
  if (xs_status st = xs_resolve_params(h, n, params, &p)) return st;
  if (n == 0) return XS_OK;
  int dev = -1;
  XS_HIP(hipGetDevice(&dev));
  if (dev != h->device)
    return fail(XS_EINVAL, "current device %d is not the tables' device %d",
                dev, h->device);
  // Only a sort uses scratch (xs_lookup_batch's workspace); an unsorted call
  // needs none and has no size limit beyond xs_lookup_batch's.
  const bool do_sort = p.sort != XS_SORT_NONE && n >= p.sort_threshold;
  const size_t need = do_sort ? sort_workspace_bytes(n, 32) : 0;
  if (need > (size_t)XS_NOALLOC_SCRATCH_BYTES)
    return fail(XS_EWORKSPACE,
                "a sorted batch of %lld lookups needs %zu bytes of scratch; "
                "the fixed scratch holds %zu (at most %lld sorted lookups)",
                (long long)n, need, (size_t)XS_NOALLOC_SCRATCH_BYTES,
                (long long)XS_NOALLOC_MAX_SORTED);
  void* ws = nullptr;
  if (need > 0) {
    ws = scratch_ptr(dev);
    if (!ws) return XS_EHIP;
  }
  return lookup_batch_into(h, n, d_E, d_mat, d_out, &p, ws,
                           ws ? (size_t)XS_NOALLOC_SCRATCH_BYTES : 0, stream);
}

}  // extern "C"
