// rs_noalloc.hip -- rs_sort_pairs_noalloc: rs_sort_pairs with its scratch in
// a static device array of the library instead of a caller's buffer.
//
// The array, `scratch`, is allocated with the library's code object on each
// device the library runs on and stays there until the process ends.  Host
// code never uses its name as an address: the name is a host-side stand-in.
// The device address is looked up once per device with hipGetSymbolAddress
// (with that device current) and kept; kernels receive that address as their
// tmp argument, exactly as rs_sort_pairs passes the caller's buffer.
//
// Every call on one device shares that device's array and leaves the last
// call's contents in it.  The launch sequences clear what must start at zero
// themselves (fill kernels over their control words and count tables), so a
// call does not depend on what an earlier call left.  Calls that overlap in
// time on one device (different streams or threads without ordering between
// them) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "rs_internal.h"

namespace {

constexpr size_t kScratchBytes = RS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up on first use.
rs_status scratch_address(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0)
    return rs::fail(RS_ERR_HIP, "hipGetDevice failed");
  if (dev >= kMaxDevices) return rs::fail(RS_ERR_UNSUPPORTED, "device ordinal beyond the static scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return rs::fail(RS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return RS_OK;
}

}  // namespace

extern "C" rs_status rs_sort_pairs_noalloc(const rs_key_desc *desc, const void *keys_in, void *keys_out,
                                           const uint32_t *vals_in, uint32_t *vals_out, uint64_t n, void *stream) {
  rs::g_last_error.clear();
  if (!desc) return rs::fail(RS_ERR_NULL_ARG, "desc is NULL");
  if (n == 0) return RS_OK;
  // the scratch this sort needs, from the same plan rs_sort_pairs makes
  rs::Plan pl;
  std::string why;
  rs_status st = rs::make_plan(desc, n, true, rs::current_tuning(desc, n, true), &pl, &why);
  if (st != RS_OK) return rs::fail(st, why);
  if (pl.total > kScratchBytes)
    return rs::fail(RS_ERR_UNSUPPORTED, "this sort needs " + std::to_string(pl.total) +
                                            " bytes of scratch; the static scratch holds " +
                                            std::to_string(kScratchBytes));
  void *tmp = nullptr;
  if ((st = scratch_address(&tmp)) != RS_OK) return st;
  return rs::sort_common(desc, keys_in, keys_out, vals_in, vals_out, n, tmp, kScratchBytes, stream, true);
}
