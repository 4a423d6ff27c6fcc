// The query without device allocation: rd_check_pairs_noalloc runs the same
// plan and kernels as rd_check_pairs, with every device buffer (descriptors,
// term tables, accumulators, bucket records, counters, re-partition and
// fallback scratch, results) carved from one fixed scratch array that the
// library holds in device memory for each GPU it runs on, from module load
// to process end.  For callers that cannot call hipMalloc.
//
// In host code the array's name is only a host-side stand-in: its device
// address on each GPU is looked up once with hipGetSymbolAddress (at
// context creation, with that device current) and only that address is
// ever handed to kernels and copies.
#include "../../include/hgrd.h"
#include "hgrd_launch.h"

#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[RD_NOALLOC_SCRATCH_BYTES];

// Device address of `scratch` per GPU (nullptr until looked up), and one
// lock per GPU: calls on one GPU share its array, so they are serialised.
void* g_scratch[kMaxDevices];
std::mutex g_lookup;
std::mutex g_busy[kMaxDevices];

}  // namespace

int hgrd::noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return 1;
  std::lock_guard<std::mutex> lk(g_lookup);
  if (g_scratch[device]) return 0;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    fprintf(stderr, "hgrd: no device address for the scratch area on device %d: %s\n",
            device, hipGetErrorString(e));
    return 1;
  }
  g_scratch[device] = p;
  return 0;
}

extern "C" int rd_check_pairs_noalloc(rd_context* ctx, const rd_kernel_model* models,
                                      uint32_t n_models, const rd_access_pair* pairs,
                                      uint32_t n_pairs, const rd_launch_domain* launch,
                                      const rd_param_sets* params, const rd_options* opt,
                                      rd_pair_result* out) {
  if (!ctx) return RD_EINVAL;
  const int dev = hgrd::context_device(ctx);  // as every other entry point
  if (dev < 0 || dev >= kMaxDevices) return RD_EDEVICE;
  if (hipSetDevice(dev) != hipSuccess) return RD_EDEVICE;
  void* base;
  {
    std::lock_guard<std::mutex> lk(g_lookup);
    base = g_scratch[dev];
  }
  if (!base) return RD_EDEVICE;  // rd_context_create looked it up on this device
  std::lock_guard<std::mutex> busy(g_busy[dev]);
  return hgrd::check_pairs_in_arena(ctx, base, RD_NOALLOC_SCRATCH_BYTES, models,
                                    n_models, pairs, n_pairs, launch, params, opt, out);
}
