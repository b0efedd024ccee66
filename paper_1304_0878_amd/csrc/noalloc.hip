// Fixed scratch memory for the entry points that allocate nothing
// (dc_potrf_noalloc): a file-scope device array holding a graph's layout
// (task descriptors, work items, level counters, status words) and a host
// staging area of the same size in the library's static data.
//
// The array's device address is looked up once per device, with that device
// current (hipGetSymbolAddress), when a runtime is created on it; host code
// only ever uses that address, never the array's name.  Every call on a
// device shares that device's array and the one staging area: calls that
// overlap (on one device, or on any device for the staging area) race.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "exec_abi.h"

namespace {

constexpr int64_t SCRATCH_BYTES = (int64_t)16 << 20;
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

alignas(256) unsigned char g_stage[SCRATCH_BYTES];
std::mutex g_mu;
void *g_dev_ptr[MAX_DEVICES] = {};

}  // namespace

int dcx_noalloc_setup(int device) {
  if (device < 0 || device >= MAX_DEVICES) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_dev_ptr[device]) return (int)hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return (int)e;
  g_dev_ptr[device] = p;
  return (int)hipSuccess;
}

int dcx_noalloc_scratch(int device, void **dev, void **host, int64_t *bytes) {
  if (device < 0 || device >= MAX_DEVICES) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_dev_ptr[device]) return -1;
  *dev = g_dev_ptr[device];
  *host = g_stage;
  *bytes = SCRATCH_BYTES;
  return 0;
}
