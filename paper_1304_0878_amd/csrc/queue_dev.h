// Device atomics policy of the ready-queue protocol (queue.h): agent-scope
// HIP atomics and fences, the 100 MHz constant wall clock, a short sleep.
#pragma once
#include <hip/hip_runtime.h>

#include "queue.h"

namespace dcq {

struct DevAT {
  template <class T> __device__ static T ld(T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  template <class T> __device__ static void st(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  template <class T> __device__ static bool cas(T *p, T *e, T d) {
    return __hip_atomic_compare_exchange_strong(p, e, d, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
  }
  template <class T> __device__ static T add(T *p, T v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __device__ static void fence_rel() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
  __device__ static void fence_acq() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
  __device__ static uint64_t now() { return wall_clock64(); }
  __device__ static void pause() { __builtin_amdgcn_s_sleep(2); }
};

// The protocol's steps as out-of-line calls made by one thread of a
// workgroup: kept out of the kernels' bodies so that their registers are not
// allocated around the tile computations.
__device__ __attribute__((noinline)) inline uint64_t pop_item(const View *q, int cls) {
  uint64_t it = 0;
  return pop<DevAT>(*q, cls, &it) == POP_ITEM ? it : 0;
}
__device__ __attribute__((noinline)) inline void complete_item(const View *q, int64_t t) {
  complete<DevAT>(*q, t);
}
__device__ __attribute__((noinline)) inline void start_worker(const View *q, int cls) {
  worker_start<DevAT>(*q, cls);
}

}  // namespace dcq
