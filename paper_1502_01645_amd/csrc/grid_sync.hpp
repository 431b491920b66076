// Cross-workgroup communication of the persistent solvers (one workgroup per compute unit, all
// resident): coherent loads and stores, and a grid-wide barrier.
//
// Data shared between workgroups is written and read with agent-scope relaxed atomics: on gfx950
// these are sc1 accesses that bypass the per-XCD L2, so no L2 write-back or invalidate is needed
// around the barrier.  Read-only data (Q) uses ordinary cached loads.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nnls {

__device__ __forceinline__ float ld_sc(const float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_sc(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_sc(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_sc(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int GS_GROUPS = 8;      // barrier arrival groups
constexpr int GS_BAR_WORDS = 1024;

// Grid barrier over G workgroups.  Every wave first waits for its own sc1 stores, so once all
// workgroups have arrived their published data is visible at the coherence point.  Arrivals go
// to one counter per group, the last arrival of a group bumps a top counter, and the last of
// those publishes the new generation that the others poll.  Counters only grow, so no reset can
// race with a later arrival; epoch is this workgroup's count of barriers passed.  The words
// must be zero at launch.
__device__ __forceinline__ void grid_barrier(unsigned* bar, int G, unsigned& epoch) {
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int ngroups = G < GS_GROUPS ? G : GS_GROUPS;
    const int grp = blockIdx.x % ngroups;
    const unsigned gsize = (unsigned)(G / ngroups + (grp < G % ngroups ? 1 : 0));
    unsigned* gen = bar;
    unsigned* top = bar + 32;
    unsigned* gc = bar + 64 + 32 * grp;
    const unsigned target = epoch + 1;
    const unsigned a = __hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (a == gsize * target - 1) {
      const unsigned b =
          __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (b == (unsigned)ngroups * target - 1)
        __hip_atomic_store(gen, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target)
      __builtin_amdgcn_s_sleep(1);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  epoch += 1;
  __syncthreads();
}

__global__ void grid_barrier_init_kernel(unsigned* bar);

}  // namespace nnls
