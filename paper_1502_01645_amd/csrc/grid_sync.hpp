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
constexpr int GS_ABORT_WORD = 16; // set to 1 by a workgroup that gave up waiting

// The abort word of a barrier area: a workgroup that stops waiting (its poll limit ran out, or
// it saw the word set) sets it, and every bounded wait of the other workgroups checks it, so
// they all leave their waits and end the launch normally instead of waiting for a workgroup
// that has gone.
__device__ __forceinline__ void grid_abort(unsigned* bar) {
  __hip_atomic_store(bar + GS_ABORT_WORD, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool grid_aborted(const unsigned* bar) {
  return __hip_atomic_load(bar + GS_ABORT_WORD, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
}

// Grid barrier over G workgroups.  Every wave first waits for its own sc1 stores, so once all
// workgroups have arrived their published data is visible at the coherence point.  Arrivals go
// to one counter per group, the last arrival of a group bumps a top counter, and the last of
// those publishes the new generation that the others poll.  Counters only grow, so no reset can
// race with a later arrival; epoch is this workgroup's count of barriers passed.  The words
// must be zero at launch.
// The wait is bounded: after spin_limit polls, or once the abort word is set, the workgroup
// sets the abort word and the barrier returns false (the same value in every thread); the
// caller then leaves its loop.
__device__ __forceinline__ bool grid_barrier(unsigned* bar, int G, unsigned& epoch,
                                             int spin_limit) {
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  bool failed = false;
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
    for (int poll = 0;
         __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target; ++poll) {
      if (poll >= spin_limit || grid_aborted(bar)) {
        grid_abort(bar);
        failed = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  }
  epoch += 1;
  return !__syncthreads_or(failed);
}

__global__ void grid_barrier_init_kernel(unsigned* bar);

}  // namespace nnls
