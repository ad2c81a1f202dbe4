// Helpers shared by the SVD kernels: the wave reduction, the round-robin (circle) order of
// one-sided Jacobi, whose rounds are sets of disjoint column pairs, and a grid barrier.
#pragma once

#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"
#include "wave_ops.hpp"

namespace nsk {

__device__ inline double wave_sum(double v) { return wave_sum64(v); }

// Positions of the circle method for N' = N rounded up to even: position 0 is fixed and
// positions 1..N'-1 hold columns 1 + (p - 1 + r) mod (N' - 1) in round r; pair i joins
// positions i and N'-1-i.
__device__ inline int circle_col(int pos, int r, int n_even) {
  return pos == 0 ? 0 : 1 + (pos - 1 + r) % (n_even - 1);
}

// Barrier over the workgroups of a cooperative launch, with one cache write-back per workgroup
// rather than one per wave.  Each wave first waits for its own memory operations, so its stores
// have reached the L2; one thread per workgroup then arrives with an agent-scope
// acquire-release (the L2's dirty lines are written back for the other XCDs), waits for the
// generation word, and takes an agent-scope acquire fence (stale cached lines are dropped)
// before the workgroup reads what the others wrote.  Arrival is two-level, so that no counter
// sees more than about nwg / 8 atomics per barrier: workgroup b arrives on the counter of group
// b mod 8, the last of a group on the top counter, and the last group publishes the next
// generation.  bar: kAgentBarWords words (one 64-byte line each for the top counter, the
// generation and the 8 group counters), zero before the first call and published by an earlier
// grid-wide synchronisation; epoch counts this workgroup's calls.  Every workgroup of the
// launch is resident, so the wait ends.
constexpr int kAgentBarGroups = 8;
constexpr int kAgentBarWords = 16 * (2 + kAgentBarGroups);

__device__ inline void agent_barrier(unsigned* bar, unsigned nwg, unsigned& epoch) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned next = epoch + 1;
    const unsigned g = blockIdx.x % kAgentBarGroups;
    const unsigned in_group = (nwg - g + kAgentBarGroups - 1) / kAgentBarGroups;
    const unsigned groups = nwg < (unsigned)kAgentBarGroups ? nwg : (unsigned)kAgentBarGroups;
    unsigned* top = bar;
    unsigned* gen = bar + 16;
    unsigned* grp = bar + 32 + 16 * g;
    bool last = __hip_atomic_fetch_add(grp, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1 == next * in_group;
    if (last) last = __hip_atomic_fetch_add(top, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1 == next * groups;
    if (last) {
      __hip_atomic_store(gen, next, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != next) __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  epoch = epoch + 1;
  __syncthreads();
}

}  // namespace nsk
