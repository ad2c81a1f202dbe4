// Helpers shared by the SVD kernels: the wave reduction and the round-robin (circle) order of
// one-sided Jacobi, whose rounds are sets of disjoint column pairs.
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

}  // namespace nsk
