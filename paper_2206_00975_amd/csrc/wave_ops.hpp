// Wavefront-wide exchanges and reductions for 64-lane waves on gfx950.
#pragma once

#include <hip/hip_runtime.h>

namespace nsk {

// Cross-lane exchanges on the VALU (no LDS round trip): v_permlane32_swap / v_permlane16_swap
// for partner distances 32 and 16, DPP row operations inside 16-lane rows for 8, 4, 2, 1.
__device__ inline double dpp_join(int lo, int hi) {
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline int dlo(double v) { return (int)(__double_as_longlong(v) & 0xffffffffll); }
__device__ inline int dhi(double v) { return (int)(__double_as_longlong(v) >> 32); }

// v + (value of lane ^ 32): swapping the upper half of one copy of v with the lower half of
// another leaves every lane holding v_l and v_{l^32} across the two results, in an order
// that a sum does not need.
__device__ inline double sum_xor32(double v) {
  const auto a = __builtin_amdgcn_permlane32_swap(dlo(v), dlo(v), false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(dhi(v), dhi(v), false, false);
  return dpp_join(a[0], b[0]) + dpp_join(a[1], b[1]);
}
// v + (value of lane ^ 16), the same way with odd/even 16-lane rows.
__device__ inline double sum_xor16(double v) {
  const auto a = __builtin_amdgcn_permlane16_swap(dlo(v), dlo(v), false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(dhi(v), dhi(v), false, false);
  return dpp_join(a[0], b[0]) + dpp_join(a[1], b[1]);
}

// Value of lane ^ H for H in {8, 4, 2, 1}, inside 16-lane rows.
//  8: row_ror:8;  4: row_half_mirror (l -> l ^ 7) then quad reverse (l -> l ^ 3);
//  2: quad_perm [2,3,0,1];  1: quad_perm [1,0,3,2].
template <int H>
__device__ inline int xor_lane_i(int x) {
  if constexpr (H == 8) return __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);
  if constexpr (H == 4) {
    const int m = __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false);
    return __builtin_amdgcn_update_dpp(0, m, 0x1B, 0xF, 0xF, false);
  }
  if constexpr (H == 2) return __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);
  return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);
}
template <int H>
__device__ inline double xor_lane(double v) {
  return dpp_join(xor_lane_i<H>(dlo(v)), xor_lane_i<H>(dhi(v)));
}

// Value of lane (l + K) mod 16 of the same 16-lane row, 1 <= K <= 15.  DPP row_ror:R rotates
// a row right (lane l receives lane l - R), so this is row_ror:(16 - K).  All lanes of the
// row must be active.
template <int K>
__device__ inline double lane_plus(double v) {
  static_assert(K >= 1 && K <= 15, "lane_plus takes 1..15");
  constexpr int ctrl = 0x120 + (16 - K);
  // every lane has a source in its row, so no old value is needed (no register initialisation)
  return dpp_join(__builtin_amdgcn_mov_dpp(dlo(v), ctrl, 0xF, 0xF, true),
                  __builtin_amdgcn_mov_dpp(dhi(v), ctrl, 0xF, 0xF, true));
}

__device__ inline double bcast_d(double v, int lane) {
  return dpp_join(__builtin_amdgcn_readlane(dlo(v), lane), __builtin_amdgcn_readlane(dhi(v), lane));
}

// Two-value swap-sums for the transposed reduction: with a in the first and b in the second
// operand, lanes whose bit 5 (resp. bit 4) is clear receive a_l + a_{l^32} (a_l + a_{l^16})
// and the others b_l + b_{l^32} (b_l + b_{l^16}).
__device__ inline double swap_sum32(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane32_swap(dlo(a), dlo(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(dhi(a), dhi(b), false, false);
  return dpp_join(lo[0], hi[0]) + dpp_join(lo[1], hi[1]);
}
__device__ inline double swap_sum16(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane16_swap(dlo(a), dlo(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(dhi(a), dhi(b), false, false);
  return dpp_join(lo[0], hi[0]) + dpp_join(lo[1], hi[1]);
}

constexpr int ceil_log2(int p) { return p <= 1 ? 0 : 1 + ceil_log2((p + 1) / 2); }

// Transposed reduction of P (<= 16) per-lane values v[0..P).  With L = ceil(log2 P), the
// steps over lane bits 5, 4, ..., 6 - L each halve the number of live values: value i is
// paired with value i + half, and a lane keeps the pair sum of the one its bit selects.  The
// remaining low lane bits are ordinary butterflies.  Afterwards lane l holds the wave total of
// value l >> (6 - L) (zero if that index is >= P).  v is clobbered.
template <int P>
__device__ inline double reduce_t(double (&v)[16], int lane) {
  constexpr int L = ceil_log2(P);
  constexpr int P2 = 1 << L;
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const int half = P2 >> (k + 1);
    const int bit = 5 - k;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const double a = i < P ? v[i] : 0.0;
      const double b = i + half < P ? v[i + half] : 0.0;
      if (bit == 5) {
        v[i] = swap_sum32(a, b);
      } else if (bit == 4) {
        v[i] = swap_sum16(a, b);
      } else {
        const bool up = (lane >> bit) & 1;
        const double keep = up ? b : a;
        const double send = up ? a : b;
        double r;
        if (bit == 3) r = xor_lane<8>(send);
        else if (bit == 2) r = xor_lane<4>(send);
        else if (bit == 1) r = xor_lane<2>(send);
        else r = xor_lane<1>(send);
        v[i] = keep + r;
      }
    }
  }
  double t = v[0];
  if (L == 0) t = sum_xor32(t);
  if (L <= 1) t = sum_xor16(t);
  if (L <= 2) t += xor_lane<8>(t);
  if (L <= 3) t += xor_lane<4>(t);
  if (L <= 4) t += xor_lane<2>(t);
  if (L <= 5) t += xor_lane<1>(t);
  return t;
}

// p as a scalar value (taken from the first active lane; p must be wave-uniform).
template <typename T>
__device__ inline T* uniform_ptr(T* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (T*)(((unsigned long long)hi << 32) | lo);
}

// A wave-uniform pointer the compiler must treat as a fresh scalar value: addresses derived
// from it are recomputed at their use instead of being kept live in vector registers.
template <typename T>
__device__ inline T* opaque_uniform(T* p) {
  p = uniform_ptr(p);
  asm volatile("" : "+s"(p));
  return p;
}

// Orders this wave's earlier LDS writes before its later LDS reads: the LDS runs a wave's
// instructions in issue order, so lanes of the wave see each other's writes once the compiler
// is kept from moving the accesses across this point.  No other wave is synchronised.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Workgroup barrier that orders LDS accesses only: unlike __syncthreads() it does not wait
// for global loads in flight, so prefetches can cross it.  Only for barriers whose producers
// and consumers communicate through LDS.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Sum over all 64 lanes, result in every lane.
__device__ inline double wave_sum64(double v) {
  v = sum_xor32(v);
  v = sum_xor16(v);
  v += xor_lane<8>(v);
  v += xor_lane<4>(v);
  v += xor_lane<2>(v);
  v += xor_lane<1>(v);
  return v;
}

__device__ inline double lane_value(double x, int src) { return bcast_d(x, src); }

}  // namespace nsk
