// Block one-sided Jacobi spread over workgroups (cooperative launch).
//
// Same sweep, schedule, rotation formulas and log as the single-workgroup version: an intra
// phase in which every block rotates its own column pairs in circle order, then nb - 1 block
// rounds in which the nb / 2 disjoint block pairs of the round meet.  Here workgroup g owns
// block pair g of every round (and blocks g, g + nb/2 of the intra phase), so the pairs of a
// round run on different CUs; a grid barrier separates the phases.  Inside a workgroup the NW
// waves split the rows: wave w holds rows 64 w .. 64 w + 63 of the two blocks, one row per
// lane.  Column dot products are reduced per wave with one transposed reduction and summed
// over the waves through LDS in wave order, so every wave derives the same rotation
// parameters.  The first wave writes the log and counts the rotations.
#pragma once

#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "jacobi_block.hpp"
#include "wave_ops.hpp"

namespace nsk {

// Per-sweep rotation counts and largest relative cosines, the two words of the Gram check
// (violation flag, largest squared cosine), then the block versions and the abort word of the
// round hand-over (kCoopVersionWords 64-bit words) and the workers' XCC ids (kCoopMaxBlocks / 2
// 32-bit words), appended to the rotation log.
constexpr int kCoopMaxBlocks = 64;
constexpr int kCoopVersionWords = kCoopMaxBlocks + 1;

__host__ __device__ inline size_t jacobi_coop_counter_bytes(int max_sweeps) {
  return ((size_t)max_sweeps * 2 + 2 + kCoopVersionWords) * sizeof(unsigned long long) +
         (size_t)(kCoopMaxBlocks / 2) * sizeof(unsigned);
}

// Hand-over of blocks between block rounds without a grid barrier.  A block is written once
// per phase (the intra phase, then each of the nb - 1 rounds), so after phase ph of sweep sw
// its version is sw * nb + ph + 1.  The workgroup that wrote a block publishes the new version
// once every wave's stores have reached the L2 (with workers on several XCDs, after an
// agent-scope release); the workgroup that takes the block in the next round polls the two
// versions it needs (one thread, bounded) and takes an agent-scope acquire, or, with all
// workers on one XCD, reads the two blocks with agent-scope loads (load_handed).  Past
// kCoopSpinLimit polls the abort word is raised, every later wait returns at once, and the
// result is marked invalid, so a protocol fault cannot hang the GPU.
constexpr unsigned kCoopSpinLimit = 1u << 20;

__device__ inline void coop_publish(unsigned long long* ver, int I, int J, unsigned long long v, bool local) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (!local) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&ver[I], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (J != I) __hip_atomic_store(&ver[J], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ inline void coop_wait(unsigned long long* ver, int I, int J, unsigned long long v,
                                 unsigned long long* abort_word, bool local) {
  if (threadIdx.x == 0) {
    unsigned spins = 0;
    while (__hip_atomic_load(&ver[I], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v ||
           __hip_atomic_load(&ver[J], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v) {
      if (__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0ull) break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins == kCoopSpinLimit) {
        __hip_atomic_store(abort_word, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    if (!local) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}



// Wave totals of the first P values of v, summed over the NW waves.  Lane l receives the
// total of value l >> (6 - ceil_log2(P)) (zero past P).  part: LDS [2][NW][16], used in turn.
template <int P, int NW>
__device__ inline double coop_reduce(double (&v)[16], int lane, int wave, double (*part)[NW][16], int& buf) {
  constexpr int SH = 6 - ceil_log2(P);
  const double t = reduce_t<P>(v, lane);
  const int pi = lane >> SH;
  if ((lane & ((1 << SH) - 1)) == 0 && pi < P) part[buf][wave][pi] = t;
  lds_barrier();
  double s = 0;
  if (pi < P)
#pragma unroll
    for (int w = 0; w < NW; ++w) s += part[buf][w][pi];
  buf ^= 1;
  return s;
}

struct CoopCount {
  int rotations;   // counted by the first wave's leading lanes only
  double offnum;   // largest squared relative cosine g^2 / (a b), kept as a fraction so that the
  double offden;   // step needs no reciprocal: (g^2, a b) replaces it when g^2 offden > offnum a b
};

__device__ inline void count_off(CoopCount& cc, double g, double ab) {
  const double g2 = g * g;
  if (ab > 0 && g2 * cc.offden > cc.offnum * ab) {
    cc.offnum = g2;
    cc.offden = ab;
  }
}

template <int NW, int B>
__device__ inline void coop_intra_block(double* __restrict__ R, int ld, int blk, double2* lg, int stride,
                                        double tol, CoopCount& cc, double (*part)[NW][16], int& buf, int lane,
                                        int wave, double2* bc) {
  constexpr int BQ = B + (B & 1);
  constexpr int H = BQ / 2;
  constexpr int SH = 6 - ceil_log2(H);
  const int pi = lane >> SH;
  const bool lead = wave == 0 && (lane & ((1 << SH) - 1)) == 0 && pi < H;
  double* p = uniform_ptr(R + (size_t)blk * B * ld) + 64 * wave + lane;
  double X[BQ];
#pragma unroll
  for (int b = 0; b < BQ; ++b) X[b] = b < B ? p[(size_t)b * ld] : 0.0;
  // The squared norms are reduced once, then carried as in the block rounds: lanes of pair pi
  // hold alpha = |x_pi|^2 and beta = |x_{BQ-1-pi}|^2, updated by each rotation and moved with
  // the circle shift; only the inner products are reduced per step.
  double alpha, beta;
  {
    constexpr int SHB = 6 - ceil_log2(B);
    double v[16];
#pragma unroll
    for (int b = 0; b < B; ++b) v[b] = X[b] * X[b];
    const double nrm = coop_reduce<B, NW>(v, lane, wave, part, buf);  // lane l: position l >> SHB
    const int pq = pi < H ? pi : 0;
    alpha = __shfl(nrm, pq << SHB, 64);
    beta = BQ - 1 - pq < B ? __shfl(nrm, (BQ - 1 - pq) << SHB, 64) : 0.0;  // the padding column is zero
  }
  const int up = lane + (1 << SH) < 64 ? lane + (1 << SH) : lane;  // a lane of pair pi + 1
  const int down = lane >= (1 << SH) ? lane - (1 << SH) : lane;    // a lane of pair pi - 1
  for (int q = 0; q < BQ - 1; ++q) {
    double g;
    {
      double v[16];
#pragma unroll
      for (int i = 0; i < H; ++i) v[i] = X[i] * X[BQ - 1 - i];
      g = coop_reduce<H, NW>(v, lane, wave, part, buf);
    }
    double c, s, t;
    bool act;
    jacobi_params(alpha, beta, g, tol, c, s, t, act);
    if (lead) {
      const double ab = alpha * beta;
      count_off(cc, g, ab);
      if (act) cc.rotations++;
      lg[pi] = make_double2(c, s);
    }
    if (act) {
      alpha = fmax(alpha - t * g, 0.0);
      beta = fmax(beta + t * g, 0.0);
    }
    if constexpr (H > 1) {
      // after the shift position b takes b + 1 (1 <= b < BQ - 1) and BQ - 1 takes 1: pair 0 keeps
      // alpha and takes pair 1's alpha as beta; pair i >= 1 takes pair i - 1's beta, and pair
      // i + 1's alpha (i < H - 1) or its own beta (i = H - 1) as alpha
      const double a_up = __shfl(alpha, up, 64), b_down = __shfl(beta, down, 64);
      const double na = pi == 0 ? alpha : pi + 1 < H ? a_up : beta;
      const double nbv = pi == 0 ? a_up : b_down;
      alpha = na;
      beta = nbv;
    }
    // every lane needs all H rotations: through this wave's LDS slots
    if ((lane & ((1 << SH) - 1)) == 0 && pi < H) bc[pi] = make_double2(c, s);
    wave_lds_sync();
    double2 csv[H];
#pragma unroll
    for (int i = 0; i < H; ++i) csv[i] = bc[i];
    __builtin_amdgcn_sched_barrier(0);  // all reads in flight before the first rotation
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double ci = csv[i].x, si = csv[i].y;
      const double a = X[i], b = X[BQ - 1 - i];
      X[i] = ci * a - si * b;
      X[BQ - 1 - i] = si * a + ci * b;
    }
    const double first = X[1];
#pragma unroll
    for (int b = 1; b < BQ - 1; ++b) X[b] = X[b + 1];
    X[BQ - 1] = first;
    lg += stride;
  }
#pragma unroll
  for (int b = 0; b < B; ++b) p[(size_t)b * ld] = X[b];
}

template <int NW, int B>
__device__ inline void coop_inter_pair(double* __restrict__ R, int ld, int I, int J, double2* lg, int stride,
                                       double tol, CoopCount& cc, double (*part)[NW][16], int& buf, int lane,
                                       int wave, double2* bc, bool local) {
  constexpr int SH = 6 - ceil_log2(B);
  const int pi = lane >> SH;
  const bool valid = pi < B;
  const bool lead = wave == 0 && (lane & ((1 << SH) - 1)) == 0 && valid;
  double* pt = uniform_ptr(R + (size_t)I * B * ld) + 64 * wave + lane;
  double* pu = uniform_ptr(R + (size_t)J * B * ld) + 64 * wave + lane;
  double T[B], U[B];
  if (local) {  // blocks handed over within the XCD: agent-scope loads, past the CU's L1
#pragma unroll
    for (int b = 0; b < B; ++b) {
      T[b] = load_handed(&pt[(size_t)b * ld]);
      U[b] = load_handed(&pu[(size_t)b * ld]);
    }
  } else {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      T[b] = pt[(size_t)b * ld];
      U[b] = pu[(size_t)b * ld];
    }
  }
  double alpha, beta;
  {
    double v[16];
#pragma unroll
    for (int i = 0; i < B; ++i) v[i] = T[i] * T[i];
    alpha = coop_reduce<B, NW>(v, lane, wave, part, buf);
  }
  {
    double v[16];
#pragma unroll
    for (int i = 0; i < B; ++i) v[i] = U[i] * U[i];
    beta = coop_reduce<B, NW>(v, lane, wave, part, buf);
  }
  const int nxt_pair = pi + 1 == B ? 0 : (valid ? pi + 1 : pi);
  const int nxt_lane = (nxt_pair << SH) | (lane & ((1 << SH) - 1));
  // sub-round j pairs T_i with U_{(i + j) mod B}; unrolled, so the pairing is a register choice
#pragma unroll
  for (int j = 0; j < B; ++j) {
    double z[16];
#pragma unroll
    for (int i = 0; i < B; ++i) z[i] = T[i] * U[(i + j) % B];
    const double g = coop_reduce<B, NW>(z, lane, wave, part, buf);
    double c, s, t;
    bool act;
    jacobi_params(alpha, beta, g, tol, c, s, t, act);
    if (!valid) {
      c = 1.0;
      s = 0.0;
      t = 0.0;
      act = false;
    }
    if (lead) {
      const double ab = alpha * beta;
      count_off(cc, g, ab);
      if (act) cc.rotations++;
      lg[pi] = make_double2(c, s);
    }
    if (act) {
      alpha = fmax(alpha - t * g, 0.0);
      beta = fmax(beta + t * g, 0.0);
    }
    // every lane needs all B rotations: through this wave's LDS slots
    if ((lane & ((1 << SH) - 1)) == 0 && valid) bc[pi] = make_double2(c, s);
    wave_lds_sync();
    double2 csv[B];
#pragma unroll
    for (int i = 0; i < B; ++i) csv[i] = bc[i];
    __builtin_amdgcn_sched_barrier(0);  // all reads in flight before the first rotation
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const double ci = csv[i].x, si = csv[i].y;
      const double a = T[i], b = U[(i + j) % B];
      T[i] = ci * a - si * b;
      U[(i + j) % B] = si * a + ci * b;
    }
    beta = __shfl(beta, nxt_lane, 64);
    lg += stride;
  }
  pt = opaque_uniform(pt - lane) + lane;
  pu = opaque_uniform(pu - lane) + lane;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    pt[(size_t)b * ld] = T[b];
    pu[(size_t)b * ld] = U[b];
  }
}

// True when no column pair of R has |x_p . x_q| > tol |x_p| |x_q|.  Collective over the grid
// (two grid barriers): column norms of each workgroup's blocks go to norms_g (N words of
// global scratch), then each workgroup takes block pairs I <= J, forms the B x B products of
// the pair's columns (one row per lane, transposed reductions in chunks of 16, wave partials
// summed through LDS) and tests them.  flags: two words (violation, largest squared cosine,
// which is returned in off2).
template <int NW, int B>
__device__ inline bool coop_gram_clear(const double* __restrict__ R, const JacobiShape& js, int N, double tol, int stride,
                                       double* __restrict__ norms_g, unsigned long long* flags,
                                       double (*part)[NW][16], int& buf, int lane, int wave, double& off2) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  constexpr int SH = 6 - ceil_log2(B);
  constexpr int NCH = (B * B + 15) / 16;
  __shared__ double norms[512];
  __shared__ double gp[NW][NCH * 16];
  __shared__ unsigned long long sh_flags[2];
  const int ld = 64 * NW;
  const int G = coop_workers(stride);
  const int me = coop_worker(stride) ? coop_worker_index(stride) : js.nb * js.nb;  // other workgroups take no work
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    flags[0] = 0;
    flags[1] = 0;
  }
  for (int b = me; b < js.nb; b += G) {
    const double* p = uniform_ptr(R + (size_t)b * B * ld) + 64 * wave + lane;
    double v[16];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const double x = p[(size_t)i * ld];
      v[i] = x * x;
    }
    const double nrm = coop_reduce<B, NW>(v, lane, wave, part, buf);
    const int pi = lane >> SH;
    if (wave == 0 && (lane & ((1 << SH) - 1)) == 0 && pi < B && b * B + pi < N) norms_g[b * B + pi] = nrm;
  }
  grid.sync();
  for (int c = threadIdx.x; c < js.nb * B; c += blockDim.x) norms[c] = c < N ? norms_g[c] : 0.0;
  __syncthreads();
  const int npairs = js.nb * (js.nb + 1) / 2;
  bool bad = false;
  double om = 0.0;
  for (int bp = me; bp < npairs; bp += G) {
    int I = 0, rem = bp;
    while (rem >= js.nb - I) {
      rem -= js.nb - I;
      ++I;
    }
    const int J = I + rem;
    const double* pt = uniform_ptr(R + (size_t)I * B * ld) + 64 * wave + lane;
    const double* pu = uniform_ptr(R + (size_t)J * B * ld) + 64 * wave + lane;
    double T[B], U[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      T[i] = pt[(size_t)i * ld];
      U[i] = pu[(size_t)i * ld];
    }
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      double v[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int q = ch * 16 + e;
        v[e] = q < B * B ? T[q / B] * U[q % B] : 0.0;
      }
      const double t = reduce_t<16>(v, lane);  // lane l: total of product ch * 16 + (l >> 2)
      if ((lane & 3) == 0) gp[wave][ch * 16 + (lane >> 2)] = t;
    }
    lds_barrier();
    if (wave == 0) {
      for (int q = lane; q < B * B; q += 64) {
        const int i = q / B, j = q % B;
        if (I == J && j <= i) continue;
        double g = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) g += gp[w][q];
        const double ab = norms[I * B + i] * norms[J * B + j];
        bad |= g * g > (tol * tol) * ab;
        if (ab > 0) om = fmax(om, g * g * rcp_nr(ab));
      }
    }
    lds_barrier();
  }
  if (wave == 0) {
    const bool any = __any(bad);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) om = fmax(om, __shfl_xor(om, o, 64));
    if (lane == 0) {
      if (any) atomicOr(&flags[0], 1ull);
      atomicMax(&flags[1], (unsigned long long)__double_as_longlong(om));
    }
  }
  grid.sync();
  if (threadIdx.x == 0) {
    sh_flags[0] = __hip_atomic_load(&flags[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sh_flags[1] = __hip_atomic_load(&flags[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  off2 = __longlong_as_double((long long)sh_flags[1]);
  const bool clear = sh_flags[0] == 0;
  __syncthreads();
  return clear;
}

// Sweeps until one performs no rotation (or max_sweeps).  Launched cooperatively with
// `stride` workgroups per worker (see coop_worker) and nb / 2 workers of NW * 64 threads,
// NW = rows / 64; the other workgroups take part in the grid barriers only.  counters:
// jacobi_coop_counter_bytes(max_sweeps).  allow_local: take the one-XCD hand-over when the
// placement allows.
template <int NW, int B>
__device__ inline void jacobi_coop_sweeps(double* __restrict__ R, int N, int max_sweeps, double2* __restrict__ log,
                                          unsigned long long* __restrict__ counters, JacobiResult* jres,
                                          double* __restrict__ scratch, int stride, bool allow_local) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  __shared__ double part[2][NW][16];
  __shared__ double2 bcs[NW][16];  // per wave: the rotations of the current step
  __shared__ int sh_rot;
  __shared__ double sh_off;
  const JacobiShape js = jacobi_shape(N);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ld = 64 * NW;
  const int nbp = js.nb / 2;
  const size_t per_sweep = jacobi_log_entries_per_sweep(js);
  const double tol = (double)N * 0x1p-53;
  unsigned long long* rot_count = counters;
  unsigned long long* off_bits = counters + max_sweeps;
  unsigned long long* ver = counters + 2 * max_sweeps + 2;
  unsigned long long* abort_word = ver + kCoopMaxBlocks;
  unsigned* xcc_ids = reinterpret_cast<unsigned*>(ver + kCoopVersionWords);
  const int G = coop_workers(stride);
  const bool worker = coop_worker(stride);
  const int me = worker ? coop_worker_index(stride) : js.nb;  // other workgroups take no blocks
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < 2 * max_sweeps; i += blockDim.x) counters[i] = 0;
    for (int i = threadIdx.x; i < kCoopVersionWords; i += blockDim.x) ver[i] = 0;
  }
  xcd_record(xcc_ids, stride);
  int buf = 0;
  int sweeps = 0, conv = 0;
  if (threadIdx.x == 0) sh_off = 0.0;
  grid.sync();
  const bool local = xcd_all_local(xcc_ids, stride, allow_local);
  for (int sw = 0; sw < max_sweeps; ++sw) {
    CoopCount cc{0, 0.0, 1.0};
    double2* sweep_log = log + (size_t)sw * per_sweep;
    // the sweep starts after a grid barrier, so the intra phase needs no wait
    const unsigned long long base_ver = (unsigned long long)sw * js.nb;
    for (int b = me; b < js.nb; b += G) {
      coop_intra_block<NW, B>(R, ld, b, sweep_log + (size_t)b * 16, js.nb * 16, tol, cc, part, buf, lane, wave,
                              bcs[wave]);
      coop_publish(ver, b, b, base_ver + 1, local);
    }
    for (int r = 0; r < js.nb - 1; ++r) {
      double2* round_log = sweep_log + jacobi_log_step_offset(js, js.bq - 1 + r * B);
      for (int i = me; i < nbp; i += G) {
        int I = circle_pos(i, r, js.nb), J = circle_pos(js.nb - 1 - i, r, js.nb);
        if (I > J) {
          const int t = I;
          I = J;
          J = t;
        }
        coop_wait(ver, I, J, base_ver + 1 + r, abort_word, local);
        coop_inter_pair<NW, B>(R, ld, I, J, round_log + (size_t)i * 16, nbp * 16, tol, cc, part, buf, lane, wave,
                               bcs[wave], local);
        coop_publish(ver, I, J, base_ver + 2 + r, local);
      }
      if (r == js.nb - 2 && wave == 0 && worker) {
        // this workgroup's counts of the sweep, published before the round's grid barrier
        int rot = cc.rotations;
        double om = cc.offnum / cc.offden;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          rot += __shfl_xor(rot, o, 64);
          om = fmax(om, __shfl_xor(om, o, 64));
        }
        if (lane == 0) {
          atomicAdd(&rot_count[sw], (unsigned long long)rot);
          atomicMax(&off_bits[sw], (unsigned long long)__double_as_longlong(om));
        }
      }
    }
    grid.sync();  // the sweep's counts are complete and every block is final
    if (threadIdx.x == 0) {
      sh_rot = (int)__hip_atomic_load(&rot_count[sw], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      sh_off = __longlong_as_double(
          (long long)__hip_atomic_load(&off_bits[sw], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    __syncthreads();
    const int total = sh_rot;
    sweeps = sw + 1;
    __syncthreads();
    if (total == 0) {
      conv = 1;
      break;
    }
    if (sh_off <= kGramCheckCos2) {
      double off2 = 0.0;
      if (coop_gram_clear<NW, B>(R, js, N, tol, stride, scratch, counters + 2 * max_sweeps, part, buf, lane, wave, off2)) {
        if (threadIdx.x == 0) sh_off = off2;
        __syncthreads();
        conv = 1;
        break;
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // a hand-over that gave up leaves wrong columns: report no convergence and poison R
    const bool aborted = __hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0ull;
    jres->sweeps = sweeps;
    jres->converged = aborted ? 0 : conv;
    jres->off = sweeps > 0 ? sqrt(sh_off) : 0.0;
    if (aborted) R[0] = __builtin_nan("");
  }
}

}  // namespace nsk
