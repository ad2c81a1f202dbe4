// Block one-sided Jacobi on R (N x N) with the column blocks held in registers.
//
// The N columns (padded with zero columns to nb * B, nb even) form nb blocks of B columns
// that stay in place in global memory (column-major, ld = 64 * NR, rows >= N zero).  One
// sweep is
//  * an intra phase: every block rotates the pairs of its own columns in circle order (B'
//    = B rounded up to even positions, position 0 fixed, one register shift per round), and
//  * an inter phase: every pair of blocks once, in circle order over the blocks; in block
//    round r the block pairs (circle(i, r), circle(nb - 1 - i, r)) are disjoint and each is
//    handled by one wave, which loads the two blocks T and U into registers (lane l holds
//    rows l + 64 j) and rotates (T_i, U_i) for all i in each of B sub-rounds, moving U's
//    registers up by one slot between sub-rounds so that every T_i meets every U_j.
// Rotation angles follow the one-sided Jacobi formulas; a pair is skipped when
// |gamma| <= tol sqrt(alpha beta).  In the inter phase only gamma = x.y is reduced per
// sub-round (one transposed reduction over the wave for all B pairs at once); the squared
// norms are exact at block load and updated as alpha - t gamma, beta + t gamma.  Every
// rotation (c, s), skipped ones as (1, 0), goes to a log in schedule order so that columns
// of V = J_1 J_2 ... are rebuilt later only for the vectors that are needed.
#pragma once

#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"
#include "wave_ops.hpp"

namespace nsk {

// ---------------------------------------------------------------- schedule arithmetic
__host__ __device__ inline int circle_pos(int pos, int r, int n) {  // n even
  return pos == 0 ? 0 : 1 + (pos - 1 + r) % (n - 1);
}

struct JacobiShape {
  int N;     // columns of R
  int NR;    // rows per lane (R has 64 * NR padded rows)
  int B;     // columns per block
  int nb;    // blocks (even)
  int bq;    // B rounded up to even (intra-block circle size)
  int spw;   // steps per sweep: (bq - 1) intra steps + B * (nb - 1) inter steps
};

__host__ __device__ inline int jacobi_nr(int N) {
  const int nr = (N + 63) / 64;
  return nr <= 5 ? nr : nr <= 8 ? 8 : 16;
}

__host__ __device__ constexpr int jacobi_block_size(int NR) {
  return NR == 1 ? 4 : NR == 2 ? 8 : NR == 3 ? 12 : NR == 4 ? 13 : NR == 5 ? 10 : NR <= 8 ? 6 : 3;
}

// Block size of the one-workgroup Jacobi (eight waves, a wave holding a whole block pair at NR
// rows per lane).  It keeps the multi-workgroup blocks while their nb / 2 pairs fit the eight
// waves in one pass.  Past that (NR = 4 with N > 208) a round takes two passes of the waves
// anyway, and blocks of 8 make those two passes full (16 pairs at N = 256) with each pair's two
// 8-column blocks in 128 registers a lane, where 13-column blocks (208 registers) spill.
__host__ __device__ constexpr int jacobi_block_size_wg(int NR, int N) {
  return NR == 4 && N > 16 * jacobi_block_size(4) ? 8 : jacobi_block_size(NR);
}

__host__ __device__ inline JacobiShape jacobi_shape_of(int N, int B) {
  JacobiShape s;
  s.N = N;
  s.NR = jacobi_nr(N);
  s.B = B;
  s.nb = (N + s.B - 1) / s.B;
  if (s.nb < 2) s.nb = 2;
  s.nb += s.nb & 1;
  s.bq = s.B + (s.B & 1);
  s.spw = (s.bq - 1) + s.B * (s.nb - 1);
  return s;
}

// shape of the multi-workgroup Jacobi (and of the one-workgroup one for NR <= 2)
__host__ __device__ inline JacobiShape jacobi_shape(int N) { return jacobi_shape_of(N, jacobi_block_size(jacobi_nr(N))); }

// shape of the one-workgroup Jacobi
__host__ __device__ inline JacobiShape jacobi_shape_wg(int N) {
  return jacobi_shape_of(N, jacobi_block_size_wg(jacobi_nr(N), N));
}

// Log layout of one sweep: intra steps have nb groups (blocks) of 16 slots, inter steps
// nb/2 groups (block pairs) of 16 slots.
__host__ __device__ inline size_t jacobi_log_step_offset(const JacobiShape& s, int st) {
  const size_t intra = (size_t)(s.bq - 1) * s.nb * 16;
  return st < s.bq - 1 ? (size_t)st * s.nb * 16 : intra + (size_t)(st - (s.bq - 1)) * (s.nb / 2) * 16;
}

__host__ __device__ inline size_t jacobi_log_entries_per_sweep(const JacobiShape& s) {
  return jacobi_log_step_offset(s, s.spw);
}

// ---------------------------------------------------------------- wave primitives
struct JacobiResult {
  int sweeps;
  int converged;
  double off;
};

struct JacobiCtx {
  double tol;
  int rotations;   // per-lane count
  double offmax;   // per-lane largest squared relative cosine g^2 / (a b)
};

// Rutishauser's rotation for the column pair with squared norms a, b and inner product g
// (the trig form of the two-sided Jacobi rotation): zeta = (b - a) / (2 g),
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), c = 1 / sqrt(1 + t^2), s = c t.  The pair is
// rotated when |g| > tol sqrt(a b), tested as g^2 > tol^2 a b.  Reciprocals and reciprocal
// square roots start from the hardware estimates and take two Newton steps each, which brings
// them to working precision: c^2 + s^2 = c^2 (1 + t^2) = 1, so the rotation stays orthogonal,
// and t solves the rotation's quadratic closely enough that the rotated pair's cosine falls
// below the tolerance (one step for t left cosines near 1e-13 and cost an extra sweep).  No branch: every quantity is computed
// and the result selected, so the dependency chains overlap.  When the pair is not rotated
// (including g = 0) the result is (c, s, t) = (1, 0, 0).
__device__ inline double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(y, fma(-x, y, 1.0), y);
  y = fma(y, fma(-x, y, 1.0), y);
  return y;
}
__device__ inline double rsq_nr(double x, int steps) {
  double y = __builtin_amdgcn_rsq(x);
  for (int k = 0; k < steps; ++k) {
    const double h = fma(-x * y, y, 1.0);  // 1 - x y^2
    y = fma(0.5 * y, h, y);
  }
  return y;
}
// Rotation of the column pair with squared norms a, b and inner product g.  The Rutishauser
// form t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)), zeta = (b - a) / (2 g), c = 1 / sqrt(1 + t^2),
// s = c t, is evaluated without zeta: with d = b - a and r = sqrt(d^2 + 4 g^2),
// t = sign(d) 2 g / (|d| + r), 1 + t^2 = 2 r / (|d| + r), so c = w u and s = sign(d) 2 g u with
// w = |d| + r and u = 1 / sqrt(2 r w).  c and s then follow from two reciprocal square roots in
// a chain instead of two reciprocals and two reciprocal square roots; t (for the norm updates
// a - t g, b + t g) takes a reciprocal of w beside the second.  c^2 + s^2 = 2 r w u^2 = 1 to
// rounding.  (sign(0) = +1.)
__device__ inline void jacobi_params(double a, double b, double g, double tol, double& c, double& s,
                                     double& t, bool& act) {
  act = g * g > (tol * tol) * (a * b);
  const double d = b - a;
  const double q = fma(d, d, 4.0 * g * g);
  const double r = q * rsq_nr(q, 2);
  const double w = fabs(d) + r;
  const double u = rsq_nr(2.0 * r * w, 2);
  const double g2 = d >= 0 ? 2.0 * g : -2.0 * g;
  c = act ? w * u : 1.0;
  s = act ? g2 * u : 0.0;
  t = act ? g2 * rcp_nr(w) : 0.0;
}

template <int NR>
__device__ inline void rot_cols(double (&x)[NR], double (&y)[NR], double c, double s) {
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const double a = x[r], b = y[r];
    x[r] = c * a - s * b;
    y[r] = s * a + c * b;
  }
}

// ---------------------------------------------------------------- intra phase
// Block `blk` alone: circle rounds q = 0..BQ-2 rotate the column at position i with the one
// at position BQ-1-i (i < BQ/2); positions 1..BQ-1 then shift down by one.  A padding
// position (B odd) holds a zero column and never rotates.  After each reduction pair i's
// sums sit in lanes i << SH .. (i << SH) + 2^SH - 1.
template <int NR, int B>
__device__ inline void jacobi_intra_block(double* __restrict__ R, int ld, int blk, double2* lg, int stride,
                                          JacobiCtx& cx, int lane) {
  constexpr int BQ = B + (B & 1);
  constexpr int H = BQ / 2;
  constexpr int SH = 6 - ceil_log2(H);
  const int pi = lane >> SH;
  const bool lead = (lane & ((1 << SH) - 1)) == 0 && pi < H;
  double X[BQ][NR];
  // wave-uniform column bases keep addressing in scalar registers plus one lane offset
  double* p = uniform_ptr(R + (size_t)blk * B * ld);
#pragma unroll
  for (int b = 0; b < BQ; ++b)
#pragma unroll
    for (int r = 0; r < NR; ++r) X[b][r] = b < B ? p[(size_t)b * ld + lane + 64 * r] : 0.0;
  // The squared norms are reduced once, then carried as in the block rounds: lanes of pair pi
  // hold alpha = |x_pi|^2 and beta = |x_{BQ-1-pi}|^2, updated by each rotation and moved with
  // the circle shift; only the inner products are reduced per step.
  double alpha, beta;
  {
    constexpr int SHB = 6 - ceil_log2(B);
    double v[16];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      v[b] = 0;
#pragma unroll
      for (int r = 0; r < NR; ++r) v[b] += X[b][r] * X[b][r];
    }
    const double nrm = reduce_t<B>(v, lane);  // lane l: position l >> SHB
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
      for (int i = 0; i < H; ++i) {
        v[i] = 0;
#pragma unroll
        for (int r = 0; r < NR; ++r) v[i] += X[i][r] * X[BQ - 1 - i][r];
      }
      g = reduce_t<H>(v, lane);
    }
    double c, s, t;
    bool act;
    jacobi_params(alpha, beta, g, cx.tol, c, s, t, act);
    if (lead) {
      const double ab = alpha * beta;
      if (ab > 0) cx.offmax = fmax(cx.offmax, g * g * rcp_nr(ab));
      if (act) cx.rotations++;
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
#pragma unroll
    for (int i = 0; i < H; ++i) rot_cols<NR>(X[i], X[BQ - 1 - i], bcast_d(c, i << SH), bcast_d(s, i << SH));
    // circle shift: position p takes position p+1 (p >= 1), the last takes position 1
    double tmp[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) tmp[r] = X[1][r];
#pragma unroll
    for (int b = 1; b < BQ - 1; ++b)
#pragma unroll
      for (int r = 0; r < NR; ++r) X[b][r] = X[b + 1][r];
#pragma unroll
    for (int r = 0; r < NR; ++r) X[BQ - 1][r] = tmp[r];
    lg += stride;
  }
  // after BQ - 1 shifts every column is back at its starting position
  p = opaque_uniform(p);
#pragma unroll
  for (int b = 0; b < B; ++b)
#pragma unroll
    for (int r = 0; r < NR; ++r) p[(size_t)b * ld + lane + 64 * r] = X[b][r];
}

// ---------------------------------------------------------------- inter phase
// Pair i's scalars (|T_i|^2, |U_i|^2, T_i . U_i, rotation) live in lanes i << SH ..
template <int NR, int B>
__device__ inline void jacobi_inter_pair(double* __restrict__ R, int ld, int I, int J, double2* lg, int stride,
                                         JacobiCtx& cx, int lane) {
  constexpr int SH = 6 - ceil_log2(B);
  const int pi = lane >> SH;
  const bool valid = pi < B;
  const bool lead = (lane & ((1 << SH) - 1)) == 0 && valid;
  double T[B][NR], U[B][NR];
  double* pt = uniform_ptr(R + (size_t)I * B * ld);
  double* pu = uniform_ptr(R + (size_t)J * B * ld);
#pragma unroll
  for (int b = 0; b < B; ++b)
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      T[b][r] = pt[(size_t)b * ld + lane + 64 * r];
      U[b][r] = pu[(size_t)b * ld + lane + 64 * r];
    }
  // exact squared norms at load
  double alpha, beta;
  {
    double v[16];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      v[i] = 0;
#pragma unroll
      for (int r = 0; r < NR; ++r) v[i] += T[i][r] * T[i][r];
    }
    alpha = reduce_t<B>(v, lane);
  }
  {
    double v[16];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      v[i] = 0;
#pragma unroll
      for (int r = 0; r < NR; ++r) v[i] += U[i][r] * U[i][r];
    }
    beta = reduce_t<B>(v, lane);
  }
  // lane of the pair whose U column moves into this lane's slot next sub-round
  const int nxt_pair = pi + 1 == B ? 0 : (valid ? pi + 1 : pi);
  const int nxt_lane = (nxt_pair << SH) | (lane & ((1 << SH) - 1));
  for (int j = 0; j < B; ++j) {
    // slot i of U holds block column (i + j) mod B
    double z[16];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      z[i] = 0;
#pragma unroll
      for (int r = 0; r < NR; ++r) z[i] += T[i][r] * U[i][r];
    }
    const double g = reduce_t<B>(z, lane);
    double c, s, t;
    bool act;
    jacobi_params(alpha, beta, g, cx.tol, c, s, t, act);
    if (!valid) {
      c = 1.0;
      s = 0.0;
      t = 0.0;
      act = false;
    }
    if (lead) {
      const double ab = alpha * beta;
      if (ab > 0) cx.offmax = fmax(cx.offmax, g * g * rcp_nr(ab));
      if (act) cx.rotations++;
      lg[pi] = make_double2(c, s);
    }
    if (act) {
      alpha = fmax(alpha - t * g, 0.0);
      beta = fmax(beta + t * g, 0.0);
    }
#pragma unroll
    for (int i = 0; i < B; ++i) rot_cols<NR>(T[i], U[i], bcast_d(c, i << SH), bcast_d(s, i << SH));
    // U slots move up by one; each pair takes the squared norm of its new U column from the
    // next pair's lanes
    double tmp[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) tmp[r] = U[0][r];
#pragma unroll
    for (int b = 0; b < B - 1; ++b)
#pragma unroll
      for (int r = 0; r < NR; ++r) U[b][r] = U[b + 1][r];
#pragma unroll
    for (int r = 0; r < NR; ++r) U[B - 1][r] = tmp[r];
    beta = __shfl(beta, nxt_lane, 64);
    lg += stride;
  }
  // after B moves the U slots are back in block order
  pt = opaque_uniform(pt);
  pu = opaque_uniform(pu);
#pragma unroll
  for (int b = 0; b < B; ++b)
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      pt[(size_t)b * ld + lane + 64 * r] = T[b][r];
      pu[(size_t)b * ld + lane + 64 * r] = U[b][r];
    }
}

// A sweep performs no rotation exactly when every column pair's cosine is already within the
// tolerance: no rotation means no column changes during the sweep, so each pair is tested on
// the columns as they stood before it.  Near convergence the largest cosine falls roughly
// quadratically from sweep to sweep (measured on the TLS sketch: 3e-2, 5e-7, 2e-14), so after a
// sweep whose largest cosine was at most 1e-6 the multi-workgroup kernel checks the condition
// directly on the Gram products of R (a fraction of a sweep's time) and stops when it holds,
// instead of running the confirming sweep.  (In the one-workgroup sweep used by the batched
// kernel the check measured slower overall on the planted-null-space instances, where it often
// fails; that sweep runs the confirming sweep.)
constexpr double kGramCheckCos2 = 1e-12;  // largest squared cosine of a sweep that triggers it

// Sweeps until a sweep performs no rotation (or max_sweeps).  All waves of the workgroup
// take part, with a barrier after the intra phase and after every block round.
// log: max_sweeps * jacobi_log_entries_per_sweep entries.  Returns sweeps; *conv, *off set.
template <int NR, int B>
__device__ inline int jacobi_block_sweeps(double* __restrict__ R, const JacobiShape& js, int max_sweeps,
                                          double2* __restrict__ log, int* sh_rot, double* sh_off, int* conv,
                                          double* off_out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int ld = 64 * NR;
  const int nbp = js.nb / 2;
  const size_t per_sweep = jacobi_log_entries_per_sweep(js);
  JacobiCtx cx;
  cx.tol = (double)js.N * 0x1p-53;
  int sweeps = 0;
  *conv = 0;
  double off = 0;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    if (threadIdx.x == 0) {
      *sh_rot = 0;
      *sh_off = 0.0;
    }
    __syncthreads();
    cx.rotations = 0;
    cx.offmax = 0.0;
    double2* sweep_log = log + (size_t)sw * per_sweep;
    for (int b = wave; b < js.nb; b += nw)
      jacobi_intra_block<NR, B>(R, ld, b, sweep_log + (size_t)b * 16, js.nb * 16, cx, lane);
    __syncthreads();
    for (int r = 0; r < js.nb - 1; ++r) {
      double2* round_log = sweep_log + jacobi_log_step_offset(js, js.bq - 1 + r * B);
      for (int i = wave; i < nbp; i += nw) {
        int I = circle_pos(i, r, js.nb), J = circle_pos(js.nb - 1 - i, r, js.nb);
        if (I > J) { const int t = I; I = J; J = t; }
        jacobi_inter_pair<NR, B>(R, ld, I, J, round_log + (size_t)i * 16, nbp * 16, cx, lane);
      }
      __syncthreads();
    }
    int rot = cx.rotations;
    double om = cx.offmax;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      rot += __shfl_xor(rot, o, 64);
      om = fmax(om, __shfl_xor(om, o, 64));
    }
    if (lane == 0) {
      atomicAdd(sh_rot, rot);
      atomicMax(reinterpret_cast<unsigned long long*>(sh_off), (unsigned long long)__double_as_longlong(om));
    }
    __syncthreads();
    sweeps = sw + 1;
    off = sqrt(*sh_off);
    const int total = *sh_rot;
    __syncthreads();
    if (total == 0) {
      *conv = 1;
      break;
    }
  }
  *off_out = off;
  return sweeps;
}

// ------------------------------------------------------------------ log replay
// x <- V x (fwd = false) takes the logged steps from last to first with [x_p, x_q] <-
// [c x_p + s x_q, -s x_p + c x_q]; x <- V^T x (fwd = true) takes them from first to last with
// [x_p, x_q] <- [c x_p - s x_q, s x_p + c x_q].  Rotations on padding columns were logged as
// (1, 0).
//
// One lane per logged rotation: in a block round, lane 16 g + i holds T_i and the U slot i of
// block pair g; in an intra phase, lane 8 g + i holds positions i and BQ-1-i of block g.
// Between steps the slots move exactly as the Jacobi kernel's registers did, here with DPP
// row rotations inside the 16- or 8-lane group.  A vector group of replay_waves(js) waves
// replays one vector (x in LDS, nb * B doubles); several groups replay different vectors at
// once.
//
// A phase is the intra phase of a sweep or one block round.  Every lane reads its own
// rotations of a phase (at most B, one per step, in processing order) straight from the log
// into registers, one phase ahead, so a step is a rotation and a slot move with no memory
// access on the chain; one barrier per phase hands x over between the lanes of a group.

// waves per vector group: 8 lanes per block in the intra phase (16 per pair in a round)
__host__ __device__ inline int replay_waves(const JacobiShape& js) { return (js.nb * 8 + 63) / 64; }

// Phase k of the replay (processing order) of `sweeps` sweeps: its sweep, round (-1 for the
// intra phase) and first log entry.
struct ReplayPhase {
  int sw, r;
  size_t begin;
};

__device__ inline ReplayPhase replay_phase(const JacobiShape& js, size_t per_sweep, int sweeps, bool fwd, int k) {
  const int per = js.nb;  // phases per sweep: intra + (nb - 1) rounds
  const int si = k / per, pi = k % per;
  ReplayPhase ph;
  ph.sw = fwd ? si : sweeps - 1 - si;
  ph.r = fwd ? pi - 1 : (pi < per - 1 ? per - 2 - pi : -1);
  const size_t intra = (size_t)(js.bq - 1) * js.nb * 16;
  const size_t round = (size_t)js.B * (js.nb / 2) * 16;
  ph.begin = (size_t)ph.sw * per_sweep + (ph.r < 0 ? 0 : intra + (size_t)ph.r * round);
  return ph;
}

template <bool FWD>
__device__ inline void rot_pair(double& x, double& y, double2 cs) {
  const double c = cs.x, s = FWD ? cs.y : -cs.y;
  const double a = x, b = y;
  x = c * a - s * b;
  y = s * a + c * b;
}

// The lane's rotations of phase ph in processing order: e[u] is step u (FWD) or step
// n - 1 - u (backward) of the phase's n steps; (1, 0) past n and for idle lanes, so that
// every lane can rotate unconditionally (idle lanes hold zeros).
template <int B, bool FWD>
__device__ inline void replay_fetch(const double2* __restrict__ log, const JacobiShape& js, const ReplayPhase& ph,
                                    int vl, bool member, double2 (&e)[B]) {
  constexpr int BQ = B + (B & 1);
  const bool intra = ph.r < 0;
  const int n = intra ? BQ - 1 : B;
  const int grp = intra ? vl >> 3 : vl >> 4, i = intra ? vl & 7 : vl & 15;
  const int groups = intra ? js.nb : js.nb / 2;  // log groups per step
  const bool act = member && grp < groups && i < (intra ? BQ / 2 : B);
  const double2* base = log + ph.begin + (size_t)grp * 16 + i;
  const size_t step = (size_t)groups * 16;
#pragma unroll
  for (int u = 0; u < B; ++u) {
    const int st = FWD ? u : n - 1 - u;
    e[u] = act && u < n ? base[st * step] : make_double2(1.0, 0.0);
  }
}

template <int B, bool FWD>
__device__ inline void jacobi_replay_dir(double* x, const double2* __restrict__ log, const JacobiShape& js,
                                         int sweeps, int vl, bool member) {
  constexpr int BQ = B + (B & 1);
  constexpr int H = BQ / 2;
  const int nb = js.nb, nbp = js.nb / 2;
  const size_t per_sweep = jacobi_log_entries_per_sweep(js);
  const int nphases = sweeps * nb;
  // lane roles: intra phase lane 8 g + i (positions i and BQ-1-i of block g), block round
  // lane 16 g + i (T_i and U slot i of pair g); idle lanes hold zeros and rotate by (1, 0)
  const int gi = vl >> 3, ii = vl & 7;
  const bool act_i = member && gi < nb && ii < H;
  const int gr = vl >> 4, ir = vl & 15;
  const bool act_r = member && gr < nbp && ir < B;
  // phase k applies cur while phase k + 1's rotations load into nxt; the two buffers swap
  // roles every phase (two phases per loop trip, so no register copies)
  auto phase = [&](int k, const double2 (&cur)[B], double2 (&nxt)[B]) {
    const ReplayPhase ph = replay_phase(js, per_sweep, sweeps, FWD, k);
    if (k + 1 < nphases)
      replay_fetch<B, FWD>(log, js, replay_phase(js, per_sweep, sweeps, FWD, k + 1), vl, member, nxt);
    lds_barrier();  // the previous phase's x updates are visible
    if (ph.r < 0) {
      const int pa = ii, pb = BQ - 1 - ii;
      double a = act_i && pa < B ? x[gi * B + pa] : 0.0;
      double b = act_i && pb < B ? x[gi * B + pb] : 0.0;
#pragma unroll
      for (int u = 0; u < BQ - 1; ++u) {
        if constexpr (!FWD && H > 1) {  // undo the circle shift that followed the step
          const double a_prev = lane_plus<15>(a), b_prev = lane_plus<15>(b), b_next = lane_plus<1>(b);
          const double na = ii == 0 ? a : ii == 1 ? b_prev : a_prev;
          const double nbv = ii + 1 < H ? b_next : a;
          a = na;
          b = nbv;
        }
        rot_pair<FWD>(a, b, cur[u]);
        if constexpr (FWD && H > 1) {  // circle shift: position p takes p + 1 (p >= 1), the last takes 1
          const double a_next = lane_plus<1>(a), b_prev = lane_plus<15>(b);
          const double na = ii == 0 ? a : ii + 1 < H ? a_next : b;
          const double nbv = ii == 0 ? a_next : b_prev;
          a = na;
          b = nbv;
        }
      }
      if (act_i) {
        if (pa < B) x[gi * B + pa] = a;
        if (pb < B) x[gi * B + pb] = b;
      }
    } else {
      const int gg = gr < nbp ? gr : 0;
      int I = circle_pos(gg, ph.r, nb), J = circle_pos(nb - 1 - gg, ph.r, nb);
      if (I > J) {
        const int u = I;
        I = J;
        J = u;
      }
      double T = act_r ? x[I * B + ir] : 0.0;
      double U = act_r ? x[J * B + ir] : 0.0;
#pragma unroll
      for (int u = 0; u < B; ++u) {
        if constexpr (!FWD) {  // undo the slot move that followed the sub-round
          const double from_prev = lane_plus<15>(U), from_last = lane_plus<(B - 1) % 16 ? (B - 1) % 16 : 15>(U);
          U = ir == 0 ? from_last : from_prev;
        }
        rot_pair<FWD>(T, U, cur[u]);
        if constexpr (FWD) {  // slot i takes slot i + 1 (mod B)
          const double from_next = lane_plus<1>(U), from_first = lane_plus<(17 - B) % 16 ? (17 - B) % 16 : 1>(U);
          U = ir == B - 1 ? from_first : from_next;
        }
      }
      if (act_r) {
        x[I * B + ir] = T;
        x[J * B + ir] = U;
      }
    }
  };
  double2 e0[B], e1[B];
  if (nphases > 0) replay_fetch<B, FWD>(log, js, replay_phase(js, per_sweep, sweeps, FWD, 0), vl, member, e0);
  for (int k = 0; k < nphases; k += 2) {
    phase(k, e0, e1);
    if (k + 1 < nphases) phase(k + 1, e1, e0);
  }
  lds_barrier();
}

// All threads of the workgroup call this with the same arguments except x and vl: vl is the
// thread's lane within its vector group (0 .. 64 * replay_waves - 1), member is false for
// threads outside any group (they take part in the barriers only), x the group's vector.
template <int B>
__device__ inline void jacobi_replay(double* x, const double2* __restrict__ log, const JacobiShape& js, int sweeps,
                                     bool fwd, int vl, bool member) {
  if (fwd)
    jacobi_replay_dir<B, true>(x, log, js, sweeps, vl, member);
  else
    jacobi_replay_dir<B, false>(x, log, js, sweeps, vl, member);
}

}  // namespace nsk
