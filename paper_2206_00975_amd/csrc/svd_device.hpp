// FP64 SVD of the sketch SA (line 3 of Algorithm 1) inside one workgroup.
//
// 1. Householder QR of SA (s x N, column-major) -> R (N x N upper triangular).  The right
//    singular vectors of SA and R coincide (SA = QR with Q orthonormal).
// 2. One-sided (Hestenes) Jacobi on the columns of R with V accumulated: a pair (p, q) with
//    alpha = |r_p|^2, beta = |r_q|^2, gamma = r_p.r_q is rotated by
//    zeta = (beta - alpha) / (2 gamma), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
//    c = 1/sqrt(1 + t^2), s = c t, unless |gamma| <= N u sqrt(alpha beta).  Pairs follow the
//    round-robin (circle) order: position 0 fixed, the others rotate by one per round, so
//    each round is a set of disjoint pairs processed concurrently by the waves.
// 3. sigma_j = |r_j|, sorted non-increasing; the trailing k columns of V are sign-normalised
//    (largest-magnitude entry positive, lowest index on ties) and written out.
//
// The working matrices R and V live in global memory (L2-resident at these sizes); all
// waves of the workgroup synchronise with barriers only, so the routine can run inside a
// persistent kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"
#include "wave_ops.hpp"

namespace nsk {

__device__ inline double wave_sum(double v) { return wave_sum64(v); }

struct SvdShared {
  double tau;
  double beta;
  int rotations;
  int pad;
  unsigned long long off_bits;
};

// Scratch needed in LDS: SvdShared + s doubles (Householder vector) + N doubles + N ints.
__host__ __device__ inline size_t svd_lds_bytes(int s, int N) {
  return sizeof(SvdShared) + (size_t)s * 8 + (size_t)N * 8 + (size_t)N * 4 + 64;
}

__device__ inline void householder_qr(double* __restrict__ A, int s, int N, double* vbuf, SvdShared* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = 0; j < N; ++j) {
    double* aj = A + (size_t)j * s;
    if (wave == 0) {
      double ss = 0;
      for (int i = j + 1 + lane; i < s; i += 64) ss += aj[i] * aj[i];
      ss = wave_sum(ss);
      const double alpha = aj[j];
      double tau = 0, beta = alpha, scal = 0;
      if (ss > 0) {
        const double nrm = sqrt(alpha * alpha + ss);
        beta = alpha >= 0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      for (int i = j + 1 + lane; i < s; i += 64) vbuf[i] = aj[i] * scal;
      if (lane == 0) {
        vbuf[j] = 1.0;
        sh->tau = tau;
        sh->beta = beta;
      }
    }
    __syncthreads();
    const double tau = sh->tau;
    if (tau != 0) {
      for (int c = j + 1 + wave; c < N; c += nw) {
        double* ac = A + (size_t)c * s;
        double d = 0;
        for (int i = j + lane; i < s; i += 64) d += vbuf[i] * ac[i];
        d = wave_sum(d) * tau;
        for (int i = j + lane; i < s; i += 64) ac[i] -= d * vbuf[i];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) aj[j] = sh->beta;
    __syncthreads();
  }
}

// Positions of the circle method for N' = N rounded up to even: position 0 is fixed and
// positions 1..N'-1 hold columns 1 + (p - 1 + r) mod (N' - 1) in round r; pair i joins
// positions i and N'-1-i.
__device__ inline int circle_col(int pos, int r, int n_even) {
  return pos == 0 ? 0 : 1 + (pos - 1 + r) % (n_even - 1);
}

// Jacobi on R (N x N column-major, ld N) accumulating V (N x N, starts as identity).
// Returns the number of sweeps; *conv = 1 if converged.
__device__ inline int jacobi(double* __restrict__ R, double* __restrict__ V, int N, int max_sweeps,
                             SvdShared* sh, int* conv, double* off_out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int n_even = N + (N & 1);
  const int P = n_even / 2;
  const double tol = (double)N * 0x1p-53;
  int sweeps = 0;
  *conv = 0;
  double off = 0;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    if (threadIdx.x == 0) {
      sh->rotations = 0;
      sh->off_bits = 0ull;
    }
    __syncthreads();
    for (int r = 0; r < n_even - 1; ++r) {
      for (int i = wave; i < P; i += nw) {
        int p = circle_col(i, r, n_even), q = circle_col(n_even - 1 - i, r, n_even);
        if (p > q) { const int tmp = p; p = q; q = tmp; }
        if (q >= N) continue;
        double* rp = R + (size_t)p * N;
        double* rq = R + (size_t)q * N;
        double a = 0, b = 0, g = 0;
        for (int e = lane; e < N; e += 64) {
          const double x = rp[e], y = rq[e];
          a += x * x;
          b += y * y;
          g += x * y;
        }
        a = wave_sum(a);
        b = wave_sum(b);
        g = wave_sum(g);
        const double nab = sqrt(a * b);
        if (nab > 0 && lane == 0) atomicMax(&sh->off_bits, (unsigned long long)__double_as_longlong(fabs(g) / nab));
        if (!(fabs(g) > tol * nab)) continue;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double sn = c * t;
        for (int e = lane; e < N; e += 64) {
          const double x = rp[e], y = rq[e];
          rp[e] = c * x - sn * y;
          rq[e] = sn * x + c * y;
        }
        double* vp = V + (size_t)p * N;
        double* vq = V + (size_t)q * N;
        for (int e = lane; e < N; e += 64) {
          const double x = vp[e], y = vq[e];
          vp[e] = c * x - sn * y;
          vq[e] = sn * x + c * y;
        }
        if (lane == 0) atomicAdd(&sh->rotations, 1);
      }
      __syncthreads();
    }
    sweeps = sw + 1;
    off = __longlong_as_double((long long)sh->off_bits);
    const int rot = sh->rotations;
    __syncthreads();
    if (rot == 0) {
      *conv = 1;
      break;
    }
  }
  *off_out = off;
  return sweeps;
}

// Full SVD pipeline for one instance.  sa: s x N column-major (overwritten).
// sigma (N, sorted) and order (N) are global outputs used by later stages.
__device__ inline void svd_instance(double* __restrict__ sa, int s, int N, int k, int max_sweeps,
                                    double* __restrict__ R, double* __restrict__ V,
                                    double* __restrict__ sigma, int* __restrict__ order,
                                    double* __restrict__ Vk, double* __restrict__ sigma_k, nsk_info* info,
                                    unsigned char* smem) {
  SvdShared* sh = reinterpret_cast<SvdShared*>(smem);
  double* vbuf = reinterpret_cast<double*>(smem + sizeof(SvdShared));
  double* nrm = vbuf + s;
  int* rk = reinterpret_cast<int*>(nrm + N);
  const int tid = threadIdx.x, nt = blockDim.x;

  householder_qr(sa, s, N, vbuf, sh);
  for (int e = tid; e < N * N; e += nt) {
    const int c = e / N, r = e % N;
    R[e] = r <= c ? sa[(size_t)c * s + r] : 0.0;
    V[e] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();
  int conv = 0;
  double off = 0;
  const int sweeps = jacobi(R, V, N, max_sweeps, sh, &conv, &off);
  // singular values = column norms
  const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  for (int c = wave; c < N; c += nw) {
    double a = 0;
    for (int e = lane; e < N; e += 64) a += R[(size_t)c * N + e] * R[(size_t)c * N + e];
    a = wave_sum(a);
    if (lane == 0) nrm[c] = sqrt(a);
  }
  __syncthreads();
  // rank by (norm descending, index ascending); NaN norms rank last, so the ranks are a
  // permutation of 0..N-1 for any input
  for (int c = tid; c < N; c += nt) {
    const double xv = nrm[c];
    const double x = xv != xv ? -1.0 : xv;
    int r = 0;
    for (int d = 0; d < N; ++d) {
      const double yv = nrm[d];
      const double y = yv != yv ? -1.0 : yv;
      r += (y > x) || (y == x && d < c);
    }
    rk[c] = r;
    order[r] = c;
    sigma[r] = xv;
  }
  __syncthreads();
  // trailing k vectors, sign-normalised
  for (int q = wave; q < k; q += nw) {
    const int c = order[N - k + q];
    const double* v = V + (size_t)c * N;
    double best = -1;
    int bi = 0;
    for (int e = lane; e < N; e += 64) {
      const double a = fabs(v[e]);
      if (a > best) { best = a; bi = e; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ob = __shfl_xor(best, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const double sgn = v[bi] < 0 ? -1.0 : 1.0;
    if (Vk)
      for (int e = lane; e < N; e += 64) Vk[(size_t)e * k + q] = sgn * v[e];
    if (sigma_k && lane == 0) sigma_k[q] = sigma[N - k + q];
  }
  if (info && tid == 0) {
    info->sweeps = sweeps;
    info->converged = conv;
    info->off = off;
    info->sigma_max = sigma[0];
  }
  __syncthreads();
}

}  // namespace nsk
