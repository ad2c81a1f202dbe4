// Householder QR of the sketch SA (s x N, column-major) in one workgroup, panel by panel.
//
// For a panel of NB columns starting at j0, wave w owns panel column j0 + w in registers
// (lane l holds rows j0 + l + 64 i).  Column j0 + jj is reduced by its owner: with
// alpha = a_jj and sigma^2 the squared norm below it, beta = -sign(alpha) sqrt(alpha^2 +
// sigma^2), tau = (beta - alpha) / beta and v = (x - beta e) / (alpha - beta) (v_jj = 1);
// v goes to LDS and the later panel columns apply H = I - tau v v^T.  The columns to the
// right of the panel are then loaded once per panel, CPW at a time per wave, receive the NB
// reflections in order and are written back, so the trailing matrix is read and written once
// per NB columns and each Householder vector is read from LDS once per CPW columns.  R is
// written into a zero-filled N_pad x N_pad column-major buffer whose extra rows/columns stay
// zero.
#pragma once

#include <hip/hip_runtime.h>

#include "nsk_internal.hpp"
#include "wave_ops.hpp"

namespace nsk {

// LDS bytes: NB * s doubles of Householder vectors + NB taus.
__host__ __device__ inline size_t qr_panel_lds_bytes(int s, int NB) { return (size_t)NB * s * 8 + NB * 8 + 64; }

template <int RPL, int NB, int CPW>
__device__ inline void qr_panel(double* __restrict__ A, int s, int N, double* __restrict__ R, int ldr,
                                unsigned char* smem) {
  double* vbuf = reinterpret_cast<double*>(smem);      // NB x s (relative rows)
  double* tau = vbuf + (size_t)NB * s;                 // NB
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j0 = 0; j0 < N; j0 += NB) {
    const int nbc = N - j0 < NB ? N - j0 : NB;
    const int rows = s - j0;  // relative rows 0..rows-1
    // cl[0] holds a wave's panel column; all of cl holds its trailing columns afterwards
    double cl[CPW][RPL];
    double (&col)[RPL] = cl[0];
    const bool owner = wave < nbc;
    if (owner) {
      const double* a = uniform_ptr(A + (size_t)(j0 + wave) * s + j0);
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int rr = lane + 64 * i;
        col[i] = rr < rows ? a[rr] : 0.0;
      }
    }
    for (int jj = 0; jj < nbc; ++jj) {
      if (wave == jj) {
        // alpha at relative row jj, sigma^2 over rows > jj
        double ss = 0, alpha_part = 0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          if (rr > jj) ss += col[i] * col[i];
          if (rr == jj) alpha_part = col[i];
        }
        ss = wave_sum64(ss);
        const double alpha = wave_sum64(alpha_part);
        double t = 0, beta = alpha, scal = 0;
        if (ss > 0) {
          const double nrm = sqrt(alpha * alpha + ss);
          beta = alpha >= 0 ? -nrm : nrm;
          t = (beta - alpha) / beta;
          scal = 1.0 / (alpha - beta);
        }
        double* v = vbuf + (size_t)jj * s;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          if (rr < rows) v[rr] = rr < jj ? 0.0 : rr == jj ? 1.0 : col[i] * scal;
          // rows above the diagonal of this column are final entries of R
          if (rr < jj) R[(size_t)(j0 + jj) * ldr + j0 + rr] = col[i];
        }
        if (lane == 0) {
          tau[jj] = t;
          R[(size_t)(j0 + jj) * ldr + j0 + jj] = beta;
        }
      }
      // v and tau travel through LDS; R is not read again in this kernel
      lds_barrier();
      if (owner && wave > jj) {
        const double* v = vbuf + (size_t)jj * s;
        const double t = tau[jj];
        double d = 0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          if (rr < rows) d += v[rr] * col[i];
        }
        d = wave_sum64(d) * t;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          if (rr < rows) col[i] -= d * v[rr];
        }
      }
    }
    // trailing columns: the panel's reflections in order, one load/store per column
    for (int c0 = j0 + nbc + wave * CPW; c0 < N; c0 += nw * CPW) {
#pragma unroll
      for (int u = 0; u < CPW; ++u) {
        const bool cu = c0 + u < N;
        const double* a = uniform_ptr(A + (size_t)(cu ? c0 + u : c0) * s + j0);
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          cl[u][i] = cu && rr < rows ? a[rr] : 0.0;
        }
      }
      for (int jj = 0; jj < nbc; ++jj) {
        const double* v = vbuf + (size_t)jj * s;
        double d[CPW];
#pragma unroll
        for (int u = 0; u < CPW; ++u) d[u] = 0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          const double vv = rr < rows ? v[rr] : 0.0;
#pragma unroll
          for (int u = 0; u < CPW; ++u) d[u] += vv * cl[u][i];
        }
        const double tj = tau[jj];
        {
          // one transposed reduction for the CPW dot products, then broadcasts
          constexpr int SH = 6 - ceil_log2(CPW);
          double v16[16];
#pragma unroll
          for (int u = 0; u < CPW; ++u) v16[u] = d[u];
          const double tot = reduce_t<CPW>(v16, lane);
#pragma unroll
          for (int u = 0; u < CPW; ++u) d[u] = bcast_d(tot, u << SH) * tj;
        }
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          const double vv = rr < rows ? v[rr] : 0.0;
#pragma unroll
          for (int u = 0; u < CPW; ++u) cl[u][i] -= d[u] * vv;
        }
      }
#pragma unroll
      for (int u = 0; u < CPW; ++u) {
        if (c0 + u >= N) continue;
        double* a = opaque_uniform(A + (size_t)(c0 + u) * s + j0);
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int rr = lane + 64 * i;
          if (rr < nbc) R[(size_t)(c0 + u) * ldr + j0 + rr] = cl[u][i];
          else if (rr < rows) a[rr] = cl[u][i];
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace nsk
