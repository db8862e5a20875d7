// Register-resident panel primitives shared by the QR and LU kernels.
//
// A panel of up to PANEL_M = 256 rows and 4*NS columns lives in the
// registers of one 256-thread workgroup: wave w owns columns w, w+4, w+8, ...
// (slot s holds column w + 4 s) and lane l holds rows l, l+64, l+128, l+192
// (slot q holds row l + 64 q).  Column operations then reduce within one
// wave (no block barrier), and only the vector that drives a step is shared
// through LDS.
#pragma once

#include "lrp_internal.h"

namespace lrp {

template <int NS>
__device__ __forceinline__ void panel_load(double (&y)[NS][4], const double *src,
                                           long ld, int m, int kk) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = wave + 4 * s;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      y[s][q] = (c < kk && i < m) ? src[i + (long)c * ld] : 0.0;
    }
  }
}

template <int NS>
__device__ __forceinline__ void panel_store(const double (&y)[NS][4], double *dst,
                                            long ld, int m, int kk) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = wave + 4 * s;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      if (c < kk && i < m) dst[i + (long)c * ld] = y[s][q];
    }
  }
}

// Column `s` of the register panel as 4 row slots (runtime s, unrolled
// selects instead of dynamic register indexing).
template <int NS>
__device__ __forceinline__ void col_get(const double (&y)[NS][4], int s, double (&x)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) x[q] = y[0][q];
#pragma unroll
  for (int s2 = 1; s2 < NS; ++s2)
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = (s2 == s) ? y[s2][q] : x[q];
}
template <int NS>
__device__ __forceinline__ void col_put(double (&y)[NS][4], int s, const double (&x)[4]) {
#pragma unroll
  for (int s2 = 0; s2 < NS; ++s2)
#pragma unroll
    for (int q = 0; q < 4; ++q) y[s2][q] = (s2 == s) ? x[q] : y[s2][q];
}

// Householder QR of the mp x kk panel (mp <= 256, kk <= 4 NS <= 64), LAPACK
// convention: H_j = I - tau_j v_j v_j^T, v_j(j) = 1, beta = -sign(alpha)||x||,
// tau = 0 when the part below the diagonal is already zero.  On return the
// panel holds R on and above the diagonal and v_j below it; taus[j] in LDS.
// vbuf: 2*256 doubles of LDS.
template <int NS>
__device__ void hh_qr_regs(double (&y)[NS][4], int mp, int kk, double *vbuf,
                           double *taus) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int jmax = min(mp, kk);
  for (int j = 0; j < jmax; ++j) {
    const int w = j & 3, s = j >> 2;
    double *vb = vbuf + (j & 1) * PANEL_M;
    if (wave == w) {
      double x[4];
      col_get(y, s, x);
      double ss = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lane + 64 * q;
        if (i > j && i < mp) ss += x[q] * x[q];
      }
      ss = wave_sum(ss);
      const double alpha = bcast_f64(x[0], j);   // j < 64: row j in slot 0
      double tj = 0.0, beta = alpha, scale = 0.0;
      if (ss != 0.0) {
        beta = -copysign(sqrt(alpha * alpha + ss), alpha);
        tj = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lane + 64 * q;
        double v = 0.0;
        if (i == j) {
          v = 1.0;
          x[q] = beta;
        } else if (i > j && i < mp) {
          x[q] *= scale;
          v = x[q];
        }
        vb[i] = v;
      }
      col_put(y, s, x);
      if (lane == 0) taus[j] = tj;
    }
    __syncthreads();
    const double tj = taus[j];
    double vv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) vv[q] = vb[lane + 64 * q];
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) {
      const int c = wave + 4 * s2;
      if (c > j && c < kk) {
        double d = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) d += vv[q] * y[s2][q];
        d = wave_sum(d) * tj;
#pragma unroll
        for (int q = 0; q < 4; ++q) y[s2][q] -= d * vv[q];
      }
    }
  }
}

// y <- H_0 H_1 ... H_{kr-1} y for reflectors stored below the diagonal of V
// (global memory, leading dimension ldv, rows >= m are zero) and taus tau[].
template <int NS>
__device__ void hh_apply_regs(double (&y)[NS][4], int m, int kr, int kk,
                              const double *V, long ldv, const double *tau) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = kr - 1; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;
    double vv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      vv[q] = (i == j) ? 1.0 : ((i > j && i < m) ? V[i + (long)j * ldv] : 0.0);
    }
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) {
      const int c = wave + 4 * s2;
      if (c < kk) {
        double d = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) d += vv[q] * y[s2][q];
        d = wave_sum(d) * tj;
#pragma unroll
        for (int q = 0; q < 4; ++q) y[s2][q] -= d * vv[q];
      }
    }
  }
}

__device__ __forceinline__ double pick4(double a, double b, double c, double d, int q) {
  return q == 0 ? a : (q == 1 ? b : (q == 2 ? c : d));
}

// Gaussian elimination with partial pivoting that only selects rows: rows are
// never moved, chosen ones are flagged.  piv_out[j] = local row of pivot j
// (j < min(mp, kk)).  A zero column picks the lowest unflagged row and
// eliminates nothing.  Ties in |value| go to the lowest row.
// lbuf: 2*256 doubles of LDS; sh_piv: int[2] of LDS.
template <int NS>
__device__ void gepp_select_regs(double (&y)[NS][4], int mp, int kk,
                                 double *lbuf, int *sh_piv, int *piv_out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int jmax = min(mp, kk);
  unsigned used = 0;   // bit q: row lane + 64 q already a pivot
  for (int j = 0; j < jmax; ++j) {
    const int w = j & 3, s = j >> 2;
    double *lb = lbuf + (j & 1) * PANEL_M;
    if (wave == w) {
      double x[4];
      col_get(y, s, x);
      double best = -1.0;
      int key = 0x7fffffff;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lane + 64 * q;
        if (i < mp && !((used >> q) & 1u)) {
          const double a = fabs(x[q]);
          if (a > best || (a == best && i < key)) {
            best = a;
            key = i;
          }
        }
      }
      wave_argmax(best, key);
      const int p = key;
      const double pv = pick4(bcast_f64(x[0], p & 63), bcast_f64(x[1], p & 63),
                              bcast_f64(x[2], p & 63), bcast_f64(x[3], p & 63),
                              p >> 6);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lane + 64 * q;
        double l = 0.0;
        if (i < mp && i != p && !((used >> q) & 1u) && pv != 0.0) l = x[q] / pv;
        lb[i] = l;
      }
      if (lane == 0) sh_piv[j & 1] = p;
    }
    __syncthreads();
    const int p = sh_piv[j & 1];
    if (threadIdx.x == 0) piv_out[j] = p;
    if ((p & 63) == lane) used |= 1u << (p >> 6);
    const int pq = p >> 6, pl = p & 63;
    double ll[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) ll[q] = lb[lane + 64 * q];
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) {
      const int c = wave + 4 * s2;
      if (c > j && c < kk) {
        // shuffle every row slot first, then choose: a select over the
        // register array itself would be turned into a scratch-memory index
        const double u = pick4(bcast_f64(y[s2][0], pl), bcast_f64(y[s2][1], pl),
                               bcast_f64(y[s2][2], pl), bcast_f64(y[s2][3], pl), pq);
#pragma unroll
        for (int q = 0; q < 4; ++q) y[s2][q] -= ll[q] * u;
      }
    }
  }
}

}  // namespace lrp
