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

template <int NS, typename T>
__device__ __forceinline__ void panel_store(const double (&y)[NS][4], T *dst,
                                            long ld, int m, int kk) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int c = wave + 4 * s;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      if (c < kk && i < m) dst[i + (long)c * ld] = (T)y[s][q];
    }
  }
}

// wave_sum of N values, stage by stage, so that the N reduction chains
// overlap (each value takes the same steps in the same order as wave_sum).
template <int N>
__device__ __forceinline__ void wave_sum_n(double (&v)[N]) {
#pragma unroll
  for (int g = 0; g < N; ++g) v[g] += dpp_f64<DPP_QUAD_1032>(v[g]);
#pragma unroll
  for (int g = 0; g < N; ++g) v[g] += dpp_f64<DPP_QUAD_2301>(v[g]);
#pragma unroll
  for (int g = 0; g < N; ++g) v[g] += dpp_f64<DPP_ROW_SHR4>(v[g]);
#pragma unroll
  for (int g = 0; g < N; ++g) v[g] += dpp_f64<DPP_ROW_SHR8>(v[g]);
#pragma unroll
  for (int g = 0; g < N; ++g) v[g] += dpp_rows_f64<DPP_ROW_BCAST15, 0xa>(v[g]);
#pragma unroll
  for (int g = 0; g < N; ++g) v[g] += dpp_rows_f64<DPP_ROW_BCAST31, 0xc>(v[g]);
#pragma unroll
  for (int g = 0; g < N; ++g) v[g] = readlane_f64(v[g], 63);
}

// Columns j = 4 S .. 4 S + 3 of the Householder QR below: column j lives in
// slot S of wave j - 4 S, so the slot index is a compile-time constant, and
// the trailing columns are the later slots of every wave plus slot S of the
// waves after the owner.
template <int NS, int S>
__device__ __forceinline__ void hh_qr_slot(double (&y)[NS][4], int mp, int kk, int jmax,
                                           double *vbuf, double *taus) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // trailing slots reduced G at a time, their reduction chains overlapping
  // (pays off once a wave holds 8 or more columns)
  constexpr int G = NS >= 8 ? 2 : 1;
  // kept rolled: the slots are already unrolled, and four copies of each
  // would double the code for no measured gain
#pragma unroll 1
  for (int w = 0; w < 4; ++w) {
    const int j = 4 * S + w;
    if (j >= jmax) return;
    double *vb = vbuf + (j & 1) * PANEL_M;
    if (wave == w) {
      double ss = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lane + 64 * q;
        if (i > j && i < mp) ss += y[S][q] * y[S][q];
      }
      ss = wave_sum(ss);
      const double alpha = bcast_f64(y[S][0], j);   // j < 64: row j in slot 0
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
          y[S][q] = beta;
        } else if (i > j && i < mp) {
          y[S][q] *= scale;
          v = y[S][q];
        }
        vb[i] = v;
      }
      if (lane == 0) taus[j] = tj;
    }
    __syncthreads();
    const double tj = taus[j];
    double vv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) vv[q] = vb[lane + 64 * q];
#pragma unroll
    for (int s0 = S; s0 < NS; s0 += G) {
      // the group's first column is wave + 4 s0, its last wave + 4 (s0 + G - 1)
      const bool any = ((s0 + G - 1 < NS ? s0 + G - 1 : NS - 1) > S || wave > w) &&
                       wave + 4 * s0 < kk;
      if (any) {
        double d[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
          d[g] = 0.0;
          if (s0 + g < NS) {
#pragma unroll
            for (int q = 0; q < 4; ++q) d[g] += vv[q] * y[s0 + g][q];
          }
        }
        wave_sum_n(d);
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int s2 = s0 + g, c = wave + 4 * s2;
          if (s2 < NS && (s2 > S || wave > w) && c < kk) {
            const double f = d[g] * tj;
#pragma unroll
            for (int q = 0; q < 4; ++q) y[s2][q] -= f * vv[q];
          }
        }
      }
    }
  }
}

template <int NS, int S>
struct HhQrSlots {
  static __device__ __forceinline__ void run(double (&y)[NS][4], int mp, int kk, int jmax,
                                             double *vbuf, double *taus) {
    if (4 * S >= jmax) return;
    hh_qr_slot<NS, S>(y, mp, kk, jmax, vbuf, taus);
    HhQrSlots<NS, S + 1>::run(y, mp, kk, jmax, vbuf, taus);
  }
};
template <int NS>
struct HhQrSlots<NS, NS> {
  static __device__ __forceinline__ void run(double (&)[NS][4], int, int, int, double *,
                                             double *) {}
};

// Householder QR of the mp x kk panel (mp <= 256, kk <= 4 NS <= 64), LAPACK
// convention: H_j = I - tau_j v_j v_j^T, v_j(j) = 1, beta = -sign(alpha)||x||,
// tau = 0 when the part below the diagonal is already zero.  On return the
// panel holds R on and above the diagonal and v_j below it; taus[j] in LDS.
// vbuf: 2*256 doubles of LDS.
template <int NS>
__device__ __forceinline__ void hh_qr_regs(double (&y)[NS][4], int mp, int kk, double *vbuf,
                           double *taus) {
  HhQrSlots<NS, 0>::run(y, mp, kk, min(mp, kk), vbuf, taus);
}

typedef double wy_d4 __attribute__((ext_vector_type(4)));

// LDS doubles that hh_apply_wy needs for rank bucket KM: a 64-row chunk of V
// (later the Gram matrix) and the KM x KM block Y (later Z, then M).
template <int KM>
constexpr int wy_lds() { return (64 + KM) * (KM + 1) + KM; }

// Entry (i, a) of the reflector matrix: zero above the diagonal and for
// a >= kr, one on it (also on the zero rows that pad a panel of m < k rows),
// the stored vector below it for i < m.
__device__ __forceinline__ double wy_v(const double *V, long ldv, int m, int kr, int i,
                                       int a) {
  if (a >= kr || i < a) return 0.0;
  if (i == a) return 1.0;
  return (i < m) ? V[i + (long)a * ldv] : 0.0;
}

// y <- H_0 H_1 ... H_{kr-1} [Y; 0], the k x k block Y (Y == nullptr: the
// identity) on top of zero rows, in compact WY form.  With V = [v_0 ..
// v_{kr-1}], applying H_{kr-1} first gives
//     H_0 ... H_{kr-1} [Y; 0] = [Y; 0] - V M,
//     m_j = tau_j (z_j - sum_{l > j} (v_j . v_l) m_l),   z_j = v_j^T [Y; 0],
// rows m_j of M by back substitution from the last.  The Gram matrix V^T V
// (a reduction over the panel rows) and Z = V^T [Y; 0] (only the top kk rows)
// run on the float64 matrix cores, so the per-reflector reductions over all
// rows of the sequential form disappear.  y is written in full (rows of the
// m-row panel, columns < kk).  lds: wy_lds<4 NS>() doubles.
template <int NS>
__device__ void hh_apply_wy(double (&y)[NS][4], int m, int kr, int kk, const double *V,
                            long ldv, const double *tau, const double *Y, long ldy,
                            double *lds) {
  constexpr int KM = 4 * NS, LD = KM + 1, NT = KM / 16, NTT = NT * NT;
  constexpr int TPW = (NTT + 3) / 4;   // Gram / Z tiles per wave
  double *sV = lds;                    // [64][LD] chunk of V, then G [KM][LD]
  double *sY = lds + 64 * LD;          // [KM][LD] Y, then Z, then M
  double *stau = sY + KM * LD;         // [KM] the reflectors' tau
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  // the thread's share of V, all loads in flight at once: rows lane + 64 q,
  // columns wave + 4 u (the register-panel layout)
  double vr[NS][4];
#pragma unroll
  for (int u = 0; u < NS; ++u)
#pragma unroll
    for (int q = 0; q < 4; ++q) vr[u][q] = wy_v(V, ldv, m, kr, lane + 64 * q, wave + 4 * u);
  // Y and tau to LDS, every load in flight at once (r, c < KM <= the Y
  // block's KMAX rows and columns, so the unmasked loads stay inside it)
  {
    constexpr int PY = KM * KM / NTHR;
    double yv[PY];
#pragma unroll
    for (int u = 0; u < PY; ++u) {
      const int e = tid + u * NTHR, r = e / KM, c = e - r * KM;
      yv[u] = Y ? Y[r + (long)c * ldy] : (r == c ? 1.0 : 0.0);
    }
    const double tv = (tid < kr) ? tau[tid] : 0.0;
#pragma unroll
    for (int u = 0; u < PY; ++u) {
      const int e = tid + u * NTHR, r = e / KM, c = e - r * KM;
      sY[r * LD + c] = (r < kk && c < kk) ? yv[u] : 0.0;
    }
    if (tid < KM) stau[tid] = tv;
  }
  // Gram tiles: only ta <= tb (the solve below reads G above its diagonal);
  // Z = V^T [Y; 0] tiles: all of them
  constexpr int NTG = NT * (NT + 1) / 2, TPG = (NTG + 3) / 4;
  int gta[TPG], gtb[TPG];
#pragma unroll
  for (int u = 0; u < TPG; ++u) {
    int ta = 0, rem = wave + 4 * u;
    while (ta < NT - 1 && rem >= NT - ta) rem -= NT - ta++;
    gta[u] = ta;
    gtb[u] = ta + rem;
  }
  wy_d4 gacc[TPG], zacc[TPW];
#pragma unroll
  for (int u = 0; u < TPG; ++u) gacc[u] = (wy_d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < TPW; ++u) zacc[u] = (wy_d4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (64 * q >= m) break;
    __syncthreads();   // the previous chunk is consumed (and sY is written)
#pragma unroll
    for (int u = 0; u < NS; ++u) sV[lane * LD + wave + 4 * u] = vr[u][q];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < TPG; ++u) {
      if (wave + 4 * u < NTG) {
        const int ta = gta[u], tb = gtb[u];
        // A[i][k] = V(row 4 ks + k, col 16 ta + i): lane i + 16 k; B likewise
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
          const double a = sV[(4 * ks + g) * LD + 16 * ta + li];
          const double b = sV[(4 * ks + g) * LD + 16 * tb + li];
          gacc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, gacc[u], 0, 0, 0);
        }
      }
    }
    if (q == 0) {
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        const int t = wave + 4 * u;
        if (t < NTT) {
          const int ta = t / NT, tb = t - ta * NT;
#pragma unroll
          for (int ks = 0; ks < KM / 4; ++ks) {
            const double a = sV[(4 * ks + g) * LD + 16 * ta + li];
            const double b = sY[(4 * ks + g) * LD + 16 * tb + li];
            zacc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, zacc[u], 0, 0, 0);
          }
        }
      }
    }
  }
  __syncthreads();
  // D[i][j]: lane j + 16 (i % 4), register i / 4
#pragma unroll
  for (int u = 0; u < TPG; ++u) {
    if (wave + 4 * u < NTG) {
      const int ta = gta[u], tb = gtb[u];
#pragma unroll
      for (int r = 0; r < 4; ++r) sV[(16 * ta + 4 * r + g) * LD + 16 * tb + li] = gacc[u][r];
    }
  }
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int t = wave + 4 * u;
    if (t < NTT) {
      const int ta = t / NT, tb = t - ta * NT;
#pragma unroll
      for (int r = 0; r < 4; ++r) sY[(16 * ta + 4 * r + g) * LD + 16 * tb + li] = zacc[u][r];
    }
  }
  __syncthreads();
  // M in place of Z, by 16-row blocks from the last.  In a block one lane
  // per column solves the rows with the block's M values in registers; then
  // all threads take the block's part out of the rows above it.
  for (int j0 = ((kr - 1) / 16) * 16; j0 >= 0; j0 -= 16) {
    const int j1 = min(kr, j0 + 16);
    if (wave == 0 && lane < kk) {
      double mb[16];
#pragma unroll
      for (int jj = 15; jj >= 0; --jj) {
        const int j = j0 + jj;
        double v = 0.0;
        if (j < j1) {
          double acc = 0.0;
#pragma unroll
          for (int ll = jj + 1; ll < 16; ++ll) acc += sV[j * LD + j0 + ll] * mb[ll];
          v = stau[j] * (sY[j * LD + lane] - acc);
          sY[j * LD + lane] = v;
        }
        mb[jj] = v;
      }
    }
    __syncthreads();
    for (int e = tid; e < j0 * kk; e += NTHR) {
      const int jr = e / kk, c = e - jr * kk;
      double acc = 0.0;
      for (int l = j0; l < j1; ++l) acc += sV[jr * LD + l] * sY[l * LD + c];
      sY[jr * LD + c] -= acc;
    }
    __syncthreads();
  }
  // y = [Y; 0] - V M  (columns >= kk of M are zero).  Y has kk <= 64 rows,
  // all in the first row slot; lane, c < KMAX stay inside the Y block, so
  // the loads go unmasked and all at once.
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int c = wave + 4 * sl;
    const double yv = Y ? Y[lane + (long)c * ldy] : (lane == c ? 1.0 : 0.0);
    y[sl][0] = (c < kk && lane < kk) ? yv : 0.0;
#pragma unroll
    for (int q = 1; q < 4; ++q) y[sl][q] = 0.0;
  }
  for (int a0 = 0; a0 < kr; a0 += 4) {
    double v[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) v[t][q] = wy_v(V, ldv, m, kr, lane + 64 * q, a0 + t);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (a0 + t >= kr) break;
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) {
        const double mv = sY[(a0 + t) * LD + wave + 4 * sl];
#pragma unroll
        for (int q = 0; q < 4; ++q) y[sl][q] -= v[t][q] * mv;
      }
    }
  }
}

__device__ __forceinline__ double pick4(double a, double b, double c, double d, int q) {
  return q == 0 ? a : (q == 1 ? b : (q == 2 ? c : d));
}

// Columns j = 4 S .. 4 S + 3 of the pivot selection below (column j in slot
// S of wave j - 4 S, the slot index a compile-time constant).
template <int NS, int S>
__device__ __forceinline__ void gepp_slot(double (&y)[NS][4], int mp, int kk, int jmax,
                                          unsigned &used, double *lbuf, int *sh_piv,
                                          int *piv_out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // kept rolled: the slots are already unrolled, and four copies of each
  // would double the code for no measured gain
#pragma unroll 1
  for (int w = 0; w < 4; ++w) {
    const int j = 4 * S + w;
    if (j >= jmax) return;
    double *lb = lbuf + (j & 1) * PANEL_M;
    if (wave == w) {
      double best = -1.0;
      int key = 0x7fffffff;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lane + 64 * q;
        if (i < mp && !((used >> q) & 1u)) {
          const double a = fabs(y[S][q]);
          if (a > best || (a == best && i < key)) {
            best = a;
            key = i;
          }
        }
      }
      wave_argmax(best, key);
      const int p = key;
      const double pv = pick4(bcast_f64(y[S][0], p & 63), bcast_f64(y[S][1], p & 63),
                              bcast_f64(y[S][2], p & 63), bcast_f64(y[S][3], p & 63),
                              p >> 6);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = lane + 64 * q;
        double l = 0.0;
        if (i < mp && i != p && !((used >> q) & 1u) && pv != 0.0) l = y[S][q] / pv;
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
    // trailing columns: the later slots, and slot S of the waves after w
#pragma unroll
    for (int s2 = S; s2 < NS; ++s2) {
      const int c = wave + 4 * s2;
      if ((s2 > S || wave > w) && c < kk) {
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

template <int NS, int S>
struct GeppSlots {
  static __device__ __forceinline__ void run(double (&y)[NS][4], int mp, int kk, int jmax,
                                             unsigned &used, double *lbuf, int *sh_piv,
                                             int *piv_out) {
    if (4 * S >= jmax) return;
    gepp_slot<NS, S>(y, mp, kk, jmax, used, lbuf, sh_piv, piv_out);
    GeppSlots<NS, S + 1>::run(y, mp, kk, jmax, used, lbuf, sh_piv, piv_out);
  }
};
template <int NS>
struct GeppSlots<NS, NS> {
  static __device__ __forceinline__ void run(double (&)[NS][4], int, int, int, unsigned &,
                                             double *, int *, int *) {}
};

// Gaussian elimination with partial pivoting that only selects rows: rows are
// never moved, chosen ones are flagged.  piv_out[j] = local row of pivot j
// (j < min(mp, kk)).  A zero column picks the lowest unflagged row and
// eliminates nothing.  Ties in |value| go to the lowest row.
// lbuf: 2*256 doubles of LDS; sh_piv: int[2] of LDS.
template <int NS>
__device__ __forceinline__ void gepp_select_regs(double (&y)[NS][4], int mp, int kk,
                                 double *lbuf, int *sh_piv, int *piv_out) {
  unsigned used = 0;   // bit q: row lane + 64 q already a pivot
  GeppSlots<NS, 0>::run(y, mp, kk, min(mp, kk), used, lbuf, sh_piv, piv_out);
}

}  // namespace lrp
