// 3D path: Tucker cross of the divided spectrum (the paper's 3D case is
// promised in Section 4.1 and left open in Section 7; Tucker cross is cited
// in Section 4.2, the Tucker format and its rounding in Section 3,
// eq. "tucker").
//
// With Uh_d = S U_d the divided spectrum is
//     Xh(i0, i1, i2) = (G x_0 Uh_0[i0] x_1 Uh_1[i1] x_2 Uh_2[i2]) / D(i0, i1, i2),
// D the operator's eigenvalue (lambda_i0 + lambda_i1 + lambda_i2 for the
// 7-point Laplacian).  Each mode d keeps a pivot set I_d (k_d indices).  An
// outer sweep approximates, for every mode at once, its fiber matrix
//     C_d[i, j + k_p l] = Xh restricted to mode d's index i and the pair
//                         (I_p[j], I_q[l]) of the other modes p < q,
//                       = (Uh_d[i] . W_d[j + k_p l]) / (lambda_i + mu_(j + k_p l)),
//     W_d[j + k_p l, a] = sum_bc G_d[a, b, c] Uh_p[I_p[j], b] Uh_q[I_q[l], c],
// an n x k_p k_q matrix of the 2D kind (rectangular, general column
// denominators), by the cross kernels of the 2D solver to eps/sqrt(3): its
// column basis Q_d (n x k_d) and maxvol rows give the new I_d and k_d.  The
// outer sweeps stop at the first one (from the second on) whose mode ranks
// k_d repeat the previous sweep's (the sweep cap ends them otherwise).  The
// final bases and pivots define the interpolating projectors
// P_d = Q_d (Q_d[I_d, :])^-1 E_{I_d}^T, and
//     X~ = Xh x_0 P_0 x_1 P_1 x_2 P_2 = C x_d Q_d,
//     C = Xh(I_0, I_1, I_2) x_0 (Q_0[I_0])^-1 x_1 (Q_1[I_1])^-1 x_2 (Q_2[I_2])^-1.
// The core C (k_0 x k_1 x k_2) is then rounded by truncated HOSVD at
// eps/sqrt(3) per mode: the left singular vectors W_d of each unfolding of C
// come from TSQR of the unfolding's transpose plus the Jacobi SVD of its R
// factor (the 2D kernels again), so the output is
//     factors S (Q_d W_d[:, :R_d])  (orthonormal columns),
//     core    C x_0 W_0^T x_1 W_1^T x_2 W_2^T.
// Work and memory are linear in n: a mode slot holds n x 64 and 4096 x 64
// panels.
#include "lrp_internal.h"

namespace lrp {
namespace {

// the two other modes of mode d, p < q
__device__ __forceinline__ void other_modes(int d, int &p, int &q) {
  p = (d == 0) ? 1 : 0;
  q = (d == 2) ? 1 : 2;
}

// The outer decision of every solve whose three mode crosses have finished
// (one thread per solve): record the mode ranks and pivot sets; restart the
// crosses on the new fibers (P3_SETUP) unless the ranks repeat the previous
// sweep's or the sweep cap is reached, then the core (P3_CORE).  A non-finite
// input or a zero mode (zero solution) finishes at once.
__global__ void k_fiber_outer(Solve3D *S) {
  Solve3D &s = S[blockIdx.x];
  if (threadIdx.x != 0 || s.phase != P3_CROSS) return;
  for (int d = 0; d < 3; ++d)
    if (s.inner[d]->active != ACT_DONE) return;
  int st = LRP_OK;
  bool zero = false;
  for (int d = 0; d < 3; ++d) {
    const int sd = s.inner[d]->status;
    if (sd == LRP_ENONFINITE) st = LRP_ENONFINITE;
    else if (sd != LRP_OK && st == LRP_OK) st = sd;
    zero |= (s.inner[d]->nrm == 0.0);
  }
  if (st == LRP_ENONFINITE || zero) {
    s.cross_status = st;
    s.R[0] = s.R[1] = s.R[2] = 0;
    s.status = (st == LRP_ENONFINITE) ? st : LRP_OK;
    s.out_ok = 1;
    s.nrm = 0.0;
    s.phase = P3_DONE;
    return;
  }
  s.outer += 1;
  bool same = s.outer >= 2;
  for (int d = 0; d < 3; ++d) {
    const Solve2D &in = *s.inner[d];
    same &= (in.k == s.kf[d]);
    s.kf[d] = in.k;
    for (int t = 0; t < in.k; ++t) s.If[d][t] = clamp_row(in.I[t], s.n);
  }
  if (st == LRP_OK && !same && s.outer < s.max_outer) {
    s.phase = P3_SETUP;
    return;
  }
  if (st == LRP_OK && !same) st = LRP_ENOCONV;
  s.cross_status = st;
  for (int d = 0; d < 3; ++d) s.k[d] = s.kf[d];
  s.phase = P3_CORE;
}

// Pivot set of mode e for the fibers of the sweep: the last outer sweep's,
// or before the first, k evenly spaced indices (k = rank + kick, capped).
__device__ int fiber_pivots(const Solve3D &s, int e, int *out, int *scratch) {
  if (s.outer > 0) {
    for (int t = 0; t < s.kf[e]; ++t) out[t] = s.If[e][t];
    return s.kf[e];
  }
  const int k = min(min(s.r[e] + s.kick, s.kcap), s.n);
  spread_indices(s.n, k, scratch, 0, out, 0);
  return k;
}

// T_d[a + r_d (b + r_p l)] = sum_c G_d[a, b, c] Uh_q[I_q[l], c] (blockIdx.z =
// 3 s + d; first block also restarts the mode slot).
__global__ __launch_bounds__(NTHR) void k_fiber_T(Solve3D *S) {
  Solve3D &s = S[blockIdx.z / 3];
  const int d = blockIdx.z % 3;
  if (s.phase != P3_SETUP) return;
  int p, q;
  other_modes(d, p, q);
  __shared__ int Iq[KMAX], scr[KMAX];
  __shared__ int kq_s;
  if (threadIdx.x == 0) kq_s = fiber_pivots(s, q, Iq, scr);
  __syncthreads();
  const int kq = kq_s;
  const int rd = s.r[d], rp = s.r[p], rq = s.r[q];
  const long idx = (long)blockIdx.x * NTHR + threadIdx.x;
  if (idx >= (long)rd * rp * kq) return;
  const int a = (int)(idx % rd);
  const int b = (int)((idx / rd) % rp);
  const int l = (int)(idx / ((long)rd * rp));
  // G index with i_d = a, i_p = b, i_q = c
  const long stg[3] = {1, s.r[0], (long)s.r[0] * s.r[1]};
  const long base = a * stg[d] + b * stg[p];
  const Solve2D &mq = *s.inner[q];
  const double *uq = mq.Uh + Iq[l];
  double acc = 0.0;
  for (int c = 0; c < rq; ++c) acc += s.G[base + c * stg[q]] * uq[(long)c * mq.ldu];
  if (!isfinite(acc)) s.inner[d]->nonfinite = 1;
  s.T[d][idx] = acc;
}

// Column side of mode d's fiber matrix: W_d rows (the slot's Vh) and the
// column tables, zero columns beyond k_p k_q; block (x, 3 s + d) covers
// columns [256 x, 256 x + 256).  Block 0 resets the mode slot to start a
// cross (as a new problem: initial column choice, k0 = rank + kick).
__global__ __launch_bounds__(NTHR) void k_fiber_cols(Solve3D *S) {
  Solve3D &s = S[blockIdx.z / 3];
  const int d = blockIdx.z % 3;
  if (s.phase != P3_SETUP) return;
  Solve2D &in = *s.inner[d];
  int p, q;
  other_modes(d, p, q);
  __shared__ int Ip[KMAX], Iq[KMAX], scr[KMAX];
  __shared__ int kk[2];
  if (threadIdx.x == 0) {
    kk[0] = fiber_pivots(s, p, Ip, scr);
    kk[1] = fiber_pivots(s, q, Iq, scr);
  }
  __syncthreads();
  const int kp = kk[0], kq = kk[1], m = kp * kq;
  const int rd = s.r[d], rp = s.r[p];
  const int col = blockIdx.x * NTHR + threadIdx.x;
  const bool prod = in.lq_r != nullptr;
  if (col < FIB_M) {
    const bool live = col < m;
    const int j = live ? col % kp : 0, l = live ? col / kp : 0;
    const int ip = Ip[j], iq = Iq[l];
    // eigenvalue factors of the column (the mode slot's row tables are the
    // grid's: lambda, or the Stokes factors p = 2 sin^2/h, q = 2 cos^2/h)
    if (!prod) {
      s.lamc[d][col] = live ? in.lam_r[ip] + in.lam_r[iq] : 1.0;
    } else {
      // 4 (s_i c_j c_l + c_i s_j c_l + c_i c_j s_l)/h^2 = p_i Qc + q_i Pc,
      // Pc = h/2 (p_j q_l + q_j p_l), Qc = h/2 q_j q_l
      const double hh = 0.5 / (double)(s.n + 1);
      s.lamc[d][col] = live ? hh * (in.lam_r[ip] * in.lq_r[iq] + in.lq_r[ip] * in.lam_r[iq]) : 1.0;
      s.lqc[d][col] = live ? hh * (in.lq_r[ip] * in.lq_r[iq]) : 0.0;
    }
    const Solve2D &mp = *s.inner[p];
    const double *T = s.T[d] + (long)rd * rp * l;
    double *out = in.Vh + col;
    for (int a0 = 0; a0 < rd; a0 += 16) {
      double acc[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) acc[t] = 0.0;
      if (live) {
        for (int b = 0; b < rp; ++b) {
          const double u = mp.Uh[ip + (long)b * mp.ldu];
#pragma unroll
          for (int t = 0; t < 16; ++t)
            if (a0 + t < rd) acc[t] += u * T[a0 + t + (long)rd * b];
        }
      }
#pragma unroll
      for (int t = 0; t < 16; ++t)
        if (a0 + t < rd) out[(long)(a0 + t) * in.ldv] = acc[t];
    }
  }
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  // restart the mode cross on the new fiber matrix
  in.lam_c = s.lamc[d];
  in.lq_c = prod ? s.lqc[d] : nullptr;
  in.kcap = min(min(s.kcap, s.n), m);
  const int k0 = min(s.r[d] + s.kick, in.kcap);
  in.k0 = k0;
  in.k = min(s.r[d], k0);
  in.kp = 0;
  in.R = 0;
  in.sweep = 0;
  in.next = NEXT_CONTINUE;
  in.status = LRP_OK;
  in.mv_done = 0;
  in.mv_swaps = 0;
  in.kgrow = 0;
  in.nrm = 0.0;
  in.change = -1.0;
  in.tail = -1.0;
  double *t;
  if (in.Ap < in.A) t = in.A, in.A = in.Ap, in.Ap = t;
  if (in.Bp < in.B) t = in.B, in.B = in.Bp, in.Bp = t;
  if (in.sigp < in.sig) t = in.sig, in.sig = in.sigp, in.sigp = t;
  in.active = (s.r[d] > 0) ? ACT_INIT : ACT_DONE;
}

// Solves whose fibers were just built start their mode crosses.
__global__ void k_fiber_go(Solve3D *S) {
  Solve3D &s = S[blockIdx.x];
  if (threadIdx.x == 0 && s.phase == P3_SETUP) s.phase = P3_CROSS;
}

// ---- mode products of the core: out = in x_ax M, M(a, t) given per stage.
//  0: G    x_0 Uh_0[I_0]  -> buf1      3: buf1 x_0 Inv_0 -> buf0
//  1: buf1 x_1 Uh_1[I_1]  -> buf0      4: buf0 x_1 Inv_1 -> buf1
//  2: buf0 x_2 Uh_2[I_2]  -> buf1,     5: buf1 x_2 Inv_2 -> buf0 (= C)
//     divided by the eigenvalue sums
//  6: buf0 x_0 W_0^T -> buf1   7: buf1 x_1 W_1^T -> buf0   8: buf0 x_2 W_2^T -> Gx
struct Stage {
  int ax;
  int din[3], dout[3];
  const double *in;
  double *out;
};

__device__ Stage stage_of(const Solve3D &s, int st) {
  Stage g;
  g.ax = st % 3;
  for (int i = 0; i < 3; ++i) {
    int v;
    if (st < 3) v = (i < st) ? s.k[i] : s.r[i];          // gathers: r -> k
    else if (st < 6) v = s.k[i];                          // inverses: k
    else v = (i < st - 6) ? s.R[i] : s.k[i];             // truncation: k -> R
    g.din[i] = v;
    g.dout[i] = (i == g.ax) ? ((st < 6) ? s.k[i] : s.R[i]) : v;
  }
  // stage st reads buf1 when st is odd, buf0 when even (stage 0: G) and
  // writes the other buffer (stage 8: Gx)
  g.in = (st == 0) ? s.G : ((st & 1) ? s.buf1 : s.buf0);
  g.out = (st == 8) ? s.Gx : ((st & 1) ? s.buf0 : s.buf1);
  return g;
}

__global__ __launch_bounds__(NTHR) void k_core_stage(int st, Solve3D *S) {
  Solve3D &s = S[blockIdx.y];
  if (st < 6) {
    if (s.phase != P3_CORE) return;
  } else {
    if (s.phase != P3_OUT || !s.out_ok) return;
  }
  const Stage g = stage_of(s, st);
  const int ax = g.ax;
  // wave-uniform selects instead of dynamically indexed arrays (no scratch)
  const int o0 = g.dout[0], o1 = g.dout[1], o2 = g.dout[2];
  const long total = (long)o0 * o1 * o2;
  const int tlen = ax == 0 ? g.din[0] : (ax == 1 ? g.din[1] : g.din[2]);
  const long s1 = g.din[0], s2 = (long)g.din[0] * g.din[1];
  const long sax = ax == 0 ? 1 : (ax == 1 ? s1 : s2);
  const Solve2D &ia = *s.inner[ax];
  for (long o = (long)blockIdx.x * NTHR + threadIdx.x; o < total; o += (long)gridDim.x * NTHR) {
    const int i0 = (int)(o % o0);
    const int i1 = (int)((o / o0) % o1);
    const int i2 = (int)(o / ((long)o0 * o1));
    const int a = ax == 0 ? i0 : (ax == 1 ? i1 : i2);
    const long base = (ax == 0 ? 0 : i0) + (ax == 1 ? 0 : i1 * s1) + (ax == 2 ? 0 : i2 * s2);
    double acc = 0.0;
    if (st < 3) {
      const double *u = ia.Uh + clamp_row(ia.I[a], s.n);
      for (int t = 0; t < tlen; ++t) acc += u[(long)t * ia.ldu] * g.in[base + t * sax];
    } else if (st < 6) {
      for (int t = 0; t < tlen; ++t) acc += ia.InvC[a + t * KMAX] * g.in[base + t * sax];
    } else {
      for (int t = 0; t < tlen; ++t) acc += ia.W[t + a * KMAX] * g.in[base + t * sax];
    }
    if (st == 2) {
      const Solve2D &m0 = *s.inner[0], &m1 = *s.inner[1];
      const int j0 = clamp_row(m0.I[i0], s.n), j1 = clamp_row(m1.I[i1], s.n),
                j2 = clamp_row(ia.I[i2], s.n);
      double den;
      if (ia.lq_r) {   // Stokes: h/2 (p0 q1 q2 + q0 p1 q2 + q0 q1 p2)
        const double p0 = m0.lam_r[j0], p1 = m1.lam_r[j1], p2 = ia.lam_r[j2];
        const double q0 = m0.lq_r[j0], q1 = m1.lq_r[j1], q2 = ia.lq_r[j2];
        den = (0.5 / (double)(s.n + 1)) * (p0 * q1 * q2 + q0 * p1 * q2 + q0 * q1 * p2);
      } else {
        den = m0.lam_r[j0] + m1.lam_r[j1] + ia.lam_r[j2];
      }
      acc /= den;
    }
    g.out[o] = acc;
  }
}

// Mode-d unfolding of the core, transposed, into the mode slot's C panel
// (rows = pairs of the other modes, p fastest; zero rows up to P), and the
// slot set to factor it (ACT_CORE).
__global__ __launch_bounds__(NTHR) void k_core_unfold(int P, Solve3D *S) {
  Solve3D &s = S[blockIdx.z / 3];
  const int d = blockIdx.z % 3;
  if (s.phase != P3_CORE) return;
  Solve2D &in = *s.inner[d];
  int p, q;
  other_modes(d, p, q);
  const int kd = s.k[d], kp = s.k[p], kq = s.k[q];
  const int row = blockIdx.x * NTHR + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) in.active = ACT_CORE;
  if (row >= P) return;
  const long st[3] = {1, s.k[0], (long)s.k[0] * s.k[1]};
  const bool live = row < kp * kq;
  const int b = live ? row % kp : 0, c = live ? row / kp : 0;
  const long base = b * st[p] + c * st[q];
  for (int a = 0; a < kd; ++a)
    in.C[row + a * in.ldc] = live ? s.buf0[base + a * st[d]] : 0.0;
}

// Output ranks: HOSVD truncation at eps/sqrt(3) per mode; the mode slots
// go back to idle.
__global__ void k_tucker_rank(Solve3D *S) {
  Solve3D &s = S[blockIdx.x];
  if (threadIdx.x != 0 || s.phase != P3_CORE) return;
  const double ed = s.eps / sqrt(3.0);
  double nrm = 0.0;
  for (int d = 0; d < 3; ++d) {
    Solve2D &in = *s.inner[d];
    const int kd = s.k[d];
    const double *sg = in.sig;
    double tot = 0.0;
    for (int i = 0; i < kd; ++i) tot += sg[i] * sg[i];
    const double nd = sqrt(tot);
    int R = kd;
    double tail = 0.0;
    for (int t = kd; t >= 0; --t) {
      if (t < kd) tail += sg[t] * sg[t];
      if (sqrt(tail) <= ed * nd) R = t;
      else break;
    }
    if (nd == 0.0) R = 0;
    s.R[d] = R;
    nrm = fmax(nrm, nd);
    in.active = ACT_DONE;
  }
  s.nrm = nrm;
  if (s.R[0] * s.R[1] * s.R[2] == 0) s.R[0] = s.R[1] = s.R[2] = 0;
  const bool fits = s.R[0] <= s.rmax[0] && s.R[1] <= s.rmax[1] && s.R[2] <= s.rmax[2];
  s.status = fits ? s.cross_status : LRP_ERANKCAP;
  s.out_ok = fits;
  s.phase = P3_OUT;
}

// A_d = Q0_d W_d[:, :R_d] (n x R_d) in the mode slot's A panel.
__global__ __launch_bounds__(NTHR) void k_tucker_factor(Solve3D *S) {
  Solve3D &s = S[blockIdx.y];
  const int d = blockIdx.z;
  if (s.phase != P3_OUT || !s.out_ok) return;
  Solve2D &in = *s.inner[d];
  const int i = blockIdx.x * NTHR + threadIdx.x;
  if (i >= s.n) return;
  const int kd = s.k[d], Rd = s.R[d];
  const long ld = in.ldu;
  for (int c = 0; c < Rd; ++c) {
    double acc = 0.0;
    for (int j = 0; j < kd; ++j) acc += in.Q0[i + j * ld] * in.W[j + c * KMAX];
    in.A[i + c * ld] = acc;
  }
}

__global__ void k_tucker_done(Solve3D *S) {
  Solve3D &s = S[blockIdx.x];
  if (threadIdx.x == 0 && s.phase == P3_OUT) s.phase = P3_DONE;
}

}  // namespace

hipError_t launch_fiber_outer(Solve3D *s, int nsolves, hipStream_t st) {
  hipLaunchKernelGGL(k_fiber_outer, dim3(nsolves), dim3(64), 0, st, s);
  return hipGetLastError();
}

hipError_t launch_fiber_setup(Solve3D *s, int nsolves, int rmax, hipStream_t st) {
  const long half = (long)rmax * rmax * KMAX;
  hipLaunchKernelGGL(k_fiber_T, dim3((unsigned)((half + NTHR - 1) / NTHR), 1, 3 * nsolves),
                     dim3(NTHR), 0, st, s);
  hipLaunchKernelGGL(k_fiber_cols, dim3(FIB_M / NTHR, 1, 3 * nsolves), dim3(NTHR), 0, st, s);
  hipLaunchKernelGGL(k_fiber_go, dim3(nsolves), dim3(64), 0, st, s);
  return hipGetLastError();
}

hipError_t launch_core_build(Solve3D *s, int nsolves, hipStream_t st) {
  for (int stg = 0; stg < 6; ++stg)
    hipLaunchKernelGGL(k_core_stage, dim3(CORE_MAX / NTHR / 4, nsolves), dim3(NTHR), 0, st,
                       stg, s);
  return hipGetLastError();
}

hipError_t launch_core_unfold(Solve3D *s, int nsolves, int P, hipStream_t st) {
  hipLaunchKernelGGL(k_core_unfold, dim3(ceil_div(P, NTHR), 1, 3 * nsolves), dim3(NTHR), 0,
                     st, P, s);
  return hipGetLastError();
}

hipError_t launch_tucker_out(Solve3D *s, int nsolves, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_tucker_rank, dim3(nsolves), dim3(64), 0, st, s);
  hipLaunchKernelGGL(k_tucker_factor, dim3(ceil_div(n, NTHR), nsolves, 3), dim3(NTHR), 0, st,
                     s);
  for (int stg = 6; stg < 9; ++stg)
    hipLaunchKernelGGL(k_core_stage, dim3(CORE_MAX / NTHR / 4, nsolves), dim3(NTHR), 0, st,
                       stg, s);
  hipLaunchKernelGGL(k_tucker_done, dim3(nsolves), dim3(64), 0, st, s);
  return hipGetLastError();
}

}  // namespace lrp
