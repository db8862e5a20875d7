// Tall-skinny Householder QR (TSQR) of an n x k panel, k <= 64, with the
// explicit orthonormal factor Q (n x k).  Used for the orthonormal bases of
// the cross columns and rows before maxvol and for the rounding of the
// skeleton (paper Section 3, "rounding": QR of the factors, then SVD of the
// small core; Section 4.2: maxvol on the cross).
//
// Tree: leaves are 256-row blocks; each internal node stacks the R factors of
// `fan` children (fan * kmax <= 256 rows) and factors them again.  Q is
// formed top-down: every node applies its reflectors to [Y; 0] and hands the
// k x k row blocks to its children; the leaves write rows of Q.
// All kernels run one 256-thread workgroup per (node, solve) with the panel
// in registers (see panel.h).
#include "panel.h"

namespace lrp {
namespace {

__device__ inline size_t lev_off(const Tree &t, int l, size_t per_node) {
  size_t o = 0;
  for (int i = 0; i < l; ++i) o += (size_t)t.nb[i] * per_node;
  return o;
}
__device__ inline size_t hlev_off(const Tree &t, int l) {   // levels >= 1
  size_t o = 0;
  for (int i = 1; i < l; ++i) o += (size_t)t.nb[i] * PANEL_M * KMAX;
  return o;
}

struct TsIO {
  const double *in;
  long ldin;
  double *out;
  long ldout;
  float *outf;   // float copy of out (same leading dimension), or null
};
__device__ inline TsIO ts_io(int which, const Solve2D &s) {
  // the cross panels are evaluated in the leaf (cross_panel), not loaded
  if (which == TS_C_TO_Q0) return {nullptr, 0, s.Q0, s.ldu, s.Q0f};
  if (which == TS_C_TO_Q1) return {nullptr, 0, s.Q1, s.ldv, s.Q1f};
  if (which == TS_VH_TO_Q1) return {s.Vh, s.ldv, s.Q1, s.ldv, s.Q1f};
  return {s.C, s.ldc, nullptr, 0, nullptr};   // TS_CORE: R only
}

__device__ inline int ts_phase(int which) {
  return which == TS_VH_TO_Q1 ? ACT_INIT : (which == TS_CORE ? ACT_CORE : ACT_SWEEP);
}

// Rows [r0, r0 + m) of the cross columns Xh[:, J] (TS_C_TO_Q0: rows of Uh
// against Vh[J]) or of the cross rows Xh[I, :]^T (TS_C_TO_Q1: rows of Vh
// against Uh[I]), evaluated straight into the register panel instead of
// being written to and read back from memory:
//     y(i, c) = (P_i . Qm_sel[c]) / D(i, sel[c]),
// the rank-r numerator summed in ascending order, D the operator's
// eigenvalue (den_of; it is symmetric in the two sides).  The selected rows
// of Qm and their eigenvalue factors are staged in LDS (qs: [alpha][c], NC
// columns; ls: [c] and [NC + c]); every wave reads the same P rows, which
// the vector cache serves.
template <int NS>
__device__ __forceinline__ void cross_panel(double (&y)[NS][4], int which,
                                            const Solve2D &s, int r0, int m,
                                            double *qs, double *ls) {
  constexpr int NC = 4 * NS;
  const bool cols = which == TS_C_TO_Q0;
  const double *P = cols ? s.Uh : s.Vh, *Qm = cols ? s.Vh : s.Uh;
  const long ldp = cols ? s.ldu : s.ldv, ldq = cols ? s.ldv : s.ldu;
  const double *lp = cols ? s.lam_r : s.lam_c, *lq = cols ? s.lam_c : s.lam_r;
  const double *lp2 = cols ? s.lq_r : s.lq_c, *lq2 = cols ? s.lq_c : s.lq_r;
  const bool prod = lp2 != nullptr;
  const int *sel = cols ? s.J : s.I;
  const int other = cols ? s.m : s.n;
  const int kk = s.k, r = s.r;
  for (int e = threadIdx.x; e < r * NC; e += NTHR) {
    const int a = e / NC, c = e - a * NC;
    qs[e] = (c < kk) ? Qm[clamp_row(sel[c], other) + (long)a * ldq] : 0.0;
  }
  for (int c = threadIdx.x; c < NC; c += NTHR) {
    ls[c] = (c < kk) ? lq[clamp_row(sel[c], other)] : 1.0;
    ls[NC + c] = (c < kk && prod) ? lq2[clamp_row(sel[c], other)] : 1.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double *Pr = P + r0 + lane;
#pragma unroll
  for (int sl = 0; sl < NS; ++sl)
#pragma unroll
    for (int q = 0; q < 4; ++q) y[sl][q] = 0.0;
  for (int a0 = 0; a0 < r; a0 += 4) {
    double p[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        p[t][q] = (a0 + t < r && lane + 64 * q < m) ? Pr[64 * q + (long)(a0 + t) * ldp] : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (a0 + t >= r) break;
#pragma unroll
      for (int sl = 0; sl < NS; ++sl) {
        const double qv = qs[(a0 + t) * NC + wave + 4 * sl];
#pragma unroll
        for (int q = 0; q < 4; ++q) y[sl][q] += p[t][q] * qv;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = lane + 64 * q;
    const double li = (i < m) ? lp[r0 + i] : 1.0;
    const double li2 = (i < m && prod) ? lp2[r0 + i] : 1.0;
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
      const int c = wave + 4 * sl;
      y[sl][q] = (c < kk && i < m) ? y[sl][q] / den_of(prod, li, li2, ls[c], ls[NC + c]) : 0.0;
    }
  }
}

template <int NS, bool CROSS>
__global__ __launch_bounds__(NTHR) void k_tsqr_leaf(int which, int n, Tree tr,
                                                   Solve2D *S) {
  Solve2D &s = S[blockIdx.y];
  if (s.active != ts_phase(which)) return;
  if (ts_phase(which) == ACT_SWEEP && rank_bucket(s.k) != 4 * NS) return;
  __shared__ double vbuf[2 * PANEL_M];
  __shared__ double taus[KMAX];
  __shared__ double qs[CROSS ? KMAX * 4 * NS : 1];
  __shared__ double ls[CROSS ? 8 * NS : 1];
  const int kk = s.k;
  const int b = blockIdx.x;
  const int r0 = b * PANEL_M;
  const int m = min(PANEL_M, n - r0);
  const int mp = max(m, kk);
  double y[NS][4];
  if constexpr (CROSS) {
    cross_panel(y, which, s, r0, m, qs, ls);
  } else {
    const TsIO io = ts_io(which, s);
    panel_load(y, io.in + r0, io.ldin, m, kk);
  }
  hh_qr_regs(y, mp, kk, vbuf, taus);
  panel_store(y, s.Hv + r0, s.ldc, m, kk);
  double *R = s.tree_R + lev_off(tr, 0, (size_t)KMAX * KMAX) + (size_t)b * KMAX * KMAX;
  double *Rf = (tr.nlev == 1) ? s.Rfin : nullptr;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int c = wave + 4 * sl;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      if (c < kk && i < kk) {
        const double v = (i <= c && i < mp) ? y[sl][q] : 0.0;
        R[i + c * KMAX] = v;
        if (Rf) Rf[i + c * KMAX] = v;
      }
    }
  }
  double *T = s.tree_tau + lev_off(tr, 0, KMAX) + (size_t)b * KMAX;
  for (int j = threadIdx.x; j < kk; j += NTHR) T[j] = (j < mp) ? taus[j] : 0.0;
}

template <int NS>
__global__ __launch_bounds__(NTHR) void k_tsqr_node(int which, int lev, Tree tr,
                                                   Solve2D *S) {
  Solve2D &s = S[blockIdx.y];
  if (s.active != ts_phase(which)) return;
  __shared__ double vbuf[2 * PANEL_M];
  __shared__ double taus[KMAX];
  const int kk = s.k;
  const int t = blockIdx.x;
  const int c0 = t * tr.fan;
  const int nch = min(tr.fan, tr.nb[lev - 1] - c0);
  const int mp = nch * kk;
  const double *Rc = s.tree_R + lev_off(tr, lev - 1, (size_t)KMAX * KMAX);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double y[NS][4];
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int c = wave + 4 * sl;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      double v = 0.0;
      if (c < kk && i < mp) {
        const int ch = i / kk, ii = i - ch * kk;
        v = Rc[(size_t)(c0 + ch) * KMAX * KMAX + ii + c * KMAX];
      }
      y[sl][q] = v;
    }
  }
  hh_qr_regs(y, mp, kk, vbuf, taus);
  double *H = s.tree_H + hlev_off(tr, lev) + (size_t)t * PANEL_M * KMAX;
  panel_store(y, H, PANEL_M, mp, kk);
  double *R = s.tree_R + lev_off(tr, lev, (size_t)KMAX * KMAX) + (size_t)t * KMAX * KMAX;
  double *Rf = (lev == tr.nlev - 1) ? s.Rfin : nullptr;
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int c = wave + 4 * sl;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      if (c < kk && i < kk) {
        const double v = (i <= c && i < mp) ? y[sl][q] : 0.0;
        R[i + c * KMAX] = v;
        if (Rf) Rf[i + c * KMAX] = v;
      }
    }
  }
  double *T = s.tree_tau + lev_off(tr, lev, KMAX) + (size_t)t * KMAX;
  for (int j = threadIdx.x; j < kk; j += NTHR) T[j] = (j < mp) ? taus[j] : 0.0;
}

// Top-down Q formation at an internal node: [Y; 0] -> child blocks.
template <int NS>
__global__ __launch_bounds__(NTHR) void k_tsqr_node_apply(int which, int lev,
                                                         Tree tr, Solve2D *S) {
  Solve2D &s = S[blockIdx.y];
  if (s.active != ts_phase(which)) return;
  const int kk = s.k;
  const int t = blockIdx.x;
  const int c0 = t * tr.fan;
  const int nch = min(tr.fan, tr.nb[lev - 1] - c0);
  const int mp = nch * kk;
  const bool top = (lev == tr.nlev - 1);
  const double *Yin = s.tree_Y + lev_off(tr, lev, (size_t)KMAX * KMAX) + (size_t)t * KMAX * KMAX;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double y[NS][4];
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int c = wave + 4 * sl;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      double v = 0.0;
      if (c < kk && i < kk) v = top ? (i == c ? 1.0 : 0.0) : Yin[i + c * KMAX];
      y[sl][q] = v;
    }
  }
  const double *H = s.tree_H + hlev_off(tr, lev) + (size_t)t * PANEL_M * KMAX;
  const double *T = s.tree_tau + lev_off(tr, lev, KMAX) + (size_t)t * KMAX;
  __shared__ double wy[wy_lds<4 * NS>()];
  hh_apply_wy(y, mp, min(mp, kk), kk, H, PANEL_M, T, top ? nullptr : Yin, KMAX, wy);
  double *Yc = s.tree_Y + lev_off(tr, lev - 1, (size_t)KMAX * KMAX);
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int c = wave + 4 * sl;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      if (c < kk && i < mp) {
        const int ch = i / kk, ii = i - ch * kk;
        Yc[(size_t)(c0 + ch) * KMAX * KMAX + ii + c * KMAX] = y[sl][q];
      }
    }
  }
}

// At NS <= 8 a budget of four waves per SIMD fits without spilling.
template <int NS>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(NS <= 8 ? 4 : 1)))
void k_tsqr_leaf_apply(int which, int n, Tree tr, Solve2D *S) {
  Solve2D &s = S[blockIdx.y];
  if (s.active != ts_phase(which)) return;
  if (ts_phase(which) == ACT_SWEEP && rank_bucket(s.k) != 4 * NS) return;
  const int kk = s.k;
  const int b = blockIdx.x;
  const int r0 = b * PANEL_M;
  const int m = min(PANEL_M, n - r0);
  const int mp = max(m, kk);
  const bool top = (tr.nlev == 1);
  const double *Yin = s.tree_Y + (size_t)b * KMAX * KMAX;   // level 0
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double y[NS][4];
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int c = wave + 4 * sl;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      double v = 0.0;
      if (c < kk && i < kk) v = top ? (i == c ? 1.0 : 0.0) : Yin[i + c * KMAX];
      y[sl][q] = v;
    }
  }
  const double *T = s.tree_tau + (size_t)b * KMAX;
  __shared__ double wy[wy_lds<4 * NS>()];
  hh_apply_wy(y, m, min(mp, kk), kk, s.Hv + r0, s.ldc, T, top ? nullptr : Yin, KMAX, wy);
  const TsIO io = ts_io(which, s);
  panel_store(y, io.out + r0, io.ldout, m, kk);
  if (io.outf) panel_store(y, io.outf + r0, io.ldout, m, kk);
}

template <int NS>
void run_leaf(int which, int n, const Tree &tr, Solve2D *s, int ns, hipStream_t st) {
  if (which == TS_C_TO_Q0 || which == TS_C_TO_Q1)
    hipLaunchKernelGGL((k_tsqr_leaf<NS, true>), dim3(tr.nb[0], ns), dim3(NTHR), 0, st,
                       which, n, tr, s);
  else
    hipLaunchKernelGGL((k_tsqr_leaf<NS, false>), dim3(tr.nb[0], ns), dim3(NTHR), 0, st,
                       which, n, tr, s);
}

template <int NS>
void run_nodes(int which, const Tree &tr, Solve2D *s, int ns, hipStream_t st) {
  for (int l = 1; l < tr.nlev; ++l)
    hipLaunchKernelGGL((k_tsqr_node<NS>), dim3(tr.nb[l], ns), dim3(NTHR), 0, st, which, l,
                       tr, s);
  if (which == TS_CORE) return;   // R only
  for (int l = tr.nlev - 1; l >= 1; --l)
    hipLaunchKernelGGL((k_tsqr_node_apply<NS>), dim3(tr.nb[l], ns), dim3(NTHR), 0, st,
                       which, l, tr, s);
}

template <int NS>
void run_leaf_apply(int which, int n, const Tree &tr, Solve2D *s, int ns, hipStream_t st) {
  hipLaunchKernelGGL((k_tsqr_leaf_apply<NS>), dim3(tr.nb[0], ns), dim3(NTHR), 0, st,
                     which, n, tr, s);
}

}  // namespace

Tree make_tree(int n, int kmax) {
  Tree t{};
  int kp = 16;
  while (kp < kmax) kp *= 2;
  t.fan = PANEL_M / kp;
  if (t.fan < 2) t.fan = 2;
  t.nb[0] = ceil_div(n, PANEL_M);
  t.nlev = 1;
  while (t.nb[t.nlev - 1] > 1 && t.nlev < 8) {
    t.nb[t.nlev] = ceil_div(t.nb[t.nlev - 1], t.fan);
    ++t.nlev;
  }
  return t;
}

// The leaf kernels (16 workgroups per slot at n = 4096) run once per bucket
// of the mask, each on its own slots; the tree nodes (a few workgroups per
// slot, latency-bound) once at the largest bucket, on every slot.
hipError_t launch_tsqr(int which, int rows, const Tree &tr, Solve2D *s,
                       int nsolves, int kmax, hipStream_t st, unsigned bmask) {
  const int n = rows;
  if (!bmask) bmask = bucket_bit(kmax);
  const int ktop = top_bucket(bmask);
  for (int kb = 16; kb <= 64; kb += 16) {
    if (!(bmask & bucket_bit(kb))) continue;
    if (kb == 16) run_leaf<4>(which, n, tr, s, nsolves, st);
    else if (kb == 32) run_leaf<8>(which, n, tr, s, nsolves, st);
    else if (kb == 48) run_leaf<12>(which, n, tr, s, nsolves, st);
    else run_leaf<16>(which, n, tr, s, nsolves, st);
  }
  if (ktop == 16) run_nodes<4>(which, tr, s, nsolves, st);
  else if (ktop == 32) run_nodes<8>(which, tr, s, nsolves, st);
  else if (ktop == 48) run_nodes<12>(which, tr, s, nsolves, st);
  else run_nodes<16>(which, tr, s, nsolves, st);
  if (which == TS_CORE) return hipGetLastError();   // R only
  for (int kb = 16; kb <= 64; kb += 16) {
    if (!(bmask & bucket_bit(kb))) continue;
    if (kb == 16) run_leaf_apply<4>(which, n, tr, s, nsolves, st);
    else if (kb == 32) run_leaf_apply<8>(which, n, tr, s, nsolves, st);
    else if (kb == 48) run_leaf_apply<12>(which, n, tr, s, nsolves, st);
    else run_leaf_apply<16>(which, n, tr, s, nsolves, st);
  }
  return hipGetLastError();
}

}  // namespace lrp
