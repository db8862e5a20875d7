// The exponential-sum comparator of Section 4.1: the kernels of one
// incremental rounding step (the TSQR and the core SVD between them are the
// cross's own, see tsqr.hip and svd.hip).
//
// With 1/x ~ sum_k w_k exp(-p_k x) on the range of the eigenvalue sums, the
// divided spectrum Xh_ij = Fh_ij / (lambda_i + lambda_j) becomes
//     Xh ~ sum_k (s_k Ea_k Uh)(s_k Ea_k Vh)^T,   s_k = sqrt(w_k),
//     Ea_k = diag(exp(-p_k lambda)),
// a product of two n x (R r) factors whose column j is term k = j / r,
// input column a = j mod r.  Section 3 rounds such a product by QR of both
// factors and an SVD of the product of the R factors.  Here the columns go
// in c at a time: the rank-K factorisation Qa diag(sig) Qb^T so far and the
// next c columns form the panels
//     Pa = [Qa diag(sig), new a columns],  Pb = [Qb, new b columns],
// n x (K + c) with K + c <= kw = min(KMAX, n); Pa = Qa~ Ra, Pb = Qb~ Rb (TSQR), Ra Rb^T
// = W S Z^T (Jacobi SVD), and the step keeps the leading K' columns of
// Qa~ W and Qb~ Z, K' the smallest rank whose dropped tail is within the
// step's share of the tolerance: (eps/2) c / (R r) of ||S|| per step, eps/2
// at the last step, so that the dropped tails add up to at most eps times
// the largest core norm.  In plain mode the same steps round a given
// product U V^T of many columns (the sums of low-rank matrices that the
// Stokes driver forms).
#include "lrp_internal.h"

namespace lrp {
namespace {

constexpr int ES_T = 256;   // threads of the row kernels (one row each)

// Panels of the step: grid (row blocks, side, solve).  Columns [0, K) copy
// the side's basis (the a side scaled by sig), columns [K, K + c) are the
// next product columns; the row's eigenvalue decides every weight of the row.
__global__ __launch_bounds__(ES_T) void k_es_panel(ExpState *E, Solve2D *jobs, int cap) {
  const ExpState &e = E[blockIdx.z];
  const int side = blockIdx.y;
  Solve2D &j = jobs[side * cap + blockIdx.z];
  const bool run = e.phase == ES_RUN;
  const int K = e.K, c = es_cols(e.K, e.j0, e.tot, e.kw);
  // the TSQR and the core act on the job records of running solves only
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    j.active = run ? ACT_INIT : ACT_DONE;
    j.k = run ? K + c : 0;
  }
  if (!run) return;
  const int n = e.n, i = blockIdx.x * ES_T + threadIdx.x;
  if (i >= n) return;
  const long ldp = j.ldv, ldq = j.ldu;
  double *P = j.Vh;
  const double *Q = j.Q0;
  for (int t = 0; t < K; ++t) P[i + t * ldp] = Q[i + t * ldq] * (side == 0 ? e.sig[t] : 1.0);
  if (e.pu) {   // plain rounding: the product's own columns
    const double *F = side == 0 ? e.pu : e.pv;
    for (int t = 0; t < c; ++t) P[i + (K + t) * ldp] = F[i + (long)(e.j0 + t) * e.ldp];
    return;
  }
  const double li = e.lam[i];
  const double *F = j.Uh;
  int k = e.j0 / e.r, a = e.j0 - k * e.r;
  double wt = e.sw[k] * exp(-e.p[k] * li);
  for (int t = 0; t < c; ++t) {
    P[i + (K + t) * ldp] = wt * F[i + a * ldq];
    if (++a == e.r && t + 1 < c) {
      a = 0;
      ++k;
      wt = e.sw[k] * exp(-e.p[k] * li);
    }
  }
}

// The step's truncation and the state's advance: one wave per solve, after
// the core SVD of the b-side record left S (descending) in its sig.
__global__ __launch_bounds__(64) void k_es_trunc(ExpState *E, const Solve2D *jobs, int cap) {
  ExpState &e = E[blockIdx.x];
  if (e.phase != ES_RUN) return;
  const Solve2D &a = jobs[blockIdx.x], &b = jobs[cap + blockIdx.x];
  const int k = b.k, c = k - e.K;
  __shared__ int keep;
  if (threadIdx.x == 0) {
    if (a.nonfinite || b.nonfinite) {
      e.status = LRP_ENONFINITE;
      e.phase = ES_DONE;
      e.K = 0;
      keep = 0;
    } else {
      const bool last = e.j0 + c >= e.tot;
      const double share = last ? 0.5 * e.eps : 0.5 * e.eps * (double)c / (double)e.tot;
      double tot2 = 0.0;
      for (int t = k - 1; t >= 0; --t) tot2 += b.sig[t] * b.sig[t];
      const double nrm = sqrt(tot2);
      // smallest rank whose tail ||S[R:]|| is within share ||S|| (the tail
      // only grows as R falls)
      int R = k;
      double tail2 = 0.0;
      for (int t = k - 1; t >= 0; --t) {
        tail2 += b.sig[t] * b.sig[t];
        if (sqrt(tail2) > share * nrm) break;
        R = t;
      }
      if (nrm == 0.0) R = 0;
      // room for the next step's columns
      if (!last && R > e.kw - ES_CMIN) {
        R = e.kw - ES_CMIN;
        e.capped = 1;
      }
      double drop2 = 0.0;
      for (int t = k - 1; t >= R; --t) drop2 += b.sig[t] * b.sig[t];
      e.drop += sqrt(drop2);
      e.nrm = nrm;
      e.K = R;
      e.j0 += c;
      e.steps += 1;
      e.phase = last ? ES_LAST : ES_RUN;
      keep = R;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < keep) e.sig[threadIdx.x] = b.sig[threadIdx.x];
}

// The new bases Qa~ W[:, :K'] and Qb~ Z[:, :K'] (grid: row blocks, side,
// solve), into Q0 while the solve runs; at its last step into the output
// staging A, the a side scaled by sig.  Writing the staging is idempotent,
// so the launches of later steps may repeat it.
__global__ __launch_bounds__(ES_T) void k_es_update(const ExpState *E, Solve2D *jobs, int cap) {
  const ExpState &e = E[blockIdx.z];
  const int ph = e.phase;
  if (ph != ES_RUN && ph != ES_LAST) return;
  const int side = blockIdx.y;
  const Solve2D &j = jobs[side * cap + blockIdx.z];
  const Solve2D &b = jobs[cap + blockIdx.z];
  const int k = j.k, Kn = e.K;
  if (k <= 0 || Kn <= 0) return;
  __shared__ double Ws[KMAX * KMAX];
  const double *W = side == 0 ? b.W : b.Z;
  const bool scale = ph == ES_LAST && side == 0;
  for (int idx = threadIdx.x; idx < KMAX * Kn; idx += ES_T) {
    const int s = idx % KMAX, t = idx / KMAX;
    Ws[idx] = (s < k) ? W[s + t * KMAX] * (scale ? e.sig[t] : 1.0) : 0.0;
  }
  __syncthreads();
  const int i = blockIdx.x * ES_T + threadIdx.x;
  if (i >= e.n) return;
  const double *Q = j.Q1;
  const long ldq = j.ldv;
  double *out = (ph == ES_LAST) ? j.A : j.Q0;
  const long ldo = j.ldu;
  for (int t0 = 0; t0 < Kn; t0 += 16) {
    double acc[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = 0.0;
    for (int s = 0; s < k; ++s) {
      const double q = Q[i + s * ldq];
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] += q * Ws[s + (t0 + u) * KMAX];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (t0 + u < Kn) out[i + (t0 + u) * ldo] = acc[u];
  }
}

}  // namespace

hipError_t launch_es_panel(ExpState *e, Solve2D *jobs, int cap, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_es_panel, dim3(ceil_div(n, ES_T), 2, cap), dim3(ES_T), 0, st, e, jobs,
                     cap);
  return hipGetLastError();
}

hipError_t launch_es_trunc(ExpState *e, Solve2D *jobs, int cap, hipStream_t st) {
  hipLaunchKernelGGL(k_es_trunc, dim3(cap), dim3(64), 0, st, e, jobs, cap);
  return hipGetLastError();
}

hipError_t launch_es_update(ExpState *e, Solve2D *jobs, int cap, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_es_update, dim3(ceil_div(n, ES_T), 2, cap), dim3(ES_T), 0, st, e, jobs,
                     cap);
  return hipGetLastError();
}

}  // namespace lrp
