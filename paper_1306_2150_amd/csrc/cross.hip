// Cross approximation of the divided spectrum (paper Section 4.2).
//
// Entries: Xh_ij = (Uh_i . Vh_j) / (lambda_i + lambda_j)   (eq. "div") -- a
// rank-r numerator over a rank-2 denominator, O(r) per entry.  The kernels
// take the general rectangular form Xh_ij = (Uh_i . Vh_j) / (lam_r[i] +
// lam_c[j]), i < n, j < m, which the 3D path uses for the unfoldings of its
// divided spectrum.  A sweep with
// column set J evaluates the columns Xh[:, J] and orthonormalises them (both
// in the TSQR, tsqr.hip), picks rows I by maxvol, evaluates and
// orthonormalises the rows Xh[I, :], picks the next columns Jn by maxvol, and rounds the
// skeleton through the k x k core (svd.hip).  This file also holds the
// per-sweep bookkeeping: the skeleton factors A = Q0 W S, B = Q1 Z, the change
// ||A B^T - Ap Bp^T||_F against the previous sweep, the truncation rank, the
// rank-growth columns and the stop decision.
//
// Change between sweeps without cancellation: with B, Bp orthonormal and
// M = Bp^T B,   ||A B^T - Ap Bp^T||^2 = ||A - Ap M||^2 + sum_a sp_a^2 ||E_a||^2,
// E = Bp - B M^T, because Ap^T Ap = diag(sp^2).  Every term is a direct
// difference of n-row panels, so the result keeps full relative accuracy
// down to changes of 1e-14 ||X||.
#include "lrp_internal.h"

namespace lrp {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// A = Q0 (W diag(sig))  (z = 0, n rows),  B = Q1 Z  (z = 1, m rows), all k
// columns.
template <int KM>
__global__ __launch_bounds__(NTHR) void k_factors(Solve2D *S) {
  Solve2D &s = S[blockIdx.y];
  if (s.active != ACT_SWEEP || rank_bucket(s.k) != KM) return;
  __shared__ double M[KMAX * KMAX];   // [j][c]
  const int kk = s.k, z = blockIdx.z;
  const double *Qz = z ? s.Q1 : s.Q0;
  double *out = z ? s.B : s.A;
  const long ld = z ? s.ldv : s.ldu;
  const int rows = z ? s.m : s.n;
  if (blockIdx.x * NTHR >= rows) return;
  // rows j < KM of M, every thread's loads in flight at once (j, c < KMAX
  // stay inside the buffers), entries past k zero
  {
    constexpr int PM = KM * KMAX / NTHR;
    const double *src = z ? s.Z : s.W;
    double tv[PM], sg[PM];
#pragma unroll
    for (int u = 0; u < PM; ++u) {
      const int e = threadIdx.x + u * NTHR, j = e / KMAX, c = e - j * KMAX;
      tv[u] = src[j + c * KMAX];
      sg[u] = s.sig[c];
    }
#pragma unroll
    for (int u = 0; u < PM; ++u) {
      const int e = threadIdx.x + u * NTHR, j = e / KMAX, c = e - j * KMAX;
      M[e] = (j < kk && c < kk) ? (z ? tv[u] : tv[u] * sg[u]) : 0.0;
    }
  }
  __syncthreads();
  const int i = blockIdx.x * NTHR + threadIdx.x;
  if (i >= rows) return;
  double acc[KM];
#pragma unroll
  for (int c = 0; c < KM; ++c) acc[c] = 0.0;
  for (int j0 = 0; j0 < kk; j0 += 8) {
    double q[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) q[t] = (j0 + t < kk) ? Qz[i + (long)(j0 + t) * ld] : 0.0;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (j0 + t >= kk) break;
#pragma unroll
      for (int c = 0; c < KM; ++c) acc[c] += q[t] * M[(j0 + t) * KMAX + c];
    }
  }
#pragma unroll
  for (int c = 0; c < KM; ++c)
    if (c < kk) out[i + (long)c * ld] = acc[c];
}

// Block b of Mc = Bp^T B (kp x k, the previous sweep's row factor against
// this one's): rows [256 b, 256 b + 256) + 256 nbm t of the m rows (nbm =
// change_blocks(m), a function of m only, so the summation order of a slot
// never depends on the batch).  Float64 matrix cores (v_mfma_f64_16x16x4):
// wave w takes rows 64 w .. 64 w + 63 of each 256-row slab, eight rows per
// step with lane group g on rows 2 g and 2 g + 1 of the step (the K order of
// the two operands is the same, so any such order gives the sum); the four
// waves' partial sums are added in LDS in wave order.
template <int KM>
__global__ __launch_bounds__(NTHR) void k_change_M(int nbm, Solve2D *S) {
  Solve2D &s = S[blockIdx.y];
  if (s.active != ACT_SWEEP || s.kp == 0 || rank_bucket(s.k) != KM) return;
  constexpr int NB = KM / 16;
  __shared__ double red[KMAX * KMAX];
  const int kk = s.k, kq = s.kp, m = s.m;
  const long ld = s.ldv;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const double *bp[NB], *bb[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int c = 16 * t + li;
    bp[t] = (c < kq) ? s.Bp + (long)c * ld : nullptr;
    bb[t] = (c < kk) ? s.B + (long)c * ld : nullptr;
  }
  d4 acc[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[a][c] = (d4){0, 0, 0, 0};
  for (int r0 = blockIdx.x * PANEL_M; r0 < m; r0 += nbm * PANEL_M) {
    for (int st = 0; st < 8; ++st) {
      const int row = r0 + 64 * wave + 8 * st + 2 * g;
      double xa[NB][2], xb[NB][2];
#pragma unroll
      for (int t = 0; t < NB; ++t)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const bool ok = row + e < m;
          xa[t][e] = (bp[t] && ok) ? bp[t][row + e] : 0.0;
          xb[t][e] = (bb[t] && ok) ? bb[t][row + e] : 0.0;
        }
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int c = 0; c < NB; ++c)
            acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a][e], xb[c][e], acc[a][c], 0, 0, 0);
    }
  }
  // D[i][j]: lane j + 16 (i % 4), register i / 4
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int c = 0; c < NB; ++c)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int e = (16 * a + 4 * r + g) * KMAX + 16 * c + li;
            red[e] = (w == 0) ? acc[a][c][r] : red[e] + acc[a][c][r];
          }
    }
    __syncthreads();
  }
  double *P = s.part + (size_t)blockIdx.x * KMAX * KMAX;
  for (int e = threadIdx.x; e < kq * kk; e += NTHR) {
    const int a = e / kk, c = e - a * kk;
    P[e] = red[a * KMAX + c];
  }
}

// Mc = the sum of the nbm block partials, in block order; one thread per
// entry (grid x covers the kp x k entries, 64 per workgroup), its loads
// independent so that many are in flight.
__global__ __launch_bounds__(64) void k_change_reduce(int nbm, int km, Solve2D *S) {
  Solve2D &s = S[blockIdx.y];
  if (s.active != ACT_SWEEP || s.kp == 0 || rank_bucket(s.k) != km) return;
  const int kk = s.k, kq = s.kp;
  const int o = blockIdx.x * 64 + threadIdx.x;
  if (o >= kq * kk) return;
  const double *p = s.part + o;
  double v = 0.0;
#pragma unroll 8
  for (int b = 0; b < nbm; ++b) v += p[(size_t)b * KMAX * KMAX];
  const int a = o / kk, c = o - a * kk;
  s.Mc[a * KMAX + c] = v;
}

// Block b: rows [256 b, 256 b + 256) of ||A - Ap M||^2 (n rows) and of
// sum_a sp_a^2 ||E_a||^2 (m rows); partial sums in part[2b], part[2b + 1].
template <int KM>
__global__ __launch_bounds__(NTHR) void k_change_norms(Solve2D *S) {
  Solve2D &s = S[blockIdx.y];
  if (s.active != ACT_SWEEP || s.kp == 0 || rank_bucket(s.k) != KM) return;
  __shared__ double M[KMAX * KMAX];
  __shared__ double sp2[KMAX];
  __shared__ double red[2][4];
  const int kk = s.k, kq = s.kp;
  if (blockIdx.x * NTHR >= max(s.n, s.m)) return;
  // rows a < KM of M = Bp^T B, every thread's loads in flight at once
  // (inside the KMAX x KMAX buffer), entries past kp x k zero
  {
    constexpr int PM = KM * KMAX / NTHR;
    double tv[PM];
#pragma unroll
    for (int u = 0; u < PM; ++u) tv[u] = s.Mc[threadIdx.x + u * NTHR];
    const double sv = s.sigp[threadIdx.x & (KMAX - 1)];
#pragma unroll
    for (int u = 0; u < PM; ++u) {
      const int e = threadIdx.x + u * NTHR, a = e / KMAX, c = e - a * KMAX;
      M[e] = (a < kq && c < kk) ? tv[u] : 0.0;
    }
    if (threadIdx.x < KMAX) sp2[threadIdx.x] = (threadIdx.x < kq) ? sv * sv : 0.0;
  }
  __syncthreads();
  const int i = blockIdx.x * NTHR + threadIdx.x;
  double n1 = 0.0, n2 = 0.0;
  // one side's row in registers, the other side's entries streamed in
  // groups of eight (half the registers of holding both rows)
  if (i < s.n) {
    const long ld = s.ldu;
    double v[KM];
#pragma unroll
    for (int a = 0; a < KM; ++a) v[a] = (a < kq) ? s.Ap[i + (long)a * ld] : 0.0;
#pragma unroll 1
    for (int c0 = 0; c0 < kk; c0 += 8) {
      double w[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) w[t] = (c0 + t < kk) ? s.A[i + (long)(c0 + t) * ld] : 0.0;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int c = c0 + t;
        if (c < kk) {
          double x = w[t];
#pragma unroll
          for (int a = 0; a < KM; ++a) x -= v[a] * M[a * KMAX + c];
          n1 += x * x;
        }
      }
    }
  }
  if (i < s.m) {
    const long ld = s.ldv;
    double v[KM];
#pragma unroll
    for (int c = 0; c < KM; ++c) v[c] = (c < kk) ? s.B[i + (long)c * ld] : 0.0;
#pragma unroll 1
    for (int a0 = 0; a0 < kq; a0 += 8) {
      double w[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) w[t] = (a0 + t < kq) ? s.Bp[i + (long)(a0 + t) * ld] : 0.0;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int a = a0 + t;
        if (a < kq) {
          double x = w[t];
#pragma unroll
          for (int c = 0; c < KM; ++c) x -= v[c] * M[a * KMAX + c];
          n2 += sp2[a] * x * x;
        }
      }
    }
  }
  n1 = wave_sum(n1);
  n2 = wave_sum(n2);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[0][wave] = n1, red[1][wave] = n2;
  __syncthreads();
  if (threadIdx.x == 0) {
    s.part[(size_t)blockIdx.x * 2 + 0] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    s.part[(size_t)blockIdx.x * 2 + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// Truncation rank, convergence and growth decision (one workgroup / solve).
__global__ __launch_bounds__(NTHR) void k_decide(Solve2D *S) {
  Solve2D &s = S[blockIdx.x];
  if (s.active != ACT_SWEEP) return;
  __shared__ int used[2 * KMAX];
  if (threadIdx.x != 0) return;
  const int kk = s.k;
  double change = -1.0;
  if (s.kp > 0) {
    const int nbn = ceil_div(max(s.n, s.m), NTHR);
    double a = 0.0, b = 0.0;
    for (int i = 0; i < nbn; ++i) a += s.part[2 * i], b += s.part[2 * i + 1];
    change = sqrt(a + b);
  }
  double tot = 0.0;
  for (int i = 0; i < kk; ++i) tot += s.sig[i] * s.sig[i];
  const double nrm = sqrt(tot);
  // smallest R with ||sig[R:]|| <= eps ||sig||
  int R = kk;
  double tail = 0.0;
  for (int t = kk; t >= 0; --t) {
    if (t < kk) tail += s.sig[t] * s.sig[t];
    if (sqrt(tail) <= s.eps * nrm) R = t;
    else break;
  }
  if (nrm == 0.0) R = 0;
  double tailR = 0.0;
  for (int t = kk - 1; t >= R; --t) tailR += s.sig[t] * s.sig[t];
  s.tail = nrm > 0.0 ? sqrt(tailR) / nrm : 0.0;
  const bool no_slack = (R > kk - s.min_slack) && (kk < min(s.n, s.m));
  int next = NEXT_CONTINUE;
  if (s.nonfinite) {
    next = NEXT_STOP;
    s.status = LRP_ENONFINITE;
  } else if (nrm == 0.0) {
    next = NEXT_STOP;
    s.status = LRP_OK;
  } else if (no_slack && kk < s.kcap) {
    next = NEXT_GROW;
    s.kgrow = min(s.kick, s.kcap - kk);
  } else if (change >= 0.0 && change <= s.eps * nrm) {
    next = NEXT_STOP;
    s.status = no_slack ? LRP_ERANKCAP : LRP_OK;
  }
  s.sweep += 1;
  if (next != NEXT_STOP && s.sweep >= s.max_sweeps) {
    next = NEXT_STOP;
    s.status = LRP_ENOCONV;
  }
  s.R = R;
  s.nrm = nrm;
  s.change = (change >= 0.0 && nrm > 0.0) ? change / nrm : -1.0;
  s.next = next;
  if (next == NEXT_GROW) {
    for (int t = 0; t < kk; ++t) used[t] = s.I[t];
    spread_indices(s.n, s.kick, used, kk, s.probe, s.off_r);
  }
}

// Residual score of every column on the probe rows (rank growth); each
// block reports its GROW_TOP best columns (score descending, ties: lower
// column first; the current columns Jn score -1).
template <int KM>
__global__ __launch_bounds__(NTHR) void k_growth_score(Solve2D *S) {
  Solve2D &s = S[blockIdx.y];
  if (s.active != ACT_SWEEP || s.next != NEXT_GROW) return;
  if (blockIdx.x * NTHR >= s.m) return;
  constexpr int PQ = 16;
  __shared__ double uP[PQ * KMAX];
  __shared__ double aP[PQ * KMAX];
  __shared__ double lP[PQ], lQ[PQ];
  __shared__ int jn[KMAX];
  __shared__ double rv[4];
  __shared__ int rk[4];
  const int kk = s.k, r = s.r, nq = min(s.kick, PQ);
  const long ldu = s.ldu, ldv = s.ldv;
  // probe rows of Uh and A, every thread's loads in flight at once (rows
  // clamped into [0, n), columns < KMAX), masked after
  {
    constexpr int PP = PQ * KMAX / NTHR;
    double tu[PP], ta[PP];
#pragma unroll
    for (int u = 0; u < PP; ++u) {
      const int e = threadIdx.x + u * NTHR, q = e / KMAX, c = e - q * KMAX;
      const int p = clamp_row(s.probe[q < nq ? q : 0], s.n);
      tu[u] = s.Uh[p + (long)c * ldu];
      ta[u] = s.A[p + (long)c * ldu];
    }
#pragma unroll
    for (int u = 0; u < PP; ++u) {
      const int e = threadIdx.x + u * NTHR, q = e / KMAX, c = e - q * KMAX;
      uP[e] = (q < nq && c < r) ? tu[u] : 0.0;
      aP[e] = (q < nq && c < kk) ? ta[u] : 0.0;
    }
  }
  const bool prod = s.lq_r != nullptr;
  for (int q = threadIdx.x; q < nq; q += NTHR) {
    const int p = clamp_row(s.probe[q], s.n);
    lP[q] = s.lam_r[p];
    lQ[q] = prod ? s.lq_r[p] : 1.0;
  }
  for (int t = threadIdx.x; t < kk; t += NTHR) jn[t] = s.Jn[t];
  __syncthreads();
  const int j = blockIdx.x * NTHR + threadIdx.x;
  double best = -2.0;   // past the end: never wins
  if (j < s.m) {
    double num[PQ], skel[PQ];
#pragma unroll
    for (int q = 0; q < PQ; ++q) num[q] = skel[q] = 0.0;
    // eight column loads in flight per step
    for (int c0 = 0; c0 < r; c0 += 8) {
      double vc[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) vc[t] = (c0 + t < r) ? s.Vh[j + (long)(c0 + t) * ldv] : 0.0;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if (c0 + t >= r) break;
#pragma unroll
        for (int q = 0; q < PQ; ++q) num[q] += uP[q * KMAX + c0 + t] * vc[t];
      }
    }
    for (int c0 = 0; c0 < kk; c0 += 8) {
      double bc[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) bc[t] = (c0 + t < kk) ? s.B[j + (long)(c0 + t) * ldv] : 0.0;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        if (c0 + t >= kk) break;
#pragma unroll
        for (int q = 0; q < PQ; ++q) skel[q] += aP[q * KMAX + c0 + t] * bc[t];
      }
    }
    const double lj = s.lam_c[j], qj = prod ? s.lq_c[j] : 1.0;
    best = 0.0;
#pragma unroll
    for (int q = 0; q < PQ; ++q)
      if (q < nq) best = fmax(best, fabs(num[q] / den_of(prod, lP[q], lQ[q], lj, qj) - skel[q]));
    for (int t = 0; t < kk; ++t)
      if (jn[t] == j) best = -1.0;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int t = 0; t < GROW_TOP; ++t) {
    double v = best;
    int key = (j < s.m) ? j : 0x7fffffff;
    wave_argmax(v, key);
    if (lane == 0) rv[wave] = v, rk[wave] = key;
    __syncthreads();
    double bv = rv[0];
    int bk = rk[0];
    for (int w = 1; w < 4; ++w)
      if (rv[w] > bv || (rv[w] == bv && rk[w] < bk)) bv = rv[w], bk = rk[w];
    if (threadIdx.x == 0) {
      s.mv_val[(size_t)blockIdx.x * GROW_TOP + t] = bv;
      s.mv_row[(size_t)blockIdx.x * GROW_TOP + t] = (bv > -1.5) ? bk : -1;
    }
    if (j == bk) best = -3.0;
    __syncthreads();
  }
}

// Next column set and state swap (one workgroup / solve).
__global__ __launch_bounds__(NTHR) void k_finalize(Solve2D *S) {
  Solve2D &s = S[blockIdx.x];
  if (s.active != ACT_SWEEP) return;
  const int m = s.m;
  __shared__ double rv[4];
  __shared__ int rk[4];
  const int kk = s.k;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (s.next == NEXT_GROW) {
    // the kgrow best reported columns, picked in order (score descending,
    // ties: lower column first): each pick is the best entry strictly after
    // the previous one in that order
    const int ntot = ceil_div(m, NTHR) * GROW_TOP;
    double lastv = INFINITY;
    int lastc = -1;
    for (int g = 0; g < s.kgrow; ++g) {
      double best = -2.0;
      int key = 0x7fffffff;
      for (int e = threadIdx.x; e < ntot; e += NTHR) {
        const int c = s.mv_row[e];
        const double v = s.mv_val[e];
        if (c < 0) continue;
        if (v > lastv || (v == lastv && c <= lastc)) continue;
        if (v > best || (v == best && c < key)) best = v, key = c;
      }
      wave_argmax(best, key);
      if (lane == 0) rv[wave] = best, rk[wave] = key;
      __syncthreads();
      double bv = rv[0];
      int bk = rk[0];
      for (int w = 1; w < 4; ++w)
        if (rv[w] > bv || (rv[w] == bv && rk[w] < bk)) bv = rv[w], bk = rk[w];
      __syncthreads();
      if (threadIdx.x == 0) s.J[kk + g] = clamp_row(bk, m);
      lastv = bv;
      lastc = bk;
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  if (s.next == NEXT_STOP) {
    s.active = ACT_DONE;
    return;
  }
  for (int t = 0; t < kk; ++t) s.J[t] = s.Jn[t];
  double *t;
  t = s.A, s.A = s.Ap, s.Ap = t;
  t = s.B, s.B = s.Bp, s.Bp = t;
  t = s.sig, s.sig = s.sigp, s.sigp = t;
  s.kp = kk;
  s.k = kk + (s.next == NEXT_GROW ? s.kgrow : 0);
}

// After the initial maxvol on the transformed V: pad J to k0 columns.
__global__ void k_init_J(Solve2D *S) {
  Solve2D &s = S[blockIdx.x];
  if (s.active != ACT_INIT || threadIdx.x != 0) return;
  if (s.nonfinite) {
    s.active = ACT_DONE;
    s.status = LRP_ENONFINITE;
    return;
  }
  __shared__ int used[2 * KMAX];
  const int kin = s.k, k0 = s.k0;
  for (int t = 0; t < kin; ++t) used[t] = s.J[t];
  if (k0 > kin) spread_indices(s.m, k0 - kin, used, kin, s.J + kin, s.off_c);
  s.k = k0;
  s.kp = 0;
  s.sweep = 0;
  s.active = ACT_SWEEP;
}

}  // namespace

#define LRP_BUCKET(KERN, GRID, ...)                                          \
  do {                                                                       \
    if (kmax <= 16) hipLaunchKernelGGL((KERN<16>), GRID, dim3(NTHR), 0, st, __VA_ARGS__); \
    else if (kmax <= 32) hipLaunchKernelGGL((KERN<32>), GRID, dim3(NTHR), 0, st, __VA_ARGS__); \
    else if (kmax <= 48) hipLaunchKernelGGL((KERN<48>), GRID, dim3(NTHR), 0, st, __VA_ARGS__); \
    else hipLaunchKernelGGL((KERN<64>), GRID, dim3(NTHR), 0, st, __VA_ARGS__); \
  } while (0)

hipError_t launch_factors(int n, int m, Solve2D *s, int nsolves, int kmax,
                          hipStream_t st) {
  dim3 g(ceil_div(max(n, m), NTHR), nsolves, 2);
  LRP_BUCKET(k_factors, g, s);
  return hipGetLastError();
}

int change_blocks(int m) { return min(ceil_div(m, PANEL_M), 256); }

hipError_t launch_change(int n, int m, Solve2D *s, int nsolves, int kmax,
                         hipStream_t st) {
  const int nbm = change_blocks(m);
  LRP_BUCKET(k_change_M, dim3(nbm, nsolves), nbm, s);
  hipLaunchKernelGGL(k_change_reduce, dim3(KMAX * KMAX / 64, nsolves), dim3(64), 0, st, nbm,
                     rank_bucket(kmax), s);
  dim3 g(ceil_div(max(n, m), NTHR), nsolves);
  LRP_BUCKET(k_change_norms, g, s);
  return hipGetLastError();
}

hipError_t launch_decide(int n, int m, Solve2D *s, int nsolves, int kmax,
                         hipStream_t st) {
  (void)n;
  hipLaunchKernelGGL(k_decide, dim3(nsolves), dim3(NTHR), 0, st, s);
  dim3 g(ceil_div(m, NTHR), nsolves);
  LRP_BUCKET(k_growth_score, g, s);
  hipLaunchKernelGGL(k_finalize, dim3(nsolves), dim3(NTHR), 0, st, s);
  return hipGetLastError();
}

hipError_t launch_init_J(Solve2D *s, int nsolves, hipStream_t st) {
  hipLaunchKernelGGL(k_init_J, dim3(nsolves), dim3(64), 0, st, s);
  return hipGetLastError();
}

}  // namespace lrp
