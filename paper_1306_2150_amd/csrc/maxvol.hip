// maxvol: k rows I of an n x k orthonormal basis Q whose k x k submatrix has
// (locally) maximal volume -- the pivot choice of the cross approximation
// (paper Section 4.2, refs. gt-maxvol-2001, gostz-maxvol-2010).  The exit
// contract is the one of the algorithm: B = Q Q[I,:]^-1 has B[I,:] =
// identity and max|B| <= tau.
//
// GPU formulation (same contract, parallel steps):
//  1. starting rows: Gaussian elimination with partial pivoting run as a
//     tournament -- every 256-row block selects its pivot rows, internal
//     nodes run the elimination again on the union of their children's
//     candidates (first sweep and after rank growth; otherwise the rows of
//     the same maxvol in the previous sweep);
//  2. Inv = Q[I,:]^-1 (Gauss-Jordan, partial pivoting), then rounds of:
//     every block forms its rows of B = Q Inv and reports its largest
//     entries above tau; one workgroup runs the classical swap loop (swap the
//     argmax row in, rank-1 update of B) on I plus the reported rows and
//     applies the same rank-1 updates to Inv.  A round that finds no entry
//     above tau ends the iteration.  Each swap multiplies |det Q[I,:]| by
//     more than tau, so the rounds terminate.  Inside a cross sweep at most
//     MV_ROUNDS rounds run (the next sweep starts from the rows reached, so
//     the iteration goes on across sweeps); launch_maxvol_rounds continues
//     one to the contract.
#include "panel.h"

namespace lrp {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));

struct MvIO {
  const double *Q;
  const float *Qf;   // float copy of Q (leading dimension ld), for the check
  long ld;
  int *out;
  double *inv;
};
__device__ inline MvIO mv_io(int which, Solve2D &s) {
  if (which == MV_Q0_TO_I) return {s.Q0, s.Q0f, s.ldu, s.I, s.InvC};
  if (which == MV_Q1_TO_JN) return {s.Q1, s.Q1f, s.ldv, s.Jn, s.Inv};
  return {s.Q1, s.Q1f, s.ldv, s.J, s.Inv};   // MV_Q1_TO_J
}

__device__ inline int mv_phase(int which) {
  return which == MV_Q1_TO_J ? ACT_INIT : ACT_SWEEP;
}

// A sweep-phase launch of the tournament leaves or the check (many
// workgroups per slot) of rank bucket km takes only the slots of that bucket.
__device__ inline bool mv_skip(const Solve2D &s, int which, int km) {
  return s.active != mv_phase(which) ||
         (mv_phase(which) == ACT_SWEEP && rank_bucket(s.k) != km);
}

// A sweep that kept the cross rank starts its maxvol from the rows the same
// maxvol chose in the previous sweep (the bases move little between sweeps,
// so those rows are nearly maximal-volume already); the tournament only
// runs on the first sweep and after the rank grew.
__device__ inline bool mv_warm(const Solve2D &s, int which) {
  return which != MV_Q1_TO_J && s.sweep >= 1 && s.kp == s.k;
}

__device__ inline size_t piv_off(const Tree &t, int l) {
  size_t o = 0;
  for (int i = 0; i < l; ++i) o += (size_t)t.nb[i] * KMAX;
  return o;
}

// ---- tournament elimination
// At NS <= 8 six waves per SIMD fit without spilling.
template <int NS>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(NS <= 8 ? 6 : 1)))
void k_mv_leaf(int which, int n, Tree tr, Solve2D *S) {
  Solve2D &s = S[blockIdx.y];
  if (mv_skip(s, which, 4 * NS)) return;
  __shared__ double lbuf[2 * PANEL_M];
  __shared__ int shp[2];
  __shared__ int piv[KMAX];
  const int kk = s.k;
  if (threadIdx.x == 0 && blockIdx.x == 0) s.mv_done = 0, s.mv_swaps = 0;
  if (mv_warm(s, which)) return;
  const MvIO io = mv_io(which, s);
  const int b = blockIdx.x, r0 = b * PANEL_M;
  const int m = min(PANEL_M, n - r0);
  double y[NS][4];
  panel_load(y, io.Q + r0, io.ld, m, kk);
  gepp_select_regs(y, m, kk, lbuf, shp, piv);
  __syncthreads();
  const int np = min(m, kk);
  int *dst = (tr.nlev == 1) ? io.out : (s.tree_piv + piv_off(tr, 0) + (size_t)b * KMAX);
  for (int j = threadIdx.x; j < kk; j += NTHR) dst[j] = (j < np) ? r0 + piv[j] : -1;
}

template <int NS>
__global__ __launch_bounds__(NTHR) void k_mv_node(int which, int n, int lev,
                                                 Tree tr, Solve2D *S) {
  Solve2D &s = S[blockIdx.y];
  if (s.active != mv_phase(which) || mv_warm(s, which)) return;
  __shared__ double lbuf[2 * PANEL_M];
  __shared__ int shp[2];
  __shared__ int piv[KMAX];
  __shared__ int rows[PANEL_M];
  __shared__ int wcnt[4];
  const int kk = s.k;
  const MvIO io = mv_io(which, s);
  const int t = blockIdx.x, c0 = t * tr.fan;
  const int nch = min(tr.fan, tr.nb[lev - 1] - c0);
  const int *cp = s.tree_piv + piv_off(tr, lev - 1) + (size_t)c0 * KMAX;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // the children's candidate rows in child order, the empty slots (-1)
  // dropped: one entry per thread (fan * kmax <= PANEL_M = NTHR), all loads
  // in flight at once, compacted by a ballot prefix count
  static_assert(PANEL_M == NTHR, "one candidate per thread");
  int rr = -1;
  if (threadIdx.x < nch * kk) {
    const int ch = threadIdx.x / kk, ii = threadIdx.x - ch * kk;
    rr = cp[(size_t)ch * KMAX + ii];
  }
  const unsigned long long keep = __ballot(rr >= 0);
  if (lane == 0) wcnt[wave] = __popcll(keep);
  __syncthreads();
  int off = 0;
  for (int w = 0; w < wave; ++w) off += wcnt[w];
  if (rr >= 0) rows[off + __popcll(keep & ((1ull << lane) - 1ull))] = rr;
  const int mp = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
  __syncthreads();
  double y[NS][4];
#pragma unroll
  for (int sl = 0; sl < NS; ++sl) {
    const int c = wave + 4 * sl;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lane + 64 * q;
      y[sl][q] = (c < kk && i < mp) ? io.Q[clamp_row(rows[i], n) + (long)c * io.ld] : 0.0;
    }
  }
  gepp_select_regs(y, mp, kk, lbuf, shp, piv);
  __syncthreads();
  const int np = min(mp, kk);
  int *dst = (lev == tr.nlev - 1) ? io.out
                                  : (s.tree_piv + piv_off(tr, lev) + (size_t)t * KMAX);
  for (int j = threadIdx.x; j < kk; j += NTHR) dst[j] = (j < np) ? rows[piv[j]] : -1;
}

// ---- Inv = Q[I,:]^-1 by Gauss-Jordan with partial pivoting (one workgroup).
// Rows are not exchanged: the pivot row of column j is flagged and scaled,
// all other rows are eliminated against it; at the end row p_j of the right
// half is row j of the inverse.  Threads: column cl = tid & 63 (and
// cl + 64), rows i0 = tid >> 6 stepping by 4.
template <int KM>
__global__ __launch_bounds__(NTHR) void k_mv_inv(int which, int n, int force,
                                                Solve2D *S) {
  Solve2D &s = S[blockIdx.x];
  if (s.active != mv_phase(which)) return;
  if (!force && s.mv_done) return;
  constexpr int W2 = 2 * KM;                   // augmented row length
  __shared__ double a[KM][W2 + 1];
  __shared__ double prow[W2];
  __shared__ double f[KM];
  __shared__ int pivrow[KM];
  __shared__ int used[KM];
  __shared__ int shp;
  __shared__ double sip;
  const int kk = s.k, w2 = 2 * kk;
  if (kk > KM) return;                         // the bucket covers every k
  const int cl = threadIdx.x & 63, i0 = threadIdx.x >> 6;
  const MvIO io = mv_io(which, s);
  for (int i = i0; i < kk; i += 4)
    for (int c = cl; c < w2; c += 64)
      a[i][c] = (c < kk) ? io.Q[clamp_row(io.out[i], n) + (long)c * io.ld]
                         : ((c - kk == i) ? 1.0 : 0.0);
  if (threadIdx.x < KM) used[threadIdx.x] = 0;
  __syncthreads();
  for (int j = 0; j < kk; ++j) {
    if (threadIdx.x < 64) {
      double best = -1.0;
      int key = 0x7fffffff;
      const int i = threadIdx.x;
      if (i < kk && !used[i]) {
        best = fabs(a[i][j]);
        key = i;
      }
      wave_argmax(best, key);
      if (threadIdx.x == 0) {
        shp = key;
        pivrow[j] = key;
        used[key] = 1;
        const double pv = a[key][j];
        sip = (pv != 0.0) ? 1.0 / pv : 0.0;
      }
    }
    __syncthreads();
    const int p = shp;
    for (int c = threadIdx.x; c < w2; c += NTHR) prow[c] = a[p][c] * sip;
    if (threadIdx.x < kk) f[threadIdx.x] = (threadIdx.x == p) ? 0.0 : a[threadIdx.x][j];
    __syncthreads();
    {
      // the thread's entries (rows i0 + 4 u, columns cl + 64 v) read first
      // (indices clamped inside the arrays), then updated; each entry is
      // read and written by its own thread only
      constexpr int RI = KM / 4, CV = (W2 + 63) / 64;
      double pr[CV], fv[RI], av[RI][CV];
#pragma unroll
      for (int v = 0; v < CV; ++v) pr[v] = prow[min(cl + 64 * v, W2 - 1)];
#pragma unroll
      for (int u = 0; u < RI; ++u) {
        const int i = min(i0 + 4 * u, KM - 1);
        fv[u] = f[i];
#pragma unroll
        for (int v = 0; v < CV; ++v) av[u][v] = a[i][min(cl + 64 * v, W2 - 1)];
      }
#pragma unroll
      for (int u = 0; u < RI; ++u)
#pragma unroll
        for (int v = 0; v < CV; ++v) {
          const int i = i0 + 4 * u, c = cl + 64 * v;
          if (i < kk && c < w2) a[i][c] = (i == p) ? pr[v] : av[u][v] - fv[u] * pr[v];
        }
    }
    __syncthreads();
  }
  for (int t = i0; t < kk; t += 4)
    for (int c = cl; c < kk; c += 64) io.inv[t + c * KMAX] = a[pivrow[t]][kk + c];
}

// One DPP step of a lane-wise max over 16 values (non-negative floats; lanes
// shifted in from outside the row read 0).
template <int CTRL>
__device__ __forceinline__ void row_max16_f32(float (&v)[16]) {
#pragma unroll
  for (int e = 0; e < 16; ++e)
    v[e] = fmaxf(v[e], __int_as_float(__builtin_amdgcn_update_dpp(
                           0, __float_as_int(v[e]), CTRL, 0xf, 0xf, true)));
}

// ---- per block: rows of B = Q Inv, report the MV_TOP largest rows > tau.
// The check only selects candidates: the swap loop recomputes every
// reported row in float64 and swaps only on those values, so B is formed
// here from the float copy of Q on the float32 matrix cores
// (v_mfma_f32_16x16x4f32; half the bytes of Q, twice the rate).  A row
// within the float32 rounding of B of tau may go unreported; maxvol then
// stops with max |B| above tau by at most that rounding.  Wave w takes rows
// 64 w .. 64 w + 63 of the block as four 16-row blocks; the B operand (Inv,
// zero past k) stays in registers for the whole K loop.  Operand layouts:
// A[i][kq] in lane i + 16 kq, B[kq][j] in lane j + 16 kq, D[i][j] in lane
// j + 16 (i / 4), register i % 4.
// At KM <= 32 the register budget of five waves per SIMD fits without
// spilling (the check is latency-bound: more waves in flight, more overlap).
template <int KM>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(KM <= 32 ? 5 : 1)))
void k_mv_check(int which, int n, Solve2D *S) {
  Solve2D &s = S[blockIdx.y];
  if (mv_skip(s, which, KM) || s.mv_done) return;
  constexpr int NC = KM / 16;                   // 16-column blocks of B
  constexpr int NK = KM / 4;                    // K steps
  __shared__ double rowmax[NTHR];
  __shared__ double sinv[KM * KM];
  __shared__ double rv[4];
  __shared__ int rk[4];
  const int kk = s.k;
  const MvIO io = mv_io(which, s);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  // the inverse staged through LDS: every thread's loads in flight at once
  // (indices below KM <= KMAX, so always inside the buffer), masked after
  {
    constexpr int PT = KM * KM / NTHR;
    double tv[PT];
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int e = threadIdx.x + u * NTHR, r = e / KM, c = e - r * KM;
      tv[u] = io.inv[r + c * KMAX];
    }
#pragma unroll
    for (int u = 0; u < PT; ++u) {
      const int e = threadIdx.x + u * NTHR, r = e / KM, c = e - r * KM;
      sinv[e] = (r < kk && c < kk) ? tv[u] : 0.0;
    }
  }
  __syncthreads();
  float binv[NK][NC];
#pragma unroll
  for (int kb = 0; kb < NK; ++kb)
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) binv[kb][cb] = (float)sinv[(4 * kb + g) * KM + 16 * cb + li];
  const int rw0 = blockIdx.x * NTHR + 64 * wave + li;   // + 16 rb
  f4 acc[4][NC];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) acc[rb][cb] = (f4){0.0f, 0.0f, 0.0f, 0.0f};
  // every load of the block first (one memory latency per workgroup), then
  // the matrix-core steps
  float a[NK][4];
#pragma unroll
  for (int kb = 0; kb < NK; ++kb) {
    const int col = 4 * kb + g;
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      const int row = rw0 + 16 * rb;
      a[kb][rb] = (row < n && col < kk) ? io.Qf[row + (long)col * io.ld] : 0.0f;
    }
  }
#pragma unroll
  for (int kb = 0; kb < NK; ++kb)
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < NC; ++cb)
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[kb][rb], binv[kb][cb], acc[rb][cb], 0, 0, 0);
  // largest |B| of each row: over the column blocks in the lane, then over
  // the 16 lanes (one DPP row) that hold the row's columns; lane 15 of the
  // DPP row ends with the row's value.  The maxima are taken in float (exact)
  // and all 16 rows' steps interleaved.
  float vm[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    float v = 0.0f;
#pragma unroll
    for (int cb = 0; cb < NC; ++cb) v = fmaxf(v, fabsf(acc[e >> 2][cb][e & 3]));
    vm[e] = v;
  }
  row_max16_f32<DPP_QUAD_1032>(vm);
  row_max16_f32<DPP_QUAD_2301>(vm);
  row_max16_f32<DPP_ROW_SHR4>(vm);
  row_max16_f32<DPP_ROW_SHR8>(vm);
  if (li == 15) {
#pragma unroll
    for (int e = 0; e < 16; ++e) rowmax[64 * wave + 16 * (e >> 2) + 4 * g + (e & 3)] = (double)vm[e];
  }
  __syncthreads();
  const int row = blockIdx.x * NTHR + threadIdx.x;
  double mx = -1.0;
  if (row < n) {
    mx = rowmax[threadIdx.x];
    if (!(mx > s.tau)) mx = -1.0;   // only violators compete
  }
  for (int t = 0; t < MV_TOP; ++t) {
    double v = mx;
    int key = (row < n) ? row : 0x7fffffff;
    wave_argmax(v, key);
    if (lane == 0) {
      rv[wave] = v;
      rk[wave] = key;
    }
    __syncthreads();
    double bv = rv[0];
    int bk = rk[0];
    for (int w = 1; w < 4; ++w)
      if (rv[w] > bv || (rv[w] == bv && rk[w] < bk)) bv = rv[w], bk = rk[w];
    if (threadIdx.x == 0) {
      s.mv_val[(size_t)blockIdx.x * MV_TOP + t] = bv;
      s.mv_row[(size_t)blockIdx.x * MV_TOP + t] = (bv > 0.0) ? bk : -1;
    }
    if (!(bv > 0.0)) {
      // no violator left in the block (uniform): the other slots report none
      if (threadIdx.x == 0)
        for (int u = t + 1; u < MV_TOP; ++u) {
          s.mv_val[(size_t)blockIdx.x * MV_TOP + u] = -1.0;
          s.mv_row[(size_t)blockIdx.x * MV_TOP + u] = -1;
        }
      break;
    }
    if (row == bk) mx = -1.0;
    __syncthreads();
  }
}

// ---- one workgroup: swap loop on I plus the reported rows
// LDS bytes of k_mv_swap<KM>
constexpr size_t mv_swap_lds(int km) {
  return (size_t)(km + MV_CAND) * km * 8 + (size_t)km * km * 8 + (size_t)2 * km * 8 +
         (size_t)(km + MV_CAND) * 8 + (size_t)(km + MV_CAND) * 4 + 16;
}

// KM: the launch's rank bucket; the LDS arrays have row length KM, so that
// small ranks leave room for more workgroups per CU.
template <int KM>
__global__ __launch_bounds__(NTHR) void k_mv_swap(int which, int n, int nb0,
                                                 Solve2D *S) {
  Solve2D &s = S[blockIdx.x];
  if (s.active != mv_phase(which) || s.mv_done) return;
  extern __shared__ __align__(16) unsigned char smem[];
  const int kk = s.k;
  if (kk > KM) return;                              // the bucket covers every k
  const MvIO io = mv_io(which, s);
  double *Bm = (double *)smem;                      // (KM+MV_CAND) x KM
  double *inv = Bm + (KM + MV_CAND) * KM;           // KM x KM
  double *prow = inv + KM * KM;                     // KM
  double *icol = prow + KM;                         // KM
  double *pcol = icol + KM;                         // KM + MV_CAND
  int *rows = (int *)(pcol + KM + MV_CAND);         // KM + MV_CAND
  int *cnt = rows + KM + MV_CAND;                   // [0] count, [1] gathered, [2] swaps
  __shared__ double rv[4];
  __shared__ int rk[4];
  const int ntot = nb0 * MV_TOP;
  int *cr = rows;
  if (threadIdx.x == 0) cnt[0] = 0;
  __syncthreads();
  // the MV_CAND largest reported violators in order (value descending,
  // ties: lower row first; reported rows are distinct).  The violators are
  // first gathered into LDS (the Bm region, built only afterwards); each then
  // finds its rank among them.  Gathering order does not matter: ranks only
  // compare values and rows.
  constexpr int CMAX = 1024;                        // 12 KB, within Bm for every KM
  static_assert((size_t)(KM + MV_CAND) * KM * 8 >= (size_t)CMAX * 12, "gather area");
  double *cv = Bm;
  int *crow = (int *)(Bm + CMAX);
  if (threadIdx.x == 0) cnt[1] = 0;
  __syncthreads();
  for (int e = threadIdx.x; e < ntot; e += NTHR) {
    const double v = s.mv_val[e];
    const int rr = s.mv_row[e];
    if (rr < 0 || !(v > s.tau)) continue;
    const int slot = atomicAdd(&cnt[1], 1);
    if (slot < CMAX) {
      cv[slot] = v;
      crow[slot] = rr;
    }
  }
  __syncthreads();
  const int nv = cnt[1];
  if (nv <= CMAX) {
    for (int e = threadIdx.x; e < nv; e += NTHR) {
      const double v = cv[e];
      const int rr = crow[e];
      // count the violators ahead of this one, eight reads in flight at once
      int rank = 0, f0 = 0;
      for (; f0 + 8 <= nv; f0 += 8) {
        double w[8];
        int r[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          w[u] = cv[f0 + u];
          r[u] = crow[f0 + u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (w[u] > v || (w[u] == v && r[u] < rr)) ++rank;
      }
      for (; f0 < nv; ++f0) {
        const double w = cv[f0];
        if (w > v || (w == v && crow[f0] < rr)) ++rank;
      }
      if (rank < MV_CAND) cr[kk + rank] = rr;
    }
    if (threadIdx.x == 0) cnt[0] = min(nv, MV_CAND);
  } else {
    // very many violators: pick them one by one, each the largest entry
    // strictly after the previous pick in that order
    double lastv = INFINITY;
    int lastr = -1, picked = 0;
    const int lane0 = threadIdx.x & 63, wave0 = threadIdx.x >> 6;
    for (int it = 0; it < MV_CAND; ++it) {
      double best = -1.0;
      int key = 0x7fffffff;
      for (int e = threadIdx.x; e < ntot; e += NTHR) {
        const double v = s.mv_val[e];
        const int rr = s.mv_row[e];
        if (rr < 0 || !(v > s.tau)) continue;
        if (v > lastv || (v == lastv && rr <= lastr)) continue;
        if (v > best || (v == best && rr < key)) best = v, key = rr;
      }
      wave_argmax(best, key);
      if (lane0 == 0) rv[wave0] = best, rk[wave0] = key;
      __syncthreads();
      double bv = rv[0];
      int bk = rk[0];
      for (int w = 1; w < 4; ++w)
        if (rv[w] > bv || (rv[w] == bv && rk[w] < bk)) bv = rv[w], bk = rk[w];
      __syncthreads();
      if (!(bv > s.tau)) break;          // uniform
      if (threadIdx.x == 0) cr[kk + it] = bk;
      lastv = bv;
      lastr = bk;
      ++picked;
    }
    if (threadIdx.x == 0) cnt[0] = picked;
  }
  __syncthreads();
  const int nc = min(cnt[0], MV_CAND);
  if (nc == 0) {
    if (threadIdx.x == 0) s.mv_done = 1;
    return;
  }
  const int nr = kk + nc;
  for (int j = threadIdx.x; j < kk; j += NTHR) rows[j] = clamp_row(io.out[j], n);
  for (int i = threadIdx.x >> 6; i < kk; i += 4)
    for (int c = threadIdx.x & 63; c < kk; c += 64) inv[i * KM + c] = io.inv[i + c * KMAX];
  __syncthreads();
  // B rows: identity for I, Q[row,:] Inv for the candidates.  Element e ->
  // (row position e / KM, column e % KM).
  const int nrk = nr * KM;
  for (int e = threadIdx.x; e < nrk; e += NTHR) {
    const int t = e / KM, c = e - t * KM;
    if (c >= kk) continue;
    double v;
    if (t < kk) {
      v = (t == c) ? 1.0 : 0.0;
    } else {
      // eight column loads in flight per step (columns past k: row 0 of the
      // panel, unused), the sum in column order
      v = 0.0;
      const int rr = clamp_row(rows[t], n);
      for (int j0 = 0; j0 < kk; j0 += 8) {
        double q[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) q[u] = io.Q[(j0 + u < kk ? rr + (long)(j0 + u) * io.ld : 0)];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (j0 + u < kk) v += q[u] * inv[(j0 + u) * KM + c];
      }
    }
    Bm[e] = v;
  }
  __shared__ int sts;
  if (threadIdx.x == 0) cnt[2] = 0, sts = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int it = 0; it < 4 * kk; ++it) {
    double best = -1.0;
    int key = 0x7fffffff;
    for (int e = threadIdx.x; e < nrk; e += NTHR) {
      const int t = e / KM, c = e - t * KM;
      if (c >= kk) continue;
      const double av = fabs(Bm[e]);
      const int kv = rows[t] * KMAX + c;
      if (av > best || (av == best && kv < key)) best = av, key = kv;
    }
    wave_argmax(best, key);
    if (lane == 0) rv[wave] = best, rk[wave] = key;
    __syncthreads();
    double bv = rv[0];
    int bk = rk[0];
    for (int w = 1; w < 4; ++w)
      if (rv[w] > bv || (rv[w] == bv && rk[w] < bk)) bv = rv[w], bk = rk[w];
    if (!(bv > s.tau)) break;            // uniform: every thread sees bv
    const int gr = bk / KMAX, cs = bk - gr * KMAX;
    // the winner's row position: one thread finds it (rows are distinct)
    for (int t = threadIdx.x; t < nr; t += NTHR)
      if (rows[t] == gr) sts = t;
    __syncthreads();
    const int ts = sts;
    const double piv = Bm[ts * KM + cs];
    for (int c = threadIdx.x; c < kk; c += NTHR)
      prow[c] = (Bm[ts * KM + c] - (c == cs ? 1.0 : 0.0)) / piv;
    for (int t = threadIdx.x; t < nr; t += NTHR) pcol[t] = Bm[t * KM + cs];
    for (int i = threadIdx.x; i < kk; i += NTHR) icol[i] = inv[i * KM + cs];
    __syncthreads();
    for (int e = threadIdx.x; e < nrk; e += NTHR) {
      const int t = e / KM, c = e - t * KM;
      if (c < kk) Bm[e] -= pcol[t] * prow[c];
    }
    // the same rank-1 update keeps Inv = Q[I,:]^-1 for the new rows:
    // B = Q Inv, so Inv' = Inv - Inv[:, cs] prow gives B' = Q Inv'
    for (int e = threadIdx.x; e < kk * KM; e += NTHR) {
      const int i = e / KM, c = e - i * KM;
      if (c < kk) inv[e] -= icol[i] * prow[c];
    }
    if (threadIdx.x == 0) {
      io.out[cs] = gr;
      cnt[2] += 1;
    }
    __syncthreads();
  }
  const int swaps = cnt[2];
  if (swaps > 0)
    for (int i = threadIdx.x >> 6; i < kk; i += 4)
      for (int c = threadIdx.x & 63; c < kk; c += 64) io.inv[i + c * KMAX] = inv[i * KM + c];
  if (threadIdx.x == 0) {
    s.mv_swaps += swaps;
    if (swaps == 0) s.mv_done = 1;
  }
}

template <int NS>
void run_mv_leaf(int which, int n, const Tree &tr, Solve2D *s, int ns, hipStream_t st) {
  hipLaunchKernelGGL((k_mv_leaf<NS>), dim3(tr.nb[0], ns), dim3(NTHR), 0, st, which, n, tr, s);
}

template <int NS>
void run_mv_nodes(int which, int n, const Tree &tr, Solve2D *s, int ns, hipStream_t st) {
  for (int l = 1; l < tr.nlev; ++l)
    hipLaunchKernelGGL((k_mv_node<NS>), dim3(tr.nb[l], ns), dim3(NTHR), 0, st,
                       which, n, l, tr, s);
}

template <int KM>
void run_check(int which, int n, const Tree &tr, Solve2D *s, int ns,
               hipStream_t st) {
  hipLaunchKernelGGL((k_mv_check<KM>), dim3(tr.nb[0], ns), dim3(NTHR), 0, st,
                     which, n, s);
}

}  // namespace

// The swap kernels' dynamic LDS limits, set once per process (before any
// launch is captured into a graph).
hipError_t maxvol_prepare() {
  static bool attr = false;
  if (attr) return hipSuccess;
  const void *fns[4] = {(const void *)k_mv_swap<16>, (const void *)k_mv_swap<32>,
                        (const void *)k_mv_swap<48>, (const void *)k_mv_swap<64>};
  const int kms[4] = {16, 32, 48, 64};
  for (int t = 0; t < 4; ++t) {
    const hipError_t e = hipFuncSetAttribute(fns[t], hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)mv_swap_lds(kms[t]));
    if (e != hipSuccess) return e;
  }
  attr = true;
  return hipSuccess;
}

// The tournament leaves and the checks run once per bucket of the mask, on
// its slots; the tournament nodes, the inverse and the swap loops (a few
// workgroups or one per slot) once at the largest bucket, on every slot.
hipError_t launch_maxvol(int which, int rows, const Tree &tr, Solve2D *s,
                         int nsolves, int kmax, hipStream_t st, unsigned bmask) {
  const int n = rows;
  if (!bmask) bmask = bucket_bit(kmax);
  const int ktop = top_bucket(bmask);
  for (int kb = 16; kb <= 64; kb += 16) {
    if (!(bmask & bucket_bit(kb))) continue;
    if (kb == 16) run_mv_leaf<4>(which, n, tr, s, nsolves, st);
    else if (kb == 32) run_mv_leaf<8>(which, n, tr, s, nsolves, st);
    else if (kb == 48) run_mv_leaf<12>(which, n, tr, s, nsolves, st);
    else run_mv_leaf<16>(which, n, tr, s, nsolves, st);
  }
  if (ktop == 16) run_mv_nodes<4>(which, n, tr, s, nsolves, st);
  else if (ktop == 32) run_mv_nodes<8>(which, n, tr, s, nsolves, st);
  else if (ktop == 48) run_mv_nodes<12>(which, n, tr, s, nsolves, st);
  else run_mv_nodes<16>(which, n, tr, s, nsolves, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = maxvol_prepare()) != hipSuccess) return e;
  // one explicit inverse of the tournament's rows; the swap rounds keep it
  // current with the rank-1 updates of their swaps
  if (ktop == 16) hipLaunchKernelGGL(k_mv_inv<16>, dim3(nsolves), dim3(NTHR), 0, st, which, n, 0, s);
  else if (ktop == 32) hipLaunchKernelGGL(k_mv_inv<32>, dim3(nsolves), dim3(NTHR), 0, st, which, n, 0, s);
  else if (ktop == 48) hipLaunchKernelGGL(k_mv_inv<48>, dim3(nsolves), dim3(NTHR), 0, st, which, n, 0, s);
  else hipLaunchKernelGGL(k_mv_inv<64>, dim3(nsolves), dim3(NTHR), 0, st, which, n, 0, s);
  return launch_maxvol_rounds(which, rows, tr, s, nsolves, kmax, MV_ROUNDS, st, bmask);
}

hipError_t launch_maxvol_rounds(int which, int rows, const Tree &tr, Solve2D *s, int nsolves,
                                int kmax, int rounds, hipStream_t st, unsigned bmask) {
  const int n = rows;
  if (!bmask) bmask = bucket_bit(kmax);
  const int ktop = top_bucket(bmask);
  for (int round = 0; round < rounds; ++round) {
    for (int kb = 16; kb <= 64; kb += 16) {
      if (!(bmask & bucket_bit(kb))) continue;
      if (kb == 16) run_check<16>(which, n, tr, s, nsolves, st);
      else if (kb == 32) run_check<32>(which, n, tr, s, nsolves, st);
      else if (kb == 48) run_check<48>(which, n, tr, s, nsolves, st);
      else run_check<64>(which, n, tr, s, nsolves, st);
    }
    if (ktop == 16)
      hipLaunchKernelGGL(k_mv_swap<16>, dim3(nsolves), dim3(NTHR), mv_swap_lds(16), st, which,
                         n, tr.nb[0], s);
    else if (ktop == 32)
      hipLaunchKernelGGL(k_mv_swap<32>, dim3(nsolves), dim3(NTHR), mv_swap_lds(32), st, which,
                         n, tr.nb[0], s);
    else if (ktop == 48)
      hipLaunchKernelGGL(k_mv_swap<48>, dim3(nsolves), dim3(NTHR), mv_swap_lds(48), st, which,
                         n, tr.nb[0], s);
    else
      hipLaunchKernelGGL(k_mv_swap<64>, dim3(nsolves), dim3(NTHR), mv_swap_lds(64), st, which,
                         n, tr.nb[0], s);
  }
  return hipGetLastError();
}

}  // namespace lrp
