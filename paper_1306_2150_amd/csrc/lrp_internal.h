// Internal declarations shared by the HIP kernels and the host orchestration.
// Not part of the public interface (include/lrpoisson.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lrpoisson.h"

namespace lrp {

// Cross-rank cap and the related LDS panel geometry.
constexpr int KMAX = LRP_MAX_RANK;   // columns of every n x k panel
constexpr int PANEL_M = 256;         // rows of one LDS-resident QR/LU panel
constexpr int NTHR = 256;            // threads of every panel kernel
constexpr int MV_TOP = 8;            // violator rows kept per block in maxvol
constexpr int MV_CAND = 128;         // candidate rows of the maxvol swap kernel
constexpr int MV_ROUNDS = 2;         // check/swap rounds launched per maxvol
constexpr int GROW_TOP = 16;         // growth candidates kept per block (>= kick)
constexpr int BLOCK_TOP = (MV_TOP > GROW_TOP) ? MV_TOP : GROW_TOP;

// Solve phases / flags written by kernels.
enum : int {
  ACT_DONE = 0,       // finished (status holds the result)
  ACT_SWEEP = 1,      // run another sweep
  ACT_INIT = 2,       // waiting for the initial column choice
  ACT_CORE = 3,       // 3D path: factoring an unfolding of the Tucker core
};
enum : int { NEXT_CONTINUE = 0, NEXT_GROW = 1, NEXT_STOP = 2 };

// Geometry of the TSQR / tournament tree over n rows.
struct Tree {
  int nlev;          // number of levels (level 0 = leaves)
  int nb[8];         // nodes per level
  int fan;           // children per internal node
};

// Per-solve device state (one per 2D solve of a batch).  Pointers are into
// the batch workspace; scalars below "control" are read and written by the
// kernels and copied back to the host once per sweep.
struct Solve2D {
  // ---- constants
  // The matrix approximated is Xh_ij = (Uh_i . Vh_j) / D_ij, i < n, j < m,
  // with the operator's eigenvalue (see den_of)
  //   D_ij = lam_r[i] + lam_c[j]                          (lq_r == nullptr)
  //   D_ij = lam_r[i] * lq_c[j] + lq_r[i] * lam_c[j]      (otherwise).
  // A 2D Laplace solve has m = n and lam_c = lam_r = lambda; the Stokes
  // operator takes lam = 2 sin^2(pi k h/2)/h, lq = 2 cos^2(pi k h/2)/h.  A
  // mode of the 3D path has m = n^2 (pairs of the other two modes) and
  // column tables over the pairs (j, l), index j + n l.
  int n, m, r, kcap, kick, max_sweeps, min_slack, rmax;
  double eps, tau;
  const double *U, *V;
  long ld;
  double *Ux, *Vx;
  long ldx;
  const double *lam_r, *lam_c;
  const double *lq_r, *lq_c;
  int off_r, off_c;         // start offsets of the spread index sequences
  // ---- workspace.  Row-side panels (n rows) have leading dimension ldu,
  // column-side panels (m rows) ldv, the shared ones (C, Hv) ldc >= both.
  long ldu, ldv, ldc;
  double *Uh, *Vh;          // n x r, m x r  transformed input factors
  double *C;                // 3D core unfolding for TS_CORE (ldc)
  double *Hv;               // leaf Householder vectors (ldc)
  double *Q0, *Q1;          // orthonormal bases: columns (n rows), rows (m rows)
  float *Q0f, *Q1f;         // their float copies (ldu, ldv), read by the maxvol check
  double *A, *B;            // skeleton factors, this sweep (n rows, m rows)
  double *Ap, *Bp;          // skeleton factors, previous sweep
  double *tree_R;           // sum_l nb[l] * KMAX*KMAX  R factors per node
  double *tree_H;           // sum_{l>=1} nb[l] * fan*KMAX*KMAX  node vectors
  double *tree_tau;         // sum_l nb[l] * KMAX
  double *tree_Y;           // sum_l nb[l] * KMAX*KMAX  Q-formation blocks
  int *tree_piv;            // sum_l nb[l] * KMAX  tournament candidates
  double *Rfin;             // KMAX x KMAX  final R of the last TSQR
  double *Inv;              // KMAX x KMAX  (Q[I,:])^-1 of the last maxvol
  double *InvC;             // KMAX x KMAX  saved inverse for the column basis
  double *W, *Z;            // KMAX x KMAX  core singular vectors
  double *Mc;               // KMAX x KMAX  Bp^T B for the change
  double *sig;              // KMAX   singular values (descending)
  double *sigp;             // KMAX   previous sweep's singular values
  double *part;             // nb0 * KMAX*KMAX  partial sums
  double *mv_val;           // nb0 * BLOCK_TOP  maxvol violators (|B|) or
  int *mv_row;              //   growth candidates: value and row / column
  int *I, *J, *Jn;          // KMAX pivot sets
  int *probe;               // KMAX probe rows
  // ---- control
  int k, kp;                // cross rank this / previous sweep
  int k0;                   // cross rank of the first sweep
  int R;                    // truncation rank this sweep
  int sweep;                // sweeps completed
  int active;               // ACT_*
  int next;                 // NEXT_* decided at the end of a sweep
  int status;               // lrp_status
  int nonfinite;            // set by the forward transform
  int mv_done;              // maxvol converged flag
  int mv_swaps;             // swaps done by the last maxvol
  int kgrow;                // columns to add on growth
  double nrm;               // ||sigma||
  double change;            // last relative change, -1 if none
  double tail;              // ||sigma[R:]|| / ||sigma|| of the last sweep
  double chg_part[2];       // change pieces
};

// Per-solve device state of a 3D (Tucker) solve.  Mode d is approximated by
// the cross of its fiber matrix, held in the Solve2D slot inner[d]: n rows,
// and as columns the pairs (j, l) of the other two modes' pivot sets
// (p < q, column index j + k_p l, k_p k_q <= FIB_M; the columns beyond are
// zero).  Outer sweeps rebuild the fiber matrices from the latest pivots.
constexpr int CORE_MAX = KMAX * KMAX * KMAX;   // entries of a Tucker core buffer
constexpr int FIB_M = KMAX * KMAX;             // fiber-matrix columns of a mode slot
struct Solve3D {
  int n;
  int r[3];                 // input Tucker ranks
  int rmax[3];              // output capacities
  double eps;               // requested accuracy
  const double *G;          // input core r0 x r1 x r2 (i0 fastest)
  double *Gx;               // output core R0 x R1 x R2
  Solve2D *inner[3];        // device addresses of the mode slots
  double *T[3];             // r_d x r_p x k_q  half-contracted core per mode
  double *lamc[3], *lqc[3]; // FIB_M column tables of each mode slot
  double *buf0, *buf1;      // CORE_MAX each, ping-pong for mode products
  int kick, kcap, max_outer;
  // ---- control
  int phase;                // P3_*
  int outer;                // outer sweeps finished
  int kf[3];                // mode ranks of the last outer sweep
  int If[3][KMAX];          // pivot sets of the last outer sweep
  int k[3];                 // cross ranks of the modes (set before the core)
  int R[3];                 // output ranks
  int cross_status;         // combined status of the three mode crosses
  int status;               // final status
  int out_ok;               // outputs written (ranks within rmax)
  double nrm;               // ||core||
};
enum : int {
  P3_IDLE = 0,    // slot free
  P3_CROSS = 1,   // mode crosses running
  P3_CORE = 2,    // core built, unfoldings being factored
  P3_OUT = 3,     // output factors and core being written
  P3_DONE = 4,    // finished (status, R valid)
  P3_SETUP = 5,   // fiber matrices to (re)build, mode crosses to restart
};

// One column of a sine-transform GEMM: dst[0:n] = S * src[0:n].
struct DstCol {
  const double *src;
  double *dst;
  int solve;     // index into the Solve2D array for the finite flag, -1 none
  int pad;
};

// ---------------------------------------------------------------- helpers
// Wave-wide reductions on DPP lane moves (VALU, no LDS round trip): quad
// permutes and row shifts reduce each 16-lane row into its lane 15, row
// broadcasts fold the four rows into lane 63, and v_readlane hands the total
// to every lane.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v, int fill) {
  return __builtin_amdgcn_update_dpp(fill, v, CTRL, 0xf, 0xf, false);
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

constexpr int DPP_QUAD_1032 = 0xb1;   // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_2301 = 0x4e;   // quad_perm [2,3,0,1]
constexpr int DPP_ROW_SHR4 = 0x114;
constexpr int DPP_ROW_SHR8 = 0x118;

constexpr int DPP_ROW_BCAST15 = 0x142;   // lane 15 of a row -> next row
constexpr int DPP_ROW_BCAST31 = 0x143;   // lane 31 -> rows 2 and 3

// Row broadcast into the rows of ROWS; the lanes of the other rows are left
// undefined (no zero fill), which the wave sums allow: they read only lane
// 63, whose inputs come from written rows only.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_rows_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, ROWS, 0xf, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<DPP_QUAD_1032>(v);
  v += dpp_f64<DPP_QUAD_2301>(v);
  v += dpp_f64<DPP_ROW_SHR4>(v);      // out-of-row lanes read 0
  v += dpp_f64<DPP_ROW_SHR8>(v);      // lane 15 of each row: row sum
  v += dpp_rows_f64<DPP_ROW_BCAST15, 0xa>(v);   // lanes 31, 63: two rows
  v += dpp_rows_f64<DPP_ROW_BCAST31, 0xc>(v);   // lane 63: all four rows
  return readlane_f64(v, 63);
}

// Larger value wins; ties go to the smaller key.
__device__ __forceinline__ void argmax_merge(double &v, int &key, double ov, int ok) {
  if (ov > v || (ov == v && ok < key)) {
    v = ov;
    key = ok;
  }
}
template <int CTRL>
__device__ __forceinline__ void argmax_step(double &v, int &key) {
  // shifted-in lanes outside the row see (-inf, INT_MAX) and never win
  const int lo = __builtin_amdgcn_update_dpp((int)0x00000000, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp((int)0xfff00000, __double2hiint(v), CTRL, 0xf, 0xf, false);
  const int ok = __builtin_amdgcn_update_dpp(0x7fffffff, key, CTRL, 0xf, 0xf, false);
  argmax_merge(v, key, __hiloint2double(hi, lo), ok);
}

// argmax of v over the wave with lowest-key tie breaking; result in all
// lanes.  Lanes that must not compete pass v = -1 (values are |.| >= 0) or
// -inf.
__device__ __forceinline__ void wave_argmax(double &v, int &key) {
  argmax_step<DPP_QUAD_1032>(v, key);
  argmax_step<DPP_QUAD_2301>(v, key);
  argmax_step<DPP_ROW_SHR4>(v, key);
  argmax_step<DPP_ROW_SHR8>(v, key);
  double bv = readlane_f64(v, 15);
  int bk = __builtin_amdgcn_readlane(key, 15);
#pragma unroll
  for (int r = 1; r < 4; ++r)
    argmax_merge(bv, bk, readlane_f64(v, 16 * r + 15),
                 __builtin_amdgcn_readlane(key, 16 * r + 15));
  v = bv;
  key = bk;
}

// Value of lane `src` (wave-uniform) in every lane.
__device__ __forceinline__ double bcast_f64(double v, int src) {
  return readlane_f64(v, src);
}

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Rank bucket of a cross of k columns: the sweep kernels are instantiated for
// k <= 16, 32, 48 and 64.  A sweep launches every bucket its slots occupy,
// and a sweep-phase kernel of bucket KM takes only the slots of that bucket,
// so a slot of 32 columns does not run at the register size and occupancy of
// a neighbour that grew to 40.
__host__ __device__ inline int rank_bucket(int k) {
  return k <= 16 ? 16 : (k <= 32 ? 32 : (k <= 48 ? 48 : 64));
}
// Bit of the bucket of k in a mask of occupied buckets, and the largest
// bucket of a mask.
__host__ __device__ inline unsigned bucket_bit(int k) { return 1u << (rank_bucket(k) / 16 - 1); }
__host__ __device__ inline int top_bucket(unsigned mask) {
  return (mask & 8u) ? 64 : (mask & 4u) ? 48 : (mask & 2u) ? 32 : 16;
}

// The operator's eigenvalue D_ij from the row-side values (a = lam_r[i],
// b = lq_r[i]) and the column-side values (c = lam_c[j], d = lq_c[j]);
// `prod` selects the product form of the Stokes operator (wave-uniform).
__device__ __forceinline__ double den_of(bool prod, double a, double b, double c, double d) {
  return prod ? a * d + b * c : a + c;
}

// Tile order of a GEMM-like launch of R x C tiles (R row tiles, C column
// tiles) on a 1D grid.  Workgroup L is dispatched to XCD L mod 8, and each
// XCD has its own L2.
//  - XCD order (xcd = true): the tiles, numbered column tile by column tile
//    (t = ct * R + rt), are cut into 8 contiguous ranges and XCD x runs range
//    x in order.  The row tiles of a column tile then share one L2, so a
//    column's data is fetched from HBM about once instead of once per XCD;
//    with fewer than 8 column tiles the row tiles of one column tile are
//    spread over all XCDs.
//  - plain order (xcd = false): tile t = L, i.e. consecutive workgroups take
//    consecutive row tiles and every XCD sees every column tile.
// Returns false for the padding workgroups of the XCD order.
__device__ __forceinline__ bool tile_of(int R, int C, bool xcd, int &rt, int &ct) {
  const int L = blockIdx.x, T = R * C;
  int t = L;
  if (xcd) {
    const int per = (T + 7) >> 3;
    const int j = L >> 3;
    t = (L & 7) * per + j;
    if (j >= per) return false;
  }
  if (t >= T) return false;
  rt = t % R;
  ct = t / R;
  return true;
}
inline int tile_grid(int R, int C, bool xcd) {
  return xcd ? 8 * ceil_div(R * C, 8) : R * C;
}

// count evenly spaced indices in [0, n) avoiding used[0:nu);
// (floor((2i+1)n/(2count)) + off) mod n moved to the next free index
// (cyclically).  Single thread.
__device__ inline void spread_indices(int n, int count, int *used, int nu, int *out, int off) {
  int have = nu;
  for (int i = 0; i < count; ++i) {
    if (have >= n) break;
    int j = (int)((((long long)(2 * i + 1) * n) / (2LL * count) + off) % n);
    for (;;) {
      bool taken = false;
      for (int t = 0; t < have; ++t)
        if (used[t] == j) {
          taken = true;
          break;
        }
      if (!taken) break;
      j = (j + 1) % n;
    }
    used[have++] = j;
    out[i] = j;
  }
}

// Row index from a pivot array, kept inside [0, n) so that a bookkeeping
// error can never turn into an out-of-bounds access.
__device__ __forceinline__ int clamp_row(int i, int n) {
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// ----------------------------------------------------------- launchers
// Each .hip file defines the host launchers for its kernels.
// `work` (work_bytes) holds the int8 slice records of the columns of one
// launch (LRP_PREC_INT8 only, see dst_i8_work_bytes).  When ev0/ev1 are
// given they are recorded on `st` right before the first and right after the
// last launch of the transform's GEMM kernel (slicing and split-K reduction
// outside the window when the columns fit one launch).
hipError_t launch_dst(int prec, int n, const void *tab, const DstCol *cols,
                      int ncols, Solve2D *solves, double *partial,
                      size_t partial_elems, void *work, size_t work_bytes,
                      hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
size_t dst_partial_elems(int n, int ncols);
// int8 slice transform (dst_i8.hip): record table of the sines, support
bool dst_i8_supported(int n);   // the sine record table fits LDS (n up to about 18000)
size_t dst_i8_table_bytes(int n);
void dst_i8_table(int n, unsigned char *out);
size_t dst_i8_work_bytes(int n, int ncols);
// columns whose slice records one work buffer holds: `want`, capped so that
// the buffer stays within 512 MiB, but never below 1024
int dst_i8_work_cols(int n, int want);
// chirp-z FFT transform in float64 (dst_fft.hip): grid sizes whose folded
// halves fit its 4096-point FFT (n <= 4096); its tables (chirp, twiddles,
// FFT of the convolution kernel) follow the int8 records in the grid's
// table block, 16-byte aligned (dst_fft_table_offset)
bool dst_fft_supported(int n);
size_t dst_fft_table_bytes(int n);
void dst_fft_table(int n, double *out);
hipError_t launch_dst_fft(int n, const void *tab, const DstCol *cols, int ncols,
                          Solve2D *solves, hipStream_t st, hipEvent_t ev0 = nullptr,
                          hipEvent_t ev1 = nullptr);
// The grid's table block, per n (Q = floor(N/2) + 1 quarter-wave entries,
// Qp8 = Q rounded up to 2, Qp4 = Q rounded up to 4):
//   [float64 x Qp8][float32 x Qp4][bf16 hi|lo x Qp4 (uint32)]
//   [bf16 hi|mid, lo x Qp4 (uint2)][int8 sine records][FFT tables]
struct TabLayout {
  size_t f32, bf2, bf3, i8, fft, end;
};
inline TabLayout tab_layout(int n) {
  const int Q = (n + 1) / 2 + 1;
  const size_t Qp8 = (size_t)((Q + 1) & ~1), Qp4 = (size_t)((Q + 3) & ~3);
  TabLayout L;
  L.f32 = Qp8 * 8;
  L.bf2 = L.f32 + Qp4 * 4;
  L.bf3 = L.bf2 + Qp4 * 4;
  L.i8 = L.bf3 + Qp4 * 8;
  L.fft = (L.i8 + dst_i8_table_bytes(n) + 255) & ~(size_t)255;
  L.end = dst_fft_supported(n) ? L.fft + dst_fft_table_bytes(n) : L.i8 + dst_i8_table_bytes(n);
  return L;
}
inline size_t dst_fft_table_offset(int n) { return tab_layout(n).fft; }
hipError_t launch_dst_i8(int n, const void *rec, DstCol *cols, int ncols, Solve2D *solves,
                         double *partial, size_t partial_elems, void *work,
                         size_t work_bytes, hipStream_t st, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);

// Row counts: calls on the column side (Xh[:, J], Q0, A) cover the n rows,
// calls on the row side (Xh[I, :]^T, Q1, B, Vh) the m columns.
// kmax selects the kernels' rank bucket (rank_bucket(kmax)), and a launch
// covers every slot with k <= its bucket -- except, in the sweep phase, the
// kernels with many workgroups per slot (the TSQR and maxvol leaves, the
// maxvol check, the factors, the change): those take only the slots of their
// own bucket.  Sweep launches therefore pass the mask of occupied buckets
// (bmask, bucket_bit): the leaf-level kernels run once per bucket in it, the
// few-workgroup ones (tree nodes, maxvol inverse and swaps, core) once at
// its largest bucket.  bmask 0: the bucket of kmax alone.
// TSQR inputs/outputs.  TS_C_TO_Q0 / TS_C_TO_Q1 evaluate the cross columns
// Xh[:, J] / rows Xh[I, :]^T in the leaf kernel itself and orthonormalise
// them.  TS_CORE factors the panel in C with `rows` rows and keeps only R
// (in Rfin); it acts on slots in the ACT_CORE phase.
enum : int { TS_C_TO_Q0 = 0, TS_C_TO_Q1 = 1, TS_VH_TO_Q1 = 2, TS_CORE = 3 };
hipError_t launch_tsqr(int which, int rows, const Tree &tr, Solve2D *s,
                       int nsolves, int kmax, hipStream_t st, unsigned bmask = 0);

enum : int { MV_Q0_TO_I = 0, MV_Q1_TO_JN = 1, MV_Q1_TO_J = 2 };
hipError_t launch_maxvol(int which, int rows, const Tree &tr, Solve2D *s,
                         int nsolves, int kmax, hipStream_t st, unsigned bmask = 0);
// host-side kernel attributes of launch_maxvol, set once (launch_maxvol
// calls it; call it before capturing launches into a graph)
hipError_t maxvol_prepare();
// more check/swap rounds of a maxvol that launch_maxvol started (its rows
// and inverse are current); rounds of a converged maxvol do nothing
hipError_t launch_maxvol_rounds(int which, int rows, const Tree &tr, Solve2D *s,
                                int nsolves, int kmax, int rounds, hipStream_t st,
                                unsigned bmask = 0);

hipError_t launch_core(int phase, Solve2D *s, int nsolves, int kmax, hipStream_t st);
hipError_t launch_factors(int n, int m, Solve2D *s, int nsolves, int kmax,
                          hipStream_t st);
// blocks of the change's partial Gram sums over m rows (fixed per m)
int change_blocks(int m);
hipError_t launch_change(int n, int m, Solve2D *s, int nsolves, int kmax,
                         hipStream_t st);
hipError_t launch_decide(int n, int m, Solve2D *s, int nsolves, int kmax,
                         hipStream_t st);
hipError_t launch_init_J(Solve2D *s, int nsolves, hipStream_t st);

// ---- 3D path (tucker.hip)
// After the mode crosses: the outer decision (restart on new fibers, or the
// core), then the fiber matrices of every solve in P3_SETUP (their column
// factors and tables, the mode slots reset to start a cross).
hipError_t launch_fiber_outer(Solve3D *s, int nsolves, hipStream_t st);
hipError_t launch_fiber_setup(Solve3D *s, int nsolves, int rmax, hipStream_t st);
hipError_t launch_core_build(Solve3D *s, int nsolves, hipStream_t st);
hipError_t launch_core_unfold(Solve3D *s, int nsolves, int P, hipStream_t st);
hipError_t launch_tucker_out(Solve3D *s, int nsolves, int n, hipStream_t st);

Tree make_tree(int n, int kmax);

// ---- exponential-sum comparator (expsum.hip, host_expsum.cpp)
// The approach Section 4.1 sets against the cross: 1/x ~ sum_k w_k e^{-p_k x}
// on the range of the eigenvalue sums makes the divided spectrum the
// Hadamard product of Fh = Uh Vh^T with a rank-R matrix, i.e. the rank R r
// product  sum_k (sqrt(w_k) e^{-p_k Lambda} Uh)(sqrt(w_k) e^{-p_k Lambda} Vh)^T,
// rounded to eps (Section 3).  The rounding runs incrementally: each step
// appends c of the R r columns to the current rank-K factorisation
// Qa diag(sig) Qb^T and rounds the rank-(K + c) product by the cross's TSQR
// (both sides) and core SVD, truncating to a share of the tolerance.
constexpr int ES_MAX_TERMS = 256;   // exponential-sum terms
constexpr int ES_CMIN = 8;          // columns every step can append at least
constexpr int ES_MIN_N = 2 * KMAX;  // smallest grid of the exponential sum
constexpr int ES_MIN_N_PLAIN = 2 * ES_CMIN;   // smallest grid of a plain rounding
enum : int { ES_DONE = 0, ES_RUN = 1, ES_LAST = 2 };
// The same steps round any product U V^T of many columns ("plain" mode,
// pu != nullptr: column j of the product is pu[:, j] pv[:, j]^T), as the
// sums of low-rank matrices of the Stokes driver need.
struct ExpState {
  int n, r, R, tot;         // grid, input rank, terms, tot = R r columns
  int kw;                   // panel width cap min(KMAX, n)
  double eps;               // requested accuracy (half for the step tails)
  const double *lam;        // lambda_k, k = 1..n
  const double *sw, *p;     // sqrt(w_k), p_k, k < R
  const double *pu, *pv;    // plain mode: the product's factors (n x tot)
  long ldp;
  // ---- control
  int phase;                // ES_*
  int K;                    // rank of the current factorisation
  int j0;                   // product columns absorbed so far
  int steps;                // rounding steps run
  int status;               // lrp_status
  int capped;               // a step truncated beyond its share (rank room)
  double drop;              // sum of the dropped tails (absolute)
  double nrm;               // ||sig|| of the last core
  double sig[KMAX];         // singular values of the current factorisation
};
// Columns the next step appends: fill the panel (kw columns).
__host__ __device__ inline int es_cols(int K, int j0, int tot, int kw) {
  const int room = kw - K, left = tot - j0;
  return room < left ? room : left;
}
// Each launcher covers `cap` solves.  jobs[i] (a side) and jobs[cap + i]
// (b side) are the Solve2D records whose TSQR and core SVD round step i's
// panels: Uh = the side's transformed factor, Q0 = the side's basis, Vh =
// the panel, Q1 = the panel's orthonormal factor, A = the output staging;
// jobs[i].Rfin points at jobs[cap + i].InvC, so that the core the b side's
// SVD takes is R_a R_b^T.
hipError_t launch_es_panel(ExpState *e, Solve2D *jobs, int cap, int n, hipStream_t st);
hipError_t launch_es_trunc(ExpState *e, Solve2D *jobs, int cap, hipStream_t st);
hipError_t launch_es_update(ExpState *e, Solve2D *jobs, int cap, int n, hipStream_t st);

// ---- low-rank Stokes driver (lowrank.hip, host_stokes.cpp)
// The shift matrices of the discrete gradients (Section 2), applied to the
// columns of a factor: out[:, c] = alpha Op in[:, c].
enum : int { SHIFT_G = 0, SHIFT_H = 1, SHIFT_GT = 2, SHIFT_HT = 3 };
hipError_t launch_shift(int op, int m_out, int cols, const double *in, long ldi, double *out,
                        long ldo, double alpha, hipStream_t st);
// dst[:, c] = alpha src[:, c], c < cols
hipError_t launch_copy_scaled(int rows, int cols, const double *src, long lds, double *dst,
                              long ldd, double alpha, hipStream_t st);
// One Frobenius inner product <Xu Xv^T, Yu Yv^T> (rows x rx, rows x ry
// factors, rx, ry <= KMAX).
struct LrDot {
  const double *xu, *xv, *yu, *yv;
  long ldx, ldy;
  int rows, rx, ry;
};
hipError_t launch_lr_dots(const LrDot *pairs, int npairs, double *out, hipStream_t st);
// C (K x L) = A^T B (A: rows x K, B: rows x L).  With a workspace of
// gemm_tn_work(rows, K, L) doubles the rows are split over up to
// GEMM_SPLIT workgroup layers whose partial products are then summed in
// layer order (the same sum for every launch shape); without one, each
// output tile sums all rows itself.
constexpr int GEMM_SPLIT = 64;
size_t gemm_tn_work(int rows, int K, int L);
hipError_t launch_gemm_tn(int rows, int K, int L, const double *A, long lda, const double *B,
                          long ldb, double *C, long ldc, hipStream_t st,
                          double *work = nullptr);
// C (rows x L) = A B diag(scale) (A: rows x K, B: K x L; scale null: ones)
hipError_t launch_gemm_nn(int rows, int K, int L, const double *A, long lda, const double *B,
                          long ldb, double *C, long ldc, const double *scale, hipStream_t st);

}  // namespace lrp
