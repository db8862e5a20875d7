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
constexpr int MV_ROUNDS = 3;         // check/swap rounds launched per maxvol

// Solve phases / flags written by kernels.
enum : int {
  ACT_DONE = 0,       // finished (status holds the result)
  ACT_SWEEP = 1,      // run another sweep
  ACT_INIT = 2,       // waiting for the initial column choice
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
  int n, r, kcap, kick, max_sweeps, min_slack, rmax;
  double eps, tau;
  const double *U, *V;
  long ld;
  double *Ux, *Vx;
  long ldx;
  // ---- workspace (n-row panels have leading dimension n)
  double *Uh, *Vh;          // n x r  transformed input factors
  double *C;                // n x KMAX  evaluated columns / rows
  double *Hv;               // n x KMAX  leaf Householder vectors
  double *Q0, *Q1;          // n x KMAX  orthonormal bases (columns, rows)
  double *A, *B;            // n x KMAX  skeleton factors, this sweep
  double *Ap, *Bp;          // n x KMAX  skeleton factors, previous sweep
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
  double *mv_val;           // nb0 * MV_TOP  maxvol violators (|B|)
  int *mv_row;              // nb0 * MV_TOP  maxvol violators (row)
  double *score;            // n  growth scores
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
  double chg_part[2];       // change pieces
};

// One column of a sine-transform GEMM: dst[0:n] = S * src[0:n].
struct DstCol {
  const double *src;
  double *dst;
  int solve;     // index into the Solve2D array for the finite flag, -1 none
  int pad;
};

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// argmax of |v| over a wave with lowest-index tie breaking; index is an
// arbitrary int key (smaller wins on ties).  Returns value and key in all
// lanes.
__device__ __forceinline__ void wave_argmax(double &v, int &key) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double ov = __shfl_xor(v, o, 64);
    int ok = __shfl_xor(key, o, 64);
    if (ov > v || (ov == v && ok < key)) {
      v = ov;
      key = ok;
    }
  }
}

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Row index from a pivot array, kept inside [0, n) so that a bookkeeping
// error can never turn into an out-of-bounds access.
__device__ __forceinline__ int clamp_row(int i, int n) {
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// ----------------------------------------------------------- launchers
// Each .hip file defines the host launchers for its kernels.
hipError_t launch_dst(int prec, int n, const void *tab, const DstCol *cols,
                      int ncols, Solve2D *solves, double *partial,
                      size_t partial_elems, hipStream_t st);
size_t dst_partial_elems(int n, int ncols);

enum : int { EV_COLS = 0, EV_ROWS = 1, EV_GROWTH = 2 };
hipError_t launch_eval(int which, int n, const double *lam, Solve2D *s,
                       int nsolves, int kmax, hipStream_t st);

enum : int { TS_C_TO_Q0 = 0, TS_C_TO_Q1 = 1, TS_VH_TO_Q0 = 2 };
hipError_t launch_tsqr(int which, int n, const Tree &tr, Solve2D *s,
                       int nsolves, int kmax, hipStream_t st);

enum : int { MV_Q0_TO_I = 0, MV_Q1_TO_JN = 1, MV_Q0_TO_J = 2 };
hipError_t launch_maxvol(int which, int n, const Tree &tr, Solve2D *s,
                         int nsolves, int kmax, hipStream_t st);

hipError_t launch_core(int n, Solve2D *s, int nsolves, hipStream_t st);
hipError_t launch_factors(int n, Solve2D *s, int nsolves, int kmax,
                          hipStream_t st);
hipError_t launch_change(int n, int nb0, Solve2D *s, int nsolves, int kmax,
                         hipStream_t st);
hipError_t launch_decide(int n, const double *lam, Solve2D *s, int nsolves,
                         int kmax, int nb0, hipStream_t st);
hipError_t launch_init_J(int n, Solve2D *s, int nsolves, hipStream_t st);

Tree make_tree(int n, int kmax);

}  // namespace lrp
