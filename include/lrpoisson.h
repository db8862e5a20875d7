/*
 * lrpoisson.h -- C interface of the MI355X low-rank Poisson solver.
 *
 * Problem (Muravleva & Oseledets, "Fast low-rank solution of the Poisson
 * equation with application to the Stokes problem", Section 4.1, eq. "pois"):
 * solve the Dirichlet Poisson problem on the uniform tensor grid of
 * [0,1]^d, d = 2 or 3, with n interior unknowns per axis, h = 1/(n+1),
 *     2D:  T X + X T = F,                 T = h^-2 tridiag(-1, 2, -1),
 *     3D:  (T(x)I(x)I + I(x)T(x)I + I(x)I(x)T) vec X = vec F,
 * where the right-hand side arrives in low-rank form -- F = U V^T
 * (Section 3, eq. "lr") or a Tucker tensor F = G x1 U1 x2 U2 x3 U3
 * (Section 3, eq. "tucker") -- and the solution is returned in the same
 * form, accurate to a relative Frobenius tolerance eps (Section 3: the
 * accuracy is chosen consistent with the discretisation error).
 *
 * Method (Sections 4.1-4.2): sine transform of the factors (eq. "diag"),
 * cross approximation with maxvol pivots of the divided spectrum
 * Xh_ij = Fh_ij / (lambda_i + lambda_j) (eq. "div"; 3D: + lambda_l),
 * rounding by QR/SVD to eps (Section 3), inverse transform of the factors.
 *
 * Conventions shared by every entry point
 *  - All matrices are float64, column-major, in DEVICE memory of the
 *    context's GPU (hipMalloc / torch CUDA tensors).  Leading dimensions are
 *    in elements.  Input buffers are read-only; output buffers are owned and
 *    allocated by the caller with capacity for ``rmax`` columns (the output
 *    rank is not known in advance).
 *  - ``stream`` is a hipStream_t (NULL = the default stream).  The
 *    synchronous calls enqueue their work on ``stream`` and return after it
 *    completed; inputs must stay valid until then.
 *  - 2D output: Vx has orthonormal columns, Ux carries the scale, so
 *    X ~= Ux Vx^T.  3D output: U1x, U2x, U3x have orthonormal columns and
 *    the core Gx (r1 x r2 x r3, i1 fastest) carries the scale.
 *  - Errors: LRP_EINVAL is returned before any device work for invalid
 *    arguments (n < 1 or n > LRP_MAX_N, LRP_MAX_N3 in 3D, rank < 0 or
 *    > LRP_MAX_RANK,
 *    eps outside (0, 1), a NULL pointer where one is needed, ld < n).
 *    A rank-0 or all-zero right-hand side returns LRP_OK with rank 0.
 *    LRP_ENONFINITE: the factors hold Inf/NaN (detected on the device).
 *    LRP_ERANKCAP: the result needs more than ``rmax`` columns (rank_out is
 *    set to the rank needed, outputs unspecified) or the cross reached the
 *    rank cap without slack (best approximation written).
 *    LRP_ENOCONV: the sweep cap was reached; the last approximation is
 *    written and info->change holds its last relative change.
 *    LRP_EDEVICE wraps a HIP runtime error; LRP_ENOMEM a failed allocation.
 */
#ifndef LRPOISSON_H
#define LRPOISSON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LRP_MAX_N 32767   /* grid points per axis (sine table lives in LDS) */
#define LRP_MAX_N3 32767  /* grid points per axis of a 3D solve            */
#define LRP_MAX_RANK 64   /* input rank and cross-rank cap (per mode in 3D) */
#define LRP_MAX_SWEEPS 64 /* largest accepted lrp_opts.max_sweeps           */

typedef enum {
  LRP_OK = 0,
  LRP_EINVAL = -1,
  LRP_ENONFINITE = -2,
  LRP_ERANKCAP = -3,
  LRP_ENOCONV = -4,
  LRP_ENOMEM = -5,
  LRP_EDEVICE = -6,
  LRP_EBUSY = -7,
  LRP_ENOTREADY = -8
} lrp_status;

/* Arithmetic of the two sine-transform contractions (forward on the input
 * factors, inverse on the output factors).  Everything else -- eigenvalue
 * denominators, maxvol, QR, SVD, truncation -- is float64 in every mode.
 *  FP64    float64 MFMA both ways.
 *  FP32    float32 MFMA (float32 accumulation inside 64-deep K blocks,
 *          float64 sum across blocks) both ways.
 *  BF16X3  bfloat16 MFMA on a two-piece split of both operands, three
 *          products (hi*hi + hi*lo + lo*hi), float32 accumulation inside
 *          K blocks, float64 across blocks, both ways.
 *  BF16X6  bfloat16 MFMA on a three-piece split of both operands (each piece
 *          the bfloat16 rounding of what the previous ones leave), the six
 *          products of piece levels a + b <= 2, float32 accumulation inside
 *          K blocks, float64 across blocks: float32-level accuracy (relative
 *          error ~1e-7) on the bfloat16 matrix cores.
 *  INT8    int8 MFMA on exact 7-bit integer slices of both operands (six
 *          slices each, the products of slice levels <= 5, int32 sums,
 *          float64 recombination: the error-free splitting of Ozaki et al.);
 *          relative error ~1e-12 or below.  Grid sizes up to about 18000
 *          (the sine record table lives in LDS); LRP_EINVAL beyond.
 *  FFT64   not a GEMM: the transform as a chirp-z (Bluestein) convolution
 *          of the even/odd folded halves through 4096-point float64 FFTs in
 *          LDS, O(n log n) work and float64 accuracy (relative error ~1e-15).
 *          Grid sizes n <= 4096; LRP_EINVAL beyond.
 *  AUTO    per-request plan: FFT64 both ways for 2048 < n <= 4096 (the
 *          fastest there, and float64-accurate); INT8 both ways wherever it
 *          is supported otherwise (n up to about 18000; there it is faster
 *          than FP64 and FP32 and accurate to ~1e-12).  Larger grids:
 *          forward transform BF16X3 when
 *          eps >= 1e-6, FP32 when eps >= 1e-7, else FP64; inverse transform
 *          FP32 when eps >= 1e-7, else FP64.  Every floating reduced-precision
 *          transform adds a relative error near its floor (measured: FP32
 *          ~2e-7, BF16X3 ~5e-6 on the bump workloads); the inverse passes it
 *          straight to the result, the forward one is damped by the division
 *          by the eigenvalue sums, but not enough for 10 eps at eps = 1e-8
 *          (measured up to 9.5e-8 in 2D and 2.6e-7 in 3D), so below 1e-7
 *          both transforms are float64. */
typedef enum {
  LRP_PREC_FP64 = 0,
  LRP_PREC_AUTO = 1,
  LRP_PREC_FP32 = 2,
  LRP_PREC_BF16X3 = 3,
  LRP_PREC_INT8 = 4,
  LRP_PREC_FFT64 = 5,
  LRP_PREC_BF16X6 = 6
} lrp_precision;

/* The discrete operator inverted.  Both are diagonalised by the same sine
 * transform (Section 4.1), so only the eigenvalue that divides the
 * transformed right-hand side differs:
 *  LAPLACE  the 5-point (2D) / 7-point (3D) Dirichlet Laplacian
 *           T (x) I + I (x) T (+ the third term): eigenvalue
 *           lambda_i + lambda_j (+ lambda_l), lambda_k = 4/h^2 sin^2(pi k h/2)
 *           (Section 4.1, eq. "diag"; eq. "div").
 *  STOKES   the Stokes-consistent Laplacian of Section 2, the sum over axes
 *           of B_d B_d^T with the discrete gradients B_x = (G (x) H)/(4h),
 *           B_y = (H (x) G)/(4h) (G, H: shift difference and shift sum); its
 *           Kronecker form A1 (x) A2 + A2 (x) A1 (Section 4.1) has, scaled
 *           by 4 so that smooth modes see -Laplacian, the eigenvalue
 *           4 (s_i c_j + c_i s_j) / h^2 in 2D and
 *           4 (s_i c_j c_l + c_i s_j c_l + c_i c_j s_l) / h^2 in 3D, with
 *           s_k = sin^2(pi k h/2), c_k = cos^2(pi k h/2).  (Section 4.2
 *           writes the 2D denominator as a sum of one-axis terms; the
 *           Kronecker form is not such a sum, and it is the one used.) */
typedef enum {
  LRP_OP_LAPLACE = 0,
  LRP_OP_STOKES = 1
} lrp_operator;

/* Optional knobs; pass NULL for defaults.  Zero fields take defaults.
 * LRP_EINVAL for max_sweeps > LRP_MAX_SWEEPS, a negative field, an
 * unknown prec or op. */
typedef struct {
  int32_t prec;         /* lrp_precision, default LRP_PREC_FP64             */
  int32_t max_sweeps;   /* cross sweeps cap, default 10, <= LRP_MAX_SWEEPS  */
  int32_t rank_cap;     /* cross rank cap k_max, default and max 64         */
  int32_t kick;         /* cross rank growth step, default 8                */
  double maxvol_tau;    /* maxvol dominance bound, default 1.05             */
  int32_t op;           /* lrp_operator, default LRP_OP_LAPLACE             */
  int32_t k0;           /* columns of the first cross sweep (capped at
                           rank_cap and n), default rank + kick             */
  uint64_t seed;        /* offset of the deterministic index sequences: the
                           evenly spaced padding of the first column set and
                           the probe rows of rank growth start at
                           seed mod n.  The method draws no random numbers;
                           different seeds give different (equally valid)
                           pivots and the same accuracy.  Default 0.        */
} lrp_opts;

/* Per-solve report (may be NULL). */
typedef struct {
  int32_t status;       /* lrp_status of this solve                          */
  int32_t sweeps;       /* cross sweeps run                                  */
  int32_t k;            /* final cross rank                                  */
  int32_t rank;         /* output rank (2D); 3D: first mode                  */
  int32_t fwd_prec;     /* lrp_precision used by the forward transform       */
  int32_t inv_prec;     /* lrp_precision used by the inverse transform       */
  double change;        /* last relative change between sweeps (-1: none)   */
  double err_est;       /* a-posteriori relative error estimate: the
                           truncation tail ||sigma[R:]|| / ||sigma|| plus
                           the last change (3D: the largest over the modes
                           plus the core truncation tails); -1 if none      */
  float us_phase[3];    /* device time in microseconds of the call's forward
                           transform, cross sweeps and inverse transform
                           (HIP events on the call's stream; a batch reports
                           the batch's phases to every problem; 0 where not
                           measured: the serving loop)                       */
  int32_t pad;
} lrp_info;

typedef struct lrp_ctx lrp_ctx;

/* Create a solver context on HIP device ``device``.  ``workspace_bytes`` is
 * the device-memory budget of the context (0 = 32 GiB); it bounds the
 * workspace of concurrent solves and the served requests admitted at once.
 * Device memory is allocated lazily inside that budget. */
lrp_status lrp_create(lrp_ctx **ctx, int device, size_t workspace_bytes);

/* Free every device allocation of the context.  Not thread-safe with
 * concurrent calls on the same context. */
lrp_status lrp_destroy(lrp_ctx *ctx);

/* Text for a status code (static storage). */
const char *lrp_strerror(int32_t status);

/* One 2D solve (Section 4.2).  U, V: n x rank (ld >= n).  Ux, Vx: n x rmax
 * (ldx >= n).  On return *rank_out holds the output rank R <= rmax and the
 * first R columns of Ux, Vx are written. */
lrp_status lrpoisson_solve2d(lrp_ctx *ctx, int64_t n, int32_t rank,
                             const double *U, const double *V, int64_t ld,
                             double eps, const lrp_opts *opts,
                             double *Ux, double *Vx, int64_t ldx, int32_t rmax,
                             int32_t *rank_out, lrp_info *info, void *stream);

/* One 2D problem of a batch: the same fields as lrpoisson_solve2d. */
typedef struct {
  const double *U;
  const double *V;
  int64_t ld;
  int32_t rank;
  int32_t rmax;
  double eps;
  double *Ux;
  double *Vx;
  int64_t ldx;
  int32_t rank_out;     /* output */
  lrp_info info;        /* output */
} lrp_problem2d;

/* ``count`` independent 2D solves on the same grid size n, run together:
 * every kernel launch covers all of them (one transform GEMM over all their
 * columns, one launch per cross step).  Each problem's own result is the
 * same as when it is solved alone.  Returns LRP_OK when every problem
 * succeeded, otherwise the first failing problem's status; per-problem
 * status is in probs[i].info.status. */
lrp_status lrpoisson_solve2d_batch(lrp_ctx *ctx, int64_t n, int32_t count,
                                   lrp_problem2d *probs, const lrp_opts *opts,
                                   void *stream);

/* One 3D solve in Tucker format (Section 3, eq. "tucker"; the 3D case of
 * Section 4.1): F = G x1 U1 x2 U2 x3 U3 on the 7-point Dirichlet Laplacian
 * (or the Stokes operator, lrp_opts.op), denominators
 * lambda_i + lambda_j + lambda_k.  Tucker cross: every mode keeps a pivot
 * set; an outer sweep approximates each mode's fiber matrix (all indices of
 * the mode against the pairs of the other two modes' pivots, n x k_p k_q)
 * by the cross of the 2D solver to eps/sqrt(3), which gives the mode's new
 * basis and pivots; the outer sweeps stop once the mode ranks repeat.  The
 * bases and pivots give an interpolating Tucker approximation whose core is
 * rounded by truncated HOSVD at eps/sqrt(3) per mode.  U1, U2, U3:
 * n x rank[d] (ld >= n), n <= LRP_MAX_N3; G: rank[0] x rank[1] x rank[2],
 * i1 fastest.  Outputs U1x, U2x, U3x: n x rmax[d] (ldx >= n); Gx: capacity
 * rmax[0]*rmax[1]*rmax[2], written as rank_out[0] x rank_out[1] x
 * rank_out[2], i1 fastest.  info: sweeps is the number of outer sweeps, k
 * the largest mode rank, rank the largest output rank, change the largest
 * last change of the mode crosses.  LRP_ENOCONV when the outer sweeps reach
 * max_sweeps without the ranks repeating.  Workspace: about 60 MB at
 * n = 512 (three n x 4096 cross slots and the cores), linear in n, taken
 * from the context budget. */
lrp_status lrpoisson_solve3d(lrp_ctx *ctx, int64_t n, const int32_t rank[3],
                             const double *U1, const double *U2,
                             const double *U3, int64_t ld, const double *G,
                             double eps, const lrp_opts *opts,
                             double *U1x, double *U2x, double *U3x,
                             int64_t ldx, double *Gx, const int32_t rmax[3],
                             int32_t rank_out[3], lrp_info *info, void *stream);

/* The exponential-sum comparator of Section 4.1 (timed against the cross in
 * Section 6.1): the same 2D problems as lrpoisson_solve2d_batch, solved
 * without the cross.  1/x is approximated on [2 lambda_1, 2 lambda_n] by the
 * sinc (trapezoidal) rule for 1/x = int exp(t - x e^t) dt,
 * 1/x ~ sum_k w_k exp(-p_k x), relative error <= eps (tails cut at eps/3
 * each, the largest step h on the grid 1.5, ..., 0.05 of 300 steps whose
 * rule meets eps at 4000 log-spaced points); the divided spectrum is then
 * the Hadamard product of Fh = Uh Vh^T with the rank-R sum
 * sum_k w_k exp(-p_k lambda_i) exp(-p_k lambda_j), a product of rank R*rank,
 * and it is rounded to eps (Section 3) incrementally: columns are appended
 * to the running factorisation up to 64 at a time and each step is rounded
 * by QR of both factors and an SVD of the small core, dropping at most
 * (eps/2) c/(R rank) of the core's norm for c appended columns, eps/2 at the
 * last step.  Only the Laplace operator (lrp_opts.op = LRP_OP_LAPLACE): the
 * Stokes eigenvalue is not a sum.  lrp_opts.prec selects the transforms;
 * the cross's options are ignored.  LRP_EINVAL also for n < 128 and for an
 * eps that needs more than 256 terms.  info: sweeps = rounding steps, k =
 * the number of terms R, rank = output rank, change = -1, err_est = eps
 * (quadrature) plus the dropped tails over the final core norm.
 * LRP_ERANKCAP when a step had to drop more than its share to keep room for
 * 8 new columns (the approximation is still written), or the output rank
 * exceeds rmax. */
lrp_status lrp_expsum_solve2d_batch(lrp_ctx *ctx, int64_t n, int32_t count,
                                    lrp_problem2d *probs, const lrp_opts *opts,
                                    void *stream);

/* The low-rank Uzawa solve of the 2D Stokes problem (Section 2, eq.
 * "stprob"; Section 5), the application the Poisson solver serves.
 * Pressure at the n x n cell centres of [0,1]^2 (h = 1/n), velocity at the
 * (n-1) x (n-1) interior vertices (zero on the boundary); with the shift
 * matrices G = E - Z and H = E + Z ((n-1) x n), and matrices whose first
 * index runs along x, the discrete gradients are B_x p = G p H^T/(4h),
 * B_y p = H p G^T/(4h), and the Laplacian is Delta = B_x B_x^T +
 * B_y B_y^T (the Stokes-consistent operator of LRP_OP_STOKES, which is
 * 4 Delta).  The system  Delta u + B_x p = f_u,  Delta v + B_y p = f_v,
 * B_x^T u + B_y^T v = g  is reduced to the Schur system (eq. "schur")
 * S p = B_x^T Delta^-1 f_u + B_y^T Delta^-1 f_v - g,
 * S = B_x^T Delta^-1 B_x + B_y^T Delta^-1 B_y, solved by restarted GMRES
 * whose vectors are low-rank matrices: every sum is rounded, each
 * application of S runs two low-rank Poisson solves, and the accuracy of
 * the products is relaxed as the residual falls (inexact GMRES, Section 5).
 * Then u = Delta^-1 (f_u - B_x p), v likewise.  S has a two-dimensional
 * kernel (the constant and the checkerboard pressure): g's components
 * along it are removed first, and p is returned without them.
 * All factors: device float64, column-major, leading dimension ld (inputs)
 * and ldx (outputs), >= n.  n >= 32; ranks <= LRP_MAX_RANK.  The call
 * returns after its work completed; status as the 2D solve (LRP_ENOCONV
 * when max_iter iterations do not reach eps, the last iterate written). */
typedef struct {
  int64_t n;
  int32_t rank_fu, rank_fv, rank_g;
  int32_t prec;               /* lrp_precision of the Poisson solves        */
  const double *fu_U, *fu_V;  /* f_u = fu_U fu_V^T, (n-1) x rank_fu each    */
  const double *fv_U, *fv_V;  /* f_v, (n-1) x rank_fv                       */
  const double *g_U, *g_V;    /* g, n x rank_g                              */
  int64_t ld;
  double eps;                 /* relative accuracy of the Schur residual    */
  int32_t max_iter;           /* GMRES iterations cap, default 200          */
  int32_t restart;            /* GMRES restart length, default 30, <= 60    */
  double *p_U, *p_V;          /* out: p = p_U p_V^T, n x rmax each          */
  double *u_U, *u_V;          /* out: u, (n-1) x rmax each                  */
  double *v_U, *v_V;          /* out: v, (n-1) x rmax each                  */
  int64_t ldx;
  int32_t rmax;
  int32_t rank_out[3];        /* out: ranks of p, u, v                      */
  int32_t iterations;         /* out: GMRES iterations (all restarts)       */
  int32_t restarts;           /* out                                        */
  int32_t max_krylov_rank;    /* out: the largest rank of a Krylov vector   */
  int32_t status;             /* out                                        */
  double residual;            /* out: GMRES's residual estimate / ||b||     */
  double true_residual;       /* out: ||b - S p|| / ||b||, recomputed       */
} lrp_stokes2d_problem;

lrp_status lrp_stokes2d(lrp_ctx *ctx, lrp_stokes2d_problem *prob, void *stream);

/* The orthonormal sine transform on its own (paper Section 4.1, eq. "diag":
 * S[j,k] = sqrt(2/(n+1)) sin(pi j k/(n+1)), the DST-I that diagonalises the
 * 1D operator; S = S^T = S^-1, so the same call transforms forward and
 * back): dst[:, c] = S src[:, c] for c < ncols.  src: n x ncols (lds >= n),
 * dst: n x ncols (ldd >= n), both float64 device memory, not overlapping.
 * ``prec`` is an lrp_precision other than AUTO (INT8 and FFT64 within their
 * grid-size limits).  Non-finite input is not checked here. */
lrp_status lrp_sine_transform(lrp_ctx *ctx, int64_t n, int32_t ncols,
                              const double *src, int64_t lds, double *dst,
                              int64_t ldd, int32_t prec, void *stream);

/* The same transform as lrp_sine_transform, allocating nothing: for callers
 * that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc).  No context: every
 * device buffer it needs beyond src and dst (sine tables, column
 * descriptors, split-K partial sums, int8 slice records) lives in one static
 * device array of about 80 MiB that each GPU the library runs on holds
 * until the process ends; the call uses the current device's copy.  Limits:
 * n <= LRP_MAX_N (INT8: n up to about 18000, as lrp_sine_transform);
 * LRP_EINVAL otherwise, and for the argument errors of lrp_sine_transform.
 * The call returns after its work completed.  Calls on one GPU share its
 * array and keep the last call's tables: calls that overlap on one GPU
 * (several host threads) race.  Results equal lrp_sine_transform's. */
lrp_status lrp_sine_transform_noalloc(int64_t n, int32_t ncols, const double *src,
                                      int64_t lds, double *dst, int64_t ldd,
                                      int32_t prec, void *stream);

/* Kernel timing of the sine-transform launches, for measurement.  While
 * enabled, the GEMM kernel of every transform call is bracketed by two HIP
 * events recorded on the stream it runs on (the int8 slicing pass and a
 * split-K reduction stay outside); lrp_kernel_stats() waits for them and
 * returns, per precision (index = lrp_precision: 0 FP64, 2 FP32, 3 BF16X3,
 * 4 INT8, 5 FFT64, 6 BF16X6), the number of timed GEMM (or FFT) dispatches (an int8
 * transform of more columns than its work buffer holds runs several),
 * columns, their summed duration in ms and the summed algorithmic work: for
 * the GEMMs the folded transform (two half-size GEMMs: 2 (H0^2 + H1^2) flops
 * per column, H0 = ceil(n/2), H1 = floor(n/2); the dense product would be
 * 2 n^2), for FFT64 two forward and two inverse 4096-point complex FFTs per
 * column at 5 M log2 M flops each.  reset != 0 clears the counters after
 * reading.  Timing adds two event records per dispatch. */
typedef struct {
  int64_t launches;
  int64_t columns;
  double ms;
  double flops;
} lrp_kernel_stat;

lrp_status lrp_set_kernel_timing(lrp_ctx *ctx, int32_t enable);
lrp_status lrp_kernel_stats(lrp_ctx *ctx, int32_t prec, lrp_kernel_stat *out,
                            int32_t reset);

/* Graph replay of the cross sweeps (the batched and served execution around
 * the cross of Section 4.2; on by default).  With it on, each sweep step of a
 * slot group (its tree QRs, maxvol, core, factors, change and decision
 * launches) is captured once per launch plan -- the live slots rounded up to
 * a power of two, the rank buckets the slots occupy -- into a HIP graph
 * (at most 64 per group; further plans run as plain launches) and replayed
 * on the caller's stream.  The graphs hold no memory set or copy nodes.  Results are the same with it off (plain launches on the
 * caller's stream covering exactly the live slots).  LRP_EINVAL for a null
 * ctx. */
lrp_status lrp_set_graph_replay(lrp_ctx *ctx, int32_t enable);

/* ---- Continuous-batching serving (same solver, asynchronous) ----------
 * A request is admitted when the context's device-memory budget has room
 * for its workspace; its factors stay resident on the device.  Each call of
 * lrp_serve_step() runs one scheduling tick on the context's own stream:
 * newly admitted requests get their forward transform, every running 2D
 * request advances one cross sweep, finished requests get their inverse
 * transform -- all grouped by grid size into shared launches -- so work of
 * requests that arrived at different times overlaps on the device.
 * Each (dimension, grid size) group runs on a stream of its own; HIP maps
 * streams onto its hardware queues round-robin, and the number of queues is
 * the process environment's GPU_MAX_HW_QUEUES (read once, when HIP
 * initialises).  With fewer queues than active groups, a group's short
 * launches can wait behind another group's long ones on a shared queue
 * (measured: 2D p99 29 ms with the default 4 queues against 15 ms with 16 on
 * a mixed 2D/3D stream), so a serving process should set it to at least the
 * number of shapes it serves. */
typedef struct {
  int32_t dim;          /* 2 or 3                                            */
  int32_t prec;         /* lrp_precision                                     */
  int64_t n;
  int32_t rank[3];      /* 2D uses rank[0]                                   */
  int32_t rmax[3];      /* output capacity; 2D uses rmax[0]                  */
  const double *U[3];   /* 2D: U[0] = U, U[1] = V                            */
  const double *G;      /* 3D core, else NULL                                */
  int64_t ld;
  double *X[3];         /* outputs; 2D: X[0] = Ux, X[1] = Vx                 */
  double *Gx;           /* 3D output core                                    */
  int64_t ldx;
  double eps;
  int32_t op;           /* lrp_operator                                      */
  int32_t reserved;     /* must be 0                                         */
} lrp_request;

/* Queue a request; never blocks.  *ticket identifies it. */
lrp_status lrp_submit(lrp_ctx *ctx, const lrp_request *req, uint64_t *ticket);

/* Run one scheduling tick (admission, one step of every running request,
 * retirement).  Returns the number of requests still queued or running in
 * *pending.  Requests of one dimension and grid size share a group of slots
 * created on first use and kept for the context's lifetime.  If a group does
 * not fit the budget, the groups the context caches for its synchronous
 * calls are freed first; if it still does not fit, the queued requests of
 * that shape finish with LRP_ENOMEM (reported by lrp_poll / lrp_wait). */
lrp_status lrp_serve_step(lrp_ctx *ctx, int32_t *pending);

/* Non-blocking completion check.  LRP_ENOTREADY while the request is queued
 * or running; otherwise *result holds its status, rank_out[] its ranks and
 * *info its report, and the ticket is released.  LRP_EINVAL for a ticket
 * that is not known (never issued, or already released). */
lrp_status lrp_poll(lrp_ctx *ctx, uint64_t ticket, int32_t *result,
                    int32_t rank_out[3], lrp_info *info);

/* Blocking completion: runs scheduling ticks (lrp_serve_step) until the
 * request of ``ticket`` has finished, then reports it as lrp_poll does.
 * Other requests advance meanwhile.  LRP_EINVAL for an unknown ticket;
 * a device error of a tick is returned as it is. */
lrp_status lrp_wait(lrp_ctx *ctx, uint64_t ticket, int32_t *result,
                    int32_t rank_out[3], lrp_info *info);

#ifdef __cplusplus
}
#endif

#endif /* LRPOISSON_H */
