// Sine transform of factor columns as an MFMA GEMM: dst = S * src, where
// S[j,k] = sqrt(2/(n+1)) sin(pi j k/(n+1)), j, k = 1..n, the orthonormal
// DST-I that diagonalises the 1D operator (paper Section 4.1, eq. "diag";
// "the DST of the factors", Section 4.1).  S is never stored: every wave
// generates its 16 x K tile on the fly from a quarter-wave table in LDS with
// exact integer argument reduction m = j k mod 2(n+1).
//
// Folding: with N = n + 1, sin(pi j (N-k)/N) = (-1)^(j+1) sin(pi j k/N), so
// the odd rows j take u_k = x_k + x_(N-k) and the even rows w_k = x_k -
// x_(N-k) over k <= n/2 (the middle point x_(N/2) of an even N joins u):
// two half-size GEMMs, half the work of the dense product.  A column tile
// holds one parity (the "parity" of its rows); the sources are folded while
// they are staged.
//
// One launch covers any set of columns with the same n (all columns of all
// solves of a batch); K is split across workgroups when the tile count alone
// cannot fill the chip, with a deterministic fixed-order reduction.
//
// Precisions (lrp_precision):
//   FP64    v_mfma_f64_16x16x4   (float64 products and sums)
//   FP32    v_mfma_f32_16x16x4   (operands rounded to float32; float32
//           accumulation over 32-deep K runs, float64 sum across runs)
//   BF16X3  v_mfma_f32_16x16x32_bf16 on hi/lo bfloat16 splits of both
//           operands, hi*hi + hi*lo + lo*hi, float32 inside 64-deep K runs,
//           float64 across runs.
//   INT8    v_mfma_i32_16x16x64_i8 on exact 7-bit integer slices
//           (dst_i8.hip).
#include <algorithm>

#include "lrp_internal.h"

namespace lrp {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int TM = 64;    // rows per workgroup (4 waves x 16)
constexpr int TN = 32;    // columns per workgroup (2 MFMA column blocks)
constexpr int KC = 64;    // K rows staged in LDS per step

// Quarter-wave lookup: value of sqrt(2/N) sin(pi m/N) for m in [0, 2N).
template <typename T>
__device__ __forceinline__ T sine_lookup(const T *tab, int m, int N) {
  T sg = (T)1;
  if (m >= N) {
    m -= N;
    sg = (T)-1;
  }
  if (2 * m > N) m = N - m;
  return sg * tab[m];
}

__device__ __forceinline__ uint32_t bf16_bits_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ __forceinline__ float bf16_to_float(uint32_t b) {
  return __uint_as_float(b << 16);
}

// Folded source value of parity par at 0-based point i (grid point i + 1):
// x_i + x_(n-1-i) (par 0) or x_i - x_(n-1-i) (par 1); x_i alone at the middle
// point of an even N (par 0 only).  Two steps, so that the loads can be in
// flight while other work runs: fold_load issues them (zero past kend or
// without a source), fold_combine forms the value once they have arrived and
// raises `bad` for a non-finite input.
__device__ __forceinline__ void fold_load(const double *x, int i, int kend, int n, double &a,
                                          double &b) {
  a = 0.0;
  b = 0.0;
  if (x && i < kend) {
    a = x[i];
    if (2 * i + 1 < n) b = x[n - 1 - i];
  }
}
__device__ __forceinline__ double fold_combine(double a, double b, int i, int n, int par,
                                               bool &bad) {
  if (!isfinite(a) || !isfinite(b)) bad = true;
  if (2 * i + 1 >= n) return a;          // middle point (or past the end: zero)
  return par ? a - b : a + b;
}

// Tile of a folded launch: R = ceil(H0 / tm) row tiles (rows a of the half
// problem, grid row j = 2a + 1 + par) times 2 ceil(ncols / tn) column tiles;
// column tile ct holds parity ct & 1 of columns (ct >> 1) tn .. + tn - 1.
struct FoldTile {
  int row0, c0, par, Kp, H0;
};
__device__ __forceinline__ bool fold_tile(int n, int ncols, int tm, int tn, bool xcd,
                                          FoldTile &t) {
  t.H0 = (n + 1) / 2;
  int rt, ct;
  if (!tile_of(ceil_div(t.H0, tm), 2 * ceil_div(ncols, tn), xcd, rt, ct)) return false;
  t.par = ct & 1;
  t.Kp = t.par ? n / 2 : t.H0;
  t.row0 = rt * tm;
  t.c0 = (ct >> 1) * tn;
  return true;
}
// 1-based grid row of half-row a (0 past the end: a zero sine row)
__device__ __forceinline__ int fold_row(int a, const FoldTile &t) {
  return a < t.Kp ? 2 * a + 1 + t.par : 0;
}

// K is cut into fixed chunks that depend on n only; each chunk is summed
// from zero and the chunk sums are added in order.  A workgroup either walks
// all chunks (gridDim.z == 1) or owns one chunk whose sum is reduced later in
// the same order, so the result never depends on how many columns share the
// launch.
__device__ __forceinline__ void chunk_range(int n, int kchunk, int &cb, int &ce) {
  if (gridDim.z > 1) {
    cb = blockIdx.z;
    ce = blockIdx.z + 1;
  } else {
    cb = 0;
    ce = (n + kchunk - 1) / kchunk;
  }
}

// Store the result of half-row a of a folded tile: grid row 2a + par of the
// column, or the chunk's partial sum (layout [z][2 col + par][a], a < H0).
__device__ __forceinline__ void store_out(double v, int a, int col, const FoldTile &t,
                                          int ncols, const DstCol *cols,
                                          double *partial, int z) {
  if (a < t.Kp && col < ncols) {
    if (partial)
      partial[((size_t)z * 2 * ncols + 2 * col + t.par) * t.H0 + a] = v;
    else
      cols[col].dst[2 * a + t.par] = v;
  }
}

// ------------------------------------------------------------------ FP64
// 128 rows x TN columns per workgroup: HW 16-row blocks per wave (HW = 2:
// four waves of 32 rows; HW = 1: eight waves of 16 rows, half the
// accumulators per wave, so two waves share a SIMD).  The source tile is
// staged in LDS as [column][k] with one double of padding per column (the
// 16 lanes that read one k for 16 columns then hit distinct banks), double
// buffered: the next K stage is fetched into registers while the MFMAs run on
// the current one.
constexpr int TM64 = 128;
constexpr int KC64 = 32;
constexpr int LDT = KC64 + 1;

template <int TN_, int HW = 2>
__global__ __launch_bounds__(512 / HW) void k_dst_f64(
    int n, int Q, const double *__restrict__ qtab,
    const DstCol *__restrict__ cols, int ncols, int kchunk,
    double *__restrict__ partial, Solve2D *solves) {
  constexpr int NT = 512 / HW;                    // threads
  constexpr int NB = TN_ / 16;                    // column blocks per wave
  constexpr int PER = KC64 * TN_ / NT;            // tile values per thread
  constexpr int CSTEP = NT / KC64;                // staged columns per pass
  extern __shared__ __align__(16) unsigned char smem[];
  const int Qp = (Q + 1) & ~1;
  double *tab = (double *)smem;
  double *xs0 = tab + Qp;                         // [TN][LDT] x 2 buffers
  const int N = n + 1, twoN = 2 * N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  FoldTile ft;
  if (!fold_tile(n, ncols, TM64, TN_, true, ft)) return;
  const int row0 = ft.row0, c0 = ft.c0;
  int cb, ce;
  chunk_range(ft.H0, kchunk, cb, ce);
  // table copy, eight loads in flight per thread
  for (int i0 = 0; i0 < Q; i0 += 8 * NT) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * NT + tid;
      v[u] = (i < Q) ? qtab[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * NT + tid;
      if (i < Q) tab[i] = v[u];
    }
  }

  // this thread's share of a K stage: k offset tk (32 lanes read 32
  // consecutive k of one column), columns tc0 + CSTEP t
  const int tk = tid & (KC64 - 1), tc0 = tid / KC64;
  const double *src[PER];
  int sidx[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int c = c0 + tc0 + CSTEP * t;
    src[t] = nullptr;
    sidx[t] = -1;
    if (c < ncols) {
      const DstCol dc = cols[c];
      src[t] = dc.src;
      sidx[t] = dc.solve;
    }
  }
  const int kbeg = cb * kchunk, kend = min(ft.Kp, ce * kchunk);
  const int nst = (kend - kbeg + KC64 - 1) / KC64;
  // a stage's loads are issued before the MFMAs of the previous stage and
  // combined (folded) only when they are stashed in LDS after them
  double pa[PER], pb[PER];
  unsigned bad = 0;
  int kf = 0;
  auto fetch = [&](int st) {
    kf = kbeg + st * KC64 + tk;
#pragma unroll
    for (int t = 0; t < PER; ++t) fold_load(src[t], kf, kend, n, pa[t], pb[t]);
  };
  auto stash = [&](int st) {
    double *xs = xs0 + (st & 1) * TN_ * LDT;
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      bool b = false;
      xs[(tc0 + CSTEP * t) * LDT + tk] = fold_combine(pa[t], pb[t], kf, n, ft.par, b);
      if (b) bad |= 1u << t;
    }
  };

  // grid rows (1-based) of the lane's half-rows row0 + 16 HW wave + 16 h + li
  const int kk = lane >> 4;
  int jr[HW], step[HW], mm[HW];
#pragma unroll
  for (int h = 0; h < HW; ++h) {
    jr[h] = fold_row(row0 + wave * 16 * HW + 16 * h + (lane & 15), ft);
    step[h] = (int)((4LL * jr[h]) % twoN);
    mm[h] = (int)(((long long)jr[h] * (kbeg + kk + 1)) % twoN);
  }
  d4 acc[HW][NB], part[HW][NB];
#pragma unroll
  for (int h = 0; h < HW; ++h)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[h][b] = part[h][b] = (d4){0, 0, 0, 0};

  fetch(0);
  __syncthreads();                                // table in LDS
  stash(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int k0 = kbeg + st * KC64;
    if (st > 0 && (k0 % kchunk) == 0) {           // a new K chunk starts
#pragma unroll
      for (int h = 0; h < HW; ++h)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          acc[h][b] += part[h][b];
          part[h][b] = (d4){0, 0, 0, 0};
        }
    }
    if (st + 1 < nst) fetch(st + 1);
    const double *xs = xs0 + (st & 1) * TN_ * LDT;
    const int kcn = min(KC64, kend - k0);
    // software pipelined: the operands of step kc + 4 are read from LDS
    // while the MFMAs of step kc run
    double av[HW], bv[NB];
#pragma unroll
    for (int h = 0; h < HW; ++h) {
      av[h] = sine_lookup(tab, mm[h], N);
      mm[h] += step[h];
      if (mm[h] >= twoN) mm[h] -= twoN;
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) bv[b] = xs[(b * 16 + (lane & 15)) * LDT + kk];
    for (int kc = 0; kc < kcn; kc += 4) {
      double na[HW], nb[NB];
#pragma unroll
      for (int h = 0; h < HW; ++h) na[h] = 0.0;
#pragma unroll
      for (int b = 0; b < NB; ++b) nb[b] = 0.0;
      if (kc + 4 < kcn) {
#pragma unroll
        for (int h = 0; h < HW; ++h) {
          na[h] = sine_lookup(tab, mm[h], N);
          mm[h] += step[h];
          if (mm[h] >= twoN) mm[h] -= twoN;
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) nb[b] = xs[(b * 16 + (lane & 15)) * LDT + kc + 4 + kk];
      }
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int h = 0; h < HW; ++h)
          part[h][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[h], bv[b], part[h][b], 0, 0, 0);
#pragma unroll
      for (int h = 0; h < HW; ++h) av[h] = na[h];
#pragma unroll
      for (int b = 0; b < NB; ++b) bv[b] = nb[b];
    }
    if (st + 1 < nst) stash(st + 1);
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < PER; ++t)
    if (((bad >> t) & 1u) && sidx[t] >= 0) solves[sidx[t]].nonfinite = 1;
#pragma unroll
  for (int h = 0; h < HW; ++h)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[h][b] += part[h][b];
  // f64 layout: D[i][jj] at lane jj + 16 (i % 4), register i / 4
#pragma unroll
  for (int h = 0; h < HW; ++h)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = row0 + wave * 16 * HW + h * 16 + (lane >> 4) + 4 * r;
        const int col = c0 + b * 16 + (lane & 15);
        store_out(acc[h][b][r], a, col, ft, ncols, cols, partial, blockIdx.z);
      }
}

// ------------------------------------------------------------------ FP32
// Same tiling as the float64 kernel (HW 16-row blocks per wave) with float32
// operands; the MFMA sums run in float32 over 32-deep K runs that are
// flushed into float64 chunk sums.
constexpr int F32_RUN = 32;   // K depth accumulated in float32
constexpr int LDT32 = KC64 + 1;

template <int TN_, int HW = 2>
__global__ __launch_bounds__(512 / HW) void k_dst_f32(
    int n, int Q, const float *__restrict__ qtab,
    const DstCol *__restrict__ cols, int ncols, int kchunk,
    double *__restrict__ partial, Solve2D *solves) {
  constexpr int NT = 512 / HW;
  constexpr int NB = TN_ / 16;
  constexpr int PER = KC64 * TN_ / NT;
  constexpr int CSTEP = NT / KC64;
  extern __shared__ __align__(16) unsigned char smem[];
  const int Qp = (Q + 3) & ~3;
  float *tab = (float *)smem;
  float *xs0 = tab + Qp;                          // [TN][LDT32] x 2 buffers
  const int N = n + 1, twoN = 2 * N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  FoldTile ft;
  if (!fold_tile(n, ncols, TM64, TN_, true, ft)) return;
  const int row0 = ft.row0, c0 = ft.c0;
  int cb, ce;
  chunk_range(ft.H0, kchunk, cb, ce);
  // table copy, eight loads in flight per thread
  for (int i0 = 0; i0 < Q; i0 += 8 * NT) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * NT + tid;
      v[u] = (i < Q) ? qtab[i] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * NT + tid;
      if (i < Q) tab[i] = v[u];
    }
  }

  const int tk = tid & (KC64 - 1), tc0 = tid / KC64;
  const double *src[PER];
  int sidx[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int c = c0 + tc0 + CSTEP * t;
    src[t] = nullptr;
    sidx[t] = -1;
    if (c < ncols) {
      const DstCol dc = cols[c];
      src[t] = dc.src;
      sidx[t] = dc.solve;
    }
  }
  const int kbeg = cb * kchunk, kend = min(ft.Kp, ce * kchunk);
  const int nst = (kend - kbeg + KC64 - 1) / KC64;
  double pa[PER], pb[PER];
  unsigned bad = 0;
  int kf = 0;
  auto fetch = [&](int st) {
    kf = kbeg + st * KC64 + tk;
#pragma unroll
    for (int t = 0; t < PER; ++t) fold_load(src[t], kf, kend, n, pa[t], pb[t]);
  };
  auto stash = [&](int st) {
    float *xs = xs0 + (st & 1) * TN_ * LDT32;
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      bool b = false;
      xs[(tc0 + CSTEP * t) * LDT32 + tk] = (float)fold_combine(pa[t], pb[t], kf, n, ft.par, b);
      if (b) bad |= 1u << t;
    }
  };

  const int kk = lane >> 4;
  int jr[HW], step[HW], mm[HW];
#pragma unroll
  for (int h = 0; h < HW; ++h) {
    jr[h] = fold_row(row0 + wave * 16 * HW + 16 * h + (lane & 15), ft);
    step[h] = (int)((4LL * jr[h]) % twoN);
    mm[h] = (int)(((long long)jr[h] * (kbeg + kk + 1)) % twoN);
  }
  f4 run[HW][NB];
  double acc[HW][NB][4], part[HW][NB][4];
#pragma unroll
  for (int h = 0; h < HW; ++h)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      run[h][b] = (f4){0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[h][b][r] = part[h][b][r] = 0.0;
    }

  fetch(0);
  __syncthreads();
  stash(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int k0 = kbeg + st * KC64;
    if (st > 0 && (k0 % kchunk) == 0) {
#pragma unroll
      for (int h = 0; h < HW; ++h)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            acc[h][b][r] += part[h][b][r];
            part[h][b][r] = 0.0;
          }
    }
    if (st + 1 < nst) fetch(st + 1);
    const float *xs = xs0 + (st & 1) * TN_ * LDT32;
    const int kcn = min(KC64, kend - k0);
    float av[HW], bv[NB];
#pragma unroll
    for (int h = 0; h < HW; ++h) {
      av[h] = sine_lookup(tab, mm[h], N);
      mm[h] += step[h];
      if (mm[h] >= twoN) mm[h] -= twoN;
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) bv[b] = xs[(b * 16 + (lane & 15)) * LDT32 + kk];
    for (int kc = 0; kc < kcn; kc += 4) {
      float na[HW], nb[NB];
#pragma unroll
      for (int h = 0; h < HW; ++h) na[h] = 0.f;
#pragma unroll
      for (int b = 0; b < NB; ++b) nb[b] = 0.f;
      if (kc + 4 < kcn) {
#pragma unroll
        for (int h = 0; h < HW; ++h) {
          na[h] = sine_lookup(tab, mm[h], N);
          mm[h] += step[h];
          if (mm[h] >= twoN) mm[h] -= twoN;
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) nb[b] = xs[(b * 16 + (lane & 15)) * LDT32 + kc + 4 + kk];
      }
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int h = 0; h < HW; ++h)
          run[h][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[h], bv[b], run[h][b], 0, 0, 0);
#pragma unroll
      for (int h = 0; h < HW; ++h) av[h] = na[h];
#pragma unroll
      for (int b = 0; b < NB; ++b) bv[b] = nb[b];
    }
    // a stage is one 32-deep float32 run
#pragma unroll
    for (int h = 0; h < HW; ++h)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) part[h][b][r] += (double)run[h][b][r];
        run[h][b] = (f4){0, 0, 0, 0};
      }
    if (st + 1 < nst) stash(st + 1);
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < PER; ++t)
    if (((bad >> t) & 1u) && sidx[t] >= 0) solves[sidx[t]].nonfinite = 1;
  // f32 layout: D[i][jj] at lane jj + 16 (i / 4), register i % 4
#pragma unroll
  for (int h = 0; h < HW; ++h)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = row0 + wave * 16 * HW + h * 16 + 4 * (lane >> 4) + r;
        const int col = c0 + b * 16 + (lane & 15);
        store_out(acc[h][b][r] + part[h][b][r], a, col, ft, ncols, cols, partial,
                  blockIdx.z);
      }
}

// ------------------------------------------------------- BF16x3 / BF16x6
// P = 2: table entries are packed (hi | lo << 16) bfloat16 splits of the
// sine and both operands are split in two: three products hi*hi + hi*lo +
// lo*hi.  P = 3: entries (hi | mid << 16, lo) and three pieces per operand,
// each the bfloat16 rounding of what the previous ones leave: the six
// products of piece levels a + b <= 2 (about 24 bits of each operand, the
// dropped products below 2^-24 relative), accumulated smallest first.
// 64 rows (4 waves x 16) x TN columns per workgroup; the folded sources of
// the next 64-deep K stage are loaded into registers while the MFMAs run on
// the current one, then split and stashed in the other LDS buffer.  A stage
// is one float32 run, added into the float64 chunk sum.
template <int P>
__global__ __launch_bounds__(NTHR) void k_dst_bf16s(
    int n, int Q, const uint32_t *__restrict__ qtab,
    const DstCol *__restrict__ cols, int ncols, int kchunk,
    double *__restrict__ partial, Solve2D *solves) {
  constexpr int PER = KC * TN / NTHR;            // tile values per thread
  constexpr int NB = TN / 16;
  constexpr int TW = P == 2 ? 1 : 2;             // table words per entry
  extern __shared__ __align__(16) unsigned char smem[];
  const int Qp = (Q + 3) & ~3;
  uint32_t *tab = (uint32_t *)smem;
  uint16_t *xb0 = (uint16_t *)(tab + TW * Qp);  // [piece][TN][KC] x 2 buffers
  const int N = n + 1, twoN = 2 * N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  FoldTile ft;
  if (!fold_tile(n, ncols, TM, TN, true, ft)) return;
  const int row0 = ft.row0, c0 = ft.c0;
  int cb, ce;
  chunk_range(ft.H0, kchunk, cb, ce);
  for (int i = tid; i < TW * Q; i += NTHR) tab[i] = qtab[i];

  // this thread stages point k0 + lane of columns wave + 4 t
  const double *src[PER];
  int sidx[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int c = c0 + wave + 4 * t;
    src[t] = nullptr;
    sidx[t] = -1;
    if (c < ncols) {
      const DstCol dc = cols[c];
      src[t] = dc.src;
      sidx[t] = dc.solve;
    }
  }
  const int kbeg = cb * kchunk, kend = min(ft.Kp, ce * kchunk);
  const int nst = (kend - kbeg + KC - 1) / KC;
  double pa[PER], pb[PER];
  unsigned bad = 0;
  int kf = 0;
  auto fetch = [&](int st) {
    kf = kbeg + st * KC + lane;
#pragma unroll
    for (int t = 0; t < PER; ++t) fold_load(src[t], kf, kend, n, pa[t], pb[t]);
  };
  auto stash = [&](int st) {
    uint16_t *xs = xb0 + (st & 1) * P * TN * KC;
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      bool b = false;
      double v = fold_combine(pa[t], pb[t], kf, n, ft.par, b);
      if (b) bad |= 1u << t;
      const int c = wave + 4 * t;
#pragma unroll
      for (int pc = 0; pc < P; ++pc) {
        const uint32_t h = bf16_bits_rne((float)v);
        xs[pc * TN * KC + c * KC + lane] = (uint16_t)h;
        v -= (double)bf16_to_float(h);
      }
    }
  };

  const int j = fold_row(row0 + wave * 16 + (lane & 15), ft);   // 1-based grid row
  const int kq = lane >> 4;                      // k offset 8*kq .. 8*kq+7
  const int jm = j % twoN;
  const int step = (int)((32LL * j) % twoN);
  // m for the lane's first point k = kbeg + 8 kq (1-based k + 1); advances
  // by 32 j per 32-deep MFMA step
  int m = (int)(((long long)j * (kbeg + 8 * kq + 1)) % twoN);
  double acc[NB][4], part[NB][4];
  f4 run[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    run[b] = (f4){0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[b][r] = part[b][r] = 0.0;
  }
  fetch(0);
  __syncthreads();                               // table in LDS
  stash(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int k0 = kbeg + st * KC;
    if (st > 0 && (k0 % kchunk) == 0) {          // a new K chunk starts
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          acc[b][r] += part[b][r];
          part[b][r] = 0.0;
        }
    }
    if (st + 1 < nst) fetch(st + 1);
    const uint16_t *xs = xb0 + (st & 1) * P * TN * KC;
    const int kcn = min(KC, kend - k0);
    for (int kc = 0; kc < kcn; kc += 32) {
      bf8 a[P];
      int mm = m;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        int q = mm;
        bool neg = false;
        if (q >= N) {
          q -= N;
          neg = true;
        }
        if (2 * q > N) q = N - q;
        uint32_t p = tab[TW * q];
        if (neg) p ^= 0x80008000u;               // negate both halves
        a[0][e] = __builtin_bit_cast(__bf16, (uint16_t)(p & 0xFFFFu));
        a[1][e] = __builtin_bit_cast(__bf16, (uint16_t)(p >> 16));
        if constexpr (P == 3) {
          uint32_t p2 = tab[TW * q + 1];
          if (neg) p2 ^= 0x8000u;
          a[2][e] = __builtin_bit_cast(__bf16, (uint16_t)(p2 & 0xFFFFu));
        }
        mm += jm;
        if (mm >= twoN) mm -= twoN;
      }
      m += step;
      if (m >= twoN) m -= twoN;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int c = b * 16 + (lane & 15);
        bf8 x[P];
#pragma unroll
        for (int pc = 0; pc < P; ++pc) x[pc] = *(const bf8 *)(xs + pc * TN * KC + c * KC + kc + 8 * kq);
        if constexpr (P == 3) {
          run[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[2], x[0], run[b], 0, 0, 0);
          run[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], x[1], run[b], 0, 0, 0);
          run[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], x[2], run[b], 0, 0, 0);
        }
        run[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], x[0], run[b], 0, 0, 0);
        run[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], x[1], run[b], 0, 0, 0);
        run[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], x[0], run[b], 0, 0, 0);
      }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int r = 0; r < 4; ++r) part[b][r] += (double)run[b][r];
      run[b] = (f4){0, 0, 0, 0};
    }
    if (st + 1 < nst) stash(st + 1);
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < PER; ++t)
    if (((bad >> t) & 1u) && sidx[t] >= 0) solves[sidx[t]].nonfinite = 1;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = row0 + wave * 16 + 4 * (lane >> 4) + r;
      const int col = c0 + b * 16 + (lane & 15);
      store_out(acc[b][r] + part[b][r], a, col, ft, ncols, cols, partial, blockIdx.z);
    }
}

// Fixed-order sum of the split-K partial results.
__global__ void k_dst_reduce(int n, int ncols, int nz,
                             const double *__restrict__ partial,
                             const DstCol *__restrict__ cols) {
  const int col = blockIdx.y;
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n || col >= ncols) return;
  const int H0 = (n + 1) / 2, par = row & 1, a = row >> 1;
  double s = 0.0;
  for (int z = 0; z < nz; ++z) s += partial[((size_t)z * 2 * ncols + 2 * col + par) * H0 + a];
  cols[col].dst[row] = s;
}

int quarter_len(int n) { return (n + 1) / 2 + 1; }

}  // namespace

size_t dst_partial_elems(int n, int ncols) {
  // room for a split of the folded K into up to 4 chunks: one float64 per
  // output and chunk, or six int32 level sums (int8)
  return (size_t)16 * (size_t)ncols * (size_t)n;
}

hipError_t launch_dst(int prec, int n, const void *tab, const DstCol *cols,
                      int ncols, Solve2D *solves, double *partial,
                      size_t partial_elems, void *work, size_t work_bytes,
                      hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (ncols <= 0) return hipSuccess;
  const int Q = quarter_len(n);
  const char *base = (const char *)tab;
  const int Qp8 = (Q + 1) & ~1, Qp4 = (Q + 3) & ~3;
  const TabLayout TL = tab_layout(n);
  if (prec == LRP_PREC_INT8)
    return launch_dst_i8(n, base + TL.i8, (DstCol *)cols, ncols, solves, partial,
                         partial_elems, work, work_bytes, st, ev0, ev1);
  if (prec == LRP_PREC_FFT64)
    return launch_dst_fft(n, base + TL.fft, cols, ncols, solves, st, ev0, ev1);
  const double *t64 = (const double *)base;
  const float *t32 = (const float *)(base + TL.f32);
  const uint32_t *tbf = (const uint32_t *)(base + (prec == LRP_PREC_BF16X6 ? TL.bf3 : TL.bf2));
  // folded length, and fixed K chunks of it that depend on n only (at most
  // 4, at least 256 deep, a multiple of every kernel's K stage)
  const int H0 = (n + 1) / 2;
  const int kchunk = std::max(256, ceil_div(ceil_div(H0, 4), KC) * KC);
  const int nchunk = ceil_div(H0, kchunk);
  // tiles of the chosen kernel; one workgroup per K chunk when the tiles
  // alone leave the 256 CUs under-filled
  const bool wide = ncols > 32;
  int tm, tn;
  if (prec == LRP_PREC_BF16X3 || prec == LRP_PREC_BF16X6) {
    tm = TM;
    tn = TN;
  } else {
    tm = TM64;
    tn = wide ? 64 : 32;
  }
  const int R = ceil_div(H0, tm), C = 2 * ceil_div(ncols, tn);
  int split = (R * C < 512) ? nchunk : 1;
  if (partial == nullptr || partial_elems < (size_t)split * 2 * ncols * H0) split = 1;
  double *out_partial = split > 1 ? partial : nullptr;
  const dim3 block(NTHR);
  size_t lds = 0;
  hipError_t e = hipSuccess;
  if (prec == LRP_PREC_FP64) {
    const dim3 g(tile_grid(R, C, true), 1, split);
    lds = (size_t)Qp8 * 8 + (size_t)2 * tn * LDT * 8;
    // 64-column tiles as eight waves of 16 rows (two waves per SIMD)
    const void *fn = wide ? (const void *)k_dst_f64<64, 1> : (const void *)k_dst_f64<32, 2>;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    if (wide)
      hipLaunchKernelGGL((k_dst_f64<64, 1>), g, dim3(512), lds, st, n, Q, t64, cols, ncols,
                         kchunk, out_partial, solves);
    else
      hipLaunchKernelGGL((k_dst_f64<32, 2>), g, dim3(256), lds, st, n, Q, t64, cols, ncols,
                         kchunk, out_partial, solves);
  } else if (prec == LRP_PREC_FP32) {
    const dim3 g(tile_grid(R, C, true), 1, split);
    lds = (size_t)Qp4 * 4 + (size_t)2 * tn * LDT32 * 4;
    const void *fn = wide ? (const void *)k_dst_f32<64, 1> : (const void *)k_dst_f32<32, 2>;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    if (wide)
      hipLaunchKernelGGL((k_dst_f32<64, 1>), g, dim3(512), lds, st, n, Q, t32, cols, ncols,
                         kchunk, out_partial, solves);
    else
      hipLaunchKernelGGL((k_dst_f32<32, 2>), g, dim3(256), lds, st, n, Q, t32, cols, ncols,
                         kchunk, out_partial, solves);
  } else if (prec == LRP_PREC_BF16X3) {
    const dim3 g(tile_grid(R, C, true), 1, split);
    lds = (size_t)Qp4 * 4 + (size_t)2 * 2 * KC * TN * 2;
    e = hipFuncSetAttribute((const void *)k_dst_bf16s<2>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_dst_bf16s<2>, g, block, lds, st, n, Q, tbf, cols,
                       ncols, kchunk, out_partial, solves);
  } else {
    const dim3 g(tile_grid(R, C, true), 1, split);
    lds = (size_t)Qp4 * 8 + (size_t)2 * 3 * KC * TN * 2;
    e = hipFuncSetAttribute((const void *)k_dst_bf16s<3>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_dst_bf16s<3>, g, block, lds, st, n, Q, tbf, cols,
                       ncols, kchunk, out_partial, solves);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev1 && (e = hipEventRecord(ev1, st)) != hipSuccess) return e;
  if (split == 1) return e;
  dim3 rg(ceil_div(n, 256), ncols);
  hipLaunchKernelGGL(k_dst_reduce, rg, dim3(256), 0, st, n, ncols, split,
                     (const double *)partial, cols);
  return hipGetLastError();
}

}  // namespace lrp
