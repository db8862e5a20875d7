// Sine transform of factor columns as an MFMA GEMM: dst = S * src, where
// S[j,k] = sqrt(2/(n+1)) sin(pi j k/(n+1)), j, k = 1..n, the orthonormal
// DST-I that diagonalises the 1D operator (paper Section 4.1, eq. "diag";
// "the DST of the factors", Section 4.1).  S is never stored: every wave
// generates its 16 x K tile on the fly from a quarter-wave table in LDS with
// exact integer argument reduction m = j k mod 2(n+1).
//
// One launch covers any set of columns with the same n (all columns of all
// solves of a batch), tiled 64 rows x 32 columns per workgroup; K is split
// across workgroups when the tile count alone cannot fill the chip, with a
// deterministic fixed-order reduction.
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

// Stage the K x TN tile of the sources in LDS (transposed to [k][c]).
// Values past the end of K or past the last column are zero.
template <typename F>
__device__ __forceinline__ void load_tile(const DstCol *__restrict__ cols,
                                          int ncols, int c0, int k0, int ke,
                                          Solve2D *solves, F store) {
  for (int idx = threadIdx.x; idx < KC * TN; idx += NTHR) {
    const int c = idx / KC, kc = idx - c * KC;
    const int k = k0 + kc;
    double v = 0.0;
    if (k < ke && c0 + c < ncols) {
      const DstCol dc = cols[c0 + c];
      v = dc.src[k];
      if (!isfinite(v) && dc.solve >= 0) solves[dc.solve].nonfinite = 1;
    }
    store(kc, c, v);
  }
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

// Write a 16x16 block held in MFMA layout.  rowOf(reg) gives the row offset.
__device__ __forceinline__ void store_out(double v, int row, int col, int n,
                                          int ncols, const DstCol *cols,
                                          double *partial, int z) {
  if (row < n && col < ncols) {
    if (partial)
      partial[((size_t)z * ncols + col) * n + row] = v;
    else
      cols[col].dst[row] = v;
  }
}

// ------------------------------------------------------------------ FP64
// 128 rows (4 waves x 32) x TN columns per workgroup.  The source tile is
// staged in LDS as [column][k] with one double of padding per column (the
// 16 lanes that read one k for 16 columns then hit distinct banks), double
// buffered: the next K stage is fetched into registers while the MFMAs run on
// the current one.
constexpr int TM64 = 128;
constexpr int KC64 = 32;
constexpr int LDT = KC64 + 1;

template <int TN_>
__global__ __launch_bounds__(NTHR) void k_dst_f64(
    int n, int Q, const double *__restrict__ qtab,
    const DstCol *__restrict__ cols, int ncols, int kchunk,
    double *__restrict__ partial, Solve2D *solves) {
  constexpr int NB = TN_ / 16;                    // column blocks per wave
  constexpr int PER = KC64 * TN_ / NTHR;          // tile values per thread
  extern __shared__ __align__(16) unsigned char smem[];
  const int Qp = (Q + 1) & ~1;
  double *tab = (double *)smem;
  double *xs0 = tab + Qp;                         // [TN][LDT] x 2 buffers
  const int N = n + 1, twoN = 2 * N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int rt, ct;
  if (!tile_of(ceil_div(n, TM64), ceil_div(ncols, TN_), false, rt, ct)) return;
  const int row0 = rt * TM64, c0 = ct * TN_;
  int cb, ce;
  chunk_range(n, kchunk, cb, ce);
  for (int i = tid; i < Q; i += NTHR) tab[i] = qtab[i];

  // this thread's share of a K stage: k offset tk (32 lanes read 32
  // consecutive k of one column), columns tc0 + 8 t
  const int tk = tid & 31, tc0 = tid >> 5;
  const double *src[PER];
  int sidx[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int c = c0 + tc0 + 8 * t;
    src[t] = nullptr;
    sidx[t] = -1;
    if (c < ncols) {
      const DstCol dc = cols[c];
      src[t] = dc.src;
      sidx[t] = dc.solve;
    }
  }
  const int kbeg = cb * kchunk, kend = min(n, ce * kchunk);
  const int nst = (kend - kbeg + KC64 - 1) / KC64;
  double pre[PER];
  unsigned bad = 0;
  auto fetch = [&](int st) {
    const int k = kbeg + st * KC64 + tk;
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      double v = 0.0;
      if (src[t] && k < kend) {
        v = src[t][k];
        if (!isfinite(v)) bad |= 1u << t;
      }
      pre[t] = v;
    }
  };
  auto stash = [&](int st) {
    double *xs = xs0 + (st & 1) * TN_ * LDT;
#pragma unroll
    for (int t = 0; t < PER; ++t) xs[(tc0 + 8 * t) * LDT + tk] = pre[t];
  };

  const int jA = row0 + wave * 32 + (lane & 15);  // S rows jA+1, jA+17
  const int jB = jA + 16;
  const int kk = lane >> 4;
  const int stepA = (int)((4LL * (jA + 1)) % twoN);
  const int stepB = (int)((4LL * (jB + 1)) % twoN);
  int mA = (int)(((long long)(jA + 1) * (kbeg + kk + 1)) % twoN);
  int mB = (int)(((long long)(jB + 1) * (kbeg + kk + 1)) % twoN);
  d4 acc[2][NB], part[2][NB];
#pragma unroll
  for (int h = 0; h < 2; ++h)
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
      for (int h = 0; h < 2; ++h)
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
    double aA = sine_lookup(tab, mA, N), aB = sine_lookup(tab, mB, N), bv[NB];
    mA += stepA;
    if (mA >= twoN) mA -= twoN;
    mB += stepB;
    if (mB >= twoN) mB -= twoN;
#pragma unroll
    for (int b = 0; b < NB; ++b) bv[b] = xs[(b * 16 + (lane & 15)) * LDT + kk];
    for (int kc = 0; kc < kcn; kc += 4) {
      double nA = 0.0, nB = 0.0, nb[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) nb[b] = 0.0;
      if (kc + 4 < kcn) {
        nA = sine_lookup(tab, mA, N);
        nB = sine_lookup(tab, mB, N);
        mA += stepA;
        if (mA >= twoN) mA -= twoN;
        mB += stepB;
        if (mB >= twoN) mB -= twoN;
#pragma unroll
        for (int b = 0; b < NB; ++b) nb[b] = xs[(b * 16 + (lane & 15)) * LDT + kc + 4 + kk];
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        part[0][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aA, bv[b], part[0][b], 0, 0, 0);
        part[1][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aB, bv[b], part[1][b], 0, 0, 0);
      }
      aA = nA;
      aB = nB;
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
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[h][b] += part[h][b];
  // f64 layout: D[i][jj] at lane jj + 16 (i % 4), register i / 4
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wave * 32 + h * 16 + (lane >> 4) + 4 * r;
        const int col = c0 + b * 16 + (lane & 15);
        store_out(acc[h][b][r], row, col, n, ncols, cols, partial, blockIdx.z);
      }
}

// ------------------------------------------------------------------ FP32
// Same tiling as the float64 kernel with float32 operands; the MFMA sums run
// in float32 over 32-deep K runs that are flushed into float64 chunk sums.
constexpr int F32_RUN = 32;   // K depth accumulated in float32
constexpr int LDT32 = KC64 + 1;

template <int TN_>
__global__ __launch_bounds__(NTHR) void k_dst_f32(
    int n, int Q, const float *__restrict__ qtab,
    const DstCol *__restrict__ cols, int ncols, int kchunk,
    double *__restrict__ partial, Solve2D *solves) {
  constexpr int NB = TN_ / 16;
  constexpr int PER = KC64 * TN_ / NTHR;
  extern __shared__ __align__(16) unsigned char smem[];
  const int Qp = (Q + 3) & ~3;
  float *tab = (float *)smem;
  float *xs0 = tab + Qp;                          // [TN][LDT32] x 2 buffers
  const int N = n + 1, twoN = 2 * N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int rt, ct;
  if (!tile_of(ceil_div(n, TM64), ceil_div(ncols, TN_), false, rt, ct)) return;
  const int row0 = rt * TM64, c0 = ct * TN_;
  int cb, ce;
  chunk_range(n, kchunk, cb, ce);
  for (int i = tid; i < Q; i += NTHR) tab[i] = qtab[i];

  const int tk = tid & 31, tc0 = tid >> 5;
  const double *src[PER];
  int sidx[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int c = c0 + tc0 + 8 * t;
    src[t] = nullptr;
    sidx[t] = -1;
    if (c < ncols) {
      const DstCol dc = cols[c];
      src[t] = dc.src;
      sidx[t] = dc.solve;
    }
  }
  const int kbeg = cb * kchunk, kend = min(n, ce * kchunk);
  const int nst = (kend - kbeg + KC64 - 1) / KC64;
  float pre[PER];
  unsigned bad = 0;
  auto fetch = [&](int st) {
    const int k = kbeg + st * KC64 + tk;
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      double v = 0.0;
      if (src[t] && k < kend) {
        v = src[t][k];
        if (!isfinite(v)) bad |= 1u << t;
      }
      pre[t] = (float)v;
    }
  };
  auto stash = [&](int st) {
    float *xs = xs0 + (st & 1) * TN_ * LDT32;
#pragma unroll
    for (int t = 0; t < PER; ++t) xs[(tc0 + 8 * t) * LDT32 + tk] = pre[t];
  };

  const int jA = row0 + wave * 32 + (lane & 15);
  const int jB = jA + 16;
  const int kk = lane >> 4;
  const int stepA = (int)((4LL * (jA + 1)) % twoN);
  const int stepB = (int)((4LL * (jB + 1)) % twoN);
  int mA = (int)(((long long)(jA + 1) * (kbeg + kk + 1)) % twoN);
  int mB = (int)(((long long)(jB + 1) * (kbeg + kk + 1)) % twoN);
  f4 run[2][NB];
  double acc[2][NB][4], part[2][NB][4];
#pragma unroll
  for (int h = 0; h < 2; ++h)
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
      for (int h = 0; h < 2; ++h)
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
    float aA = sine_lookup(tab, mA, N), aB = sine_lookup(tab, mB, N), bv[NB];
    mA += stepA;
    if (mA >= twoN) mA -= twoN;
    mB += stepB;
    if (mB >= twoN) mB -= twoN;
#pragma unroll
    for (int b = 0; b < NB; ++b) bv[b] = xs[(b * 16 + (lane & 15)) * LDT32 + kk];
    for (int kc = 0; kc < kcn; kc += 4) {
      float nA = 0.f, nB = 0.f, nb[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) nb[b] = 0.f;
      if (kc + 4 < kcn) {
        nA = sine_lookup(tab, mA, N);
        nB = sine_lookup(tab, mB, N);
        mA += stepA;
        if (mA >= twoN) mA -= twoN;
        mB += stepB;
        if (mB >= twoN) mB -= twoN;
#pragma unroll
        for (int b = 0; b < NB; ++b) nb[b] = xs[(b * 16 + (lane & 15)) * LDT32 + kc + 4 + kk];
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        run[0][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(aA, bv[b], run[0][b], 0, 0, 0);
        run[1][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(aB, bv[b], run[1][b], 0, 0, 0);
      }
      aA = nA;
      aB = nB;
#pragma unroll
      for (int b = 0; b < NB; ++b) bv[b] = nb[b];
    }
    // a stage is one 32-deep float32 run
#pragma unroll
    for (int h = 0; h < 2; ++h)
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
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wave * 32 + h * 16 + 4 * (lane >> 4) + r;
        const int col = c0 + b * 16 + (lane & 15);
        store_out(acc[h][b][r] + part[h][b][r], row, col, n, ncols, cols, partial,
                  blockIdx.z);
      }
}

// ---------------------------------------------------------------- BF16x3
// Table entries are packed (hi | lo << 16) bfloat16 splits of the sine.
__global__ __launch_bounds__(NTHR) void k_dst_bf16x3(
    int n, int Q, const uint32_t *__restrict__ qtab,
    const DstCol *__restrict__ cols, int ncols, int kchunk,
    double *__restrict__ partial, Solve2D *solves) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int Qp = (Q + 3) & ~3;
  uint32_t *tab = (uint32_t *)smem;
  uint16_t *xhi = (uint16_t *)(tab + Qp);        // [TN][KC]
  uint16_t *xlo = xhi + TN * KC;
  const int N = n + 1, twoN = 2 * N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int rt, ct;
  if (!tile_of(ceil_div(n, TM), ceil_div(ncols, TN), true, rt, ct)) return;
  const int row0 = rt * TM, c0 = ct * TN;
  int cb, ce;
  chunk_range(n, kchunk, cb, ce);
  for (int i = tid; i < Q; i += NTHR) tab[i] = qtab[i];

  const int j = row0 + wave * 16 + (lane & 15);
  const int kq = lane >> 4;                      // k offset 8*kq .. 8*kq+7
  const int jm = (j + 1) % twoN;
  const int step = (int)((32LL * (j + 1)) % twoN);
  double acc[TN / 16][4], part[TN / 16][4];
  f4 run[TN / 16];
#pragma unroll
  for (int b = 0; b < TN / 16; ++b) {
    run[b] = (f4){0, 0, 0, 0};
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[b][r] = 0.0;
  }
  for (int ch = cb; ch < ce; ++ch) {
  const int kb = ch * kchunk, ke = min(n, kb + kchunk);
  // m for k = kb + 8 kq (1-based k + 1); advances by 32 (j+1) per step
  int m = (int)(((long long)(j + 1) * (kb + 8 * kq + 1)) % twoN);
#pragma unroll
  for (int b = 0; b < TN / 16; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) part[b][r] = 0.0;
  for (int k0 = kb; k0 < ke; k0 += KC) {
    __syncthreads();
    load_tile(cols, ncols, c0, k0, ke, solves, [&](int kc, int c, double v) {
      const uint32_t h = bf16_bits_rne((float)v);
      const uint32_t l = bf16_bits_rne((float)(v - (double)bf16_to_float(h)));
      xhi[c * KC + kc] = (uint16_t)h;
      xlo[c * KC + kc] = (uint16_t)l;
    });
    __syncthreads();
    const int kcn = min(KC, ke - k0);
    for (int kc = 0; kc < kcn; kc += 32) {
      bf8 ah, al;
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
        uint32_t p = tab[q];
        if (neg) p ^= 0x80008000u;               // negate both halves
        ah[e] = __builtin_bit_cast(__bf16, (uint16_t)(p & 0xFFFFu));
        al[e] = __builtin_bit_cast(__bf16, (uint16_t)(p >> 16));
        mm += jm;
        if (mm >= twoN) mm -= twoN;
      }
      m += step;
      if (m >= twoN) m -= twoN;
#pragma unroll
      for (int b = 0; b < TN / 16; ++b) {
        const int c = b * 16 + (lane & 15);
        const bf8 bh = *(const bf8 *)(xhi + c * KC + kc + 8 * kq);
        const bf8 bl = *(const bf8 *)(xlo + c * KC + kc + 8 * kq);
        run[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, run[b], 0, 0, 0);
        run[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, run[b], 0, 0, 0);
        run[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, run[b], 0, 0, 0);
      }
    }
#pragma unroll
    for (int b = 0; b < TN / 16; ++b) {
#pragma unroll
      for (int r = 0; r < 4; ++r) part[b][r] += (double)run[b][r];
      run[b] = (f4){0, 0, 0, 0};
    }
  }
#pragma unroll
  for (int b = 0; b < TN / 16; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[b][r] += part[b][r];
  }
#pragma unroll
  for (int b = 0; b < TN / 16; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = row0 + wave * 16 + 4 * (lane >> 4) + r;
      const int col = c0 + b * 16 + (lane & 15);
      store_out(acc[b][r], row, col, n, ncols, cols, partial, blockIdx.z);
    }
}

// Fixed-order sum of the split-K partial results.
__global__ void k_dst_reduce(int n, int ncols, int nz,
                             const double *__restrict__ partial,
                             const DstCol *__restrict__ cols) {
  const int col = blockIdx.y;
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n || col >= ncols) return;
  double s = 0.0;
  for (int z = 0; z < nz; ++z) s += partial[((size_t)z * ncols + col) * n + row];
  cols[col].dst[row] = s;
}

int quarter_len(int n) { return (n + 1) / 2 + 1; }

}  // namespace

size_t dst_partial_elems(int n, int ncols) {
  // room for a split of up to 8
  return (size_t)8 * (size_t)ncols * (size_t)n;
}

hipError_t launch_dst(int prec, int n, const void *tab, const DstCol *cols,
                      int ncols, Solve2D *solves, double *partial,
                      size_t partial_elems, void *work, size_t work_bytes,
                      hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (ncols <= 0) return hipSuccess;
  const int Q = quarter_len(n);
  const int gx = ceil_div(n, TM), gy = ceil_div(ncols, TN);
  // Fixed K chunks (at most 8, at least 256 deep); one workgroup per chunk
  // when the tiles alone leave the 256 CUs under-filled.
  const int kchunk = std::max(256, ceil_div(ceil_div(n, 8), KC) * KC);
  const int nchunk = ceil_div(n, kchunk);
  int split = (gx * gy < 512) ? nchunk : 1;
  if (partial == nullptr ||
      partial_elems < (size_t)split * (size_t)ncols * (size_t)n)
    split = 1;
  double *out_partial = split > 1 ? partial : nullptr;
  dim3 grid(tile_grid(gx, gy, true), 1, split), block(NTHR);
  size_t lds = 0;
  hipError_t e = hipSuccess;
  const char *base = (const char *)tab;
  const int Qp8 = (Q + 1) & ~1, Qp4 = (Q + 3) & ~3;
  // table layout: [f64 x Qp8][f32 x Qp4][u32 x Qp4][int8 records]
  if (prec == LRP_PREC_INT8)
    return launch_dst_i8(n, base + (size_t)Qp8 * 8 + (size_t)Qp4 * 8, (DstCol *)cols, ncols,
                         kchunk, solves, partial, partial_elems, work, work_bytes, st, ev0,
                         ev1);
  const double *t64 = (const double *)base;
  const float *t32 = (const float *)(base + (size_t)Qp8 * 8);
  const uint32_t *tbf = (const uint32_t *)(base + (size_t)Qp8 * 8 + (size_t)Qp4 * 4);
  if (prec == LRP_PREC_FP64) {
    const bool wide = ncols > 32;
    const int tn = wide ? 64 : 32;
    const int R64 = ceil_div(n, TM64), C64 = ceil_div(ncols, tn);
    dim3 g64(tile_grid(R64, C64, false), 1, grid.z);
    if (R64 * C64 >= 512) g64.z = 1;
    if (g64.z == 1) out_partial = nullptr;
    lds = (size_t)Qp8 * 8 + (size_t)2 * tn * LDT * 8;
    const void *fn = wide ? (const void *)k_dst_f64<64> : (const void *)k_dst_f64<32>;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    if (wide)
      hipLaunchKernelGGL(k_dst_f64<64>, g64, block, lds, st, n, Q, t64, cols, ncols,
                         kchunk, out_partial, solves);
    else
      hipLaunchKernelGGL(k_dst_f64<32>, g64, block, lds, st, n, Q, t64, cols, ncols,
                         kchunk, out_partial, solves);
    split = g64.z;
  } else if (prec == LRP_PREC_FP32) {
    const bool wide = ncols > 32;
    const int tn = wide ? 64 : 32;
    const int R32 = ceil_div(n, TM64), C32 = ceil_div(ncols, tn);
    dim3 g32(tile_grid(R32, C32, false), 1, grid.z);
    if (R32 * C32 >= 512) g32.z = 1;
    if (g32.z == 1) out_partial = nullptr;
    lds = (size_t)Qp4 * 4 + (size_t)2 * tn * LDT32 * 4;
    const void *fn = wide ? (const void *)k_dst_f32<64> : (const void *)k_dst_f32<32>;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    if (wide)
      hipLaunchKernelGGL(k_dst_f32<64>, g32, block, lds, st, n, Q, t32, cols, ncols,
                         kchunk, out_partial, solves);
    else
      hipLaunchKernelGGL(k_dst_f32<32>, g32, block, lds, st, n, Q, t32, cols, ncols,
                         kchunk, out_partial, solves);
    split = g32.z;
  } else {
    lds = (size_t)Qp4 * 4 + (size_t)KC * TN * 2 * 2;
    e = hipFuncSetAttribute((const void *)k_dst_bf16x3,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_dst_bf16x3, grid, block, lds, st, n, Q, tbf, cols,
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
