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
__global__ __launch_bounds__(NTHR) void k_dst_f64(
    int n, int Q, const double *__restrict__ qtab,
    const DstCol *__restrict__ cols, int ncols, int kchunk,
    double *__restrict__ partial, Solve2D *solves) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int Qp = (Q + 1) & ~1;
  double *tab = (double *)smem;
  double *xs = tab + Qp;                         // [KC][TN]
  const int N = n + 1, twoN = 2 * N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row0 = blockIdx.x * TM, c0 = blockIdx.y * TN;
  int cb, ce;
  chunk_range(n, kchunk, cb, ce);
  for (int i = tid; i < Q; i += NTHR) tab[i] = qtab[i];

  const int j = row0 + wave * 16 + (lane & 15);  // S row j+1
  const int kk = lane >> 4;
  const int step = (int)((4LL * (j + 1)) % twoN);
  d4 acc[TN / 16];
#pragma unroll
  for (int b = 0; b < TN / 16; ++b) acc[b] = (d4){0, 0, 0, 0};

  for (int ch = cb; ch < ce; ++ch) {
    const int kb = ch * kchunk, ke = min(n, kb + kchunk);
    int m = (int)(((long long)(j + 1) * (kb + kk + 1)) % twoN);
    d4 part[TN / 16];
#pragma unroll
    for (int b = 0; b < TN / 16; ++b) part[b] = (d4){0, 0, 0, 0};
    for (int k0 = kb; k0 < ke; k0 += KC) {
      __syncthreads();
      load_tile(cols, ncols, c0, k0, ke, solves,
                [&](int kc, int c, double v) { xs[kc * TN + c] = v; });
      __syncthreads();
      const int kcn = min(KC, ke - k0);
      for (int kc = 0; kc < kcn; kc += 4) {
        const double a = sine_lookup(tab, m, N);
        m += step;
        if (m >= twoN) m -= twoN;
#pragma unroll
        for (int b = 0; b < TN / 16; ++b) {
          const double bv = xs[(kc + kk) * TN + b * 16 + (lane & 15)];
          part[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, part[b], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int b = 0; b < TN / 16; ++b) acc[b] += part[b];
  }
  // f64 layout: D[i][jj] at lane jj + 16 (i % 4), register i / 4
#pragma unroll
  for (int b = 0; b < TN / 16; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = row0 + wave * 16 + (lane >> 4) + 4 * r;
      const int col = c0 + b * 16 + (lane & 15);
      store_out(acc[b][r], row, col, n, ncols, cols, partial, blockIdx.z);
    }
}

// ------------------------------------------------------------------ FP32
constexpr int F32_RUN = 32;   // K depth accumulated in float32

__global__ __launch_bounds__(NTHR) void k_dst_f32(
    int n, int Q, const float *__restrict__ qtab,
    const DstCol *__restrict__ cols, int ncols, int kchunk,
    double *__restrict__ partial, Solve2D *solves) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int Qp = (Q + 3) & ~3;
  float *tab = (float *)smem;
  float *xs = tab + Qp;                          // [KC][TN]
  const int N = n + 1, twoN = 2 * N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row0 = blockIdx.x * TM, c0 = blockIdx.y * TN;
  int cb, ce;
  chunk_range(n, kchunk, cb, ce);
  for (int i = tid; i < Q; i += NTHR) tab[i] = qtab[i];

  const int j = row0 + wave * 16 + (lane & 15);
  const int kk = lane >> 4;
  const int step = (int)((4LL * (j + 1)) % twoN);
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
  int m = (int)(((long long)(j + 1) * (kb + kk + 1)) % twoN);
#pragma unroll
  for (int b = 0; b < TN / 16; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) part[b][r] = 0.0;
  for (int k0 = kb; k0 < ke; k0 += KC) {
    __syncthreads();
    load_tile(cols, ncols, c0, k0, ke, solves,
              [&](int kc, int c, double v) { xs[kc * TN + c] = (float)v; });
    __syncthreads();
    const int kcn = min(KC, ke - k0);
    for (int kc = 0; kc < kcn; kc += 4) {
      const float a = sine_lookup(tab, m, N);
      m += step;
      if (m >= twoN) m -= twoN;
#pragma unroll
      for (int b = 0; b < TN / 16; ++b) {
        const float bv = xs[(kc + kk) * TN + b * 16 + (lane & 15)];
        run[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, run[b], 0, 0, 0);
      }
      if (((kc + 4) % F32_RUN) == 0 || kc + 4 >= kcn) {
#pragma unroll
        for (int b = 0; b < TN / 16; ++b) {
#pragma unroll
          for (int r = 0; r < 4; ++r) part[b][r] += (double)run[b][r];
          run[b] = (f4){0, 0, 0, 0};
        }
      }
    }
  }
#pragma unroll
  for (int b = 0; b < TN / 16; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[b][r] += part[b][r];
  }
  // f32 layout: D[i][jj] at lane jj + 16 (i / 4), register i % 4
#pragma unroll
  for (int b = 0; b < TN / 16; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = row0 + wave * 16 + 4 * (lane >> 4) + r;
      const int col = c0 + b * 16 + (lane & 15);
      store_out(acc[b][r], row, col, n, ncols, cols, partial, blockIdx.z);
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
  const int row0 = blockIdx.x * TM, c0 = blockIdx.y * TN;
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
                      size_t partial_elems, hipStream_t st) {
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
  dim3 grid(gx, gy, split), block(NTHR);
  size_t lds = 0;
  hipError_t e = hipSuccess;
  const char *base = (const char *)tab;
  const int Qp8 = (Q + 1) & ~1, Qp4 = (Q + 3) & ~3;
  // table layout: [f64 x Qp8][f32 x Qp4][u32 x Qp4]
  const double *t64 = (const double *)base;
  const float *t32 = (const float *)(base + (size_t)Qp8 * 8);
  const uint32_t *tbf = (const uint32_t *)(base + (size_t)Qp8 * 8 + (size_t)Qp4 * 4);
  if (prec == LRP_PREC_FP64) {
    lds = (size_t)Qp8 * 8 + (size_t)KC * TN * 8;
    e = hipFuncSetAttribute((const void *)k_dst_f64,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dst_f64, grid, block, lds, st, n, Q, t64, cols, ncols,
                       kchunk, out_partial, solves);
  } else if (prec == LRP_PREC_FP32) {
    lds = (size_t)Qp4 * 4 + (size_t)KC * TN * 4;
    e = hipFuncSetAttribute((const void *)k_dst_f32,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dst_f32, grid, block, lds, st, n, Q, t32, cols, ncols,
                       kchunk, out_partial, solves);
  } else {
    lds = (size_t)Qp4 * 4 + (size_t)KC * TN * 2 * 2;
    e = hipFuncSetAttribute((const void *)k_dst_bf16x3,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dst_bf16x3, grid, block, lds, st, n, Q, tbf, cols,
                       ncols, kchunk, out_partial, solves);
  }
  e = hipGetLastError();
  if (e != hipSuccess || split == 1) return e;
  dim3 rg(ceil_div(n, 256), ncols);
  hipLaunchKernelGGL(k_dst_reduce, rg, dim3(256), 0, st, n, ncols, split,
                     (const double *)partial, cols);
  return hipGetLastError();
}

}  // namespace lrp
