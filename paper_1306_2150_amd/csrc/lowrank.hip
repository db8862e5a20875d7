// Elementwise and small-reduction kernels of the low-rank Stokes driver
// (Sections 2 and 5): the shift-matrix factors of the discrete gradients
// applied to the columns of a factor, scaled column copies (the
// concatenations that a sum of low-rank matrices starts from), and
// Frobenius inner products of low-rank matrices.
#include "lrp_internal.h"

#include <algorithm>

namespace lrp {
namespace {

constexpr int LR_T = 256;

// out[:, c] = alpha * Op in[:, c], Op one of the (m-1) x m shift matrices
// G = E - Z, H = E + Z or their transposes (Section 2):
//   G:   out_i = in_{i+1} - in_i          (m_out = m_in - 1)
//   H:   out_i = in_{i+1} + in_i
//   G^T: out_i = in_{i-1} - in_i          (m_out = m_in + 1; in_{-1} = in_{m_in} = 0)
//   H^T: out_i = in_{i-1} + in_i
__global__ __launch_bounds__(LR_T) void k_shift(int op, int m_out, const double *in, long ldi,
                                               double *out, long ldo, double alpha) {
  const int i = blockIdx.x * LR_T + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= m_out) return;
  const double *x = in + (long)c * ldi;
  double v;
  if (op == SHIFT_G || op == SHIFT_H) {
    const double a = x[i + 1], b = x[i];
    v = (op == SHIFT_G) ? a - b : a + b;
  } else {
    const int m_in = m_out - 1;
    const double a = (i >= 1) ? x[i - 1] : 0.0, b = (i < m_in) ? x[i] : 0.0;
    v = (op == SHIFT_GT) ? a - b : a + b;
  }
  out[i + (long)c * ldo] = alpha * v;
}

__global__ __launch_bounds__(LR_T) void k_copy_scaled(int rows, const double *src, long lds,
                                                     double *dst, long ldd, double alpha) {
  const int i = blockIdx.x * LR_T + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= rows) return;
  dst[i + (long)c * ldd] = alpha * src[i + (long)c * lds];
}

// <X, Y>_F = sum_ab (Xu^T Yu)_ab (Xv^T Yv)_ab for X = Xu Xv^T, Y = Yu Yv^T
// (rows x rx and rows x ry factors, rx, ry <= KMAX): one workgroup per pair.
// The rows go through LDS in chunks of LR_CH (both factors of both sides,
// coalesced), each thread accumulates its entries of the two Gram matrices,
// and the products are summed over the workgroup.
constexpr int LR_CH = 16;
constexpr int LR_LD = LR_CH + 1;   // column stride in LDS (odd: no bank conflicts)
__global__ __launch_bounds__(LR_T) void k_lr_dot(const LrDot *pairs, double *out) {
  const LrDot d = pairs[blockIdx.x];
  __shared__ double xs[2][LR_LD * KMAX], ys[2][LR_LD * KMAX];
  __shared__ double red[LR_T / 64];
  constexpr int PER = KMAX * KMAX / LR_T;   // Gram entries per thread
  double gu[PER], gv[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) gu[q] = gv[q] = 0.0;
  const int rx = d.rx, ry = d.ry;
  for (int i0 = 0; i0 < d.rows; i0 += LR_CH) {
    const int m = min(LR_CH, d.rows - i0);
    for (int e = threadIdx.x; e < LR_CH * KMAX; e += LR_T) {
      const int i = e % LR_CH, a = e / LR_CH, o = i + a * LR_LD;
      const bool in = i < m;
      xs[0][o] = (in && a < rx) ? d.xu[i0 + i + (long)a * d.ldx] : 0.0;
      xs[1][o] = (in && a < rx) ? d.xv[i0 + i + (long)a * d.ldx] : 0.0;
      ys[0][o] = (in && a < ry) ? d.yu[i0 + i + (long)a * d.ldy] : 0.0;
      ys[1][o] = (in && a < ry) ? d.yv[i0 + i + (long)a * d.ldy] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = threadIdx.x + q * LR_T, a = e % KMAX, b = e / KMAX;
      if (a < rx && b < ry) {
        double su = 0.0, sv = 0.0;
        for (int i = 0; i < m; ++i) {
          su += xs[0][i + a * LR_LD] * ys[0][i + b * LR_LD];
          sv += xs[1][i + a * LR_LD] * ys[1][i + b * LR_LD];
        }
        gu[q] += su;
        gv[q] += sv;
      }
    }
    __syncthreads();
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < PER; ++q) s += gu[q] * gv[q];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < LR_T / 64; ++w) t += red[w];
    out[blockIdx.x] = t;
  }
}

// Tall-skinny products of the randomized rounding, 64 x 64 output tiles,
// 256 threads each owning a 4 x 4 block, operands staged through LDS in
// chunks of 16 along the summed index.
constexpr int GT = 64, GK = 16;

// C (K x L) = A^T B, A: rows x K, B: rows x L (sum over the rows).  Layer
// z = blockIdx.z sums the rows [z chunk, (z + 1) chunk) into C + z * ldc * L
// (its own K x L partial; one layer: C itself).
__global__ __launch_bounds__(LR_T) void k_gemm_tn(int rows, int chunk, int K, int L,
                                                 const double *A, long lda, const double *B,
                                                 long ldb, double *C, long ldc) {
  __shared__ double as[GK][GT + 1], bs[GK][GT + 1];
  const int k0 = blockIdx.x * GT, l0 = blockIdx.y * GT;
  const int tk = (threadIdx.x & 15) * 4, tl = (threadIdx.x >> 4) * 4;
  const int r0 = blockIdx.z * chunk, r1 = min(rows, r0 + chunk);
  C += (long)blockIdx.z * ldc * L;
  double acc[4][4] = {};
  for (int i0 = r0; i0 < r1; i0 += GK) {
    for (int e = threadIdx.x; e < GK * GT; e += LR_T) {
      const int i = e % GK, c = e / GK;
      const bool in = i0 + i < r1;
      as[i][c] = (in && k0 + c < K) ? A[i0 + i + (long)(k0 + c) * lda] : 0.0;
      bs[i][c] = (in && l0 + c < L) ? B[i0 + i + (long)(l0 + c) * ldb] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < GK; ++i) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = as[i][tk + u], b[u] = bs[i][tl + u];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (k0 + tk + u < K && l0 + tl + v < L) C[k0 + tk + u + (long)(l0 + tl + v) * ldc] = acc[u][v];
}

// C[e] = sum over the layers z < nz of P[z * per + e], in layer order, for
// the K x L entries e of a partial (leading dimension K), into C (ldc).
__global__ __launch_bounds__(LR_T) void k_sum_layers(int nz, int K, int L, const double *P,
                                                    double *C, long ldc) {
  const long per = (long)K * L;
  const long e = (long)blockIdx.x * LR_T + threadIdx.x;
  if (e >= per) return;
  double v = 0.0;
  for (int z = 0; z < nz; ++z) v += P[z * per + e];
  const int k = (int)(e % K), l = (int)(e / K);
  C[k + (long)l * ldc] = v;
}

// C (rows x L) = A B diag(scale), A: rows x K, B: K x L (sum over K);
// scale may be null (ones).
__global__ __launch_bounds__(LR_T) void k_gemm_nn(int rows, int K, int L, const double *A,
                                                 long lda, const double *B, long ldb,
                                                 double *C, long ldc, const double *scale) {
  __shared__ double as[GK][GT + 1], bs[GK][GT + 1];
  const int r0 = blockIdx.x * GT, l0 = blockIdx.y * GT;
  const int tr = (threadIdx.x & 15) * 4, tl = (threadIdx.x >> 4) * 4;
  double acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += GK) {
    for (int e = threadIdx.x; e < GK * GT; e += LR_T) {
      const int r = e % GT, k = e / GT;          // A tile: rows fastest (coalesced)
      as[k][r] = (r0 + r < rows && k0 + k < K) ? A[r0 + r + (long)(k0 + k) * lda] : 0.0;
      const int kk = e % GK, c = e / GK;         // B tile: k fastest (coalesced)
      bs[kk][c] = (k0 + kk < K && l0 + c < L) ? B[k0 + kk + (long)(l0 + c) * ldb] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < GK; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = as[k][tr + u], b[u] = bs[k][tl + u];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int l = l0 + tl + v;
    if (l >= L) continue;
    const double sc = scale ? scale[l] : 1.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (r0 + tr + u < rows) C[r0 + tr + u + (long)l * ldc] = acc[u][v] * sc;
  }
}

}  // namespace

hipError_t launch_shift(int op, int m_out, int cols, const double *in, long ldi, double *out,
                        long ldo, double alpha, hipStream_t st) {
  if (cols <= 0 || m_out <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_shift, dim3(ceil_div(m_out, LR_T), cols), dim3(LR_T), 0, st, op, m_out,
                     in, ldi, out, ldo, alpha);
  return hipGetLastError();
}

hipError_t launch_copy_scaled(int rows, int cols, const double *src, long lds, double *dst,
                              long ldd, double alpha, hipStream_t st) {
  if (cols <= 0 || rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_scaled, dim3(ceil_div(rows, LR_T), cols), dim3(LR_T), 0, st, rows,
                     src, lds, dst, ldd, alpha);
  return hipGetLastError();
}

// Layers of the split sum over the rows: ceil(rows / 128) of them, at most
// GEMM_SPLIT, each a chunk of equal length rounded up to a multiple of GK
// (the last one takes the rest).
static int gemm_tn_layers(int rows, int *chunk) {
  int nz = std::min(GEMM_SPLIT, std::max(1, ceil_div(rows, 128)));
  int c = ceil_div(ceil_div(rows, nz), GK) * GK;
  nz = ceil_div(rows, c);
  *chunk = c;
  return nz;
}

size_t gemm_tn_work(int rows, int K, int L) {
  int chunk;
  const int nz = gemm_tn_layers(rows, &chunk);
  return nz > 1 ? (size_t)nz * K * L : 0;
}

hipError_t launch_gemm_tn(int rows, int K, int L, const double *A, long lda, const double *B,
                          long ldb, double *C, long ldc, hipStream_t st, double *work) {
  if (K <= 0 || L <= 0) return hipSuccess;
  int chunk;
  const int nz = work ? gemm_tn_layers(rows, &chunk) : 1;
  if (nz <= 1) {
    hipLaunchKernelGGL(k_gemm_tn, dim3(ceil_div(K, GT), ceil_div(L, GT), 1), dim3(LR_T), 0, st,
                       rows, std::max(rows, 1), K, L, A, lda, B, ldb, C, ldc);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_gemm_tn, dim3(ceil_div(K, GT), ceil_div(L, GT), nz), dim3(LR_T), 0, st,
                     rows, chunk, K, L, A, lda, B, ldb, work, (long)K);
  const long per = (long)K * L;
  hipLaunchKernelGGL(k_sum_layers, dim3((unsigned)ceil_div((int)per, LR_T)), dim3(LR_T), 0, st,
                     nz, K, L, (const double *)work, C, ldc);
  return hipGetLastError();
}

hipError_t launch_gemm_nn(int rows, int K, int L, const double *A, long lda, const double *B,
                          long ldb, double *C, long ldc, const double *scale, hipStream_t st) {
  if (rows <= 0 || L <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm_nn, dim3(ceil_div(rows, GT), ceil_div(L, GT)), dim3(LR_T), 0, st,
                     rows, K, L, A, lda, B, ldb, C, ldc, scale);
  return hipGetLastError();
}

hipError_t launch_lr_dots(const LrDot *pairs, int npairs, double *out, hipStream_t st) {
  if (npairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lr_dot, dim3(npairs), dim3(LR_T), 0, st, pairs, out);
  return hipGetLastError();
}

}  // namespace lrp
