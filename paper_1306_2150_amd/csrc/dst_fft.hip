// Sine transform by chirp-z convolution (Bluestein) of the folded halves, in
// float64: the O(n log n) form of the transform (paper Section 4.1: the DST
// of the factors costs O(n r log n)), for grid sizes whose folded halves fit
// one 4096-point FFT in LDS.
//
// With N = n + 1 the folded transform (see dst.hip) splits into
//   odd rows   y_(2a+1) = sqrt(2/N) sum_{k=1..H0} u_k sin(pi (2a+1) k / N),
//   even rows  y_(2a+2) = sqrt(2/N) sum_{k=1..H1} w_k sin(pi (2a+2) k / N),
// u_k = x_k + x_(N-k), w_k = x_k - x_(N-k) (the middle point of an even N
// joins u alone), H0 = ceil(n/2), H1 = floor(n/2).  With k' = k - 1 and
// W = e^(2 pi i/N), both are imaginary parts of W^(a k') times a pre-factor
// in k' and a post-factor in a, and
//   W^(a k') = d_a d_k' conj(d_(a-k')),   d_m = e^(i pi m^2 / N),
// so each half is a cyclic convolution of length M >= 2 H0 - 1 with the
// fixed kernel beta_m = conj(d_min(m, M-m)):
//   alpha_k' = v_k' e^(i pi p(k') / N),     p = k'^2 + k' + 1 (odd), k'^2 + 2k' (even)
//   z = IFFT_M(FFT_M(alpha) * FFT_M(beta))
//   y = sqrt(2/N) Im(e^(i pi q(a) / N) z_a), q = a^2 + 2a (odd), a^2 + 2a + 2 (even).
// Every phase is an exact integer mod 2N, looked up in a table of e^(i pi q/N).
//
// One workgroup (256 threads) transforms one column: the two halves in turn,
// each through a 4096-point FFT as three radix-16 passes (a 16-point DFT in
// registers per thread and pass, radix 4 x 4), the pointwise product with
// FFT_M(beta) between the last forward pass and the first inverse pass (the
// thread that holds X[k1 + 16 k2 + 256 k3] for all k3 also starts the inverse
// over k3), and four LDS exchanges whose layout (stride 257) keeps every
// eight consecutive lanes on distinct banks.  The inputs are read once,
// coalesced (x_k ascending, x_(N-k) descending), and the two halves' outputs
// are written interleaved as they belong, rows 2a+1 and 2a+2 side by side.
#include <algorithm>
#include <vector>

#include "lrp_internal.h"

namespace lrp {
namespace {

constexpr int FM = 4096;     // FFT length
constexpr int FT = 256;      // threads per workgroup
constexpr int FP = 257;      // LDS stride between the 16 rows of an exchange
constexpr int FLDS = 16 * FP;

struct cd {
  double x, y;
};
__device__ __forceinline__ cd operator+(cd a, cd b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cd operator-(cd a, cd b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cd cmul(cd a, cd b) {
  return {fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}
// a * conj(b)
__device__ __forceinline__ cd cmulc(cd a, cd b) {
  return {fma(a.x, b.x, a.y * b.y), fma(a.y, b.x, -a.x * b.y)};
}
__device__ __forceinline__ cd ld2(const double2 *p) {
  const double2 v = *p;
  return {v.x, v.y};
}

// 4-point DFT in place, natural order; forward e^(-2 pi i/4) = -i.
template <bool INV>
__device__ __forceinline__ void dft4(cd &a0, cd &a1, cd &a2, cd &a3) {
  const cd t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = a1 - a3;
  a0 = t0 + t2;
  a2 = t0 - t2;
  if (!INV) {
    a1 = {t1.x + t3.y, t1.y - t3.x};
    a3 = {t1.x - t3.y, t1.y + t3.x};
  } else {
    a1 = {t1.x - t3.y, t1.y + t3.x};
    a3 = {t1.x + t3.y, t1.y - t3.x};
  }
}

// multiply by e^(-+2 pi i e/16) (forward: minus), e in {1, 2, 3, 4, 6, 9}
template <bool INV, int E>
__device__ __forceinline__ cd tw16(cd a) {
  constexpr double C = 0x1.d906bcf328d46p-1;   // cos(pi/8)
  constexpr double S = 0x1.87de2a6aea963p-2;   // sin(pi/8)
  constexpr double R = 0x1.6a09e667f3bcdp-1;   // sqrt(2)/2
  constexpr double sg = INV ? 1.0 : -1.0;      // sign of the sine part
  if constexpr (E == 4) return INV ? cd{-a.y, a.x} : cd{a.y, -a.x};
  double c, s;
  if constexpr (E == 1) c = C, s = S;
  else if constexpr (E == 2) c = R, s = R;
  else if constexpr (E == 3) c = S, s = C;
  else if constexpr (E == 6) c = -R, s = R;
  else c = -C, s = -S;                          // E == 9
  return cmul(a, cd{c, sg * s});
}

// 16-point DFT in place, natural order (radix 4 x 4).
template <bool INV>
__device__ __forceinline__ void dft16(cd (&v)[16]) {
#pragma unroll
  for (int a = 0; a < 4; ++a) dft4<INV>(v[a], v[a + 4], v[a + 8], v[a + 12]);
  v[5] = tw16<INV, 1>(v[5]);
  v[9] = tw16<INV, 2>(v[9]);
  v[13] = tw16<INV, 3>(v[13]);
  v[6] = tw16<INV, 2>(v[6]);
  v[10] = tw16<INV, 4>(v[10]);
  v[14] = tw16<INV, 6>(v[14]);
  v[7] = tw16<INV, 3>(v[7]);
  v[11] = tw16<INV, 6>(v[11]);
  v[15] = tw16<INV, 9>(v[15]);
#pragma unroll
  for (int b = 0; b < 4; ++b) dft4<INV>(v[4 * b], v[4 * b + 1], v[4 * b + 2], v[4 * b + 3]);
  // v[4 k1 + k2] holds X[k1 + 4 k2]: transpose
  cd t;
  t = v[1], v[1] = v[4], v[4] = t;
  t = v[2], v[2] = v[8], v[8] = t;
  t = v[3], v[3] = v[12], v[12] = t;
  t = v[6], v[6] = v[9], v[9] = t;
  t = v[7], v[7] = v[13], v[13] = t;
  t = v[11], v[11] = v[14], v[14] = t;
}

__device__ __forceinline__ void lds_put(double2 *L, int i, cd v) { L[i] = make_double2(v.x, v.y); }
__device__ __forceinline__ cd lds_get(const double2 *L, int i) { return ld2(L + i); }
// A zero the compiler cannot see through.  Added to the index of a load whose
// address depends on the thread only, it keeps the load inside the loop over
// the two halves: hoisted out of it, the sixteen loads of FFT_M(beta) would
// hold 64 registers across the whole kernel.
__device__ __forceinline__ int opaque_zero() {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return z;
}

// One half: alpha in v (positions t + 256 j) -> z in v (same positions).
// Twiddles come from two LDS tables: W1[e] = e^(-2 pi i e/256) and
// W2[e] = e^(-2 pi i e/4096), e < 256; a pass-2 twiddle
// e^(-2 pi i n1 (k1 + 16 k2)/4096) is W2[n1 k1] W1[n1 k2 mod 256].
// bh = FFT_M(beta) (global, L2-resident).
__device__ __forceinline__ void conv4096(cd (&v)[16], double2 *L, const double2 *W1,
                                         const double2 *W2, const double2 *__restrict__ bh) {
  const int t = threadIdx.x, lo = t & 15, hi = t >> 4;
  // pass 1: thread (n1, n2) = (lo, hi), DFT over n3
  dft16<false>(v);
#pragma unroll
  for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], lds_get(W1, (hi * k1) & 255));
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) lds_put(L, lo + 16 * k1 + FP * hi, v[k1]);
  __syncthreads();
  // pass 2: thread (n1, k1) = (lo, hi), DFT over n2
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) v[n2] = lds_get(L, t + FP * n2);
  dft16<false>(v);
  {
    const cd b = lds_get(W2, lo * hi);
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) {
      v[k2] = cmul(v[k2], cmul(b, lds_get(W1, (lo * k2) & 255)));
    }
  }
  __syncthreads();
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) lds_put(L, hi + 16 * k2 + FP * lo, v[k2]);
  __syncthreads();
  // pass 3: thread (k1, k2) = (lo, hi), DFT over n1 -> X[t + 256 k3]; the
  // loads of FFT_M(beta) go out first and complete under the pass
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) v[n1] = lds_get(L, t + FP * n1);
  cd bv[8];
  int z = opaque_zero();
#pragma unroll
  for (int k3 = 0; k3 < 8; ++k3) bv[k3] = ld2(bh + (t + 256 * k3 + z));
  dft16<false>(v);
  // pointwise product with FFT_M(beta) (in two groups of eight loads), then
  // the inverse over k3
#pragma unroll
  for (int k3 = 0; k3 < 8; ++k3) v[k3] = cmul(v[k3], bv[k3]);
  z = opaque_zero();
#pragma unroll
  for (int k3 = 8; k3 < 16; ++k3) bv[k3 - 8] = ld2(bh + (t + 256 * k3 + z));
#pragma unroll
  for (int k3 = 8; k3 < 16; ++k3) v[k3] = cmul(v[k3], bv[k3 - 8]);
  dft16<true>(v);
  // inverse twiddle e^(+2 pi i n1 (k1 + 16 k2)/4096), thread (k1, k2) = (lo, hi)
#pragma unroll
  for (int n1 = 1; n1 < 16; ++n1) {
    v[n1] = cmulc(v[n1], cmul(lds_get(W2, n1 * lo), lds_get(W1, (n1 * hi) & 255)));
  }
  __syncthreads();
#pragma unroll
  for (int n1 = 0; n1 < 16; ++n1) lds_put(L, lo + 16 * n1 + FP * hi, v[n1]);
  __syncthreads();
  // inverse pass 2: thread (k1, n1) = (lo, hi), DFT over k2
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) v[k2] = lds_get(L, t + FP * k2);
  dft16<true>(v);
#pragma unroll
  for (int n2 = 1; n2 < 16; ++n2) v[n2] = cmulc(v[n2], lds_get(W1, (n2 * lo) & 255));
  __syncthreads();
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) lds_put(L, hi + 16 * n2 + FP * lo, v[n2]);
  __syncthreads();
  // inverse pass 3: thread (n1, n2) = (lo, hi), DFT over k1 -> z[t + 256 n3]
#pragma unroll
  for (int k1 = 0; k1 < 16; ++k1) v[k1] = lds_get(L, t + FP * k1);
  dft16<true>(v);
}

// One workgroup per column.  tab = [e^(i pi q/N), q < 2N][W1, 256][W2, 256][bh, 4096].
__global__ __launch_bounds__(FT, 2) void k_dst_fft4096(int n, const double2 *__restrict__ tab,
                                                    const DstCol *__restrict__ cols,
                                                    Solve2D *solves) {
  extern __shared__ double2 lds[];
  const DstCol col = cols[blockIdx.x];
  const int t = threadIdx.x, N = n + 1, N2 = 2 * N;
  const int H0 = (n + 1) / 2, H1 = n / 2;
  const double2 *ch = tab, *bh = tab + N2 + 2 * 256;
  double2 *W1 = lds + FLDS, *W2 = W1 + 256;
  W1[t] = tab[N2 + t];
  W2[t] = tab[N2 + 256 + t];
  __syncthreads();
  // folded inputs at k' = t + 256 j (k = k' + 1); K <= 2048, so j < 8: read
  // once, both halves formed from them
  double u[8], w[8];
  bool bad = false;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int kp = t + 256 * j, k = kp + 1;
    double xa = 0.0, xb = 0.0;
    if (kp < H0) {
      xa = col.src[kp];
      if (N - k != k) xb = col.src[N - k - 1];
    }
    bad |= !(isfinite(xa) && isfinite(xb));
    u[j] = xa + xb;
    w[j] = (kp < H1) ? xa - xb : 0.0;
  }
  if (bad && col.solve >= 0 && solves) solves[col.solve].nonfinite = 1;
  const double scale = sqrt(2.0 / (double)N) / (double)FM;
  // the odd half's outputs wait in registers, so that rows 2a+1 and 2a+2 go
  // out together (whole cache lines: stride-2 stores of each half alone
  // would write every line twice)
  double yo[8];
#pragma unroll 1
  for (int half = 0; half < 2; ++half) {
    cd v[16];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int kp = t + 256 * j;
      const int ph = (kp * kp + (half ? 2 * kp : kp + 1)) % N2;
      const double val = half ? w[j] : u[j];
      const cd e = ld2(ch + ph);
      v[j] = {val * e.x, val * e.y};
    }
#pragma unroll
    for (int j = 8; j < 16; ++j) v[j] = {0.0, 0.0};
    conv4096(v, lds, W1, W2, bh);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int a = t + 256 * j;
      const int ph = (a * a + 2 * a + (half ? 2 : 0)) % N2;
      const cd e = ld2(ch + ph);
      const double y = scale * fma(e.x, v[j].y, e.y * v[j].x);
      if (!half) {
        yo[j] = y;
      } else {
        // rows 2a + 1 (odd half, a < H0) and 2a + 2 (even half, a < H1)
        if (a < H0) col.dst[2 * a] = yo[j];
        if (a < H1) col.dst[2 * a + 1] = y;
      }
    }
    __syncthreads();   // the last exchange's reads are done before the next half writes
  }
}

}  // namespace

bool dst_fft_supported(int n) { return n >= 1 && (n + 1) / 2 <= FM / 2; }

size_t dst_fft_table_bytes(int n) { return ((size_t)2 * (n + 1) + 512 + FM) * 16; }

// e^(i pi q/N) for q < 2N, e^(-2 pi i e/256) and e^(-2 pi i e/4096) for
// e < 256, and FFT_M(beta) with beta_m = conj(e^(i pi min(m, M-m)^2 / N)),
// in long double, rounded once.
void dst_fft_table(int n, double *out) {
  const int N = n + 1, N2 = 2 * N;
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int q = 0; q < N2; ++q) {
    // angle pi q/N through the quadrant of the smaller argument
    const long double a = pi * (long double)q / (long double)N;
    out[2 * q] = (double)cosl(a);
    out[2 * q + 1] = (double)sinl(a);
  }
  double *tw = out + 2 * (size_t)N2;
  for (int e = 0; e < 256; ++e) {
    const long double a1 = 2.0L * pi * (long double)e / 256.0L;
    const long double a2 = 2.0L * pi * (long double)e / (long double)FM;
    tw[2 * e] = (double)cosl(a1);
    tw[2 * e + 1] = (double)-sinl(a1);
    tw[512 + 2 * e] = (double)cosl(a2);
    tw[512 + 2 * e + 1] = (double)-sinl(a2);
  }
  // FFT of beta in long double: iterative radix-2, bit-reversed input order
  std::vector<long double> re(FM), im(FM);
  int lg = 0;
  while ((1 << lg) < FM) ++lg;
  for (int m = 0; m < FM; ++m) {
    const long long mm = std::min(m, FM - m);
    const long long ph = (mm * mm) % N2;
    const long double a = pi * (long double)ph / (long double)N;
    int r = 0;
    for (int b = 0; b < lg; ++b) r |= ((m >> b) & 1) << (lg - 1 - b);
    re[r] = cosl(a);
    im[r] = -sinl(a);
  }
  for (int len = 2; len <= FM; len <<= 1) {
    for (int s = 0; s < FM; s += len) {
      for (int k = 0; k < len / 2; ++k) {
        const long double a = -2.0L * pi * (long double)k / (long double)len;
        const long double c = cosl(a), sn = sinl(a);
        const int i0 = s + k, i1 = s + k + len / 2;
        const long double xr = re[i1] * c - im[i1] * sn, xi = re[i1] * sn + im[i1] * c;
        re[i1] = re[i0] - xr;
        im[i1] = im[i0] - xi;
        re[i0] += xr;
        im[i0] += xi;
      }
    }
  }
  double *bh = tw + 2 * (size_t)512;
  for (int k = 0; k < FM; ++k) {
    bh[2 * k] = (double)re[k];
    bh[2 * k + 1] = (double)im[k];
  }
}

hipError_t launch_dst_fft(int n, const void *tab, const DstCol *cols, int ncols,
                          Solve2D *solves, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (ncols <= 0) return hipSuccess;
  if (!dst_fft_supported(n)) return hipErrorInvalidValue;
  const size_t lds = (size_t)(FLDS + 512) * 16;
  hipError_t e = hipFuncSetAttribute((const void *)k_dst_fft4096,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (ev0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
  // grid dimension x holds up to 2^31 - 1 workgroups: one per column
  hipLaunchKernelGGL(k_dst_fft4096, dim3((unsigned)ncols), dim3(FT), lds, st, n,
                     (const double2 *)tab, cols, solves);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev1 && (e = hipEventRecord(ev1, st)) != hipSuccess) return e;
  return hipSuccess;
}

}  // namespace lrp
