// Sine transform on the int8 matrix cores with exact integer products (the
// error-free splitting of Ozaki, Ogita and Oishi, "Error-free transformations
// of matrix multiplication by using fast routines of matrix multiplication",
// 2012, with integer slices as in Ootomo, Ozaki and Yokota, 2024).
//
// Both operands are cut into 7-bit integer slices:
//   sin(pi m/N) * 2^6   = T_0 + T_1 2^-7 + ... + T_5 2^-35 + r,  |r| <= 2^-36,
//   x_k 2^(-e_c) * 2^6  = X_0 + X_1 2^-7 + ... + X_5 2^-35 + r,
// with T_a, X_b in [-64, 64] and e_c the exponent of the column's largest
// entry.  Every product T_a X_b is exact in int32, and so is every sum over
// K (|sum| <= 2^12 K * 6 < 2^31 for K < 2^15).  The products of one level
// t = a + b share an accumulator; levels t <= 5 are kept, so the dropped
// terms are below 2^-42 of the leading one:
//   y_j = sqrt(2/N) 2^(e_c - 12) sum_{t<=5} 2^(-7t) acc_t[j],
//   acc_t[j] = sum_k sum_{a+b=t} T_a[j,k] X_b[k].
//
// A first pass writes every column's reversed slice records (8 bytes per
// point); the GEMM stages them in LDS as two dword planes and forms the six
// byte windows below in registers (v_alignbyte).
//
// MFMA formulation (v_mfma_i32_16x16x64_i8): the 64-deep MFMA K runs over 16
// grid points k times 4 slice positions.  Lane (i, g) of the A operand holds,
// for the four points 4g..4g+3, the 4 bytes [T_0 T_1 T_2 T_3] of
// sin(pi j k/N) (one dword per point, read from an LDS record table with the
// sign folded in); lane (c, g) of the B operand holds the 4 bytes
// [X_t X_(t-1) X_(t-2) X_(t-3)] (zero for negative indices) of x_k, a byte
// window of the reversed slice record [X_5 .. X_0 0 0 0] (v_alignbyte).  So
// one MFMA per level t adds sum_{a<=3} T_a X_(t-a) into acc_t, and two more
// with [T_4 T_5 0 0] add the a = 4, 5 terms to levels 4 and 5: 8 MFMAs per
// 16 grid points and 16 x 16 output tile.
//
// Folding: with N = n + 1, sin(pi j (N-k)/N) = (-1)^(j+1) sin(pi j k/N), so
//   y_j = sum_{k=1}^{H0} sin(pi j k/N) u_k  (j odd),   u_k = x_k + x_(N-k),
//   y_j = sum_{k=1}^{H1} sin(pi j k/N) w_k  (j even),  w_k = x_k - x_(N-k),
// with H0 = ceil(n/2), H1 = floor(n/2) and, for even N, the middle point
// u_(N/2) = x_(N/2).  The transform is two half-size GEMMs (half the work of
// the dense one): a column becomes two "parity columns", u with the odd
// rows and w with the even rows, each sliced with its own exponent.
//
// The level sums are exact integers, so a split of K over workgroups (used
// when the tiles alone cannot fill the chip) changes nothing: results do not
// depend on how many columns share a launch.
#include <algorithm>
#include <cmath>

#include "lrp_internal.h"

namespace lrp {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int TMI = 128;         // rows per workgroup: 512 / HW threads, HW 16-row blocks per wave
constexpr int TNI = 32;          // columns per workgroup
// Grid points staged per LDS buffer: KC = 64 for the 64-column tiles where
// the planes fit beside the table (half the barriers of KC = 32), else 32.
// Staged columns are KC + 4 dwords apart (bank skew).
constexpr int KCW = 64, KCN = 32;
constexpr int KPAD = 64;         // the parity records are padded to a multiple of this

// Reversed 7-bit slice record of x * 2^-e: dword 0 = bytes [X5 X4 X3 X2],
// dword 1 = [X1 X0 0 0].
__device__ __forceinline__ uint2 slice_record(double x, int e) {
  double w = ldexp(x, 6 - e);
  if (!isfinite(w)) w = 0.0;
  int s[6];
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    const double q = rint(w);
    s[b] = (int)q;
    w = (w - q) * 128.0;
  }
  uint2 r;
  r.x = (uint32_t)(s[5] & 0xff) | ((uint32_t)(s[4] & 0xff) << 8) |
        ((uint32_t)(s[3] & 0xff) << 16) | ((uint32_t)(s[2] & 0xff) << 24);
  r.y = (uint32_t)(s[1] & 0xff) | ((uint32_t)(s[0] & 0xff) << 8);
  return r;
}

// One block per column c: its parity vectors u (k = 1..H0) and w (k =
// 1..H1), their exponents e with max|v| = f 2^e, f in [0.5, 1) (ex[2c + p],
// p = 0 for u, 1 for w), then the slice records of both, hpad points each
// (zero past H_p), at out + (2c + p) hpad.  Non-finite columns raise their
// solve's flag.
__global__ __launch_bounds__(NTHR) void k_x_slices(int n, int hpad, const DstCol *cols,
                                                   int ncols, uint2 *__restrict__ out,
                                                   int *__restrict__ ex, Solve2D *solves) {
  const int c = blockIdx.x;
  if (c >= ncols) return;
  const double *x = cols[c].src;
  const int N = n + 1, H0 = (n + 1) / 2, H1 = n / 2;
  // parity values at points k = k0 + t NTHR (1-based) for t < FP, all loads
  // in flight at once: indices are clamped into the column (k <= H0, so
  // N - k - 1 >= 0) and the values past H0 masked
  constexpr int FP = 4;
  auto fold4 = [&](int k0, double (&u)[FP], double (&w)[FP], bool &bad) {
    double a[FP], b[FP];
#pragma unroll
    for (int t = 0; t < FP; ++t) {
      const int k = min(k0 + t * NTHR, H0);
      a[t] = x[k - 1];
      b[t] = x[N - k - 1];
    }
#pragma unroll
    for (int t = 0; t < FP; ++t) {
      const int k = k0 + t * NTHR;
      const bool in = k <= H0, pair = 2 * k < N;   // pair: not the middle point
      if (in && (!isfinite(a[t]) || (pair && !isfinite(b[t])))) bad = true;
      u[t] = in ? (pair ? a[t] + b[t] : a[t]) : 0.0;
      w[t] = (in && pair) ? a[t] - b[t] : 0.0;
    }
  };
  // every entry of x is read by the fold (x[k-1] for k <= H0, x[N-k-1] for
  // 2k < N), which also finds the non-finite ones
  // Up to NCACHE passes (hpad <= 4096, n <= 8192) the folded values stay in
  // registers for the slicing below, so the column is read once; past that
  // the slicing folds the column again.
  constexpr int NCACHE = 4;
  const int npass = (max(hpad, H0) + FP * NTHR - 1) / (FP * NTHR);
  const bool cached = npass <= NCACHE;
  double cu[NCACHE][FP], cw[NCACHE][FP];
  double mu = 0.0, mw = 0.0;
  bool bad = false;
  if (cached) {
    // points up to hpad: past H0 the fold gives zeros (no maxima, no flags)
#pragma unroll
    for (int it = 0; it < NCACHE; ++it) {
      if (it < npass) {
        fold4(threadIdx.x + 1 + it * FP * NTHR, cu[it], cw[it], bad);
#pragma unroll
        for (int t = 0; t < FP; ++t) {
          mu = fmax(mu, fabs(cu[it][t]));
          mw = fmax(mw, fabs(cw[it][t]));
        }
      }
    }
  } else {
    for (int k0 = threadIdx.x + 1; k0 <= H0; k0 += FP * NTHR) {
      double u[FP], w[FP];
      fold4(k0, u, w, bad);
#pragma unroll
      for (int t = 0; t < FP; ++t) {
        mu = fmax(mu, fabs(u[t]));
        mw = fmax(mw, fabs(w[t]));
      }
    }
  }
  __shared__ double red[2][4];
  __shared__ int badw[4];
  __shared__ int exs[2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int key = 0;
  wave_argmax(mu, key);                 // wave maxima (keys unused)
  wave_argmax(mw, key);
  const unsigned long long anyb = __ballot(bad);
  if (lane == 0) {
    red[0][wave] = mu;
    red[1][wave] = mw;
    badw[wave] = anyb != 0ull;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int p = threadIdx.x;
    const double m = fmax(fmax(red[p][0], red[p][1]), fmax(red[p][2], red[p][3]));
    int e = 0;
    if (m > 0.0 && isfinite(m)) (void)frexp(m, &e);
    exs[p] = e;
    ex[2 * c + p] = e;
    if (p == 0 && (badw[0] | badw[1] | badw[2] | badw[3]) && cols[c].solve >= 0)
      solves[cols[c].solve].nonfinite = 1;
  }
  __syncthreads();
  const int e0 = exs[0], e1 = exs[1];
  uint2 *o0 = out + (size_t)(2 * c) * hpad, *o1 = o0 + hpad;
  if (cached) {
#pragma unroll
    for (int it = 0; it < NCACHE; ++it) {
      if (it < npass) {
#pragma unroll
        for (int t = 0; t < FP; ++t) {
          const int k = threadIdx.x + 1 + it * FP * NTHR + t * NTHR;
          if (k <= hpad) {
            o0[k - 1] = slice_record(cu[it][t], e0);
            o1[k - 1] = slice_record(k <= H1 ? cw[it][t] : 0.0, e1);
          }
        }
      }
    }
    return;
  }
  bool unused = false;
  for (int k0 = threadIdx.x + 1; k0 <= hpad; k0 += FP * NTHR) {
    double u[FP], w[FP];
    fold4(k0, u, w, unused);
#pragma unroll
    for (int t = 0; t < FP; ++t) {
      const int k = k0 + t * NTHR;
      if (k <= hpad) {
        o0[k - 1] = slice_record(u[t], e0);
        o1[k - 1] = slice_record(k <= H1 ? w[t] : 0.0, e1);
      }
    }
  }
}

// Value of an output from its exact level sums: Horner in powers of 2^-7
// (every step but the last two is exact), then the column scale.  The GEMM
// and the split-K reduction both call this on the same integers, so a
// result does not depend on how K was split.
__device__ __forceinline__ double recombine(const int (&acc)[6], double sc) {
#pragma clang fp contract(off)
  double v = (double)acc[5];
  v = v * 0x1p-7 + (double)acc[4];
  v = v * 0x1p-7 + (double)acc[3];
  v = v * 0x1p-7 + (double)acc[2];
  v = v * 0x1p-7 + (double)acc[1];
  v = v * 0x1p-7 + (double)acc[0];
  return v * sc;
}

// FULL: the LDS table holds the records of all m in [0, 2N) (no folding in
// the inner loop); otherwise the quarter wave q in [0, N/2] with both signs.
//
// The level sums over all of K are exact in int32 (|sum| <= 6 2^12 K < 2^31
// for K < 87000), so one pass needs no intermediate rounding.  With a K
// split (gridDim.z > 1) workgroup z sums chunk z and writes its six level
// sums as int32 to `partial` ([z][p][level][a][c], consecutive lanes on
// consecutive columns); k_dst_i8_reduce adds them exactly and recombines.
//
// HW: 16-row blocks per wave.  HW = 2: four waves of 32 rows (256 threads);
// HW = 1: eight waves of 16 rows (512 threads), half the accumulators per
// wave, so that the 64-column tiles run two waves per SIMD.
template <int TN_, int KC, bool FULL, int HW = 2>
__global__ __launch_bounds__(512 / HW) void k_dst_i8(int n, int Q, const uint2 *__restrict__ rec,
                                                const DstCol *__restrict__ cols, int ncols,
                                                int kchunk, const uint2 *__restrict__ xrec,
                                                int hpad, const int *__restrict__ xex,
                                                int *__restrict__ partial) {
  constexpr int NB = TN_ / 16;
  constexpr int XST = KC + 4;
  constexpr int NT = 512 / HW;
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = n + 1, twoN = 2 * N;
  const int ntab = FULL ? twoN : 2 * Q;
  uint2 *tab = (uint2 *)smem;                    // records, see FULL
  uint32_t *xs0 = (uint32_t *)(tab + ntab);      // record planes [c][k] x 2 buffers
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int H0 = (n + 1) / 2;
  int rt, ct;
  if (!tile_of(ceil_div(H0, TMI), 2 * ceil_div(ncols, TN_), true, rt, ct)) return;
  const int par = ct & 1;
  const int Kp = par ? n / 2 : H0;               // points and rows of this parity
  const int row0 = rt * TMI, c0 = (ct >> 1) * TN_;
  const bool split = gridDim.z > 1;
  const int kbeg = split ? blockIdx.z * kchunk : 0;
  const int kend = split ? min(Kp, kbeg + kchunk) : Kp;
  // table copy, eight loads in flight per thread
  for (int i0 = 0; i0 < ntab; i0 += 8 * NT) {
    uint2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * NT + tid;
      v[u] = (i < ntab) ? rec[i] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * NT + tid;
      if (i < ntab) tab[i] = v[u];
    }
  }
  // staging share: thread stages grid points tk of columns tc0 + 8 t; the
  // columns' records lie 2 hpad apart
  constexpr int PER = KC * TN_ / NT;
  constexpr int CSTEP = NT / KC;
  constexpr int LVL = TN_ * XST;                 // dwords per record plane and buffer
  const int tk = tid & (KC - 1), tc0 = tid / KC;
  const int nsrc = max(0, min(PER, ceil_div(ncols - c0 - tc0, CSTEP)));
  const uint2 *xsrc = xrec + (size_t)(2 * (c0 + tc0) + par) * hpad;
  const size_t sstep = (size_t)2 * CSTEP * hpad;
  const int nst = (kend - kbeg + KC - 1) / KC;
  uint2 pre[PER];
  auto fetch = [&](int st) {
    const int k = kbeg + st * KC + tk;
#pragma unroll
    for (int t = 0; t < PER; ++t)
      pre[t] = (t < nsrc && k < kend) ? xsrc[t * sstep + k] : make_uint2(0u, 0u);
  };
  // the two dwords of the records in two planes [c][k], so that one 16-byte
  // read gives a dword of four consecutive points
  auto stash = [&](int st) {
    uint32_t *xs = xs0 + (st & 1) * 2 * LVL;
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      uint32_t *p = xs + (tc0 + CSTEP * t) * XST + tk;
      p[0] = pre[t].x;
      p[LVL] = pre[t].y;
    }
  };
  // rows of this lane: a = row0 + 16 HW wave + 16 h + (lane & 15), grid row
  // j = 2 a + 1 + par (1-based)
  const int g = lane >> 4, li = lane & 15;
  int jr[HW], d16[HW], mk[HW];
#pragma unroll
  for (int h = 0; h < HW; ++h) {
    const int a = row0 + 16 * HW * wave + 16 * h + li;
    jr[h] = (a < Kp) ? 2 * a + 1 + par : 0;    // rows past the end: sin(0) = 0
    d16[h] = (int)(((long long)jr[h] * 16) % twoN);
    // m = j k mod 2N at this lane's first grid point, k = kbeg + 4 g + 1
    mk[h] = (int)(((long long)jr[h] * (kbeg + 4 * g + 1)) % twoN);
  }
  v4i acc[HW][NB][6];
#pragma unroll
  for (int h = 0; h < HW; ++h)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int t = 0; t < 6; ++t) acc[h][b][t] = (v4i){0, 0, 0, 0};
  if (nst > 0) {
    fetch(0);
    stash(0);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int k0 = kbeg + st * KC;
    if (st + 1 < nst) fetch(st + 1);
    const uint32_t *xs = xs0 + (st & 1) * 2 * LVL;
    const int kcn = min(KC, kend - k0);
    for (int kk = 0; kk < kcn; kk += 16) {
      // A operands: records of points k0 + kk + 4g + e (1-based k)
      v4i ahi[HW], alo[HW];
#pragma unroll
      for (int h = 0; h < HW; ++h) {
        int m = mk[h];
        mk[h] += d16[h];                 // the lane's first point of the next step
        if (mk[h] >= twoN) mk[h] -= twoN;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          uint2 r;
          if (FULL) {
            r = tab[m];
          } else {
            int mm = m, sg = 0;
            if (mm >= N) {
              mm -= N;
              sg = 1;
            }
            if (2 * mm > N) mm = N - mm;
            r = tab[2 * mm + sg];
          }
          // points past the end of K contribute zero through the B side
          ahi[h][e] = (int)r.x;
          alo[h][e] = (int)r.y;
          m += jr[h];
          if (m >= twoN) m -= twoN;
        }
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        // records of points kk + 4g .. +3 of column 16 b + li, and their
        // windows t of [X5 .. X0 0 0 0]: bytes [X_t X_(t-1) X_(t-2) X_(t-3)]
        const uint32_t *xw = xs + (16 * b + li) * XST + kk + 4 * g;
        const v4i d0 = *(const v4i *)xw, d1 = *(const v4i *)(xw + LVL);
        v4i w[6];
        w[5] = d0;
        w[1] = d1;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          w[4][e] = (int)__builtin_amdgcn_alignbyte((uint32_t)d1[e], (uint32_t)d0[e], 1);
          w[3][e] = (int)__builtin_amdgcn_alignbyte((uint32_t)d1[e], (uint32_t)d0[e], 2);
          w[2][e] = (int)__builtin_amdgcn_alignbyte((uint32_t)d1[e], (uint32_t)d0[e], 3);
          w[0][e] = (int)((uint32_t)d1[e] >> 8);
        }
#pragma unroll
        for (int h = 0; h < HW; ++h) {
#pragma unroll
          for (int t = 0; t < 6; ++t)
            acc[h][b][t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ahi[h], w[t], acc[h][b][t], 0, 0, 0);
          acc[h][b][4] = __builtin_amdgcn_mfma_i32_16x16x64_i8(alo[h], w[0], acc[h][b][4], 0, 0, 0);
          acc[h][b][5] = __builtin_amdgcn_mfma_i32_16x16x64_i8(alo[h], w[1], acc[h][b][5], 0, 0, 0);
        }
      }
    }
    __syncthreads();
    if (st + 1 < nst) stash(st + 1);
    __syncthreads();
  }
  // D[i][c]: lane c + 16 (i / 4), register i % 4
  const double sc0 = sqrt(2.0 / (double)N);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int c = c0 + 16 * b + li;
    const int e = (c < ncols) ? xex[2 * c + par] : 0;
    const double sc = ldexp(sc0, e - 12);
#pragma unroll
    for (int h = 0; h < HW; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int a = row0 + 16 * HW * wave + 16 * h + 4 * g + q;
        if (a < Kp && c < ncols) {
          if (split) {
            int *pp = partial + (((size_t)blockIdx.z * 2 + par) * 6 * H0 + a) * ncols + c;
#pragma unroll
            for (int t = 0; t < 6; ++t) pp[(size_t)t * H0 * ncols] = acc[h][b][t][q];
          } else {
            int lv[6];
#pragma unroll
            for (int t = 0; t < 6; ++t) lv[t] = acc[h][b][t][q];
            cols[c].dst[2 * a + par] = recombine(lv, sc);
          }
        }
      }
  }
}

// Exact sum of the split-K level sums, then the same recombination as the
// GEMM's.
// Threads run along columns (x) so that the partial reads coalesce.
__global__ void k_dst_i8_reduce(int n, int ncols, int nz, const int *__restrict__ partial,
                                const int *__restrict__ xex, const DstCol *__restrict__ cols) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int row = blockIdx.y * blockDim.y + threadIdx.y;
  if (row >= n || col >= ncols) return;
  const int H0 = (n + 1) / 2, par = row & 1, a = row >> 1;
  long long s[6] = {0, 0, 0, 0, 0, 0};
  for (int z = 0; z < nz; ++z) {
    const int *pp = partial + (((size_t)z * 2 + par) * 6 * H0 + a) * ncols + col;
#pragma unroll
    for (int t = 0; t < 6; ++t) s[t] += pp[(size_t)t * H0 * ncols];
  }
  // the total over K is bounded like one pass's sum, so it fits int32
  int lv[6];
#pragma unroll
  for (int t = 0; t < 6; ++t) lv[t] = (int)s[t];
  const double sc = ldexp(sqrt(2.0 / (double)(n + 1)), xex[2 * col + par] - 12);
  cols[col].dst[row] = recombine(lv, sc);
}

}  // namespace

// Two record tables of sin(pi m/N) slices, bytes [T_0 T_1 T_2 T_3 | T_4 T_5 0 0]:
// the quarter wave with both signs, rec[2q + s] for q = 0 .. N/2, followed by
// the full period, rec[m] for m = 0 .. 2N-1.
static size_t i8_quarter_bytes(int n) { return (size_t)((n + 1) / 2 + 1) * 2 * 8; }
static size_t i8_full_bytes(int n) { return (size_t)2 * (n + 1) * 8; }

size_t dst_i8_table_bytes(int n) { return i8_quarter_bytes(n) + i8_full_bytes(n); }

static void slice_sine(long double v, unsigned char *o) {
  long double w = v * 64.0L;
  signed char sl[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int a = 0; a < 6; ++a) {
    const long double r = roundl(w);
    sl[a] = (signed char)(long)r;
    w = (w - r) * 128.0L;
  }
  for (int a = 0; a < 8; ++a) o[a] = (unsigned char)sl[a];
}

void dst_i8_table(int n, unsigned char *out) {
  const int N = n + 1, Q = N / 2 + 1;
  const long double pi = 3.14159265358979323846264338327950288L;
  for (int q = 0; q < Q; ++q) {
    const long double v = sinl(pi * (long double)q / (long double)N);
    slice_sine(v, out + ((size_t)2 * q) * 8);
    slice_sine(-v, out + ((size_t)2 * q + 1) * 8);
  }
  unsigned char *full = out + i8_quarter_bytes(n);
  for (int m = 0; m < 2 * N; ++m) {
    // sin(pi m/N) from the quarter wave, so both tables hold identical slices
    int mm = m;
    bool neg = false;
    if (mm >= N) {
      mm -= N;
      neg = true;
    }
    if (2 * mm > N) mm = N - mm;
    const long double v = sinl(pi * (long double)mm / (long double)N);
    slice_sine(neg ? -v : v, full + (size_t)m * 8);
  }
}

static size_t i8_lds(int n, int tn, int kc, bool full) {
  return (full ? i8_full_bytes(n) : i8_quarter_bytes(n)) + (size_t)2 * 2 * tn * (kc + 4) * 4;
}

constexpr size_t LDS_MAX = 160 * 1024;
bool dst_i8_supported(int n) { return i8_lds(n, TNI, KCN, false) <= LDS_MAX; }

// work per column: two parity records of hpad points, then two exponents
static int i8_hpad(int n) { return ceil_div((n + 1) / 2, KPAD) * KPAD; }
static size_t i8_col_bytes(int n) { return (size_t)2 * i8_hpad(n) * 8 + 8; }

size_t dst_i8_work_bytes(int n, int ncols) { return (size_t)ncols * i8_col_bytes(n); }

int dst_i8_work_cols(int n, int want) {
  const size_t per = i8_col_bytes(n);
  const int cap = (int)std::max<size_t>(1024, ((size_t)512 << 20) / per);
  return std::min(want, cap);
}

hipError_t launch_dst_i8(int n, const void *rec, DstCol *cols, int ncols, Solve2D *solves,
                         double *partial, size_t partial_elems, void *work,
                         size_t work_bytes, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (ncols <= 0) return hipSuccess;
  if (!dst_i8_supported(n)) return hipErrorInvalidValue;
  const int Q = (n + 1) / 2 + 1;
  const int H0 = (n + 1) / 2, hpad = i8_hpad(n);
  // fixed K chunks of the folded length (at most 4, at least 256 deep)
  const int kchunk = std::max(256, ceil_div(ceil_div(H0, 4), KPAD) * KPAD);
  const int nchunk = ceil_div(H0, kchunk);
  // the slice records of a launch's columns must fit the work buffer; larger
  // column sets run in several launches (results per column are unchanged)
  const int per = (int)std::min<size_t>((size_t)ncols, work_bytes / i8_col_bytes(n));
  if (per <= 0) return hipErrorInvalidValue;
  for (int c0 = 0; c0 < ncols; c0 += per) {
    const int nc = std::min(per, ncols - c0);
    DstCol *cc = cols + c0;
    uint2 *xrec = (uint2 *)work;
    int *xex = (int *)(xrec + (size_t)2 * nc * hpad);
    hipLaunchKernelGGL(k_x_slices, dim3(nc), dim3(NTHR), 0, st, n, hpad, cc, nc, xrec, xex,
                       solves);
    // 64-column tiles (eight waves of 16 rows where the 64-point stages fit,
    // two waves per SIMD; faster on large launches than 32-column tiles)
    // when they alone give every CU a workgroup; 32-column tiles, twice as
    // many, on small launches
    const int R = ceil_div(H0, TMI);
    const bool wide = R * 2 * ceil_div(nc, 64) >= 256 && i8_lds(n, 64, KCN, false) <= LDS_MAX;
    const int tn = wide ? 64 : TNI;
    const int kc = (wide && i8_lds(n, 64, KCW, false) <= LDS_MAX) ? KCW : KCN;
    const bool full = i8_lds(n, tn, kc, true) <= LDS_MAX;
    const unsigned char *tabs = (const unsigned char *)rec;
    const uint2 *trec = (const uint2 *)(full ? tabs + i8_quarter_bytes(n) : tabs);
    const int C = 2 * ceil_div(nc, tn);
    dim3 g(tile_grid(R, C, true), 1, 1);
    // split-K partials: six int32 level sums per output and chunk
    if (R * C < 512 && partial && partial_elems * 2 >= (size_t)nchunk * 2 * nc * 6 * H0)
      g.z = nchunk;
    int *out_partial = g.z > 1 ? (int *)partial : nullptr;
    const size_t lds = i8_lds(n, tn, kc, full);
    const void *fn = nullptr;
    if (wide && kc == KCW)
      fn = full ? (const void *)k_dst_i8<64, KCW, true, 1> : (const void *)k_dst_i8<64, KCW, false, 1>;
    else if (wide)
      fn = full ? (const void *)k_dst_i8<64, KCN, true> : (const void *)k_dst_i8<64, KCN, false>;
    else
      fn = full ? (const void *)k_dst_i8<TNI, KCN, true> : (const void *)k_dst_i8<TNI, KCN, false>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (ev0 && c0 == 0 && (e = hipEventRecord(ev0, st)) != hipSuccess) return e;
#define LRP_I8_LAUNCH(TNV, KCV, FV)                                                         \
  hipLaunchKernelGGL((k_dst_i8<TNV, KCV, FV>), g, dim3(NTHR), lds, st, n, Q, trec, cc, nc,  \
                     kchunk, xrec, hpad, xex, out_partial)
    if (wide && kc == KCW) {
      if (full)
        hipLaunchKernelGGL((k_dst_i8<64, KCW, true, 1>), g, dim3(512), lds, st, n, Q, trec, cc, nc,
                           kchunk, xrec, hpad, xex, out_partial);
      else
        hipLaunchKernelGGL((k_dst_i8<64, KCW, false, 1>), g, dim3(512), lds, st, n, Q, trec, cc, nc,
                           kchunk, xrec, hpad, xex, out_partial);
    } else if (wide) {
      if (full) LRP_I8_LAUNCH(64, KCN, true);
      else LRP_I8_LAUNCH(64, KCN, false);
    } else if (full) {
      LRP_I8_LAUNCH(TNI, KCN, true);
    } else {
      LRP_I8_LAUNCH(TNI, KCN, false);
    }
#undef LRP_I8_LAUNCH
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev1 && c0 + nc >= ncols && (e = hipEventRecord(ev1, st)) != hipSuccess) return e;
    if (g.z > 1) {
      hipLaunchKernelGGL(k_dst_i8_reduce, dim3(ceil_div(nc, 64), ceil_div(n, 4)), dim3(64, 4), 0,
                         st, n, nc, (int)g.z, (const int *)partial, (const int *)xex, cc);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace lrp
