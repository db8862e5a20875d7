// Rounding of the skeleton (paper Section 3, "rounding": QR of the factors
// plus SVD of the small core, O((n+m) r^2 + r^3)).
//
// After the column basis Q0 (n x k, orthonormal), the rows I picked by
// maxvol, and the rows' QR  Xh[I,:]^T = Q1 R1, the skeleton of the cross is
//     X~ = Q0 (Q0[I,:])^-1 Xh[I,:] = Q0 K Q1^T,   K = (Q0[I,:])^-1 R1^T,
// so its SVD only needs the k x k core K = W S Z^T:  X~ = (Q0 W) S (Q1 Z)^T.
// The core SVD is one-sided (Hestenes) Jacobi, which keeps small singular
// values to high relative accuracy (needed for tail truncation at 1e-10);
// one 256-thread workgroup per solve, K and the accumulated right rotations
// in LDS (sized for the launch's rank bucket, so several workgroups share a
// CU), rotations applied to disjoint column pairs in parallel (round-robin
// ordering).
#include "lrp_internal.h"

namespace lrp {
namespace {

// Sums over each row of 16 lanes (every lane of the row gets its row's sum)
// of N values, stage by stage so that their chains overlap.
template <int N>
__device__ __forceinline__ void row_sum16_n(double (&v)[N]) {
#pragma unroll
  for (int g = 0; g < N; ++g) v[g] += dpp_f64<0x128>(v[g]);
#pragma unroll
  for (int g = 0; g < N; ++g) v[g] += dpp_f64<0x124>(v[g]);
#pragma unroll
  for (int g = 0; g < N; ++g) v[g] += dpp_f64<0x122>(v[g]);
#pragma unroll
  for (int g = 0; g < N; ++g) v[g] += dpp_f64<0x121>(v[g]);
}

// phase ACT_SWEEP: K = InvC Rfin^T (the cross core); phase ACT_CORE (3D
// path): K = Rfin^T, whose left singular vectors W are those of the Tucker
// core unfolding that the preceding TSQR factored.
// NT = 16 threads per column pair (one DPP row), all pairs of the bucket in
// flight at once: 256 threads up to k = 32, 384 and 512 for the larger
// buckets (few-solve launches, as in the 3D path and serving, are bound by
// the latency of the rounds, not by occupancy).
template <int KM>
constexpr int core_threads() { return KM / 2 * 16 < NTHR ? NTHR : KM / 2 * 16; }

template <int KM>
__global__ __launch_bounds__(core_threads<KM>()) void k_core(int phase, Solve2D *S) {
  constexpr int LD = KM + 1;
  constexpr int NT = core_threads<KM>();
  constexpr int NW = NT / 64;     // waves
  Solve2D &s = S[blockIdx.x];
  if (s.active != phase) return;
  const bool plain = phase == ACT_CORE;
  __shared__ double K[KM * LD];   // column c at K[c*LD + i]
  __shared__ double V[KM * LD];
  __shared__ double sg[KM];
  __shared__ int perm[KM];
  __shared__ int rot;
  const int kk = s.k;
  if (kk > KM) return;            // the launch's bucket covers every k
  const int kp = (kk + 1) & ~1;   // even number of players
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // stage InvC (in V): every thread's loads in flight at once (indices below
  // KM <= KMAX stay inside the buffer), masked after
  {
    constexpr int PV = (KM * KM + NT - 1) / NT;
    double tv[PV];
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int e = threadIdx.x + u * NT, j = e / KM, i = e - j * KM;
      tv[u] = s.InvC[(e < KM * KM ? i + j * KMAX : 0)];
    }
#pragma unroll
    for (int u = 0; u < PV; ++u) {
      const int e = threadIdx.x + u * NT, j = e / KM, i = e - j * KM;
      if (e < KM * KM) V[j * LD + i] = (i < kk && j < kk) ? (plain ? (i == j ? 1.0 : 0.0) : tv[u]) : 0.0;
    }
  }
  // rows c = wv + NW t of Rfin, lane j holding Rfin[c][j] (one load per lane
  // and row, all in flight before the products; c < KM and j < 64 stay
  // inside the KMAX x KMAX buffer)
  constexpr int NCW = (KM + NW - 1) / NW;
  static_assert(NW * NCW <= KMAX, "rows of Rfin inside the buffer");
  double rrow[NCW];
#pragma unroll
  for (int t = 0; t < NCW; ++t) {
    const int c = wv + NW * t;
    rrow[t] = s.Rfin[c + lane * KMAX];
  }
  __syncthreads();
  // K[i][c] = sum_{j >= c} InvC[i][j] * Rfin[c][j]   (Rfin upper triangular;
  // Rfin[c][j] broadcast from lane j)
#pragma unroll
  for (int t = 0; t < NCW; ++t) {
    const int c = wv + NW * t;
    if (c >= kp) break;
    for (int i = lane; i < kp; i += 64) {
      double v = 0.0;
      if (i < kk && c < kk)
        for (int j = c; j < kk; ++j) v += V[j * LD + i] * readlane_f64(rrow[t], j);
      K[c * LD + i] = v;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x >> 6; c < kp; c += NW)
    for (int i = threadIdx.x & 63; i < kp; i += 64) V[c * LD + i] = (i == c) ? 1.0 : 0.0;
  __syncthreads();
  // ||K||_F^2, which the rotations keep: a pair of columns whose norms are
  // both at the rounding level of ||K||_F (geometric mean below u ||K||_F,
  // u = 2^-52) holds no information, and rotating it only stirs rounding
  // noise that the relative test below would chase for dozens of sweeps
  __shared__ double fro_w[NW];
  {
    double v = 0.0;
    for (int e = threadIdx.x; e < kp * KM; e += NT) {
      const int c = e / KM, i = e - c * KM;
      const double x = (i < kp) ? K[c * LD + i] : 0.0;
      v += x * x;
    }
    v = wave_sum(v);
    if (lane == 0) fro_w[wv] = v;
  }
  __syncthreads();
  double fro2 = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) fro2 += fro_w[w];
  const double floor2 = 0x1p-104 * fro2;   // (u ||K||_F)^2
  const int npairs = kp / 2;
  // 16 threads (one DPP row) per column pair, NT / 16 pairs in flight
  constexpr int NP = NT / 16;
  const int pr0 = threadIdx.x >> 4, gl = threadIdx.x & 15;
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (threadIdx.x == 0) rot = 0;
    __syncthreads();
    for (int st = 0; st < kp - 1; ++st) {
      for (int pr = pr0; pr < ((npairs + NP - 1) / NP) * NP; pr += NP) {
        const bool live = pr < npairs;
        const int pa = pr, pb = kp - 1 - pr;
        const int a = live ? ((pa == 0) ? 0 : 1 + (pa - 1 + st) % (kp - 1)) : 0;
        const int b = live ? 1 + (pb - 1 + st) % (kp - 1) : 0;
        // the pair's column entries gl, gl + 16, ... below kp (KM / 16 at
        // most, loaded together, then masked)
        constexpr int NI = (KM + 15) / 16;
        double xa[NI], xb[NI];
#pragma unroll
        for (int u = 0; u < NI; ++u) {
          const int i = min(gl + 16 * u, KM - 1);
          xa[u] = K[a * LD + i];
          xb[u] = K[b * LD + i];
        }
        double sums[3] = {0.0, 0.0, 0.0};   // al, be, ga
#pragma unroll
        for (int u = 0; u < NI; ++u)
          if (live && gl + 16 * u < kp) {
            sums[0] += xa[u] * xa[u];
            sums[1] += xb[u] * xb[u];
            sums[2] += xa[u] * xb[u];
          }
        row_sum16_n(sums);
        const double al = sums[0], be = sums[1], ga = sums[2];
        if (live && al > 0.0 && be > 0.0 && fabs(ga) > tol * sqrt(al * be) &&
            sqrt(al * be) > floor2) {
          const double zeta = (be - al) / (2.0 * ga);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) /
                           (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
          double va[NI], vb[NI];
#pragma unroll
          for (int u = 0; u < NI; ++u) {
            const int i = min(gl + 16 * u, KM - 1);
            va[u] = V[a * LD + i];
            vb[u] = V[b * LD + i];
          }
#pragma unroll
          for (int u = 0; u < NI; ++u) {
            const int i = gl + 16 * u;
            if (i < kp) {
              K[a * LD + i] = cs * xa[u] - sn * xb[u];
              K[b * LD + i] = sn * xa[u] + cs * xb[u];
              V[a * LD + i] = cs * va[u] - sn * vb[u];
              V[b * LD + i] = sn * va[u] + cs * vb[u];
            }
          }
          if (gl == 0) rot = 1;
        }
      }
      __syncthreads();
    }
    if (rot == 0) break;
    __syncthreads();
  }
  // singular values and descending order (ties: lower index first)
  if (threadIdx.x < kk) {
    double v = 0.0;
    for (int i = 0; i < kk; ++i) v += K[threadIdx.x * LD + i] * K[threadIdx.x * LD + i];
    sg[threadIdx.x] = sqrt(v);
  }
  __syncthreads();
  if (threadIdx.x < kk) {
    const int c = threadIdx.x;
    int rank = 0;
    for (int d = 0; d < kk; ++d)
      if (sg[d] > sg[c] || (sg[d] == sg[c] && d < c)) ++rank;
    perm[rank] = c;
  }
  __syncthreads();
  for (int t = threadIdx.x >> 6; t < kk; t += NW)
    for (int i = threadIdx.x & 63; i < kk; i += 64) {
      const int c = perm[t];
      const double sv = sg[c];
      s.W[i + t * KMAX] = (sv > 0.0) ? K[c * LD + i] / sv : 0.0;
      s.Z[i + t * KMAX] = V[c * LD + i];
    }
  if (threadIdx.x < kk) s.sig[threadIdx.x] = sg[perm[threadIdx.x]];
}

}  // namespace

hipError_t launch_core(int phase, Solve2D *s, int nsolves, int kmax, hipStream_t st) {
  if (kmax <= 16)
    hipLaunchKernelGGL(k_core<16>, dim3(nsolves), dim3(core_threads<16>()), 0, st, phase, s);
  else if (kmax <= 32)
    hipLaunchKernelGGL(k_core<32>, dim3(nsolves), dim3(core_threads<32>()), 0, st, phase, s);
  else if (kmax <= 48)
    hipLaunchKernelGGL(k_core<48>, dim3(nsolves), dim3(core_threads<48>()), 0, st, phase, s);
  else
    hipLaunchKernelGGL(k_core<64>, dim3(nsolves), dim3(core_threads<64>()), 0, st, phase, s);
  return hipGetLastError();
}

}  // namespace lrp
