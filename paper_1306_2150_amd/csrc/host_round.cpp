// Rounding of a sum of low-rank matrices by a randomized range finder: the
// Stokes driver's sums (Section 5: every operation of the Uzawa iteration
// is followed by a rounding to the working accuracy) have partial sums of
// far higher rank than their result, so the incremental rounding of the
// exponential-sum comparator, which keeps the running factorisation inside
// a 64-column panel, cannot take them.  This one never forms a partial sum:
// for X = U V^T (K columns),
//   Y = X Omega, Omega an n x L Gaussian sketch (L = min(64, n)), one power
//   step Y = X X^T Y with re-orthonormalisation, Q = orth(Y)   (TSQR),
//   X^T Q = Q2 R2                                                (TSQR),
//   X ~ Q Q^T X = Q R2^T Q2^T,  R2^T = W S Z^T                  (Jacobi),
// then the smallest rank R whose tail ||S[R:]|| is within eps ||S|| (the
// relative tolerance of the result itself, not of a partial sum; or an
// absolute tolerance when that is larger), and
// Ux = Q W[:, :R] S[:R], Vx = Q2 Z[:, :R].  A rank that reaches L - 8 is
// refused (LRP_ERANKCAP): the sketch could no longer vouch for the tail.
// The products are the tall-skinny GEMMs of lowrank.hip, the QR the cross's
// TSQR and the SVD its Jacobi core, on one slot of a one-slot group.
#include "../../include/lrpoisson_kernels.h"
#include "host.h"

#include <cmath>
#include <cstring>
#include <vector>

namespace lrp {
namespace {

#define HIPCHK(x)                             \
  do {                                        \
    hipError_t e_ = (x);                      \
    if (e_ != hipSuccess) return LRP_EDEVICE; \
  } while (0)

constexpr int RR_GUARD = 8;   // columns of the sketch kept above the rank

// Standard normal draws from a counter-based generator (splitmix64, then
// Box-Muller on pairs of 53-bit uniforms), a fixed seed per grid size.
void gaussian(std::vector<double> &out, uint64_t seed) {
  uint64_t x = seed;
  auto next = [&x]() {
    uint64_t z = (x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  };
  const double two_pi = 6.283185307179586476925286766559;
  for (size_t i = 0; i < out.size(); i += 2) {
    const double u1 = ((double)(next() >> 11) + 1.0) * 0x1p-53;   // (0, 1]
    const double u2 = (double)(next() >> 11) * 0x1p-53;
    const double r = std::sqrt(-2.0 * std::log(u1));
    out[i] = r * std::cos(two_pi * u2);
    if (i + 1 < out.size()) out[i + 1] = r * std::sin(two_pi * u2);
  }
}

}  // namespace

RoundGroup::~RoundGroup() {
  g.reset();
  dev_free(ctx, buf, bytes);
}

static lrp_status round_group(lrp_ctx *ctx, int n, int K, RoundGroup **out) {
  auto &slot = ctx->round_groups[n];
  const int L = std::min(KMAX, n);
  if (!slot || slot->kcap < K) {
    if (slot) (void)hipDeviceSynchronize();   // its buffers may still be read
    slot.reset();
    std::unique_ptr<RoundGroup> r(new RoundGroup);
    r->ctx = ctx;
    r->n = n;
    r->L = L;
    r->kcap = std::max(K, 4 * KMAX);
    r->g.reset(new Group2D(ctx, n, 1));
    lrp_status e = r->g->init();
    if (e != LRP_OK) return e;
    const size_t om = (size_t)n * L, z = (size_t)r->kcap * L, qk = (size_t)n * L;
    const size_t zp = gemm_tn_work(n, r->kcap, L);
    r->bytes = (om + z + qk + zp) * 8 + 4 * 256;
    void *p = nullptr;
    if ((e = dev_alloc(ctx, &p, r->bytes)) != LRP_OK) return e;
    r->buf = (double *)p;
    r->omega = r->buf;
    r->Z = r->omega + ((om + 31) & ~(size_t)31);
    r->Qk = r->Z + ((z + 31) & ~(size_t)31);
    r->zpart = zp ? r->Qk + ((qk + 31) & ~(size_t)31) : nullptr;
    std::vector<double> h(om);
    gaussian(h, 0x5EEDULL * 1000003ULL + (uint64_t)n);
    Solve2D &s = r->g->host(0);
    // the core takes K = InvC Rfin^T with InvC = I: the transpose of the R
    // factor the last TSQR left in Rfin
    std::vector<double> eye((size_t)KMAX * KMAX, 0.0);
    for (int i = 0; i < KMAX; ++i) eye[i + (size_t)i * KMAX] = 1.0;
    if (hipMemcpy(r->omega, h.data(), om * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s.InvC, eye.data(), eye.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
      return LRP_EDEVICE;
    s.Q1f = nullptr;
    s.k = L;
    s.r = L;
    s.active = ACT_INIT;
    s.nonfinite = 0;
    slot = std::move(r);
  }
  *out = slot.get();
  return LRP_OK;
}

lrp_status round_random(lrp_ctx *ctx, int n, int K, const double *U, const double *V, long ld,
                        double eps, double *Ux, double *Vx, long ldx, int rmax, int *rank,
                        double *err, hipStream_t st, double abs_tol) {
  *rank = 0;
  *err = 0.0;
  if (K <= 0) return LRP_OK;
  if (n < 16 || ld < n || ldx < n) return LRP_EINVAL;
  RoundGroup *rp = nullptr;
  lrp_status e = round_group(ctx, n, K, &rp);
  if (e != LRP_OK) return e;
  RoundGroup &r = *rp;
  Group2D &G = *r.g;
  Solve2D &s = G.host(0);
  Solve2D *d = G.dev_solves();
  const int L = r.L;
  const Tree tr = make_tree(n, KMAX);
  if ((e = G.upload_slot(0, st)) != LRP_OK) return e;
  auto orth = [&]() -> hipError_t {   // slot Vh (n x L) -> Q1, Rfin
    return launch_tsqr(TS_VH_TO_Q1, n, tr, d, 1, L, st);
  };
  // Y = X Omega = U (V^T Omega), Q = orth(Y)
  HIPCHK(launch_gemm_tn(n, K, L, V, ld, r.omega, n, r.Z, K, st, r.zpart));
  HIPCHK(launch_gemm_nn(n, K, L, U, ld, r.Z, K, s.Vh, s.ldv, nullptr, st));
  HIPCHK(orth());
  // one power step: Q' = orth(X^T Q), Q = orth(X Q')
  HIPCHK(launch_gemm_tn(n, K, L, U, ld, s.Q1, s.ldv, r.Z, K, st, r.zpart));
  HIPCHK(launch_gemm_nn(n, K, L, V, ld, r.Z, K, s.Vh, s.ldv, nullptr, st));
  HIPCHK(orth());
  HIPCHK(launch_gemm_tn(n, K, L, V, ld, s.Q1, s.ldv, r.Z, K, st, r.zpart));
  HIPCHK(launch_gemm_nn(n, K, L, U, ld, r.Z, K, s.Vh, s.ldv, nullptr, st));
  HIPCHK(orth());
  HIPCHK(hipMemcpy2DAsync(r.Qk, (size_t)n * 8, s.Q1, (size_t)s.ldv * 8, (size_t)n * 8, L,
                          hipMemcpyDeviceToDevice, st));
  // X^T Q = V (U^T Q) = Q2 R2
  HIPCHK(launch_gemm_tn(n, K, L, U, ld, r.Qk, n, r.Z, K, st, r.zpart));
  HIPCHK(launch_gemm_nn(n, K, L, V, ld, r.Z, K, s.Vh, s.ldv, nullptr, st));
  HIPCHK(orth());
  // R2^T = W S Z^T
  HIPCHK(launch_core(ACT_INIT, d, 1, L, st));
  double sig[KMAX];
  HIPCHK(hipMemcpyAsync(sig, s.sig, sizeof(double) * L, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double tot2 = 0.0;
  for (int t = L - 1; t >= 0; --t) tot2 += sig[t] * sig[t];
  const double nrm = std::sqrt(tot2);
  int R = L;
  double tail2 = 0.0;
  for (int t = L - 1; t >= 0; --t) {
    tail2 += sig[t] * sig[t];
    if (std::sqrt(tail2) > std::max(eps * nrm, abs_tol)) break;
    R = t;
  }
  if (nrm == 0.0) R = 0;
  double drop2 = 0.0;
  for (int t = L - 1; t >= R; --t) drop2 += sig[t] * sig[t];
  *err = nrm > 0.0 ? std::sqrt(drop2) / nrm : 0.0;
  *rank = R;
  if (R > L - RR_GUARD || R > rmax) return LRP_ERANKCAP;
  if (R == 0) return LRP_OK;
  // Ux = Q W[:, :R] S[:R], Vx = Q2 Z[:, :R]
  HIPCHK(launch_gemm_nn(n, L, R, r.Qk, n, s.W, KMAX, Ux, ldx, s.sig, st));
  HIPCHK(launch_gemm_nn(n, L, R, s.Q1, s.ldv, s.Z, KMAX, Vx, ldx, nullptr, st));
  return LRP_OK;
}

}  // namespace lrp

using namespace lrp;

extern "C" lrp_status lrp_lowrank_round(lrp_ctx *ctx, int64_t n, int32_t K, const double *U,
                                        const double *V, int64_t ld, double eps, double *Ux,
                                        double *Vx, int64_t ldx, int32_t rmax,
                                        int32_t *rank_out, void *stream) {
  if (!ctx || !rank_out || n < 16 || n > LRP_MAX_N || K < 0 || rmax < 0) return LRP_EINVAL;
  if (!(eps > 0.0 && eps < 1.0) || ld < n || ldx < n) return LRP_EINVAL;
  if (K > 0 && (!U || !V)) return LRP_EINVAL;
  if (rmax > 0 && (!Ux || !Vx)) return LRP_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return LRP_EDEVICE;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(ctx->mu);
  int rank = 0;
  double err = 0.0;
  lrp_status e = round_random(ctx, (int)n, K, U, V, ld, eps, Ux, Vx, ldx, rmax, &rank, &err, st);
  *rank_out = rank;
  if (hipStreamSynchronize(st) != hipSuccess) return LRP_EDEVICE;
  return e;
}
