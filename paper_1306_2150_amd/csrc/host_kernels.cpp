// The component entry points of include/lrpoisson_kernels.h: the TSQR +
// maxvol and the Jacobi core SVD of the cross, run on caller data through a
// one-slot group (the slot's own buffers hold the panel and the small
// matrices, as in a solve).
#include "../../include/lrpoisson_kernels.h"

#include <cstring>
#include <vector>

#include "host.h"

namespace lrp {
namespace {

#define HIPCHK(x)                             \
  do {                                        \
    hipError_t e_ = (x);                      \
    if (e_ != hipSuccess) return LRP_EDEVICE; \
  } while (0)

Group2D *kernel_group(lrp_ctx *ctx, int n, lrp_status *err) {
  auto &g = ctx->kernel_groups[n];
  if (!g) {
    std::unique_ptr<Group2D> ng(new Group2D(ctx, n, 1));
    if ((*err = ng->init()) != LRP_OK) return nullptr;
    g = std::move(ng);
  }
  *err = LRP_OK;
  return g.get();
}

// the slot's control fields for one pass of an ACT_INIT launch sequence
void reset_slot(Solve2D &s, int k, double tau) {
  s.k = k;
  s.kp = 0;
  s.r = k;
  s.sweep = 0;
  s.tau = tau;
  s.mv_done = 0;
  s.mv_swaps = 0;
  s.nonfinite = 0;
  s.status = LRP_OK;
  s.active = ACT_INIT;
}

}  // namespace
}  // namespace lrp

using namespace lrp;

extern "C" lrp_status lrp_kernel_qr_maxvol(lrp_ctx *ctx, int64_t n, int32_t k, const double *A,
                                           int64_t lda, double tau, double *Q, int64_t ldq,
                                           double *R, int64_t ldr, int32_t *rows,
                                           int32_t *converged, void *stream) {
  if (!ctx || !A || !Q || !R || !rows || !converged) return LRP_EINVAL;
  if (k < 1 || k > KMAX || n < k || n > LRP_MAX_N) return LRP_EINVAL;
  if (lda < n || ldq < n || ldr < k) return LRP_EINVAL;
  if (tau == 0.0) tau = 1.05;
  if (!(tau > 1.0)) return LRP_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return LRP_EDEVICE;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(ctx->mu);
  lrp_status err;
  Group2D *g = kernel_group(ctx, (int)n, &err);
  if (!g) return err;
  Solve2D &s = g->host(0);
  reset_slot(s, k, tau);
  // the panel goes where the initial column choice reads Vh
  HIPCHK(hipMemcpy2DAsync(s.Vh, (size_t)s.ldv * 8, A, (size_t)lda * 8, (size_t)n * 8, k,
                          hipMemcpyDeviceToDevice, st));
  if ((err = g->upload_slot(0, st)) != LRP_OK) return err;
  const Tree tr = make_tree((int)n, KMAX);
  HIPCHK(launch_tsqr(TS_VH_TO_Q1, (int)n, tr, g->dev_solves(), 1, k, st));
  HIPCHK(launch_maxvol(MV_Q1_TO_J, (int)n, tr, g->dev_solves(), 1, k, st));
  // a cross step stops after three rounds and resumes in the next sweep;
  // here the rounds go on until one finds no entry above tau (each swap
  // multiplies the volume by more than tau, so this ends)
  for (int extra = 0; extra < 64; ++extra) {
    if ((err = g->fetch(st)) != LRP_OK) return err;
    if (g->host(0).mv_done) break;
    HIPCHK(launch_maxvol_rounds(MV_Q1_TO_J, (int)n, tr, g->dev_solves(), 1, k, 1, st));
  }
  HIPCHK(hipMemcpy2DAsync(Q, (size_t)ldq * 8, s.Q1, (size_t)s.ldv * 8, (size_t)n * 8, k,
                          hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpy2DAsync(R, (size_t)ldr * 8, s.Rfin, (size_t)KMAX * 8, (size_t)k * 8, k,
                          hipMemcpyDeviceToDevice, st));
  int32_t J[KMAX];
  HIPCHK(hipMemcpyAsync(J, s.J, sizeof(int32_t) * k, hipMemcpyDeviceToHost, st));
  if ((err = g->fetch(st)) != LRP_OK) return err;   // synchronises
  std::memcpy(rows, J, sizeof(int32_t) * k);
  *converged = g->host(0).mv_done ? 1 : 0;
  g->host(0).active = ACT_DONE;
  return LRP_OK;
}

extern "C" lrp_status lrp_kernel_core_svd(lrp_ctx *ctx, int32_t k, const double *M, int64_t ldm,
                                          double *W, double *sigma, double *Z, void *stream) {
  if (!ctx || !M || !W || !sigma || !Z) return LRP_EINVAL;
  if (k < 1 || k > KMAX || ldm < k) return LRP_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return LRP_EDEVICE;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(ctx->mu);
  lrp_status err;
  Group2D *g = kernel_group(ctx, KMAX, &err);
  if (!g) return err;
  Solve2D &s = g->host(0);
  reset_slot(s, k, 1.05);
  // the core K = InvC Rfin^T of a cross step, with InvC = M and Rfin = I
  static const std::vector<double> eye = [] {
    std::vector<double> e((size_t)KMAX * KMAX, 0.0);
    for (int i = 0; i < KMAX; ++i) e[i + (size_t)i * KMAX] = 1.0;
    return e;
  }();
  HIPCHK(hipMemcpyAsync(s.Rfin, eye.data(), eye.size() * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpy2DAsync(s.InvC, (size_t)KMAX * 8, M, (size_t)ldm * 8, (size_t)k * 8, k,
                          hipMemcpyDeviceToDevice, st));
  if ((err = g->upload_slot(0, st)) != LRP_OK) return err;
  HIPCHK(launch_core(ACT_INIT, g->dev_solves(), 1, k, st));
  HIPCHK(hipMemcpy2DAsync(W, (size_t)k * 8, s.W, (size_t)KMAX * 8, (size_t)k * 8, k,
                          hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpy2DAsync(Z, (size_t)k * 8, s.Z, (size_t)KMAX * 8, (size_t)k * 8, k,
                          hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(sigma, s.sig, (size_t)k * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  g->host(0).active = ACT_DONE;
  return LRP_OK;
}
