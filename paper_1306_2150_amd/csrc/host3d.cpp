// Host runtime of the 3D (Tucker) path: slot groups and the synchronous
// lrpoisson_solve3d entry point.  The kernels and the method are described
// in tucker.hip.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "host.h"

namespace lrp {

#define HIPCHK3(x)                        \
  do {                                    \
    hipError_t e_ = (x);                  \
    if (e_ != hipSuccess) return LRP_EDEVICE; \
  } while (0)

Group3D::Group3D(lrp_ctx *ctx, int n, int cap) : ctx_(ctx), n_(n), cap_(cap) {}

Group3D::~Group3D() {
  inner_.reset();
  dev_free(ctx_, ws_, bytes_);
  if (h_s_) (void)hipHostFree(h_s_);
}

size_t Group3D::bytes() const { return bytes_ + (inner_ ? inner_->bytes() : 0); }

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// half-contracted cores (r_d x r_p x k_q <= KMAX^3), the column tables of
// the three fiber matrices, two core buffers
static constexpr size_t T_ELEMS = (size_t)KMAX * KMAX * KMAX;
static size_t own_slot_bytes() {
  return 3 * align256(T_ELEMS * 8) + 6 * align256((size_t)FIB_M * 8) +
         2 * align256((size_t)CORE_MAX * 8);
}

size_t solve3d_slot_bytes(int n) { return own_slot_bytes() + 3 * cross_slot_bytes(n, FIB_M); }

lrp_status Group3D::init() {
  lrp_status err;
  const GridTables *tabs = get_tables(ctx_, n_, &err);
  if (!tabs) return err;
  const size_t per_slot = own_slot_bytes();
  const size_t solves_b = align256(sizeof(Solve3D) * cap_);
  bytes_ = solves_b + per_slot * cap_;
  void *p = nullptr;
  if ((err = dev_alloc(ctx_, &p, bytes_)) != LRP_OK) return err;
  ws_ = (char *)p;
  d_s_ = (Solve3D *)ws_;
  char *slots = ws_ + solves_b;
  // mode slots: n rows, the FIB_M fiber columns (column tables per slot)
  inner_.reset(new Group2D(ctx_, n_, 3 * cap_, FIB_M, nullptr));
  if ((err = inner_->init()) != LRP_OK) {
    inner_.reset();
    return err;
  }
  if (hipHostMalloc((void **)&h_s_, sizeof(Solve3D) * cap_, 0) != hipSuccess) return LRP_ENOMEM;
  std::memset(h_s_, 0, sizeof(Solve3D) * cap_);
  plans_.resize(cap_);
  io_.resize(cap_);
  for (int i = cap_ - 1; i >= 0; --i) free_slots.push_back(i);
  for (int i = 0; i < cap_; ++i) {
    Solve3D &s = h_s_[i];
    char *b = slots + per_slot * i;
    s.n = n_;
    for (int d = 0; d < 3; ++d) {
      s.T[d] = (double *)(b + d * align256(T_ELEMS * 8));
      s.inner[d] = inner_->dev_solves() + 3 * i + d;
    }
    char *c = b + 3 * align256(T_ELEMS * 8);
    for (int d = 0; d < 3; ++d) {
      s.lamc[d] = (double *)(c + (2 * d) * align256((size_t)FIB_M * 8));
      s.lqc[d] = (double *)(c + (2 * d + 1) * align256((size_t)FIB_M * 8));
    }
    c += 6 * align256((size_t)FIB_M * 8);
    s.buf0 = (double *)c;
    s.buf1 = (double *)(c + align256((size_t)CORE_MAX * 8));
    s.phase = P3_IDLE;
  }
  HIPCHK3(hipMemcpy(d_s_, h_s_, sizeof(Solve3D) * cap_, hipMemcpyHostToDevice));
  return LRP_OK;
}

void Group3D::setup_slot(int i, const double *const U[3], long ld, const int r[3],
                         const double *G, double eps, double *const X[3], long ldx,
                         double *Gx, const int rmax[3], const Plan &plan) {
  Solve3D &s = h_s_[i];
  plans_[i] = plan;
  IO &io = io_[i];
  for (int d = 0; d < 3; ++d) {
    s.r[d] = r[d];
    s.rmax[d] = rmax[d];
    s.k[d] = 0;
    s.R[d] = 0;
    io.U[d] = U[d];
    io.X[d] = X[d];
  }
  io.ld = ld;
  io.ldx = ldx;
  s.eps = eps;
  s.G = G;
  s.Gx = Gx;
  s.phase = P3_SETUP;
  s.outer = 0;
  s.kick = plan.kick;
  s.kcap = plan.kcap;
  s.max_outer = plan.max_sweeps;
  for (int d = 0; d < 3; ++d) s.kf[d] = 0;
  s.cross_status = LRP_OK;
  s.status = LRP_OK;
  s.out_ok = 0;
  s.nrm = 0.0;
  // every mode cross works at eps / sqrt(3) on its fiber matrix; its
  // numerator rank is the mode's Tucker rank.  The column tables are the
  // slot's own (filled when the fibers are built).
  const double ed = eps / std::sqrt(3.0);
  for (int d = 0; d < 3; ++d) {
    // the first width the device gives a mode cross when it (re)starts it on
    // new fibers (rank + kick, k_fiber_cols): the host mirror must agree, as
    // the launches take their rank bucket from it
    Plan pm = plan;
    pm.k0 = r[d] + plan.kick;
    inner_->setup_slot(3 * i + d, nullptr, nullptr, 0, r[d], ed, nullptr, nullptr, 0,
                       KMAX, pm);
    Solve2D &m = inner_->host(3 * i + d);
    m.lam_c = s.lamc[d];
    m.lq_c = (plan.op == LRP_OP_STOKES) ? s.lqc[d] : nullptr;
  }
}

lrp_status Group3D::start(const std::vector<int> &slots, hipStream_t st) {
  if (slots.empty()) return LRP_OK;
  int rmax_in = 1;
  for (int i : slots) {
    HIPCHK3(hipMemcpyAsync(d_s_ + i, h_s_ + i, sizeof(Solve3D), hipMemcpyHostToDevice, st));
    for (int d = 0; d < 3; ++d) {
      lrp_status e = inner_->upload_slot(3 * i + d, st);
      if (e != LRP_OK) return e;
      rmax_in = std::max(rmax_in, h_s_[i].r[d]);
    }
  }
  // forward transforms of the three factors into the mode slots' Uh
  for (int prec : ALL_PRECS) {
    std::vector<DstCol> cols;
    for (int i : slots) {
      if (plans_[i].fwd_prec != prec) continue;
      for (int d = 0; d < 3; ++d) {
        const Solve2D &m = inner_->host(3 * i + d);
        for (int c = 0; c < h_s_[i].r[d]; ++c)
          cols.push_back({io_[i].U[d] + (long)c * io_[i].ld, m.Uh + (long)c * m.ldu,
                          3 * i + d, 0});
      }
    }
    if (!cols.empty()) {
      lrp_status e = inner_->transform(cols, prec, st);
      if (e != LRP_OK) return e;
    }
  }
  int hi = 0;
  for (int i : slots) hi = std::max(hi, i + 1);
  // the first fibers (evenly spaced pivots) and the mode crosses' start
  HIPCHK3(launch_fiber_setup(d_s_, hi, rmax_in, st));
  return LRP_OK;
}

lrp_status Group3D::step(hipStream_t st) {
  int hi = 0;
  for (int i = 0; i < cap_; ++i)
    if (h_s_[i].phase != P3_IDLE && h_s_[i].phase != P3_DONE) hi = i + 1;
  if (hi == 0) return LRP_OK;
  lrp_status e = inner_->step(st);
  if (e != LRP_OK) return e;
  // solves whose three crosses just finished: another outer sweep on new
  // fibers, or the core, its unfoldings' TSQR and Jacobi SVD, output ranks,
  // factors and core (all gated on the device)
  int rmax_in = 1;
  for (int i = 0; i < hi; ++i)
    for (int d = 0; d < 3; ++d) rmax_in = std::max(rmax_in, h_s_[i].r[d]);
  HIPCHK3(launch_fiber_outer(d_s_, hi, st));
  HIPCHK3(launch_fiber_setup(d_s_, hi, rmax_in, st));
  const int P = KMAX * KMAX;
  const Tree tp = make_tree(P, KMAX);
  HIPCHK3(launch_core_build(d_s_, hi, st));
  HIPCHK3(launch_core_unfold(d_s_, hi, P, st));
  HIPCHK3(launch_tsqr(TS_CORE, P, tp, inner_->dev_solves(), 3 * hi, KMAX, st));
  HIPCHK3(launch_core(ACT_CORE, inner_->dev_solves(), 3 * hi, KMAX, st));
  HIPCHK3(launch_tucker_out(d_s_, hi, n_, st));
  return LRP_OK;
}

lrp_status Group3D::fetch(hipStream_t st, bool sync) {
  HIPCHK3(hipMemcpyAsync(h_s_, d_s_, sizeof(Solve3D) * cap_, hipMemcpyDeviceToHost, st));
  lrp_status e = inner_->fetch(st, false);
  if (e != LRP_OK) return e;
  if (sync) HIPCHK3(hipStreamSynchronize(st));
  return LRP_OK;
}

lrp_status Group3D::finish(const std::vector<int> &slots, hipStream_t st) {
  for (int prec : ALL_PRECS) {
    std::vector<DstCol> cols;
    for (int i : slots) {
      const Solve3D &s = h_s_[i];
      if (plans_[i].inv_prec != prec || !s.out_ok) continue;
      for (int d = 0; d < 3; ++d) {
        const Solve2D &m = inner_->host(3 * i + d);
        for (int c = 0; c < s.R[d]; ++c)
          cols.push_back({m.A + (long)c * m.ldu, io_[i].X[d] + (long)c * io_[i].ldx, -1, 0});
      }
    }
    if (!cols.empty()) {
      lrp_status e = inner_->transform(cols, prec, st);
      if (e != LRP_OK) return e;
    }
  }
  return LRP_OK;
}

// Result report of a finished slot.
void fill_info3d(Group3D &g, int i, int32_t rank_out[3], lrp_info *info) {
  const Solve3D &s = g.host(i);
  int sweeps = s.outer, k = 0, R = 0;
  double change = -1.0, est = 0.0;
  for (int d = 0; d < 3; ++d) {
    const Solve2D &m = g.modes().host(3 * i + d);
    k = std::max(k, m.k);
    R = std::max(R, s.R[d]);
    change = std::max(change, m.change);
    // mode cross: its truncation tail and last change
    est = std::max(est, std::max(m.tail, 0.0) + std::max(m.change, 0.0));
    if (rank_out) rank_out[d] = s.R[d];
  }
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->status = s.status;
    info->sweeps = sweeps;
    info->k = k;
    info->rank = R;
    info->fwd_prec = g.plan(i).fwd_prec;
    info->inv_prec = g.plan(i).inv_prec;
    info->change = change;
    // the core's HOSVD truncation at eps/sqrt(3) per mode adds at most
    // sqrt(3 (eps/sqrt(3))^2) = eps
    info->err_est = (s.nrm == 0.0) ? 0.0 : est + s.eps;
  }
}

lrp_status check_problem3d(int64_t n, const int32_t rank[3], const double *const U[3],
                           int64_t ld, const double *G, double eps,
                           double *const X[3], int64_t ldx, const double *Gx,
                           const int32_t rmax[3]) {
  if (n < 1 || n > LRP_MAX_N3 || !rank || !rmax) return LRP_EINVAL;
  if (!(eps > 0.0 && eps < 1.0)) return LRP_EINVAL;
  bool any_zero = false, all_cap = true;
  for (int d = 0; d < 3; ++d) {
    if (rank[d] < 0 || rank[d] > LRP_MAX_RANK || rmax[d] < 0) return LRP_EINVAL;
    any_zero |= rank[d] == 0;
    all_cap &= rmax[d] > 0;
  }
  if (!any_zero) {
    if (!G || ld < n) return LRP_EINVAL;
    for (int d = 0; d < 3; ++d)
      if (!U[d]) return LRP_EINVAL;
  }
  if (all_cap) {
    if (!Gx || ldx < n) return LRP_EINVAL;
    for (int d = 0; d < 3; ++d)
      if (!X[d]) return LRP_EINVAL;
  }
  return LRP_OK;
}

}  // namespace lrp

using namespace lrp;

extern "C" lrp_status lrpoisson_solve3d(lrp_ctx *ctx, int64_t n, const int32_t rank[3],
                                        const double *U1, const double *U2,
                                        const double *U3, int64_t ld, const double *G,
                                        double eps, const lrp_opts *opts,
                                        double *U1x, double *U2x, double *U3x,
                                        int64_t ldx, double *Gx, const int32_t rmax[3],
                                        int32_t rank_out[3], lrp_info *info, void *stream) {
  if (!ctx || !rank_out) return LRP_EINVAL;
  if (check_opts(opts) != LRP_OK) return LRP_EINVAL;
  if (opts && opts->prec != LRP_PREC_AUTO && !transform_prec_ok(opts->prec, (int)n))
    return LRP_EINVAL;
  const double *U[3] = {U1, U2, U3};
  double *X[3] = {U1x, U2x, U3x};
  lrp_status e = check_problem3d(n, rank, U, ld, G, eps, X, ldx, Gx, rmax);
  if (e != LRP_OK) return e;
  for (int d = 0; d < 3; ++d) rank_out[d] = 0;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->change = -1.0;
  }
  if (rank[0] == 0 || rank[1] == 0 || rank[2] == 0) return LRP_OK;   // zero solution
  if (hipSetDevice(ctx->device) != hipSuccess) return LRP_EDEVICE;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(ctx->mu);
  auto &slot = ctx->batch3_groups[(int)n];
  if (!slot) {
    std::unique_ptr<Group3D> g(new Group3D(ctx, (int)n, 1));
    if ((e = g->init()) != LRP_OK) return e;
    slot = std::move(g);
  }
  Group3D &g = *slot;
  g.begin_batch();
  const Plan plan = make_plan(opts, eps, (int)n);
  const int r[3] = {rank[0], rank[1], rank[2]};
  const int rm[3] = {rmax[0], rmax[1], rmax[2]};
  g.setup_slot(0, U, ld, r, G, eps, X, ldx, Gx, rm, plan);
  phase_mark(ctx, 0, st);
  if ((e = g.start({0}, st)) != LRP_OK) return e;
  phase_mark(ctx, 1, st);
  // at most max_sweeps outer sweeps, each of at most max_sweeps mode-cross
  // sweeps plus its initial step; the core and its rounding take a few more
  bool done = false;
  const int cap = (plan.max_sweeps + 2) * (plan.max_sweeps + 1) + 8;
  for (int it = 0; it <= cap && !done; ++it) {
    if ((e = g.step(st)) != LRP_OK) return e;
    if ((e = g.fetch(st)) != LRP_OK) return e;
    done = g.host(0).phase == P3_DONE;
  }
  if (!done) return LRP_EDEVICE;
  phase_mark(ctx, 2, st);
  if ((e = g.finish({0}, st)) != LRP_OK) return e;
  phase_mark(ctx, 3, st);
  if (hipStreamSynchronize(st) != hipSuccess) return LRP_EDEVICE;
  g.host(0).phase = P3_IDLE;
  fill_info3d(g, 0, rank_out, info);
  if (info) phase_times(ctx, info->us_phase);
  return (lrp_status)g.host(0).status;
}
