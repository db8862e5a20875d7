// The low-rank Uzawa-GMRES Stokes driver (Sections 2 and 5): the Schur
// system S p = B^T Delta^-1 f - g solved by restarted GMRES on low-rank
// matrices, each product with S running two low-rank Poisson solves of the
// Stokes-consistent operator and every sum rounded.  Host code orchestrates;
// the arithmetic on the matrices runs in the library's kernels (shift
// factors, scaled copies and inner products in lowrank.hip, the rounding of
// sums through the incremental TSQR + Jacobi steps, the Poisson solves).
// The host only updates GMRES's small Hessenberg system.
#include "host.h"

#include <algorithm>
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
#define LRPCHK(x)                    \
  do {                               \
    lrp_status e_ = (x);             \
    if (e_ != LRP_OK) return e_;     \
  } while (0)

constexpr int ST_MAX_RESTART = 60;

// A low-rank matrix U V^T: rows x r factors, leading dimension ld.
struct LR {
  double *U = nullptr, *V = nullptr;
  long ld = 0;
  int rows = 0, r = 0;
};

class Driver {
 public:
  Driver(lrp_ctx *ctx, lrp_stokes2d_problem &p, hipStream_t st)
      : ctx_(ctx), P_(p), st_(st), n_((int)p.n), nv_((int)p.n - 1), h_(1.0 / (double)p.n) {
    m_ = p.restart > 0 ? p.restart : 30;
    max_iter_ = p.max_iter > 0 ? p.max_iter : 200;
  }
  ~Driver() {
    if (ws_) {
      (void)hipStreamSynchronize(st_);
      std::lock_guard<std::mutex> lock(ctx_->mu);
      dev_free(ctx_, ws_, ws_bytes_);
    }
  }
  lrp_status run();

 private:
  double *take(size_t doubles) {
    double *p = (double *)(ws_ + ws_used_);
    ws_used_ += (doubles * 8 + 255) & ~(size_t)255;
    return p;
  }
  LR make(int rows) {
    LR x;
    x.rows = rows;
    x.ld = rows;
    x.U = take((size_t)rows * KMAX);
    x.V = take((size_t)rows * KMAX);
    return x;
  }
  lrp_status setup();
  lrp_status dots(const std::vector<std::pair<const LR *, const LR *>> &pairs,
                  std::vector<double> &out);
  double norm(const LR &x, lrp_status *err) {
    std::vector<double> v;
    *err = dots({{&x, &x}}, v);
    return *err == LRP_OK ? std::sqrt(std::max(v[0], 0.0)) : 0.0;
  }
  // panel columns [off, off + x.r) = (alpha x.U, x.V)
  lrp_status put(int &off, const LR &x, double alpha) {
    if (off + x.r > pan_cols_ || x.rows > pld_) return LRP_EDEVICE;   // cannot happen
    HIPCHK(launch_copy_scaled(x.rows, x.r, x.U, x.ld, panU_ + (long)off * pld_, pld_, alpha, st_));
    HIPCHK(launch_copy_scaled(x.rows, x.r, x.V, x.ld, panV_ + (long)off * pld_, pld_, 1.0, st_));
    off += x.r;
    return LRP_OK;
  }
  // round the panel's first K columns into out: relative eps, or an
  // absolute tail up to abs_tol when that is larger
  lrp_status round(int rows, int K, double eps, LR &out, double abs_tol = 0.0);
  lrp_status grad(const LR &p, LR &bx, LR &by);
  lrp_status poisson2(const LR &a, const LR &b, double eps, LR &ya, LR &yb);
  // panel columns: alpha (B_x^T Delta^-1 a + B_y^T Delta^-1 b) from the
  // solves ya = Delta^-1 a / 4, yb (the solver's operator is 4 Delta)
  lrp_status put_div(int &off, const LR &ya, const LR &yb, double alpha);
  // S x rounded to eps; the two Poisson solves inside to eps_solve (the
  // terms B_x^T Delta^-1 B_x x and B_y^T Delta^-1 B_y x can cancel, so a
  // residual needs them tighter than the sum)
  lrp_status schur(const LR &x, double eps, LR &out, double eps_solve = 0.0);
  lrp_status copy_out(const LR &x, double alpha, double *U, double *V);

  lrp_ctx *ctx_;
  lrp_stokes2d_problem &P_;
  hipStream_t st_;
  int n_, nv_, m_, max_iter_;
  double h_;
  char *ws_ = nullptr;
  size_t ws_bytes_ = 0, ws_used_ = 0;
  double *panU_ = nullptr, *panV_ = nullptr;
  long pld_ = 0;
  int pan_cols_ = 0;
  LrDot *d_dots_ = nullptr;
  double *d_dout_ = nullptr;
  int max_dots_ = 0;
  LR one_, chk_;             // the kernel directions 1 1^T and c c^T, c_i = (-1)^i
  std::vector<LR> basis_;    // Krylov vectors
  LR b_, x_, r_, w_, t_;     // pressure grid
  LR ax_, ay_, yx_, yy_, tu_, tv_;   // velocity grid
  int max_rank_ = 0;
};

lrp_status Driver::setup() {
  pld_ = n_;
  pan_cols_ = KMAX * (m_ + 3);
  max_dots_ = 2 * (m_ + 2);
  const size_t lr_n = 2 * (size_t)n_ * KMAX, lr_v = 2 * (size_t)nv_ * KMAX;
  ws_bytes_ = (size_t)(m_ + 1 + 5) * (lr_n * 8 + 512) + 6 * (lr_v * 8 + 512) +
              2 * ((size_t)pld_ * pan_cols_ * 8 + 256) + 2 * ((size_t)n_ * 8 * 2 + 256) +
              (size_t)max_dots_ * (sizeof(LrDot) + 8) + 1024;
  {
    std::lock_guard<std::mutex> lock(ctx_->mu);
    void *p = nullptr;
    LRPCHK(dev_alloc(ctx_, &p, ws_bytes_));
    ws_ = (char *)p;
  }
  panU_ = take((size_t)pld_ * pan_cols_);
  panV_ = take((size_t)pld_ * pan_cols_);
  basis_.resize(m_ + 1);
  for (auto &v : basis_) v = make(n_);
  b_ = make(n_);
  x_ = make(n_);
  r_ = make(n_);
  w_ = make(n_);
  t_ = make(n_);
  ax_ = make(nv_);
  ay_ = make(nv_);
  yx_ = make(nv_);
  yy_ = make(nv_);
  tu_ = make(nv_);
  tv_ = make(nv_);
  d_dots_ = (LrDot *)take((max_dots_ * sizeof(LrDot) + 7) / 8);
  d_dout_ = take(max_dots_);
  double *kv = take(2 * (size_t)n_);
  if (ws_used_ > ws_bytes_) return LRP_EDEVICE;   // cannot happen: sized above
  std::vector<double> one(n_), chk(n_);
  for (int i = 0; i < n_; ++i) {
    one[i] = 1.0;
    chk[i] = (i & 1) ? -1.0 : 1.0;
  }
  one_.rows = chk_.rows = n_;
  one_.ld = chk_.ld = n_;
  one_.r = chk_.r = 1;
  one_.U = one_.V = kv;
  chk_.U = chk_.V = kv + n_;
  HIPCHK(hipMemcpyAsync(one_.U, one.data(), (size_t)n_ * 8, hipMemcpyHostToDevice, st_));
  HIPCHK(hipMemcpyAsync(chk_.U, chk.data(), (size_t)n_ * 8, hipMemcpyHostToDevice, st_));
  HIPCHK(hipStreamSynchronize(st_));
  return LRP_OK;
}

lrp_status Driver::dots(const std::vector<std::pair<const LR *, const LR *>> &pairs,
                        std::vector<double> &out) {
  std::vector<LrDot> h;
  for (const auto &pr : pairs) {
    const LR &x = *pr.first, &y = *pr.second;
    h.push_back({x.U, x.V, y.U, y.V, x.ld, y.ld, x.rows, x.r, y.r});
  }
  out.assign(pairs.size(), 0.0);
  for (size_t i0 = 0; i0 < h.size(); i0 += max_dots_) {
    const int cnt = (int)std::min(h.size() - i0, (size_t)max_dots_);
    HIPCHK(hipMemcpyAsync(d_dots_, h.data() + i0, sizeof(LrDot) * cnt, hipMemcpyHostToDevice,
                          st_));
    HIPCHK(launch_lr_dots(d_dots_, cnt, d_dout_, st_));
    HIPCHK(hipMemcpyAsync(out.data() + i0, d_dout_, 8 * cnt, hipMemcpyDeviceToHost, st_));
    HIPCHK(hipStreamSynchronize(st_));
  }
  return LRP_OK;
}

lrp_status Driver::round(int rows, int K, double eps, LR &out, double abs_tol) {
  out.rows = rows;
  out.ld = rows;
  if (K == 0) {
    out.r = 0;
    return LRP_OK;
  }
  int rank = 0;
  double rerr = 0.0;
  lrp_status e;
  {
    std::lock_guard<std::mutex> lock(ctx_->mu);
    e = round_random(ctx_, rows, K, panU_, panV_, pld_, eps, out.U, out.V, rows, KMAX, &rank,
                     &rerr, st_, abs_tol);
  }
  (void)rerr;
  if (e != LRP_OK) return e;
  out.r = rank;
  max_rank_ = std::max(max_rank_, out.r);
  return LRP_OK;
}

lrp_status Driver::grad(const LR &p, LR &bx, LR &by) {
  const double s = 1.0 / (4.0 * h_);
  bx.r = by.r = p.r;
  HIPCHK(launch_shift(SHIFT_G, nv_, p.r, p.U, p.ld, bx.U, bx.ld, s, st_));
  HIPCHK(launch_shift(SHIFT_H, nv_, p.r, p.V, p.ld, bx.V, bx.ld, 1.0, st_));
  HIPCHK(launch_shift(SHIFT_H, nv_, p.r, p.U, p.ld, by.U, by.ld, s, st_));
  HIPCHK(launch_shift(SHIFT_G, nv_, p.r, p.V, p.ld, by.V, by.ld, 1.0, st_));
  return LRP_OK;
}

lrp_status Driver::poisson2(const LR &a, const LR &b, double eps, LR &ya, LR &yb) {
  lrp_problem2d pr[2];
  std::memset(pr, 0, sizeof(pr));
  const LR *in[2] = {&a, &b};
  LR *out[2] = {&ya, &yb};
  for (int i = 0; i < 2; ++i) {
    pr[i].U = in[i]->U;
    pr[i].V = in[i]->V;
    pr[i].ld = std::max<long>(in[i]->ld, nv_);
    pr[i].rank = in[i]->r;
    pr[i].rmax = KMAX;
    pr[i].eps = eps;
    pr[i].Ux = out[i]->U;
    pr[i].Vx = out[i]->V;
    pr[i].ldx = out[i]->ld;
  }
  lrp_opts o;
  std::memset(&o, 0, sizeof(o));
  o.prec = P_.prec;
  o.op = LRP_OP_STOKES;
  o.max_sweeps = 20;
  lrp_status e = lrpoisson_solve2d_batch(ctx_, nv_, 2, pr, &o, st_);
  // a solve that ran out of sweeps still wrote its last approximation; the
  // recomputed Schur residual judges the outcome
  if (e == LRP_ENOCONV) e = LRP_OK;
  if (e != LRP_OK) return e;
  for (int i = 0; i < 2; ++i) out[i]->r = pr[i].rank_out;
  return LRP_OK;
}

lrp_status Driver::put_div(int &off, const LR &ya, const LR &yb, double alpha) {
  // B_x^T (4 ya) = G^T ya.U (4/(4h)) (H^T ya.V)^T, B_y^T (4 yb) likewise
  const double s = alpha / h_;
  HIPCHK(launch_shift(SHIFT_GT, n_, ya.r, ya.U, ya.ld, panU_ + (long)off * pld_, pld_, s, st_));
  HIPCHK(launch_shift(SHIFT_HT, n_, ya.r, ya.V, ya.ld, panV_ + (long)off * pld_, pld_, 1.0, st_));
  off += ya.r;
  HIPCHK(launch_shift(SHIFT_HT, n_, yb.r, yb.U, yb.ld, panU_ + (long)off * pld_, pld_, s, st_));
  HIPCHK(launch_shift(SHIFT_GT, n_, yb.r, yb.V, yb.ld, panV_ + (long)off * pld_, pld_, 1.0, st_));
  off += yb.r;
  return LRP_OK;
}

lrp_status Driver::schur(const LR &x, double eps, LR &out, double eps_solve) {
  if (x.r == 0) {
    out.r = 0;
    return LRP_OK;
  }
  LRPCHK(grad(x, ax_, ay_));
  LRPCHK(poisson2(ax_, ay_, eps_solve > 0.0 ? eps_solve : eps, yx_, yy_));
  int off = 0;
  LRPCHK(put_div(off, yx_, yy_, 1.0));
  return round(n_, off, eps, out);
}

lrp_status Driver::copy_out(const LR &x, double alpha, double *U, double *V) {
  HIPCHK(launch_copy_scaled(x.rows, x.r, x.U, x.ld, U, P_.ldx, alpha, st_));
  HIPCHK(launch_copy_scaled(x.rows, x.r, x.V, x.ld, V, P_.ldx, 1.0, st_));
  return LRP_OK;
}

lrp_status Driver::run() {
  LRPCHK(setup());
  const double eps = P_.eps;
  const double eps_in = 0.1 * eps;   // the products and sums that feed b and x
  lrp_status err;
  // ---- right-hand side b = B^T Delta^-1 f - g, g off the kernel
  LR fu, fv, g;
  fu.U = (double *)P_.fu_U;
  fu.V = (double *)P_.fu_V;
  fu.ld = P_.ld;
  fu.rows = nv_;
  fu.r = P_.rank_fu;
  fv = fu;
  fv.U = (double *)P_.fv_U;
  fv.V = (double *)P_.fv_V;
  fv.r = P_.rank_fv;
  g.U = (double *)P_.g_U;
  g.V = (double *)P_.g_V;
  g.ld = P_.ld;
  g.rows = n_;
  g.r = P_.rank_g;
  std::vector<double> kd;
  LRPCHK(dots({{&g, &one_}, {&g, &chk_}}, kd));
  const double nn = (double)n_ * (double)n_;
  LRPCHK(poisson2(fu, fv, eps_in, yx_, yy_));
  int off = 0;
  LRPCHK(put_div(off, yx_, yy_, 1.0));
  LRPCHK(put(off, g, -1.0));
  LRPCHK(put(off, one_, kd[0] / nn));
  LRPCHK(put(off, chk_, kd[1] / nn));
  LRPCHK(round(n_, off, eps_in, b_));
  const double beta0 = norm(b_, &err);
  LRPCHK(err);
  x_.r = 0;
  int its = 0, restarts = 0;
  double res = beta0;
  bool converged = beta0 == 0.0;
  std::vector<double> H((size_t)(m_ + 1) * m_), cs(m_), sn(m_), gv(m_ + 1), y(m_);
  while (!converged && its < max_iter_) {
    // residual of the current iterate
    LR *r = &b_;
    if (x_.r > 0) {
      // the residual is needed to eps_in beta0 in absolute terms
      LRPCHK(schur(x_, eps_in, t_, 0.1 * eps_in));
      off = 0;
      LRPCHK(put(off, b_, 1.0));
      LRPCHK(put(off, t_, -1.0));
      LRPCHK(round(n_, off, eps_in, r_, eps_in * beta0));
      r = &r_;
    }
    const double beta = norm(*r, &err);
    LRPCHK(err);
    if (beta <= eps * beta0) {
      res = beta;
      converged = true;
      break;
    }
    HIPCHK(launch_copy_scaled(n_, r->r, r->U, r->ld, basis_[0].U, basis_[0].ld, 1.0 / beta, st_));
    HIPCHK(launch_copy_scaled(n_, r->r, r->V, r->ld, basis_[0].V, basis_[0].ld, 1.0, st_));
    basis_[0].r = r->r;
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int J = 0;   // columns of H in use
    for (int j = 0; j < m_ && its < max_iter_; ++j) {
      // inexact products: the accuracy may fall as the residual does
      const double rj = std::fabs(gv[j]);
      const double delta = std::min(1e-2, std::max(eps_in, 0.5 * eps * beta0 / rj));
      LRPCHK(schur(basis_[j], delta, w_));
      // classical Gram-Schmidt, twice, each pass one rounded sum
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<std::pair<const LR *, const LR *>> pr;
        for (int i = 0; i <= j; ++i) pr.push_back({&w_, &basis_[i]});
        std::vector<double> hv;
        LRPCHK(dots(pr, hv));
        off = 0;
        LRPCHK(put(off, w_, 1.0));
        for (int i = 0; i <= j; ++i) {
          LRPCHK(put(off, basis_[i], -hv[i]));
          H[i + (size_t)j * (m_ + 1)] += hv[i];
        }
        LRPCHK(round(n_, off, delta, w_));
      }
      const double hn = norm(w_, &err);
      LRPCHK(err);
      H[j + 1 + (size_t)j * (m_ + 1)] = hn;
      // Givens rotations of the Hessenberg column
      for (int i = 0; i < j; ++i) {
        double &a = H[i + (size_t)j * (m_ + 1)], &b = H[i + 1 + (size_t)j * (m_ + 1)];
        const double t = cs[i] * a + sn[i] * b;
        b = -sn[i] * a + cs[i] * b;
        a = t;
      }
      double &a = H[j + (size_t)j * (m_ + 1)], &b = H[j + 1 + (size_t)j * (m_ + 1)];
      const double d = std::hypot(a, b);
      cs[j] = d > 0.0 ? a / d : 1.0;
      sn[j] = d > 0.0 ? b / d : 0.0;
      a = d;
      b = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      ++its;
      J = j + 1;
      res = std::fabs(gv[j + 1]);
      if (res <= eps * beta0 || hn == 0.0) break;
      if (j + 1 < m_) {
        HIPCHK(launch_copy_scaled(n_, w_.r, w_.U, w_.ld, basis_[j + 1].U, basis_[j + 1].ld,
                                  1.0 / hn, st_));
        HIPCHK(launch_copy_scaled(n_, w_.r, w_.V, w_.ld, basis_[j + 1].V, basis_[j + 1].ld, 1.0,
                                  st_));
        basis_[j + 1].r = w_.r;
      }
    }
    // y from the triangular system, x += sum_i y_i v_i (one rounded sum)
    for (int i = J - 1; i >= 0; --i) {
      double s = gv[i];
      for (int k = i + 1; k < J; ++k) s -= H[i + (size_t)k * (m_ + 1)] * y[k];
      const double d = H[i + (size_t)i * (m_ + 1)];
      y[i] = d != 0.0 ? s / d : 0.0;
    }
    off = 0;
    if (x_.r > 0) LRPCHK(put(off, x_, 1.0));
    for (int i = 0; i < J; ++i) LRPCHK(put(off, basis_[i], y[i]));
    LRPCHK(round(n_, off, eps_in, t_));
    std::swap(x_, t_);
    ++restarts;
    // the relaxed products and sums leave the basis orthonormal only to
    // their accuracy, so the estimate res may be optimistic: the next pass
    // of the loop recomputes the residual and restarts if it is too large
  }
  // the kernel components that the rounding let into p
  LRPCHK(dots({{&x_, &one_}, {&x_, &chk_}}, kd));
  off = 0;
  LRPCHK(put(off, x_, 1.0));
  LRPCHK(put(off, one_, -kd[0] / nn));
  LRPCHK(put(off, chk_, -kd[1] / nn));
  LRPCHK(round(n_, off, eps_in, t_));
  std::swap(x_, t_);
  // recomputed residual
  double true_res = 0.0;
  if (beta0 > 0.0) {
    LRPCHK(schur(x_, eps_in, t_, 0.1 * eps_in));
    off = 0;
    LRPCHK(put(off, b_, 1.0));
    LRPCHK(put(off, t_, -1.0));
    LRPCHK(round(n_, off, eps_in, r_, 0.1 * eps_in * beta0));
    true_res = norm(r_, &err) / beta0;
    LRPCHK(err);
  }
  // velocity: Delta^-1 (f - B p)
  LRPCHK(grad(x_, ax_, ay_));
  off = 0;
  if (fu.r > 0) LRPCHK(put(off, fu, 1.0));
  LRPCHK(put(off, ax_, -1.0));
  LRPCHK(round(nv_, off, eps_in, tu_));
  off = 0;
  if (fv.r > 0) LRPCHK(put(off, fv, 1.0));
  LRPCHK(put(off, ay_, -1.0));
  LRPCHK(round(nv_, off, eps_in, tv_));
  LRPCHK(poisson2(tu_, tv_, eps, yx_, yy_));
  P_.rank_out[0] = x_.r;
  P_.rank_out[1] = yx_.r;
  P_.rank_out[2] = yy_.r;
  P_.iterations = its;
  P_.restarts = restarts;
  P_.max_krylov_rank = max_rank_;
  P_.residual = beta0 > 0.0 ? res / beta0 : 0.0;
  P_.true_residual = true_res;
  if (x_.r > P_.rmax || yx_.r > P_.rmax || yy_.r > P_.rmax) return LRP_ERANKCAP;
  LRPCHK(copy_out(x_, 1.0, P_.p_U, P_.p_V));
  LRPCHK(copy_out(yx_, 4.0, P_.u_U, P_.u_V));
  LRPCHK(copy_out(yy_, 4.0, P_.v_U, P_.v_V));
  HIPCHK(hipStreamSynchronize(st_));
  return converged ? LRP_OK : LRP_ENOCONV;
}

}  // namespace
}  // namespace lrp

using namespace lrp;

extern "C" lrp_status lrp_stokes2d(lrp_ctx *ctx, lrp_stokes2d_problem *p, void *stream) {
  if (!ctx || !p) return LRP_EINVAL;
  const int64_t n = p->n;
  if (n < 32 || n - 1 > LRP_MAX_N) return LRP_EINVAL;
  if (!(p->eps > 0.0 && p->eps < 1.0)) return LRP_EINVAL;
  if (p->restart < 0 || p->restart > ST_MAX_RESTART || p->max_iter < 0 || p->rmax < 0)
    return LRP_EINVAL;
  const int32_t ranks[3] = {p->rank_fu, p->rank_fv, p->rank_g};
  const double *facs[3][2] = {{p->fu_U, p->fu_V}, {p->fv_U, p->fv_V}, {p->g_U, p->g_V}};
  for (int t = 0; t < 3; ++t) {
    if (ranks[t] < 0 || ranks[t] > LRP_MAX_RANK) return LRP_EINVAL;
    if (ranks[t] > 0 && (!facs[t][0] || !facs[t][1])) return LRP_EINVAL;
  }
  if (p->ld < n || p->ldx < n) return LRP_EINVAL;
  if (p->rmax > 0 && (!p->p_U || !p->p_V || !p->u_U || !p->u_V || !p->v_U || !p->v_V))
    return LRP_EINVAL;
  if (p->prec != LRP_PREC_AUTO && !transform_prec_ok(p->prec, (int)n - 1)) return LRP_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return LRP_EDEVICE;
  std::memset(p->rank_out, 0, sizeof(p->rank_out));
  p->iterations = p->restarts = p->max_krylov_rank = 0;
  p->residual = p->true_residual = 0.0;
  lrp_status e;
  {
    Driver d(ctx, *p, (hipStream_t)stream);
    e = d.run();
  }
  p->status = e;
  return e;
}
