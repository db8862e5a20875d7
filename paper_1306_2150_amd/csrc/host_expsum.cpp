// Host side of the exponential-sum comparator (Section 4.1; the device steps
// are in expsum.hip): the quadrature nodes, the slot group and the C entry.
#include "host.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace lrp {
namespace {

#define HIPCHK(x)                             \
  do {                                        \
    hipError_t e_ = (x);                      \
    if (e_ != hipSuccess) return LRP_EDEVICE; \
  } while (0)

constexpr int ES_STEPS_PER_FETCH = 8;   // steps enqueued between state fetches

// Weights and exponents of 1/x ~ sum_k w_k exp(-p_k x) on [a, b] to relative
// accuracy eps.  With p = e^t, 1/x = int_0^inf exp(-p x) dp =
// int_R exp(t - x e^t) dt; the integrand is analytic in the strip
// |Im t| < pi/2, so the trapezoidal rule t_k = t0 + k h converges
// exponentially in 1/h, and p_k = e^{t_k}, w_k = h e^{t_k}.  The tails are
// cut at eps/3 each: below t0 the integral is at most e^{t0}, relative
// x e^{t0} <= b e^{t0}; above t1 it is exp(-x e^{t1})/x, relative
// exp(-a e^{t1}).  The step is the largest of 300 evenly spaced values from
// 1.5 down to 0.05 whose rule meets eps at 4000 log-spaced points of [a, b]
// (ends included).  Returns false when no step does within ES_MAX_TERMS.
bool expsum_nodes(double a, double b, double eps, std::vector<double> &sw,
                  std::vector<double> &p) {
  const double t0 = std::log(eps / (3.0 * b));
  const double t1 = std::log(std::log(3.0 / eps) / a);
  constexpr int NPTS = 4000, NSTEP = 300;
  std::vector<double> x(NPTS);
  const double la = std::log(a), lb = std::log(b);
  for (int q = 0; q < NPTS; ++q) x[q] = std::exp(la + (lb - la) * (double)q / (NPTS - 1));
  x[0] = a;
  x[NPTS - 1] = b;
  std::vector<double> w;
  for (int s = 0; s < NSTEP; ++s) {
    const double h = 1.5 + (0.05 - 1.5) * (double)s / (NSTEP - 1);
    const int K = (int)std::ceil((t1 - t0) / h) + 1;
    if (K > ES_MAX_TERMS) return false;   // smaller steps need more terms
    p.resize(K);
    w.resize(K);
    for (int k = 0; k < K; ++k) {
      p[k] = std::exp(t0 + h * (double)k);
      w[k] = h * p[k];
    }
    bool ok = true;
    for (int q = 0; q < NPTS && ok; ++q) {
      double acc = 0.0;
      for (int k = 0; k < K; ++k) acc += w[k] * std::exp(-x[q] * p[k]);
      ok = std::fabs(x[q] * acc - 1.0) <= eps;
    }
    if (ok) {
      sw.resize(K);
      for (int k = 0; k < K; ++k) sw[k] = std::sqrt(w[k]);
      return true;
    }
  }
  return false;
}

// [2 lambda_1, 2 lambda_n]: the range of lambda_i + lambda_j on grid size n
// (lambda_k = 4/h^2 sin^2(pi k h/2), h = 1/(n+1), as the device tables)
void sum_range(int n, double *a, double *b) {
  const long double pi = 3.14159265358979323846264338327950288L;
  const long double N = (long double)(n + 1);
  const long double s1 = sinl(pi / (2.0L * N)), sn = sinl(pi * (long double)n / (2.0L * N));
  *a = (double)(2.0L * 4.0L * N * N * s1 * s1);
  *b = (double)(2.0L * 4.0L * N * N * sn * sn);
}

size_t states_bytes(int cap) { return ((size_t)cap * sizeof(ExpState) + 255) & ~(size_t)255; }

}  // namespace

// The rounding steps of slots [0, count) of g (their states uploaded): until
// every slot has left ES_RUN, ES_STEPS_PER_FETCH steps between read-backs
// of the states (a finished slot's launches exit at once).
lrp_status run_steps(ExpGroup &g, int count, hipStream_t st) {
  const int cap = g.cap, n = g.n;
  // every step appends at least min(ES_CMIN, what is left) columns
  int max_steps = 0;
  for (int i = 0; i < count; ++i)
    max_steps = std::max(max_steps, 1 + ceil_div(g.h_e[i].tot, ES_CMIN));
  const Tree tree = make_tree(n, KMAX);
  Solve2D *d_jobs = g.jobs->dev_solves();
  bool running = true;
  for (int done = 0; running && done <= max_steps; done += ES_STEPS_PER_FETCH) {
    for (int s = 0; s < ES_STEPS_PER_FETCH; ++s) {
      HIPCHK(launch_es_panel(g.d_e, d_jobs, cap, n, st));
      HIPCHK(launch_tsqr(TS_VH_TO_Q1, n, tree, d_jobs, 2 * cap, KMAX, st));
      HIPCHK(launch_core(ACT_INIT, d_jobs + cap, cap, KMAX, st));
      HIPCHK(launch_es_trunc(g.d_e, d_jobs, cap, st));
      HIPCHK(launch_es_update(g.d_e, d_jobs, cap, n, st));
    }
    HIPCHK(hipMemcpyAsync(g.h_e, g.d_e, sizeof(ExpState) * cap, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    running = false;
    for (int i = 0; i < count; ++i) running |= g.h_e[i].phase == ES_RUN;
  }
  return LRP_OK;
}

ExpGroup *expsum_group(lrp_ctx *ctx, int n, int count, lrp_status *err) {
  auto &slot = ctx->expsum_groups[n];
  if (!slot || slot->cap < count) {
    slot.reset();
    std::unique_ptr<ExpGroup> g(new ExpGroup(ctx, n, count));
    if ((*err = g->init()) != LRP_OK) return nullptr;
    slot = std::move(g);
  }
  *err = LRP_OK;
  return slot.get();
}

// Reset slot i's state and both job records for a new problem (host mirror).
static void reset_state(ExpGroup &g, int i) {
  ExpState &e = g.h_e[i];
  std::memset(&e, 0, sizeof(e));
  e.phase = ES_DONE;
  e.n = g.n;
  e.kw = std::min(KMAX, g.n);
  e.status = LRP_OK;
  Solve2D &a = g.jobs->host(i), &b = g.jobs->host(g.cap + i);
  a.active = b.active = ACT_DONE;
  a.k = b.k = 0;
  a.nonfinite = b.nonfinite = 0;
}

lrp_status round_products(lrp_ctx *ctx, int n, int count, RoundJob *jobs, hipStream_t st) {
  if (count == 0) return LRP_OK;
  if (n < ES_MIN_N_PLAIN) return LRP_EINVAL;
  lrp_status err;
  ExpGroup *gp = expsum_group(ctx, n, count, &err);
  if (!gp) return err;
  ExpGroup &g = *gp;
  for (int i = 0; i < g.cap; ++i) {
    reset_state(g, i);
    if (i >= count) continue;
    ExpState &e = g.h_e[i];
    const RoundJob &J = jobs[i];
    e.tot = J.K;
    e.eps = J.eps;
    e.pu = J.U;
    e.pv = J.V;
    e.ldp = J.ld;
    e.phase = J.K > 0 ? ES_RUN : ES_DONE;
  }
  HIPCHK(hipMemcpyAsync(g.d_e, g.h_e, sizeof(ExpState) * g.cap, hipMemcpyHostToDevice, st));
  if ((err = g.jobs->upload_all(2 * g.cap, st)) != LRP_OK) return err;
  if ((err = run_steps(g, count, st)) != LRP_OK) return err;
  for (int i = 0; i < count; ++i) {
    const ExpState &e = g.h_e[i];
    RoundJob &J = jobs[i];
    J.status = e.phase == ES_RUN ? LRP_EDEVICE : e.status;
    J.rank = (e.phase == ES_LAST && e.status == LRP_OK) ? e.K : 0;
    if (J.status == LRP_OK && e.capped) J.status = LRP_ERANKCAP;
    J.err = e.nrm > 0.0 ? e.drop / e.nrm : 0.0;
    if (J.rank > J.rmax) {
      J.status = LRP_ERANKCAP;
      continue;
    }
    if (J.rank == 0) continue;
    const Solve2D &a = g.jobs->host(i), &b = g.jobs->host(g.cap + i);
    HIPCHK(hipMemcpy2DAsync(J.Ux, (size_t)J.ldx * 8, a.A, (size_t)a.ldu * 8, (size_t)n * 8,
                            J.rank, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpy2DAsync(J.Vx, (size_t)J.ldx * 8, b.A, (size_t)b.ldu * 8, (size_t)n * 8,
                            J.rank, hipMemcpyDeviceToDevice, st));
  }
  return LRP_OK;
}

ExpGroup::ExpGroup(lrp_ctx *c, int n_, int cap_) : ctx(c), n(n_), cap(cap_) {}

ExpGroup::~ExpGroup() {
  jobs.reset();
  dev_free(ctx, d_e, bytes);
  if (h_e) (void)hipHostFree(h_e);
  if (h_nodes) (void)hipHostFree(h_nodes);
}

lrp_status ExpGroup::init() {
  jobs.reset(new Group2D(ctx, n, 2 * cap));
  lrp_status e = jobs->init();
  if (e != LRP_OK) return e;
  const size_t nodes_b = (size_t)cap * 2 * ES_MAX_TERMS * 8;
  bytes = states_bytes(cap) + nodes_b;
  void *p = nullptr;
  if ((e = dev_alloc(ctx, &p, bytes)) != LRP_OK) return e;
  d_e = (ExpState *)p;
  d_nodes = (double *)((char *)p + states_bytes(cap));
  if (hipHostMalloc((void **)&h_e, sizeof(ExpState) * cap, 0) != hipSuccess) return LRP_ENOMEM;
  if (hipHostMalloc((void **)&h_nodes, nodes_b, 0) != hipSuccess) return LRP_ENOMEM;
  std::memset(h_e, 0, sizeof(ExpState) * cap);
  std::memset(h_nodes, 0, nodes_b);
  // job records: the a side's R goes where the b side's core reads InvC
  for (int i = 0; i < cap; ++i) {
    Solve2D &a = jobs->host(i), &b = jobs->host(cap + i);
    a.Rfin = b.InvC;
    a.Q1f = b.Q1f = nullptr;
  }
  return LRP_OK;
}

}  // namespace lrp

using namespace lrp;

extern "C" lrp_status lrp_expsum_solve2d_batch(lrp_ctx *ctx, int64_t n, int32_t count,
                                               lrp_problem2d *probs, const lrp_opts *opts,
                                               void *stream) {
  if (!ctx || !probs || count < 0) return LRP_EINVAL;
  if (n < ES_MIN_N || n > LRP_MAX_N) return LRP_EINVAL;
  if (check_opts(opts) != LRP_OK) return LRP_EINVAL;
  if (opts && opts->op != LRP_OP_LAPLACE) return LRP_EINVAL;
  if (opts && opts->prec != LRP_PREC_AUTO && !transform_prec_ok(opts->prec, (int)n))
    return LRP_EINVAL;
  for (int i = 0; i < count; ++i) {
    const lrp_problem2d &p = probs[i];
    if (p.rank < 0 || p.rank > LRP_MAX_RANK) return LRP_EINVAL;
    if (!(p.eps > 0.0 && p.eps < 1.0) || p.rmax < 0) return LRP_EINVAL;
    if (p.rank > 0 && (!p.U || !p.V || p.ld < n)) return LRP_EINVAL;
    if (p.rmax > 0 && (!p.Ux || !p.Vx || p.ldx < n)) return LRP_EINVAL;
  }
  if (count == 0) return LRP_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return LRP_EDEVICE;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(ctx->mu);
  lrp_status err;
  ExpGroup *gp = expsum_group(ctx, (int)n, count, &err);
  if (!gp) return err;
  ExpGroup &g = *gp;
  Group2D &J = *g.jobs;
  const int cap = g.cap;
  // the nodes of every problem, before any device work
  double ra, rb;
  sum_range((int)n, &ra, &rb);
  std::vector<const std::vector<double> *> nodes(count);
  for (int i = 0; i < count; ++i) {
    auto it = g.node_cache.find(probs[i].eps);
    if (it == g.node_cache.end()) {
      std::vector<double> sw, p;
      if (!expsum_nodes(ra, rb, probs[i].eps, sw, p)) return LRP_EINVAL;
      sw.insert(sw.end(), p.begin(), p.end());
      it = g.node_cache.emplace(probs[i].eps, std::move(sw)).first;
    }
    nodes[i] = &it->second;
  }
  std::vector<Plan> plans(count);
  for (int i = 0; i < cap; ++i) {
    reset_state(g, i);
    ExpState &e = g.h_e[i];
    if (i >= count) continue;
    const lrp_problem2d &p = probs[i];
    plans[i] = make_plan(opts, p.eps, (int)n);
    const int R = (int)nodes[i]->size() / 2;
    double *hn = g.h_nodes + (size_t)i * 2 * ES_MAX_TERMS;
    std::memcpy(hn, nodes[i]->data(), sizeof(double) * R);
    std::memcpy(hn + ES_MAX_TERMS, nodes[i]->data() + R, sizeof(double) * R);
    e.r = p.rank;
    e.R = R;
    e.tot = R * p.rank;
    e.eps = p.eps;
    e.lam = J.tables()->lam;
    e.sw = g.d_nodes + (size_t)i * 2 * ES_MAX_TERMS;
    e.p = e.sw + ES_MAX_TERMS;
    e.phase = p.rank > 0 ? ES_RUN : ES_DONE;
    e.status = LRP_OK;
  }
  HIPCHK(hipMemcpyAsync(g.d_e, g.h_e, sizeof(ExpState) * cap, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(g.d_nodes, g.h_nodes, (size_t)cap * 2 * ES_MAX_TERMS * 8,
                        hipMemcpyHostToDevice, st));
  if ((err = J.upload_all(2 * cap, st)) != LRP_OK) return err;
  J.begin_batch();
  phase_mark(ctx, 0, st);
  for (int prec : ALL_PRECS) {
    std::vector<DstCol> cols;
    for (int i = 0; i < count; ++i) {
      const lrp_problem2d &p = probs[i];
      if (plans[i].fwd_prec != prec || p.rank == 0) continue;
      const Solve2D &a = J.host(i), &b = J.host(cap + i);
      for (int c = 0; c < p.rank; ++c)
        cols.push_back({p.U + (long)c * p.ld, a.Uh + (long)c * a.ldu, i, 0});
      for (int c = 0; c < p.rank; ++c)
        cols.push_back({p.V + (long)c * p.ld, b.Uh + (long)c * b.ldu, cap + i, 0});
    }
    if (!cols.empty() && (err = J.transform(cols, prec, st)) != LRP_OK) return err;
  }
  phase_mark(ctx, 1, st);
  if ((err = run_steps(g, count, st)) != LRP_OK) return err;
  phase_mark(ctx, 2, st);
  std::vector<int> status(count, LRP_OK), rank(count, 0);
  for (int i = 0; i < count; ++i) {
    const ExpState &e = g.h_e[i];
    if (e.phase == ES_RUN) {   // cannot happen: every step appends columns
      status[i] = LRP_EDEVICE;
      continue;
    }
    if (e.status != LRP_OK) {
      status[i] = e.status;
      continue;
    }
    rank[i] = e.phase == ES_LAST ? e.K : 0;
    if (e.capped) status[i] = LRP_ERANKCAP;
    if (rank[i] > probs[i].rmax) status[i] = LRP_ERANKCAP;
  }
  for (int prec : ALL_PRECS) {
    std::vector<DstCol> cols;
    for (int i = 0; i < count; ++i) {
      const lrp_problem2d &p = probs[i];
      if (plans[i].inv_prec != prec || rank[i] == 0 || rank[i] > p.rmax) continue;
      if (status[i] != LRP_OK && status[i] != LRP_ERANKCAP) continue;
      const Solve2D &a = J.host(i), &b = J.host(cap + i);
      for (int c = 0; c < rank[i]; ++c)
        cols.push_back({a.A + (long)c * a.ldu, p.Ux + (long)c * p.ldx, -1, 0});
      for (int c = 0; c < rank[i]; ++c)
        cols.push_back({b.A + (long)c * b.ldu, p.Vx + (long)c * p.ldx, -1, 0});
    }
    if (!cols.empty() && (err = J.transform(cols, prec, st)) != LRP_OK) return err;
  }
  phase_mark(ctx, 3, st);
  HIPCHK(hipStreamSynchronize(st));
  float us[3];
  phase_times(ctx, us);
  lrp_status first = LRP_OK;
  for (int i = 0; i < count; ++i) {
    const ExpState &e = g.h_e[i];
    lrp_problem2d &p = probs[i];
    std::memset(&p.info, 0, sizeof(p.info));
    p.rank_out = rank[i];
    p.info.status = status[i];
    p.info.sweeps = e.steps;
    p.info.k = e.R;
    p.info.rank = rank[i];
    p.info.fwd_prec = plans[i].fwd_prec;
    p.info.inv_prec = plans[i].inv_prec;
    p.info.change = -1.0;
    p.info.err_est = (e.nrm > 0.0) ? e.eps + e.drop / e.nrm : 0.0;
    for (int t = 0; t < 3; ++t) p.info.us_phase[t] = us[t];
    if (first == LRP_OK && status[i] != LRP_OK) first = (lrp_status)status[i];
  }
  return first;
}
