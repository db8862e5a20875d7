// Host runtime: context, per-grid tables, 2D slot groups, synchronous C API.
#include "host.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace lrp {

// AUTO takes the chirp-z FFT transform above this grid size (its 4096-point
// FFT costs the same at any supported n; below, the int8 GEMM is cheaper)
constexpr int FFT_AUTO_MIN_N = 2048;

#define HIPCHK(x)                         \
  do {                                    \
    hipError_t e_ = (x);                  \
    if (e_ != hipSuccess) return LRP_EDEVICE; \
  } while (0)

lrp_status dev_alloc(lrp_ctx *ctx, void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return LRP_OK;
  if (ctx->used + bytes > ctx->budget) return LRP_ENOMEM;
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    return LRP_ENOMEM;
  }
  ctx->used += bytes;
  return LRP_OK;
}

void dev_free(lrp_ctx *ctx, void *p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  ctx->used -= std::min(ctx->used, bytes);
}

double transform_flops(int prec, int n) {
  if (prec == LRP_PREC_FFT64) {
    // two halves, each a forward and an inverse 4096-point complex FFT
    return 2.0 * 2.0 * 5.0 * 4096.0 * 12.0;
  }
  // the folded transform: two half-size GEMMs of H0 = ceil(n/2), H1 = floor(n/2)
  const double h0 = (double)((n + 1) / 2), h1 = (double)(n / 2);
  return 2.0 * (h0 * h0 + h1 * h1);
}

hipError_t timed_dst(lrp_ctx *ctx, int prec, int n, const void *tab,
                     const DstCol *cols, int ncols, Solve2D *solves,
                     double *partial, size_t partial_elems, void *work,
                     size_t work_bytes, hipStream_t st) {
  if (!ctx->timing)
    return launch_dst(prec, n, tab, cols, ncols, solves, partial, partial_elems, work,
                      work_bytes, st);
  // one timing window per GEMM dispatch: the int8 transform runs one
  // dispatch per work-buffer load of columns, so it is called per load here
  int per = ncols;
  if (prec == LRP_PREC_INT8) {
    const size_t cb = dst_i8_work_bytes(n, 1);
    per = (int)std::max<size_t>(1, std::min<size_t>((size_t)ncols, work_bytes / cb));
  }
  for (int c0 = 0; c0 < ncols; c0 += per) {
    const int cnt = std::min(per, ncols - c0);
    lrp_ctx::PendingTime pt;
    hipError_t e = hipEventCreate(&pt.a);
    if (e != hipSuccess) return e;
    if ((e = hipEventCreate(&pt.b)) != hipSuccess) return e;
    // the window covers the GEMM kernel only, as a kernel trace reports it
    e = launch_dst(prec, n, tab, cols + c0, cnt, solves, partial, partial_elems, work,
                   work_bytes, st, pt.a, pt.b);
    if (e != hipSuccess) return e;
    pt.prec = prec;
    pt.cols = cnt;
    pt.flops = transform_flops(prec, n) * (double)cnt;
    ctx->pending_times.push_back(pt);
  }
  return hipSuccess;
}

static uint32_t bf16_rne_host(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}
static float bf16_float_host(uint32_t b) {
  uint32_t u = b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

size_t sine_table_bytes(int n) { return tab_layout(n).end; }

// Quarter-wave tables of sqrt(2/N) sin(pi q/N), q = 0..floor(N/2), in the
// layout launch_dst reads ([f64][f32][bf16 hi|lo][int8 records]), evaluated
// in long double and rounded once.  out: sine_table_bytes(n) bytes.
void build_sine_table(int n, char *out) {
  const int N = n + 1;
  const int Q = N / 2 + 1;
  const TabLayout L = tab_layout(n);
  std::memset(out, 0, L.end);
  dst_i8_table(n, (unsigned char *)out + L.i8);
  if (dst_fft_supported(n)) dst_fft_table(n, (double *)(out + L.fft));
  double *t64 = (double *)out;
  float *t32 = (float *)(out + L.f32);
  uint32_t *tbf = (uint32_t *)(out + L.bf2);
  uint32_t *tb3 = (uint32_t *)(out + L.bf3);   // pairs: hi | mid << 16, lo
  const long double pi = 3.14159265358979323846264338327950288L;
  const long double scale = sqrtl(2.0L / (long double)N);
  for (int q = 0; q < Q; ++q) {
    const long double v = scale * sinl(pi * (long double)q / (long double)N);
    t64[q] = (double)v;
    t32[q] = (float)v;
    const uint32_t hi = bf16_rne_host((float)v);
    const uint32_t lo = bf16_rne_host((float)(v - (long double)bf16_float_host(hi)));
    tbf[q] = hi | (lo << 16);
    // three-piece split: each piece the bfloat16 rounding of what the
    // previous pieces leave (about 24 significant bits together)
    const long double r1 = v - (long double)bf16_float_host(hi);
    const uint32_t mid = bf16_rne_host((float)r1);
    const uint32_t lo3 = bf16_rne_host((float)(r1 - (long double)bf16_float_host(mid)));
    tb3[2 * q] = hi | (mid << 16);
    tb3[2 * q + 1] = lo3;
  }
}

// The sine tables and the eigenvalues lambda_k = 4/h^2 sin^2(pi k/(2N)),
// h = 1/N, N = n+1 (long double, rounded once) of grid size n.
const GridTables *get_tables(lrp_ctx *ctx, int n, lrp_status *err) {
  *err = LRP_OK;
  auto it = ctx->tables.find(n);
  if (it != ctx->tables.end()) return &it->second;
  const int N = n + 1;
  const size_t tab_bytes = sine_table_bytes(n);
  std::vector<char> host(tab_bytes, 0);
  build_sine_table(n, host.data());
  const long double pi = 3.14159265358979323846264338327950288L;
  // lambda_k, then the Stokes operator's factors 2 sin^2 / h and 2 cos^2 / h
  // of the half angle pi k/(2N) (cos^2 as sin^2 of the complementary angle)
  std::vector<double> lam(3 * (size_t)n);
  const long double N2 = (long double)N * (long double)N;
  for (int k = 1; k <= n; ++k) {
    const long double s = sinl(pi * (long double)k / (2.0L * (long double)N));
    const long double c = sinl(pi * (long double)(N - k) / (2.0L * (long double)N));
    lam[k - 1] = (double)(4.0L * N2 * s * s);
    lam[n + k - 1] = (double)(2.0L * (long double)N * s * s);
    lam[2 * n + k - 1] = (double)(2.0L * (long double)N * c * c);
  }
  GridTables g;
  g.n = n;
  g.bytes = tab_bytes + (size_t)n * 24;
  void *p = nullptr;
  *err = dev_alloc(ctx, &p, g.bytes);
  if (*err != LRP_OK) return nullptr;
  g.tab = p;
  g.lam = (double *)((char *)p + tab_bytes);
  g.sp = g.lam + n;
  g.sq = g.lam + 2 * (size_t)n;
  if (hipMemcpy(g.tab, host.data(), tab_bytes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(g.lam, lam.data(), (size_t)n * 24, hipMemcpyHostToDevice) != hipSuccess) {
    dev_free(ctx, p, g.bytes);
    *err = LRP_EDEVICE;
    return nullptr;
  }
  auto res = ctx->tables.emplace(n, g);
  return &res.first->second;
}

Plan make_plan(const lrp_opts *o, double eps, int n) {
  Plan p;
  int prec = o ? o->prec : LRP_PREC_FP64;
  p.max_sweeps = (o && o->max_sweeps > 0) ? o->max_sweeps : 10;
  p.kcap = (o && o->rank_cap > 0) ? std::min(o->rank_cap, KMAX) : KMAX;
  p.kcap = std::min(p.kcap, n);
  p.kick = (o && o->kick > 0) ? std::min(o->kick, 16) : 8;
  p.min_slack = std::max(1, p.kick / 2);
  p.tau = (o && o->maxvol_tau > 1.0) ? o->maxvol_tau : 1.05;
  p.op = o ? o->op : LRP_OP_LAPLACE;
  p.k0 = o ? o->k0 : 0;
  p.seed = o ? o->seed : 0;
  if (prec == LRP_PREC_AUTO) {
    if (dst_fft_supported(n) && n > FFT_AUTO_MIN_N) {
      // float64 chirp-z FFT: the fewest operations and float64 accuracy
      p.fwd_prec = p.inv_prec = LRP_PREC_FFT64;
    } else if (dst_i8_supported(n)) {
      // exact int8 slices: about 1e-12, faster than the float64 and float32
      // transforms wherever the sine record table fits in LDS
      p.fwd_prec = p.inv_prec = LRP_PREC_INT8;
    } else {
      // the inverse transform's relative error reaches the result undamped;
      // the forward one is damped by the eigenvalue division, not enough
      // for 10 eps below 1e-7
      p.fwd_prec = eps >= 1e-6 ? LRP_PREC_BF16X3 : (eps >= 1e-7 ? LRP_PREC_FP32 : LRP_PREC_FP64);
      p.inv_prec = eps >= 1e-7 ? LRP_PREC_FP32 : LRP_PREC_FP64;
    }
  } else if (prec == LRP_PREC_FP32 || prec == LRP_PREC_BF16X3 || prec == LRP_PREC_INT8 ||
             prec == LRP_PREC_FFT64 || prec == LRP_PREC_BF16X6) {
    // INT8 / FFT64 callers check dst_i8_supported(n) / dst_fft_supported(n)
    p.fwd_prec = p.inv_prec = prec;
  } else {
    p.fwd_prec = p.inv_prec = LRP_PREC_FP64;
  }
  return p;
}

bool transform_prec_ok(int prec, int n) {
  switch (prec) {
    case LRP_PREC_FP64:
    case LRP_PREC_FP32:
    case LRP_PREC_BF16X3:
    case LRP_PREC_BF16X6: return true;
    case LRP_PREC_INT8: return dst_i8_supported(n);
    case LRP_PREC_FFT64: return dst_fft_supported(n);
    default: return false;
  }
}

lrp_status check_opts(const lrp_opts *o) {
  if (!o) return LRP_OK;
  if (o->prec < 0 || o->prec > LRP_PREC_BF16X6) return LRP_EINVAL;
  if (o->max_sweeps < 0 || o->max_sweeps > LRP_MAX_SWEEPS) return LRP_EINVAL;
  if (o->rank_cap < 0 || o->kick < 0 || o->maxvol_tau < 0.0) return LRP_EINVAL;
  if (o->op != LRP_OP_LAPLACE && o->op != LRP_OP_STOKES) return LRP_EINVAL;
  if (o->k0 < 0) return LRP_EINVAL;
  return LRP_OK;
}

void phase_mark(lrp_ctx *ctx, int i, hipStream_t st) {
  if (!ctx->phase_ev[i] && hipEventCreate(&ctx->phase_ev[i]) != hipSuccess) {
    ctx->phase_ev[i] = nullptr;
    return;
  }
  (void)hipEventRecord(ctx->phase_ev[i], st);
}

void phase_times(lrp_ctx *ctx, float us[3]) {
  for (int i = 0; i < 3; ++i) {
    float ms = 0.f;
    if (ctx->phase_ev[i] && ctx->phase_ev[i + 1] &&
        hipEventElapsedTime(&ms, ctx->phase_ev[i], ctx->phase_ev[i + 1]) == hipSuccess)
      us[i] = 1000.f * ms;
    else
      us[i] = 0.f;
  }
}

// ------------------------------------------------------------- Group2D
struct Layout {
  size_t off_Uh, off_Vh, off_upan, off_vpan, off_cpan, off_treeR, off_treeH,
      off_treeTau, off_treeY, off_small, off_part, off_mvval, off_ints, off_qf, total;
};

static size_t tree_nodes(const Tree &t, int from) {
  size_t s = 0;
  for (int l = from; l < t.nlev; ++l) s += t.nb[l];
  return s;
}

// Per-slot workspace: row-side panels (n rows: Uh, Q0, A, Ap), column-side
// panels (m rows: Vh, Q1, B, Bp), shared panels (max(n, m) rows: C, Hv),
// the TSQR / tournament tree over max(n, m) rows, small matrices, partial
// sums and index sets.
static Layout slot_layout(int n, int m, const Tree &t) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o += (bytes + 255) & ~(size_t)255;
    return r;
  };
  const size_t nb0 = t.nb[0];
  const size_t mx = std::max(n, m);
  L.off_Uh = take((size_t)n * KMAX * 8);
  L.off_Vh = take((size_t)m * KMAX * 8);
  L.off_upan = take((size_t)3 * n * KMAX * 8);
  L.off_vpan = take((size_t)3 * m * KMAX * 8);
  L.off_cpan = take((size_t)2 * mx * KMAX * 8);
  L.off_treeR = take(tree_nodes(t, 0) * KMAX * KMAX * 8);
  L.off_treeH = take(std::max<size_t>(1, tree_nodes(t, 1)) * PANEL_M * KMAX * 8);
  L.off_treeTau = take(tree_nodes(t, 0) * KMAX * 8);
  L.off_treeY = take(tree_nodes(t, 0) * KMAX * KMAX * 8);
  L.off_small = take((size_t)(7 * KMAX * KMAX + 2 * KMAX) * 8);
  L.off_part = take(std::max<size_t>((size_t)change_blocks(m) * KMAX * KMAX, 2 * nb0) * 8);
  L.off_mvval = take(nb0 * BLOCK_TOP * 8);
  L.off_ints = take((tree_nodes(t, 0) * KMAX + nb0 * BLOCK_TOP + 4 * KMAX) * 4);
  L.off_qf = take((size_t)(n + m) * KMAX * 4);
  L.total = o;
  return L;
}

size_t cross_slot_bytes(int n, int m) {
  return slot_layout(n, m, make_tree(std::max(n, m), KMAX)).total;
}

Group2D::Group2D(lrp_ctx *ctx, int n, int cap, int m, const double *const *col)
    : ctx_(ctx), n_(n), cap_(cap), m_(m > 0 ? m : n) {
  if (col)
    for (int t = 0; t < 3; ++t) col_[t] = col[t];
}

Group2D::~Group2D() {
  if (stream_) {
    (void)hipStreamSynchronize(stream_);
    (void)hipStreamDestroy(stream_);
  }
  for (auto &kv : graphs_) (void)hipGraphExecDestroy(kv.second);
  dev_free(ctx_, ws_, bytes_);
  dev_free(ctx_, d_work_, work_bytes_);
  if (h_s_) (void)hipHostFree(h_s_);
  if (h_cols_) (void)hipHostFree(h_cols_);
}

hipStream_t Group2D::stream() {
  if (!stream_ && hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking) != hipSuccess)
    stream_ = nullptr;
  return stream_;
}

lrp_status Group2D::init() {
  lrp_status err;
  tabs_ = get_tables(ctx_, n_, &err);
  if (!tabs_) return err;
  talloc_ = make_tree(std::max(n_, m_), KMAX);
  const Layout L = slot_layout(n_, m_, talloc_);
  per_slot_ = L.total;
  cols_cap_ = cap_ * 4 * KMAX;   // forward and inverse columns of one tick
  partial_elems_ = dst_partial_elems(n_, std::min(cols_cap_, 4 * KMAX));
  const size_t solves_b = ((size_t)cap_ * sizeof(Solve2D) + 255) & ~(size_t)255;
  const size_t cols_b = ((size_t)cols_cap_ * sizeof(DstCol) + 255) & ~(size_t)255;
  const size_t part_b = partial_elems_ * 8;
  bytes_ = per_slot_ * cap_ + solves_b + cols_b + part_b;
  void *p = nullptr;
  err = dev_alloc(ctx_, &p, bytes_);
  if (err != LRP_OK) return err;
  ws_ = (char *)p;
  d_s_ = (Solve2D *)(ws_ + per_slot_ * cap_);
  d_cols_ = (DstCol *)((char *)d_s_ + solves_b);
  d_partial_ = (double *)((char *)d_cols_ + cols_b);
  if (hipHostMalloc((void **)&h_s_, sizeof(Solve2D) * cap_, 0) != hipSuccess) return LRP_ENOMEM;
  if (hipHostMalloc((void **)&h_cols_, sizeof(DstCol) * cols_cap_, 0) != hipSuccess) return LRP_ENOMEM;
  std::memset(h_s_, 0, sizeof(Solve2D) * cap_);
  plans_.resize(cap_);
  kin_.assign(cap_, 0);
  for (int i = cap_ - 1; i >= 0; --i) free_slots.push_back(i);
  // carve fixed pointers of every slot once
  const size_t mx = std::max(n_, m_);
  for (int i = 0; i < cap_; ++i) {
    Solve2D &s = h_s_[i];
    char *b = ws_ + per_slot_ * i;
    s.n = n_;
    s.m = m_;
    s.ldu = n_;
    s.ldv = m_;
    s.ldc = (long)mx;
    s.lam_r = tabs_->lam;
    s.lam_c = col_[0] ? col_[0] : tabs_->lam;
    s.lq_r = s.lq_c = nullptr;
    s.Uh = (double *)(b + L.off_Uh);
    s.Vh = (double *)(b + L.off_Vh);
    double *up = (double *)(b + L.off_upan);
    double *vp = (double *)(b + L.off_vpan);
    double *cp = (double *)(b + L.off_cpan);
    const size_t nk = (size_t)n_ * KMAX, mk = (size_t)m_ * KMAX, ck = mx * KMAX;
    s.Q0 = up;
    s.A = up + nk;
    s.Ap = up + 2 * nk;
    s.Q1 = vp;
    s.Q0f = (float *)(b + L.off_qf);
    s.Q1f = s.Q0f + nk;
    s.B = vp + mk;
    s.Bp = vp + 2 * mk;
    s.C = cp;
    s.Hv = cp + ck;
    s.tree_R = (double *)(b + L.off_treeR);
    s.tree_H = (double *)(b + L.off_treeH);
    s.tree_tau = (double *)(b + L.off_treeTau);
    s.tree_Y = (double *)(b + L.off_treeY);
    double *sm = (double *)(b + L.off_small);
    const size_t k2 = (size_t)KMAX * KMAX;
    s.Rfin = sm;
    s.Inv = sm + k2;
    s.InvC = sm + 2 * k2;
    s.W = sm + 3 * k2;
    s.Z = sm + 4 * k2;
    s.Mc = sm + 5 * k2;
    s.sig = sm + 7 * k2;
    s.sigp = sm + 7 * k2 + KMAX;
    s.part = (double *)(b + L.off_part);
    s.mv_val = (double *)(b + L.off_mvval);
    int *ip = (int *)(b + L.off_ints);
    s.tree_piv = ip;
    ip += tree_nodes(talloc_, 0) * KMAX;
    s.mv_row = ip;
    ip += (size_t)talloc_.nb[0] * BLOCK_TOP;
    s.I = ip;
    s.J = ip + KMAX;
    s.Jn = ip + 2 * KMAX;
    s.probe = ip + 3 * KMAX;
    s.active = ACT_DONE;
  }
  HIPCHK(hipMemcpy(d_s_, h_s_, sizeof(Solve2D) * cap_, hipMemcpyHostToDevice));
  return LRP_OK;
}

void Group2D::setup_slot(int i, const double *U, const double *V, long ld, int r,
                         double eps, double *Ux, double *Vx, long ldx, int rmax,
                         const Plan &plan) {
  Solve2D &s = h_s_[i];
  plans_[i] = plan;
  s.n = n_;
  s.r = r;
  s.kick = plan.kick;
  s.max_sweeps = plan.max_sweeps;
  s.min_slack = plan.min_slack;
  s.rmax = rmax;
  s.eps = eps;
  s.tau = plan.tau;
  s.U = U;
  s.V = V;
  s.ld = ld;
  s.Ux = Ux;
  s.Vx = Vx;
  s.ldx = ldx;
  // the operator's eigenvalue tables (Solve2D: D_ij from lam and lq)
  if (plan.op == LRP_OP_STOKES) {
    s.lam_r = tabs_->sp;
    s.lq_r = tabs_->sq;
    s.lam_c = col_[0] ? col_[1] : tabs_->sp;
    s.lq_c = col_[0] ? col_[2] : tabs_->sq;
  } else {
    s.lam_r = tabs_->lam;
    s.lq_r = nullptr;
    s.lam_c = col_[0] ? col_[0] : tabs_->lam;
    s.lq_c = nullptr;
  }
  s.off_r = (int)(plan.seed % (uint64_t)n_);
  s.off_c = (int)(plan.seed % (uint64_t)m_);
  // reset pointer roles that a previous occupant may have swapped
  double *lo = std::min(s.A, s.Ap), *hi = std::max(s.A, s.Ap);
  s.A = lo;
  s.Ap = hi;
  lo = std::min(s.B, s.Bp);
  hi = std::max(s.B, s.Bp);
  s.B = lo;
  s.Bp = hi;
  lo = std::min(s.sig, s.sigp);
  hi = std::max(s.sig, s.sigp);
  s.sig = lo;
  s.sigp = hi;
  s.kcap = std::min(plan.kcap, std::min(n_, m_));
  const int k0 = std::min(plan.k0 > 0 ? plan.k0 : r + plan.kick, s.kcap);
  s.k0 = k0;
  s.k = std::min(r, k0);   // columns of the initial maxvol on Vh
  kin_[i] = s.k;
  s.kp = 0;
  s.R = 0;
  s.sweep = 0;
  s.next = NEXT_CONTINUE;
  s.status = LRP_OK;
  s.nonfinite = 0;
  s.mv_done = 0;
  s.mv_swaps = 0;
  s.kgrow = 0;
  s.nrm = 0.0;
  s.change = -1.0;
  s.tail = -1.0;
  s.active = (r > 0) ? ACT_INIT : ACT_DONE;
}

lrp_status Group2D::upload_slot(int i, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(d_s_ + i, h_s_ + i, sizeof(Solve2D), hipMemcpyHostToDevice, st));
  return LRP_OK;
}

lrp_status Group2D::upload_all(int count, hipStream_t st) {
  HIPCHK(hipMemcpyAsync(d_s_, h_s_, sizeof(Solve2D) * count, hipMemcpyHostToDevice, st));
  return LRP_OK;
}

lrp_status Group2D::dst_cols(std::vector<DstCol> &cols, int prec, hipStream_t st) {
  if (prec == LRP_PREC_INT8 && !d_work_) {
    const size_t wb = dst_i8_work_bytes(n_, dst_i8_work_cols(n_, cols_cap_));
    lrp_status e = dev_alloc(ctx_, &d_work_, wb);
    if (e != LRP_OK) return e;
    work_bytes_ = wb;
  }
  size_t done = 0;
  while (done < cols.size()) {
    const int cnt = (int)std::min(cols.size() - done, (size_t)cols_cap_);
    // the staging ring is reused only after the stream drained it
    if (cols_used_ + cnt > cols_cap_) {
      HIPCHK(hipStreamSynchronize(st));
      cols_used_ = 0;
    }
    DstCol *h = h_cols_ + cols_used_, *d = d_cols_ + cols_used_;
    std::memcpy(h, cols.data() + done, sizeof(DstCol) * cnt);
    HIPCHK(hipMemcpyAsync(d, h, sizeof(DstCol) * cnt, hipMemcpyHostToDevice, st));
    HIPCHK(timed_dst(ctx_, prec, n_, tabs_->tab, d, cnt, d_s_, d_partial_,
                     partial_elems_, d_work_, work_bytes_, st));
    cols_used_ += cnt;
    done += cnt;
  }
  return LRP_OK;
}

lrp_status Group2D::forward(const std::vector<int> &slots, hipStream_t st) {
  for (int prec : ALL_PRECS) {
    std::vector<DstCol> cols;
    for (int i : slots) {
      const Solve2D &s = h_s_[i];
      if (plans_[i].fwd_prec != prec || s.r == 0) continue;
      for (int c = 0; c < s.r; ++c) cols.push_back({s.U + (long)c * s.ld, s.Uh + (long)c * s.ldu, i, 0});
      for (int c = 0; c < s.r; ++c) cols.push_back({s.V + (long)c * s.ld, s.Vh + (long)c * s.ldv, i, 0});
    }
    if (!cols.empty()) {
      lrp_status e = dst_cols(cols, prec, st);
      if (e != LRP_OK) return e;
    }
  }
  return LRP_OK;
}

uint64_t Group2D::StepPlan::key() const {
  // hi < 2^24; the three rank buckets in 2 bits each, the mask in 4
  const auto b2 = [](int k) { return (uint64_t)(rank_bucket(std::max(k, 1)) / 16 - 1); };
  return (uint64_t)hi | (b2(kin) << 24) | (b2(km) << 26) | (b2(kev) << 28) |
         ((uint64_t)bmask << 30) | ((uint64_t)init << 34) | ((uint64_t)sweep << 35);
}

lrp_status Group2D::launch_step(const StepPlan &p, hipStream_t st) {
  // trees depend on the shape only, so a slot's arithmetic does not depend
  // on which other slots share the launch
  const Tree tn = make_tree(n_, KMAX), tm = make_tree(m_, KMAX);
  const int hi = p.hi;
  if (p.init) {
    HIPCHK(launch_tsqr(TS_VH_TO_Q1, m_, tm, d_s_, hi, p.kin, st));
    HIPCHK(launch_maxvol(MV_Q1_TO_J, m_, tm, d_s_, hi, p.kin, st));
    HIPCHK(launch_init_J(d_s_, hi, st));
  }
  // k of a slot only grows at the end of a sweep, so kmax and the buckets
  // hold for this sweep: the kernels with many workgroups per slot run once
  // per occupied bucket, on its slots, the rest once at the largest
  HIPCHK(launch_tsqr(TS_C_TO_Q0, n_, tn, d_s_, hi, p.km, st, p.bmask));
  HIPCHK(launch_maxvol(MV_Q0_TO_I, n_, tn, d_s_, hi, p.km, st, p.bmask));
  HIPCHK(launch_tsqr(TS_C_TO_Q1, m_, tm, d_s_, hi, p.km, st, p.bmask));
  HIPCHK(launch_maxvol(MV_Q1_TO_JN, m_, tm, d_s_, hi, p.km, st, p.bmask));
  HIPCHK(launch_core(ACT_SWEEP, d_s_, hi, p.km, st));
  for (int kb = 16; kb <= 64; kb += 16) {
    if (!(p.bmask & bucket_bit(kb))) continue;
    HIPCHK(launch_factors(n_, m_, d_s_, hi, kb, st));
    HIPCHK(launch_change(n_, m_, d_s_, hi, kb, st));
  }
  HIPCHK(launch_decide(n_, m_, d_s_, hi, p.kev, st));
  return LRP_OK;
}

// Graphs kept per group; a plan beyond them runs as plain launches.
constexpr size_t GRAPH_CACHE = 64;

lrp_status Group2D::step(hipStream_t st) {
  StepPlan p{0, 0, 0, 0, 0u, false, false};
  int kmax = 0, rmax = 0;
  int live = 0;   // launches cover slots [0, hi): the live ones
  for (int i = 0; i < cap_; ++i) {
    const Solve2D &s = h_s_[i];
    if (s.active != ACT_DONE) live = i + 1;
    if (s.active == ACT_INIT) {
      p.init = true;
      p.kin = std::max(p.kin, s.k);
      kmax = std::max(kmax, s.k0);
      rmax = std::max(rmax, s.r);
      p.bmask |= bucket_bit(s.k0);   // k_init_J sets k = k0
    } else if (s.active == ACT_SWEEP) {
      p.sweep = true;
      kmax = std::max(kmax, s.k);
      rmax = std::max(rmax, s.r);
      p.bmask |= bucket_bit(s.k);
    }
  }
  if (!p.init && !p.sweep) return LRP_OK;
  p.km = std::max(kmax, 1);
  p.kev = std::max(p.km, rmax);
  if (!ctx_->graphs) {
    p.hi = live;
    return launch_step(p, st);
  }
  // Replayed: the launches cover the live slots rounded up to a power of
  // two (finished and unused slots return at once), so that a few graphs
  // serve every step of a batch.  Every slot of [0, cap) holds a valid
  // state (init uploads them all as finished).
  int hi = 1;
  while (hi < live) hi *= 2;
  p.hi = std::min(hi, cap_);
  auto it = graphs_.find(p.key());
  if (it == graphs_.end()) {
    if (graphs_.size() >= GRAPH_CACHE) return launch_step(p, st);
    hipStream_t gs = stream();
    if (!gs) return LRP_EDEVICE;
    HIPCHK(maxvol_prepare());   // no host-side attribute calls inside a capture
    hipGraph_t gr = nullptr;
    HIPCHK(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
    const lrp_status e = launch_step(p, gs);
    const hipError_t ce = hipStreamEndCapture(gs, &gr);
    if (e != LRP_OK || ce != hipSuccess) {
      if (gr) (void)hipGraphDestroy(gr);
      return e != LRP_OK ? e : LRP_EDEVICE;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (ie != hipSuccess) return LRP_EDEVICE;
    it = graphs_.emplace(p.key(), ex).first;
  }
  // captured on the group's own stream (capture needs one that is not the
  // legacy default stream), replayed on the caller's
  HIPCHK(hipGraphLaunch(it->second, st));
  return LRP_OK;
}

lrp_status Group2D::fetch(hipStream_t st, bool sync) {
  HIPCHK(hipMemcpyAsync(h_s_, d_s_, sizeof(Solve2D) * cap_, hipMemcpyDeviceToHost, st));
  if (sync) HIPCHK(hipStreamSynchronize(st));
  return LRP_OK;
}

lrp_status Group2D::inverse(const std::vector<int> &slots, hipStream_t st) {
  for (int prec : ALL_PRECS) {
    std::vector<DstCol> cols;
    for (int i : slots) {
      const Solve2D &s = h_s_[i];
      if (plans_[i].inv_prec != prec) continue;
      for (int c = 0; c < s.R; ++c) cols.push_back({s.A + (long)c * s.ldu, s.Ux + (long)c * s.ldx, -1, 0});
      for (int c = 0; c < s.R; ++c) cols.push_back({s.B + (long)c * s.ldv, s.Vx + (long)c * s.ldx, -1, 0});
    }
    if (!cols.empty()) {
      lrp_status e = dst_cols(cols, prec, st);
      if (e != LRP_OK) return e;
    }
  }
  return LRP_OK;
}

void fill_info2d(const Solve2D &s, const Plan &plan, lrp_info *info) {
  info->status = s.status;
  info->sweeps = s.sweep;
  info->k = s.k;
  info->rank = s.R;
  info->fwd_prec = plan.fwd_prec;
  info->inv_prec = plan.inv_prec;
  info->change = s.change;
  // truncation tail plus the last change between sweeps
  info->err_est = (s.tail >= 0.0) ? s.tail + (s.change >= 0.0 ? s.change : 0.0) : -1.0;
  if (s.r == 0 || s.nrm == 0.0) info->err_est = 0.0;
}

}  // namespace lrp

using namespace lrp;

// ---------------------------------------------------------------- C API
extern "C" {

const char *lrp_strerror(int32_t s) {
  switch (s) {
    case LRP_OK: return "ok";
    case LRP_EINVAL: return "invalid argument";
    case LRP_ENONFINITE: return "right-hand side holds Inf or NaN";
    case LRP_ERANKCAP: return "rank cap reached";
    case LRP_ENOCONV: return "cross sweeps did not converge";
    case LRP_ENOMEM: return "out of device memory budget";
    case LRP_EDEVICE: return "HIP runtime error";
    case LRP_EBUSY: return "busy";
    case LRP_ENOTREADY: return "not ready";
    default: return "unknown status";
  }
}

lrp_status lrp_create(lrp_ctx **ctx, int device, size_t workspace_bytes) {
  if (!ctx) return LRP_EINVAL;
  *ctx = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return LRP_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return LRP_EDEVICE;
  lrp_ctx *c = new lrp_ctx();
  c->device = device;
  c->budget = workspace_bytes ? workspace_bytes : ((size_t)32 << 30);
  *ctx = c;
  return LRP_OK;
}

lrp_status lrp_sine_transform(lrp_ctx *ctx, int64_t n, int32_t ncols,
                              const double *src, int64_t lds, double *dst,
                              int64_t ldd, int32_t prec, void *stream) {
  if (!ctx || n < 1 || n > LRP_MAX_N || ncols < 0) return LRP_EINVAL;
  if (!transform_prec_ok(prec, (int)n)) return LRP_EINVAL;
  if (ncols == 0) return LRP_OK;
  if (!src || !dst || lds < n || ldd < n) return LRP_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return LRP_EDEVICE;
  std::lock_guard<std::mutex> lock(ctx->mu);
  lrp_status err;
  const GridTables *t = get_tables(ctx, (int)n, &err);
  if (!t) return err;
  hipStream_t st = (hipStream_t)stream;
  const int chunk = 1024;
  const size_t pe = dst_partial_elems((int)n, 64);
  if (ctx->tx_cap < chunk || ctx->tx_partial_elems < pe) {
    if (ctx->tx_dcols) dev_free(ctx, ctx->tx_dcols, ctx->tx_bytes);
    if (ctx->tx_hcols) (void)hipHostFree(ctx->tx_hcols);
    ctx->tx_dcols = nullptr;
    ctx->tx_hcols = nullptr;
    ctx->tx_cap = 0;
    const size_t cb = ((size_t)chunk * sizeof(DstCol) + 255) & ~(size_t)255;
    void *p = nullptr;
    if ((err = dev_alloc(ctx, &p, cb + pe * 8)) != LRP_OK) return err;
    ctx->tx_bytes = cb + pe * 8;
    ctx->tx_dcols = (DstCol *)p;
    ctx->tx_partial = (double *)((char *)p + cb);
    ctx->tx_partial_elems = pe;
    if (hipHostMalloc((void **)&ctx->tx_hcols, sizeof(DstCol) * chunk, 0) != hipSuccess)
      return LRP_ENOMEM;
    ctx->tx_cap = chunk;
  }
  if (prec == LRP_PREC_INT8 && !ctx->tx_work) {
    const size_t wb = dst_i8_work_bytes((int)n, chunk);
    if ((err = dev_alloc(ctx, &ctx->tx_work, wb)) != LRP_OK) return err;
    ctx->tx_work_bytes = wb;
  }
  if (prec == LRP_PREC_INT8 && ctx->tx_work_bytes < dst_i8_work_bytes((int)n, chunk)) {
    dev_free(ctx, ctx->tx_work, ctx->tx_work_bytes);
    ctx->tx_work = nullptr;
    ctx->tx_work_bytes = 0;
    const size_t wb = dst_i8_work_bytes((int)n, chunk);
    if ((err = dev_alloc(ctx, &ctx->tx_work, wb)) != LRP_OK) return err;
    ctx->tx_work_bytes = wb;
  }
  for (int c0 = 0; c0 < ncols; c0 += chunk) {
    const int cnt = std::min(chunk, ncols - c0);
    if (hipStreamSynchronize(st) != hipSuccess) return LRP_EDEVICE;
    for (int c = 0; c < cnt; ++c)
      ctx->tx_hcols[c] = {src + (long)(c0 + c) * lds, dst + (long)(c0 + c) * ldd, -1, 0};
    if (hipMemcpyAsync(ctx->tx_dcols, ctx->tx_hcols, sizeof(DstCol) * cnt,
                       hipMemcpyHostToDevice, st) != hipSuccess)
      return LRP_EDEVICE;
    if (timed_dst(ctx, prec, (int)n, t->tab, ctx->tx_dcols, cnt, nullptr,
                  ctx->tx_partial, ctx->tx_partial_elems, ctx->tx_work, ctx->tx_work_bytes,
                  st) != hipSuccess)
      return LRP_EDEVICE;
  }
  // the staging buffers belong to the context: the call returns after its
  // work completed, so that a call on another stream may reuse them
  if (hipStreamSynchronize(st) != hipSuccess) return LRP_EDEVICE;
  return LRP_OK;
}

lrp_status lrp_set_kernel_timing(lrp_ctx *ctx, int32_t enable) {
  if (!ctx) return LRP_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  ctx->timing = enable != 0;
  return LRP_OK;
}

lrp_status lrp_set_graph_replay(lrp_ctx *ctx, int32_t enable) {
  if (!ctx) return LRP_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  ctx->graphs = enable != 0;
  return LRP_OK;
}

lrp_status lrp_kernel_stats(lrp_ctx *ctx, int32_t prec, lrp_kernel_stat *out,
                            int32_t reset) {
  if (!ctx || prec < 0 || prec > LRP_PREC_BF16X6 || prec == LRP_PREC_AUTO) return LRP_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  if (hipSetDevice(ctx->device) != hipSuccess) return LRP_EDEVICE;
  for (auto &pt : ctx->pending_times) {
    if (hipEventSynchronize(pt.b) != hipSuccess) return LRP_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pt.a, pt.b) != hipSuccess) return LRP_EDEVICE;
    lrp_kernel_stat &k = ctx->kstat[pt.prec];
    k.launches += 1;
    k.columns += pt.cols;
    k.ms += ms;
    k.flops += pt.flops;
    (void)hipEventDestroy(pt.a);
    (void)hipEventDestroy(pt.b);
  }
  ctx->pending_times.clear();
  if (out) *out = ctx->kstat[prec];
  if (reset) ctx->kstat[prec] = lrp_kernel_stat{};
  return LRP_OK;
}

lrp_status lrp_destroy(lrp_ctx *ctx) {
  if (!ctx) return LRP_EINVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->tx_dcols) dev_free(ctx, ctx->tx_dcols, ctx->tx_bytes);
  if (ctx->tx_hcols) (void)hipHostFree(ctx->tx_hcols);
  if (ctx->tx_work) dev_free(ctx, ctx->tx_work, ctx->tx_work_bytes);
  ctx->batch_groups.clear();
  ctx->batch3_groups.clear();
  ctx->expsum_groups.clear();
  ctx->kernel_groups.clear();
  ctx->round_groups.clear();
  ctx->serve_groups.clear();
  ctx->serve3_groups.clear();
  for (auto &kv : ctx->tables) dev_free(ctx, kv.second.tab, kv.second.bytes);
  if (ctx->serve_stream) (void)hipStreamDestroy(ctx->serve_stream);
  for (hipEvent_t e : ctx->phase_ev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
  return LRP_OK;
}

static lrp_status check_problem(int64_t n, const lrp_problem2d &p) {
  if (p.rank < 0 || p.rank > LRP_MAX_RANK) return LRP_EINVAL;
  if (!(p.eps > 0.0 && p.eps < 1.0)) return LRP_EINVAL;
  if (p.rmax < 0) return LRP_EINVAL;
  if (p.rank > 0 && (!p.U || !p.V || p.ld < n)) return LRP_EINVAL;
  if (p.rmax > 0 && (!p.Ux || !p.Vx || p.ldx < n)) return LRP_EINVAL;
  return LRP_OK;
}

lrp_status lrpoisson_solve2d_batch(lrp_ctx *ctx, int64_t n, int32_t count,
                                   lrp_problem2d *probs, const lrp_opts *opts,
                                   void *stream) {
  if (!ctx || !probs || count < 0) return LRP_EINVAL;
  if (n < 1 || n > LRP_MAX_N) return LRP_EINVAL;
  if (check_opts(opts) != LRP_OK) return LRP_EINVAL;
  if (opts && opts->prec != LRP_PREC_AUTO && !transform_prec_ok(opts->prec, (int)n))
    return LRP_EINVAL;
  for (int i = 0; i < count; ++i) {
    lrp_status e = check_problem(n, probs[i]);
    if (e != LRP_OK) return e;
  }
  if (count == 0) return LRP_OK;
  if (hipSetDevice(ctx->device) != hipSuccess) return LRP_EDEVICE;
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(ctx->mu);
  auto &slot = ctx->batch_groups[(int)n];
  if (!slot || slot->cap() < count) {
    slot.reset();
    std::unique_ptr<Group2D> g(new Group2D(ctx, (int)n, count));
    lrp_status e = g->init();
    if (e != LRP_OK) return e;
    slot = std::move(g);
  }
  Group2D &g = *slot;
  g.begin_batch();
  std::vector<int> all;
  for (int i = 0; i < g.cap(); ++i) {
    if (i < count) {
      const lrp_problem2d &p = probs[i];
      const Plan plan = make_plan(opts, p.eps, (int)n);
      g.setup_slot(i, p.U, p.V, p.ld, p.rank, p.eps, p.Ux, p.Vx, p.ldx, p.rmax, plan);
      all.push_back(i);
    } else {
      g.host(i).active = ACT_DONE;
    }
  }
  lrp_status e = g.upload_all(g.cap(), st);
  if (e != LRP_OK) return e;
  phase_mark(ctx, 0, st);
  if ((e = g.forward(all, st)) != LRP_OK) return e;
  phase_mark(ctx, 1, st);
  // one step for the initial column choice, then at most max_sweeps
  // (<= LRP_MAX_SWEEPS) sweeps: the device stops every slot by then
  for (int step = 0; step <= LRP_MAX_SWEEPS; ++step) {
    if ((e = g.step(st)) != LRP_OK) return e;
    if ((e = g.fetch(st)) != LRP_OK) return e;
    bool any = false;
    for (int i = 0; i < count; ++i) any |= g.host(i).active != ACT_DONE;
    if (!any) break;
  }
  phase_mark(ctx, 2, st);
  std::vector<int> out;
  for (int i = 0; i < count; ++i) {
    Solve2D &s = g.host(i);
    if (s.active != ACT_DONE) {   // cannot happen: the device caps the sweeps
      s.status = LRP_EDEVICE;
      s.R = 0;
      continue;
    }
    if (s.status == LRP_ENONFINITE || s.r == 0) {
      s.R = 0;
      continue;
    }
    if (s.R > s.rmax) {
      s.status = LRP_ERANKCAP;
      continue;
    }
    out.push_back(i);
  }
  if ((e = g.inverse(out, st)) != LRP_OK) return e;
  phase_mark(ctx, 3, st);
  if (hipStreamSynchronize(st) != hipSuccess) return LRP_EDEVICE;
  float us[3];
  phase_times(ctx, us);
  lrp_status first = LRP_OK;
  for (int i = 0; i < count; ++i) {
    const Solve2D &s = g.host(i);
    lrp_problem2d &p = probs[i];
    std::memset(&p.info, 0, sizeof(p.info));
    p.rank_out = s.R;
    fill_info2d(s, g.plan(i), &p.info);
    for (int t = 0; t < 3; ++t) p.info.us_phase[t] = us[t];
    if (first == LRP_OK && s.status != LRP_OK) first = (lrp_status)s.status;
  }
  return first;
}

lrp_status lrpoisson_solve2d(lrp_ctx *ctx, int64_t n, int32_t rank,
                             const double *U, const double *V, int64_t ld,
                             double eps, const lrp_opts *opts, double *Ux,
                             double *Vx, int64_t ldx, int32_t rmax,
                             int32_t *rank_out, lrp_info *info, void *stream) {
  if (!rank_out) return LRP_EINVAL;
  lrp_problem2d p;
  std::memset(&p, 0, sizeof(p));
  p.U = U;
  p.V = V;
  p.ld = ld;
  p.rank = rank;
  p.rmax = rmax;
  p.eps = eps;
  p.Ux = Ux;
  p.Vx = Vx;
  p.ldx = ldx;
  lrp_status e = lrpoisson_solve2d_batch(ctx, n, 1, &p, opts, stream);
  *rank_out = p.rank_out;
  if (info) {
    *info = p.info;
    if (e == LRP_EINVAL) info->status = LRP_EINVAL;
  }
  return e;
}



}  // extern "C"
