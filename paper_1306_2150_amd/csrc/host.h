// Host-side runtime of the solver: context, per-grid tables, slot groups.
#pragma once

#include <array>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "lrp_internal.h"

namespace lrp {

// Serving-loop bookkeeping of one slot group (see serve.cpp).
struct ServeInfo {
  bool inflight = false;           // launches enqueued, completion not yet seen
  std::vector<int> retiring;       // finished slots whose results are in flight
  std::vector<uint64_t> ticket;    // request of each slot, 0 = free
  std::vector<lrp_info> result;    // report of each retiring slot
  std::vector<std::array<int32_t, 3>> ranks;
};

// Sine-transform tables and eigenvalues of one grid size n (device memory).
struct GridTables {
  int n = 0;
  void *tab = nullptr;      // [f64 quarter][f32 quarter][bf16 pair quarter]
  double *lam = nullptr;    // lambda_k, k = 1..n
  double *sp = nullptr;     // Stokes operator factors 2 sin^2(pi k h/2)/h,
  double *sq = nullptr;     //   2 cos^2(pi k h/2)/h, k = 1..n
  size_t bytes = 0;
};

// Resolved per-request options.
struct Plan {
  int fwd_prec, inv_prec;
  int max_sweeps, kcap, kick, min_slack;
  double tau;
  int op;             // lrp_operator
  int k0;             // columns of the first sweep, 0: rank + kick
  uint64_t seed;      // offset of the spread index sequences
};

// A group of cross-approximation slots of one shape.  Every kernel launch
// covers all slots; each slot's `active` flag selects which launches act on
// it.  2D solves: n x n with the grid's tables on both sides.  3D path: the
// n x n^2 mode unfoldings, with column tables over the n^2 pairs
// (col[0]: Laplace mu, col[1], col[2]: the Stokes factors).
class Group2D {
 public:
  Group2D(lrp_ctx *ctx, int n, int cap, int m = 0, const double *const *col = nullptr);
  ~Group2D();
  lrp_status init();                       // allocate
  size_t bytes() const { return bytes_; }
  int n() const { return n_; }
  int m() const { return m_; }
  int cap() const { return cap_; }
  const GridTables *tables() const { return tabs_; }

  // Fill slot `i` for a new problem (host mirror only) -- call upload().
  void setup_slot(int i, const double *U, const double *V, long ld, int r,
                  double eps, double *Ux, double *Vx, long ldx, int rmax,
                  const Plan &plan);
  lrp_status upload_slot(int i, hipStream_t st);
  lrp_status upload_all(int count, hipStream_t st);
  // Forward transform of the listed slots (grouped by precision).
  lrp_status forward(const std::vector<int> &slots, hipStream_t st);
  // Initial maxvol for INIT slots, then one sweep for SWEEP slots.
  lrp_status step(hipStream_t st);
  // Copy the control state of all slots back; with sync, wait for it.
  lrp_status fetch(hipStream_t st, bool sync = true);
  // Inverse transform of the listed finished slots.
  lrp_status inverse(const std::vector<int> &slots, hipStream_t st);

  // Start of a batch of launches on an idle stream: the transform-column
  // staging ring may be reused from its start.
  void begin_batch() { cols_used_ = 0; }
  // Sine transform of arbitrary columns; a column's `solve` index names a
  // slot of this group whose non-finite flag it sets.
  lrp_status transform(std::vector<DstCol> &cols, int prec, hipStream_t st) {
    return dst_cols(cols, prec, st);
  }

  Solve2D &host(int i) { return h_s_[i]; }
  Solve2D *dev_solves() { return d_s_; }
  // own stream (default priority) for the serving loop
  hipStream_t stream();
  const Plan &plan(int i) const { return plans_[i]; }
  std::vector<int> free_slots;
  ServeInfo serve;

 private:
  lrp_status dst_cols(std::vector<DstCol> &cols, int prec, hipStream_t st);
  lrp_ctx *ctx_;
  int n_, cap_, m_;
  const double *col_[3] = {nullptr, nullptr, nullptr};
  Tree talloc_;
  size_t per_slot_ = 0, bytes_ = 0;
  char *ws_ = nullptr;
  Solve2D *d_s_ = nullptr, *h_s_ = nullptr;
  DstCol *d_cols_ = nullptr, *h_cols_ = nullptr;
  int cols_cap_ = 0, cols_used_ = 0;
  double *d_partial_ = nullptr;
  size_t partial_elems_ = 0;
  void *d_work_ = nullptr;         // int8 slice records (allocated on first use)
  size_t work_bytes_ = 0;
  std::vector<Plan> plans_;
  std::vector<int> kin_;
  const GridTables *tabs_ = nullptr;
  hipStream_t stream_ = nullptr;
  // sweep steps captured as graphs (on stream_), keyed by their launch plan,
  // replayed on the caller's stream
  struct StepPlan {
    int hi, kin, km, kev;
    unsigned bmask;
    bool init, sweep;
    uint64_t key() const;
  };
  lrp_status launch_step(const StepPlan &p, hipStream_t st);
  std::map<uint64_t, hipGraphExec_t> graphs_;
};

// A group of 3D (Tucker) solve slots of one grid size n.  Slot i owns the
// mode slots 3i, 3i+1, 3i+2 of a cross group of n x FIB_M fiber matrices.
class Group3D {
 public:
  Group3D(lrp_ctx *ctx, int n, int cap);
  ~Group3D();
  lrp_status init();
  int n() const { return n_; }
  int cap() const { return cap_; }
  size_t bytes() const;
  // Fill slot i (host mirror).  U[d]: n x r[d] (ld), G: r0 x r1 x r2.
  void setup_slot(int i, const double *const U[3], long ld, const int r[3],
                  const double *G, double eps, double *const X[3], long ldx,
                  double *Gx, const int rmax[3], const Plan &plan);
  // Upload, forward transforms and mode-unfolding factors of new slots.
  lrp_status start(const std::vector<int> &slots, hipStream_t st);
  // One sweep of every running mode cross, then the core, its rounding and
  // the output core of every solve whose three crosses have finished.
  lrp_status step(hipStream_t st);
  lrp_status fetch(hipStream_t st, bool sync = true);
  // Inverse transforms of the output factors of finished slots.
  lrp_status finish(const std::vector<int> &slots, hipStream_t st);
  Solve3D &host(int i) { return h_s_[i]; }
  const Plan &plan(int i) const { return plans_[i]; }
  Group2D &modes() { return *inner_; }
  hipStream_t stream() { return inner_->stream(); }
  void begin_batch() { inner_->begin_batch(); }
  std::vector<int> free_slots;
  ServeInfo serve;

 private:
  struct IO {
    const double *U[3];
    long ld;
    double *X[3];
    long ldx;
  };
  lrp_ctx *ctx_;
  int n_, cap_;
  size_t bytes_ = 0;
  char *ws_ = nullptr;
  std::unique_ptr<Group2D> inner_;
  Solve3D *d_s_ = nullptr, *h_s_ = nullptr;
  std::vector<Plan> plans_;
  std::vector<IO> io_;
};

// Slots of the exponential-sum comparator for one grid size n: the Solve2D
// job records of both sides (a Group2D of 2 cap slots, see ExpState), the
// device states and the quadrature nodes of every slot.
struct ExpGroup {
  ExpGroup(lrp_ctx *ctx, int n, int cap);
  ~ExpGroup();
  lrp_status init();
  lrp_ctx *ctx;
  int n, cap;
  std::unique_ptr<Group2D> jobs;
  ExpState *d_e = nullptr, *h_e = nullptr;
  double *d_nodes = nullptr, *h_nodes = nullptr;   // per slot: sqrt(w), p
  size_t bytes = 0;
  // nodes of each (eps) met so far: sqrt(w_k), then p_k
  std::map<double, std::vector<double>> node_cache;
};
ExpGroup *expsum_group(lrp_ctx *ctx, int n, int count, lrp_status *err);
// the incremental rounding steps of slots [0, count) (states uploaded)
lrp_status run_steps(ExpGroup &g, int count, hipStream_t st);

// One product U V^T (n x K factors, device, leading dimension ld) to round
// to eps (relative Frobenius): Ux (the scale) and Vx (orthonormal columns)
// receive `rank` <= rmax columns; status LRP_ERANKCAP when the rank exceeds
// rmax (outputs unwritten) or a step lacked room.
struct RoundJob {
  const double *U, *V;
  long ld;
  int K;
  double eps;
  double *Ux, *Vx;
  long ldx;
  int rmax;
  int rank;       // out
  int status;     // out
  double err;     // out: the dropped tails over the final core norm
};
// Rounds `count` products of grid size n >= ES_MIN_N_PLAIN together; the
// outputs are enqueued on st (the call waits only for the rank read-backs).
lrp_status round_products(lrp_ctx *ctx, int n, int count, RoundJob *jobs, hipStream_t st);

// The randomized rounding of one product U V^T (n x K, host_round.cpp): a
// one-slot group for its TSQR and core, the Gaussian sketch and buffers.
struct RoundGroup {
  ~RoundGroup();
  lrp_ctx *ctx = nullptr;
  int n = 0, L = 0, kcap = 0;
  std::unique_ptr<Group2D> g;
  // zpart: the row layers' partial products of the A^T B steps
  double *buf = nullptr, *omega = nullptr, *Z = nullptr, *Qk = nullptr, *zpart = nullptr;
  size_t bytes = 0;
};
// Ux (scale) and Vx (orthonormal) of rank <= rmax with relative error
// <= eps (*err: the dropped tail over the result's norm); LRP_ERANKCAP when
// the rank exceeds rmax or comes within 8 of the sketch width min(64, n).
// Enqueued on st; waits for the singular values only.
// A tail up to abs_tol (absolute Frobenius) may also be dropped.
lrp_status round_random(lrp_ctx *ctx, int n, int K, const double *U, const double *V, long ld,
                        double eps, double *Ux, double *Vx, long ldx, int rmax, int *rank,
                        double *err, hipStream_t st, double abs_tol = 0.0);

}  // namespace lrp

// Requests of the serving loop.
struct ServeReq {
  uint64_t ticket;
  lrp_request req;
  int state;            // 0 queued, 1 running, 2 done
  int group_slot;
  lrp::Group2D *group;      // 2D requests
  lrp::Group3D *group3;     // 3D requests
  int32_t status;
  int32_t rank_out[3];
  lrp_info info;
  size_t bytes;
};

struct lrp_ctx {
  int device = 0;
  size_t budget = 0;
  size_t used = 0;
  std::map<int, lrp::GridTables> tables;
  // cached groups for synchronous calls, keyed by n
  std::map<int, std::unique_ptr<lrp::Group2D>> batch_groups;
  std::map<int, std::unique_ptr<lrp::Group3D>> batch3_groups;
  std::map<int, std::unique_ptr<lrp::ExpGroup>> expsum_groups;
  // one-slot groups of the component entry points, keyed by n
  std::map<int, std::unique_ptr<lrp::Group2D>> kernel_groups;
  // randomized rounding of the Stokes driver's sums, keyed by n
  std::map<int, std::unique_ptr<lrp::RoundGroup>> round_groups;
  // serving
  hipStream_t serve_stream = nullptr;
  std::map<int, std::unique_ptr<lrp::Group2D>> serve_groups;
  std::map<int, std::unique_ptr<lrp::Group3D>> serve3_groups;
  std::deque<ServeReq> queue;
  std::map<uint64_t, ServeReq> running;
  std::map<uint64_t, ServeReq> finished;
  uint64_t next_ticket = 1;
  // standalone sine transform staging
  lrp::DstCol *tx_dcols = nullptr, *tx_hcols = nullptr;
  int tx_cap = 0;
  double *tx_partial = nullptr;
  size_t tx_partial_elems = 0, tx_bytes = 0;
  void *tx_work = nullptr;
  size_t tx_work_bytes = 0;
  // transform kernel timing (events recorded around each launch)
  bool timing = false;
  struct PendingTime {
    hipEvent_t a, b;
    int prec;
    long cols;
    double flops;
  };
  std::vector<PendingTime> pending_times;
  lrp_kernel_stat kstat[LRP_PREC_BF16X6 + 1] = {};
  // phase events of the synchronous calls (forward, cross, inverse)
  hipEvent_t phase_ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // replay the cross sweep steps as captured HIP graphs (lrp_set_graph_replay)
  bool graphs = true;
  std::mutex mu;
};

namespace lrp {
const GridTables *get_tables(lrp_ctx *ctx, int n, lrp_status *err);
// bytes and host construction of the sine tables of grid size n (the
// layout launch_dst reads)
size_t sine_table_bytes(int n);
void build_sine_table(int n, char *out);
Plan make_plan(const lrp_opts *o, double eps, int n);
// LRP_EINVAL for options outside their documented ranges
lrp_status check_opts(const lrp_opts *o);
// an explicit transform precision that grid size n supports
bool transform_prec_ok(int prec, int n);
// algorithmic flops of one transformed column (lrp_kernel_stat.flops)
double transform_flops(int prec, int n);
// every transform precision, in the order the groups launch them
constexpr int ALL_PRECS[] = {LRP_PREC_FP64, LRP_PREC_FP32, LRP_PREC_BF16X3, LRP_PREC_INT8,
                             LRP_PREC_FFT64, LRP_PREC_BF16X6};
// phase timing of a synchronous call: record event i (0..3) on st
void phase_mark(lrp_ctx *ctx, int i, hipStream_t st);
// after the stream completed: the three phase durations in microseconds
void phase_times(lrp_ctx *ctx, float us[3]);
lrp_status dev_alloc(lrp_ctx *ctx, void **p, size_t bytes);
// launch_dst with optional event timing for the context
hipError_t timed_dst(lrp_ctx *ctx, int prec, int n, const void *tab,
                     const DstCol *cols, int ncols, Solve2D *solves,
                     double *partial, size_t partial_elems, void *work,
                     size_t work_bytes, hipStream_t st);
void dev_free(lrp_ctx *ctx, void *p, size_t bytes);
// 3D helpers shared by the synchronous call and the serving loop
lrp_status check_problem3d(int64_t n, const int32_t rank[3], const double *const U[3],
                           int64_t ld, const double *G, double eps,
                           double *const X[3], int64_t ldx, const double *Gx,
                           const int32_t rmax[3]);
void fill_info3d(Group3D &g, int i, int32_t rank_out[3], lrp_info *info);
// report of a finished 2D slot (status, sweeps, ranks, plan, estimates)
void fill_info2d(const Solve2D &s, const Plan &plan, lrp_info *info);
// device bytes of one slot of a cross group of shape n x m
size_t cross_slot_bytes(int n, int m);
// device bytes of one 3D slot of grid size n (its three mode slots included)
size_t solve3d_slot_bytes(int n);
}  // namespace lrp
