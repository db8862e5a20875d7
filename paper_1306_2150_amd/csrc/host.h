// Host-side runtime of the solver: context, per-grid tables, slot groups.
#pragma once

#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "lrp_internal.h"

namespace lrp {

// Sine-transform tables and eigenvalues of one grid size n (device memory).
struct GridTables {
  int n = 0;
  void *tab = nullptr;      // [f64 quarter][f32 quarter][bf16 pair quarter]
  double *lam = nullptr;    // lambda_k, k = 1..n
  size_t bytes = 0;
};

// Resolved per-request options.
struct Plan {
  int fwd_prec, inv_prec;
  int max_sweeps, kcap, kick, min_slack;
  double tau;
};

// A group of 2D solve slots on one grid size.  Every kernel launch covers all
// slots; each slot's `active` flag selects which launches act on it.
class Group2D {
 public:
  Group2D(lrp_ctx *ctx, int n, int cap);
  ~Group2D();
  lrp_status init();                       // allocate
  size_t bytes() const { return bytes_; }
  int n() const { return n_; }
  int cap() const { return cap_; }

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

  Solve2D &host(int i) { return h_s_[i]; }
  Solve2D *dev_solves() { return d_s_; }
  // own stream (default priority) for the serving loop
  hipStream_t stream();
  const Plan &plan(int i) const { return plans_[i]; }
  std::vector<int> free_slots;

 private:
  lrp_status dst_cols(std::vector<DstCol> &cols, int prec, hipStream_t st);
  lrp_ctx *ctx_;
  int n_, cap_;
  Tree talloc_;
  size_t per_slot_ = 0, bytes_ = 0;
  char *ws_ = nullptr;
  Solve2D *d_s_ = nullptr, *h_s_ = nullptr;
  DstCol *d_cols_ = nullptr, *h_cols_ = nullptr;
  int cols_cap_ = 0;
  double *d_partial_ = nullptr;
  size_t partial_elems_ = 0;
  std::vector<Plan> plans_;
  std::vector<int> kin_;
  const GridTables *tabs_ = nullptr;
  hipStream_t stream_ = nullptr;
};

}  // namespace lrp

// Requests of the serving loop.
struct ServeReq {
  uint64_t ticket;
  lrp_request req;
  int state;            // 0 queued, 1 running, 2 done
  int group_slot;
  lrp::Group2D *group;
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
  // cached group for synchronous batches, keyed by n
  std::map<int, std::unique_ptr<lrp::Group2D>> batch_groups;
  // serving
  hipStream_t serve_stream = nullptr;
  std::map<int, std::unique_ptr<lrp::Group2D>> serve_groups;
  std::deque<ServeReq> queue;
  std::map<uint64_t, ServeReq> running;
  std::map<uint64_t, ServeReq> finished;
  uint64_t next_ticket = 1;
  // standalone sine transform staging
  lrp::DstCol *tx_dcols = nullptr, *tx_hcols = nullptr;
  int tx_cap = 0;
  double *tx_partial = nullptr;
  size_t tx_partial_elems = 0, tx_bytes = 0;
  // transform kernel timing (events recorded around each launch)
  bool timing = false;
  struct PendingTime {
    hipEvent_t a, b;
    int prec;
    long cols;
    double flops;
  };
  std::vector<PendingTime> pending_times;
  lrp_kernel_stat kstat[4] = {};
  std::mutex mu;
};

namespace lrp {
const GridTables *get_tables(lrp_ctx *ctx, int n, lrp_status *err);
Plan make_plan(const lrp_opts *o, double eps, int n);
lrp_status dev_alloc(lrp_ctx *ctx, void **p, size_t bytes);
// launch_dst with optional event timing for the context
hipError_t timed_dst(lrp_ctx *ctx, int prec, int n, const void *tab,
                     const DstCol *cols, int ncols, Solve2D *solves,
                     double *partial, size_t partial_elems, hipStream_t st);
void dev_free(lrp_ctx *ctx, void *p, size_t bytes);
}  // namespace lrp
