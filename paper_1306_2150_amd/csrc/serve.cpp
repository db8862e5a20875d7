// Continuous-batching request loop over the slot groups (host side).
//
// Requests wait in a FIFO until the group of their dimension and grid size
// has a free slot (groups are created on demand inside the context's
// device-memory budget, which is the admission limit; a 3D group holds as
// many slots as fit a fixed share of it).  Every group advances on its own
// stream and at its own pace: lrp_serve_step never waits for the device.
// For each group whose previously enqueued work has completed (a stream
// query), one call
//   1. reports the requests whose inverse transforms were in that work and
//      frees their slots;
//   2. reads the slot states fetched by that work: slots that finished get
//      their inverse transforms (3D: of the three output factors);
//   3. admits queued requests of the group into free slots (upload, forward
//      transforms; 3D also forms its mode-unfolding factors);
//   4. enqueues one step of every running slot -- the initial column choice
//      of new slots and one cross sweep of the others, requests admitted at
//      different times sharing every launch; 3D solves whose mode crosses
//      finished also get their core and its rounding -- and the copy of the
//      slot states back to the host.
// A slow group (a large 3D grid) therefore never holds back a fast one.
#include <algorithm>
#include <cstring>
#include <map>
#include <thread>

#include "host.h"

using namespace lrp;

namespace {

constexpr int SERVE_SLOTS = 32;                      // slots per 2D group
constexpr size_t SERVE3_SHARE = (size_t)16 << 30;   // bytes per 3D group

lrp_status check_request(const lrp_request &q) {
  if (q.prec < 0 || q.prec > LRP_PREC_BF16X6) return LRP_EINVAL;
  if (q.op != LRP_OP_LAPLACE && q.op != LRP_OP_STOKES) return LRP_EINVAL;
  if (q.reserved != 0) return LRP_EINVAL;
  if (q.prec != LRP_PREC_AUTO &&
      (q.n < 1 || q.n > LRP_MAX_N || !transform_prec_ok(q.prec, (int)q.n)))
    return LRP_EINVAL;
  if (q.dim == 3) {
    const int32_t *rk = q.rank, *rm = q.rmax;
    return check_problem3d(q.n, rk, q.U, q.ld, q.G, q.eps, q.X, q.ldx, q.Gx, rm);
  }
  if (q.dim != 2) return LRP_EINVAL;
  if (q.n < 1 || q.n > LRP_MAX_N) return LRP_EINVAL;
  if (!(q.eps > 0.0 && q.eps < 1.0)) return LRP_EINVAL;
  if (q.rank[0] < 0 || q.rank[0] > LRP_MAX_RANK || q.rmax[0] < 0) return LRP_EINVAL;
  if (q.rank[0] > 0 && (!q.U[0] || !q.U[1] || q.ld < q.n)) return LRP_EINVAL;
  if (q.rmax[0] > 0 && (!q.X[0] || !q.X[1] || q.ldx < q.n)) return LRP_EINVAL;
  return LRP_OK;
}

Group2D *serve_group(lrp_ctx *ctx, int n, lrp_status *err) {
  *err = LRP_OK;
  auto &g = ctx->serve_groups[n];
  if (!g) {
    std::unique_ptr<Group2D> ng(new Group2D(ctx, n, SERVE_SLOTS));
    *err = ng->init();
    if (*err != LRP_OK) {
      ctx->serve_groups.erase(n);
      return nullptr;
    }
    ng->serve.ticket.assign(ng->cap(), 0);
    ng->serve.result.resize(ng->cap());
    ng->serve.ranks.resize(ng->cap());
    g = std::move(ng);
  }
  return g.get();
}

Group3D *serve_group3(lrp_ctx *ctx, int n, lrp_status *err) {
  *err = LRP_OK;
  auto &g = ctx->serve3_groups[n];
  if (!g) {
    const size_t per = solve3d_slot_bytes(n);
    const int cap = (int)std::max<size_t>(1, std::min<size_t>(SERVE_SLOTS, SERVE3_SHARE / per));
    std::unique_ptr<Group3D> ng(new Group3D(ctx, n, cap));
    *err = ng->init();
    if (*err != LRP_OK) {
      ctx->serve3_groups.erase(n);
      return nullptr;
    }
    ng->serve.ticket.assign(ng->cap(), 0);
    ng->serve.result.resize(ng->cap());
    ng->serve.ranks.resize(ng->cap());
    g = std::move(ng);
  }
  return g.get();
}

// A request that needs no device work (a zero Tucker rank): done at once.
bool trivially_done(const lrp_request &q) {
  return q.dim == 3 && (q.rank[0] == 0 || q.rank[1] == 0 || q.rank[2] == 0);
}

Plan request_plan(const lrp_request &q) {
  lrp_opts o;
  std::memset(&o, 0, sizeof(o));
  o.prec = q.prec;
  o.op = q.op;
  return make_plan(&o, q.eps, (int)q.n);
}

void finish_request(lrp_ctx *ctx, uint64_t t, const lrp_info &info,
                    const int32_t rank_out[3]) {
  auto it = ctx->running.find(t);
  if (it == ctx->running.end()) return;
  ServeReq r = it->second;
  ctx->running.erase(it);
  r.state = 2;
  r.status = info.status;
  r.info = info;
  for (int d = 0; d < 3; ++d) r.rank_out[d] = rank_out[d];
  ctx->finished[t] = r;
}

// Has the group's previously enqueued work completed?  False while it runs
// (or on a device error, then *err is set).
bool group_idle(ServeInfo &sv, hipStream_t st, lrp_status *err) {
  *err = LRP_OK;
  if (!sv.inflight) return true;
  const hipError_t q = hipStreamQuery(st);
  if (q == hipErrorNotReady) return false;
  if (q != hipSuccess) {
    *err = LRP_EDEVICE;
    return false;
  }
  sv.inflight = false;
  return true;
}

// Moves the queued requests that `admit` takes (in arrival order) to the
// running set.
template <class Admit>
lrp_status admit_queued(lrp_ctx *ctx, Admit admit) {
  for (auto it = ctx->queue.begin(); it != ctx->queue.end();) {
    int taken = 0;
    lrp_status e = admit(*it, &taken);
    if (e != LRP_OK) return e;
    if (taken < 0) break;   // group full
    if (taken) {
      ctx->running[it->ticket] = *it;
      it = ctx->queue.erase(it);
    } else {
      ++it;
    }
  }
  return LRP_OK;
}

lrp_status tick2d(lrp_ctx *ctx, Group2D *g) {
  lrp_status e;
  ServeInfo &sv = g->serve;
  hipStream_t st = g->stream();
  if (!st) return LRP_EDEVICE;
  if (!group_idle(sv, st, &e)) return e;
  g->begin_batch();
  // 1. report what the completed work finished
  for (int slot : sv.retiring) {
    finish_request(ctx, sv.ticket[slot], sv.result[slot], sv.ranks[slot].data());
    sv.ticket[slot] = 0;
    g->free_slots.push_back(slot);
  }
  sv.retiring.clear();
  // 2. slots that finished: their reports (the state copy of the next step
  // overwrites the host mirror) and inverse transforms
  std::vector<int> inv;
  for (int slot = 0; slot < g->cap(); ++slot) {
    if (!sv.ticket[slot]) continue;
    const Solve2D &s = g->host(slot);
    if (s.active != ACT_DONE) continue;
    lrp_info &info = sv.result[slot];
    std::memset(&info, 0, sizeof(info));
    fill_info2d(s, g->plan(slot), &info);
    if (s.status == LRP_ENONFINITE || s.r == 0) {
      info.rank = 0;
    } else if (s.R > s.rmax) {
      info.status = LRP_ERANKCAP;
    } else {
      inv.push_back(slot);
    }
    sv.ranks[slot] = {info.rank, 0, 0};
    sv.retiring.push_back(slot);
  }
  bool launched = false;
  if (!inv.empty()) {
    if ((e = g->inverse(inv, st)) != LRP_OK) return e;
    launched = true;
  }
  // 3. admission
  std::vector<int> fresh;
  const int64_t n = g->n();
  e = admit_queued(ctx, [&](ServeReq &r, int *taken) -> lrp_status {
    const lrp_request &q = r.req;
    if (q.dim != 2 || q.n != n) return LRP_OK;
    if (g->free_slots.empty()) {
      *taken = -1;
      return LRP_OK;
    }
    const int slot = g->free_slots.back();
    g->free_slots.pop_back();
    g->setup_slot(slot, q.U[0], q.U[1], q.ld, q.rank[0], q.eps, q.X[0], q.X[1], q.ldx,
                  q.rmax[0], request_plan(q));
    lrp_status ee = g->upload_slot(slot, st);
    if (ee != LRP_OK) return ee;
    fresh.push_back(slot);
    r.state = 1;
    r.group = g;
    r.group3 = nullptr;
    r.group_slot = slot;
    sv.ticket[slot] = r.ticket;
    *taken = 1;
    return LRP_OK;
  });
  if (e != LRP_OK) return e;
  if (!fresh.empty() && (e = g->forward(fresh, st)) != LRP_OK) return e;
  // 4. one step of every running slot and the state copy back
  bool live = false;
  for (int slot = 0; slot < g->cap(); ++slot)
    live |= sv.ticket[slot] && g->host(slot).active != ACT_DONE;
  if (live) {
    if ((e = g->step(st)) != LRP_OK) return e;
    if ((e = g->fetch(st, false)) != LRP_OK) return e;
    launched = true;
  }
  sv.inflight = launched || !sv.retiring.empty();
  return LRP_OK;
}

lrp_status tick3d(lrp_ctx *ctx, Group3D *g) {
  lrp_status e;
  ServeInfo &sv = g->serve;
  hipStream_t st = g->stream();
  if (!st) return LRP_EDEVICE;
  if (!group_idle(sv, st, &e)) return e;
  g->begin_batch();
  for (int slot : sv.retiring) {
    finish_request(ctx, sv.ticket[slot], sv.result[slot], sv.ranks[slot].data());
    sv.ticket[slot] = 0;
    g->host(slot).phase = P3_IDLE;
    g->free_slots.push_back(slot);
  }
  sv.retiring.clear();
  for (int slot = 0; slot < g->cap(); ++slot) {
    if (!sv.ticket[slot] || g->host(slot).phase != P3_DONE) continue;
    fill_info3d(*g, slot, sv.ranks[slot].data(), &sv.result[slot]);
    sv.retiring.push_back(slot);
  }
  bool launched = false;
  if (!sv.retiring.empty()) {
    if ((e = g->finish(sv.retiring, st)) != LRP_OK) return e;
    launched = true;
  }
  std::vector<int> fresh;
  const int64_t n = g->n();
  e = admit_queued(ctx, [&](ServeReq &r, int *taken) -> lrp_status {
    const lrp_request &q = r.req;
    if (q.dim != 3 || q.n != n) return LRP_OK;
    if (g->free_slots.empty()) {
      *taken = -1;
      return LRP_OK;
    }
    const int slot = g->free_slots.back();
    g->free_slots.pop_back();
    const int rk[3] = {q.rank[0], q.rank[1], q.rank[2]};
    const int rm[3] = {q.rmax[0], q.rmax[1], q.rmax[2]};
    g->setup_slot(slot, q.U, q.ld, rk, q.G, q.eps, q.X, q.ldx, q.Gx, rm, request_plan(q));
    fresh.push_back(slot);
    r.state = 1;
    r.group = nullptr;
    r.group3 = g;
    r.group_slot = slot;
    sv.ticket[slot] = r.ticket;
    *taken = 1;
    return LRP_OK;
  });
  if (e != LRP_OK) return e;
  if (!fresh.empty() && (e = g->start(fresh, st)) != LRP_OK) return e;
  bool live = false;
  for (int slot = 0; slot < g->cap(); ++slot)
    live |= sv.ticket[slot] && g->host(slot).phase != P3_DONE && g->host(slot).phase != P3_IDLE;
  if (live) {
    if ((e = g->step(st)) != LRP_OK) return e;
    if ((e = g->fetch(st, false)) != LRP_OK) return e;
    launched = true;
  }
  sv.inflight = launched || !sv.retiring.empty();
  return LRP_OK;
}

}  // namespace

extern "C" {

lrp_status lrp_submit(lrp_ctx *ctx, const lrp_request *req, uint64_t *ticket) {
  if (!ctx || !req || !ticket) return LRP_EINVAL;
  lrp_status e = check_request(*req);
  if (e != LRP_OK) return e;
  std::lock_guard<std::mutex> lock(ctx->mu);
  ServeReq r;
  std::memset(&r, 0, sizeof(r));
  r.ticket = ctx->next_ticket++;
  r.req = *req;
  r.state = 0;
  r.group_slot = -1;
  r.group = nullptr;
  r.group3 = nullptr;
  r.status = LRP_ENOTREADY;
  if (trivially_done(*req)) {
    r.state = 2;
    r.status = LRP_OK;
    r.info.change = -1.0;
    ctx->finished[r.ticket] = r;
  } else {
    ctx->queue.push_back(r);
  }
  *ticket = r.ticket;
  return LRP_OK;
}

lrp_status lrp_serve_step(lrp_ctx *ctx, int32_t *pending) {
  if (!ctx) return LRP_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return LRP_EDEVICE;
  std::lock_guard<std::mutex> lock(ctx->mu);
  lrp_status e;
  // Groups for queued requests are created on first use.  A group that does
  // not fit the budget first frees the groups that the context caches for
  // its synchronous calls (they are rebuilt when next needed).  Serving
  // groups are kept for the context's lifetime, so a group that still does
  // not fit never will: the queued requests of its shape finish with that
  // error instead of waiting for memory that cannot free up.
  std::map<std::pair<int, int>, lrp_status> failed;   // (dim, n) -> status
  auto make = [&](int dim, int n) -> bool {
    return dim == 3 ? serve_group3(ctx, n, &e) != nullptr : serve_group(ctx, n, &e) != nullptr;
  };
  for (const auto &q : ctx->queue) {
    const int dim = q.req.dim, n = (int)q.req.n;
    const bool have = dim == 3 ? ctx->serve3_groups.count(n) > 0 : ctx->serve_groups.count(n) > 0;
    if (have || failed.count({dim, n})) continue;
    if (make(dim, n)) continue;
    if (e == LRP_ENOMEM && (!ctx->batch_groups.empty() || !ctx->batch3_groups.empty() ||
                            !ctx->expsum_groups.empty())) {
      ctx->batch_groups.clear();
      ctx->batch3_groups.clear();
      ctx->expsum_groups.clear();
      if (make(dim, n)) continue;
    }
    failed[{dim, n}] = e;
  }
  for (auto it = ctx->queue.begin(); it != ctx->queue.end();) {
    auto f = failed.find({it->req.dim, (int)it->req.n});
    if (f == failed.end()) {
      ++it;
      continue;
    }
    it->state = 2;
    it->status = f->second;
    ctx->finished[it->ticket] = *it;
    it = ctx->queue.erase(it);
  }
  for (auto &kv : ctx->serve_groups)
    if ((e = tick2d(ctx, kv.second.get())) != LRP_OK) return e;
  for (auto &kv : ctx->serve3_groups)
    if ((e = tick3d(ctx, kv.second.get())) != LRP_OK) return e;
  if (pending) *pending = (int32_t)(ctx->queue.size() + ctx->running.size());
  return LRP_OK;
}

lrp_status lrp_poll(lrp_ctx *ctx, uint64_t ticket, int32_t *result,
                    int32_t rank_out[3], lrp_info *info) {
  if (!ctx) return LRP_EINVAL;
  std::lock_guard<std::mutex> lock(ctx->mu);
  auto it = ctx->finished.find(ticket);
  if (it == ctx->finished.end()) {
    for (const auto &q : ctx->queue)
      if (q.ticket == ticket) return LRP_ENOTREADY;
    if (ctx->running.count(ticket)) return LRP_ENOTREADY;
    return LRP_EINVAL;
  }
  if (result) *result = it->second.status;
  if (rank_out)
    for (int d = 0; d < 3; ++d) rank_out[d] = it->second.rank_out[d];
  if (info) *info = it->second.info;
  ctx->finished.erase(it);
  return LRP_OK;
}

lrp_status lrp_wait(lrp_ctx *ctx, uint64_t ticket, int32_t *result,
                    int32_t rank_out[3], lrp_info *info) {
  if (!ctx) return LRP_EINVAL;
  for (;;) {
    const lrp_status p = lrp_poll(ctx, ticket, result, rank_out, info);
    if (p != LRP_ENOTREADY) return p;
    // every tick of a group waits for nothing: a group whose enqueued work
    // has not completed is skipped, so give the device time between ticks
    int32_t pending = 0;
    const lrp_status e = lrp_serve_step(ctx, &pending);
    if (e != LRP_OK) return e;
    std::this_thread::yield();
  }
}

}  // extern "C"
