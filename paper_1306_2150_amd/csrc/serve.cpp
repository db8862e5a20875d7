// Continuous-batching request loop over the slot groups (host side).
//
// Requests wait in a FIFO until the group of their dimension and grid size
// has a free slot (groups are created on demand inside the context's
// device-memory budget, which is the admission limit; a 3D group holds as
// many slots as fit a fixed share of it).  One tick (lrp_serve_step):
//   1. admit: fill free slots, upload their state, forward transforms of all
//      newly admitted requests (one launch per group and precision; 3D also
//      forms its mode-unfolding factors);
//   2. advance: for every group with work, on the group's own stream, one
//      launch sequence that runs the initial column choice of the new slots
//      and one cross sweep of every running slot -- requests admitted at
//      different ticks share launches; 3D solves whose three mode crosses
//      finished also get their core and its rounding in the same tick;
//   3. retire: inverse transforms of the slots that finished, results
//      recorded, slots freed for the next tick.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "host.h"

using namespace lrp;

namespace {

constexpr int SERVE_SLOTS = 32;   // slots per grid-size group

constexpr size_t SERVE3_SHARE = (size_t)16 << 30;   // bytes per 3D group

lrp_status check_request(const lrp_request &q) {
  if (q.prec < 0 || q.prec > LRP_PREC_BF16X3) return LRP_EINVAL;
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
    g = std::move(ng);
  }
  return g.get();
}

// A request that needs no device work (a zero Tucker rank): done at once.
bool trivially_done(const lrp_request &q) {
  return q.dim == 3 && (q.rank[0] == 0 || q.rank[1] == 0 || q.rank[2] == 0);
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
  ctx->queue.push_back(r);
  *ticket = r.ticket;
  return LRP_OK;
}

lrp_status lrp_serve_step(lrp_ctx *ctx, int32_t *pending) {
  if (!ctx) return LRP_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return LRP_EDEVICE;
  std::lock_guard<std::mutex> lock(ctx->mu);
  lrp_status e;
  // 1. admission (FIFO per group: a request waits only for its own group)
  std::map<Group2D *, std::vector<int>> fresh;
  std::map<Group3D *, std::vector<int>> fresh3;
  for (auto it = ctx->queue.begin(); it != ctx->queue.end();) {
    const lrp_request &q = it->req;
    ServeReq r = *it;
    lrp_opts o;
    std::memset(&o, 0, sizeof(o));
    o.prec = q.prec;
    const Plan plan = make_plan(&o, q.eps, (int)q.n);
    if (trivially_done(q)) {
      r.state = 2;
      r.status = LRP_OK;
      std::memset(&r.info, 0, sizeof(r.info));
      r.info.change = -1.0;
      ctx->finished[r.ticket] = r;
      it = ctx->queue.erase(it);
      continue;
    }
    if (q.dim == 3) {
      Group3D *g = serve_group3(ctx, (int)q.n, &e);
      if (!g || g->free_slots.empty()) {
        ++it;
        continue;
      }
      const int slot = g->free_slots.back();
      g->free_slots.pop_back();
      const int rk[3] = {q.rank[0], q.rank[1], q.rank[2]};
      const int rm[3] = {q.rmax[0], q.rmax[1], q.rmax[2]};
      g->setup_slot(slot, q.U, q.ld, rk, q.G, q.eps, q.X, q.ldx, q.Gx, rm, plan);
      fresh3[g].push_back(slot);
      r.group3 = g;
      r.group = nullptr;
      r.group_slot = slot;
    } else {
      Group2D *g = serve_group(ctx, (int)q.n, &e);
      if (!g || g->free_slots.empty()) {
        ++it;
        continue;
      }
      const int slot = g->free_slots.back();
      g->free_slots.pop_back();
      g->setup_slot(slot, q.U[0], q.U[1], q.ld, q.rank[0], q.eps, q.X[0], q.X[1],
                    q.ldx, q.rmax[0], plan);
      if (!g->stream()) return LRP_EDEVICE;
      if ((e = g->upload_slot(slot, g->stream())) != LRP_OK) return e;
      fresh[g].push_back(slot);
      r.group = g;
      r.group3 = nullptr;
      r.group_slot = slot;
    }
    r.state = 1;
    ctx->running[r.ticket] = r;
    it = ctx->queue.erase(it);
  }
  // 2. every group with live slots, on its own stream so that the groups'
  // latency-bound launches overlap on the device
  std::vector<Group2D *> live;
  for (auto &kv : ctx->serve_groups) {
    Group2D *g = kv.second.get();
    if ((int)g->free_slots.size() < g->cap()) live.push_back(g);
  }
  std::vector<Group3D *> live3;
  for (auto &kv : ctx->serve3_groups) {
    Group3D *g = kv.second.get();
    if ((int)g->free_slots.size() < g->cap()) live3.push_back(g);
  }
  for (Group2D *g : live) {
    auto it = fresh.find(g);
    if (it != fresh.end() && (e = g->forward(it->second, g->stream())) != LRP_OK) return e;
    if ((e = g->step(g->stream())) != LRP_OK) return e;
    if ((e = g->fetch(g->stream(), false)) != LRP_OK) return e;
  }
  for (Group3D *g : live3) {
    if (!g->stream()) return LRP_EDEVICE;
    auto it = fresh3.find(g);
    if (it != fresh3.end() && (e = g->start(it->second, g->stream())) != LRP_OK) return e;
    if ((e = g->step(g->stream())) != LRP_OK) return e;
    if ((e = g->fetch(g->stream(), false)) != LRP_OK) return e;
  }
  for (Group2D *g : live)
    if (hipStreamSynchronize(g->stream()) != hipSuccess) return LRP_EDEVICE;
  for (Group3D *g : live3)
    if (hipStreamSynchronize(g->stream()) != hipSuccess) return LRP_EDEVICE;
  // 3. retirement
  std::map<Group2D *, std::vector<int>> done;
  std::map<Group3D *, std::vector<int>> done3;
  std::vector<uint64_t> finished;
  for (auto &kv : ctx->running) {
    ServeReq &r = kv.second;
    if (r.group3) {
      if (r.group3->host(r.group_slot).phase != P3_DONE) continue;
      done3[r.group3].push_back(r.group_slot);
      finished.push_back(kv.first);
      continue;
    }
    Solve2D &s = r.group->host(r.group_slot);
    if (s.active != ACT_DONE) continue;
    if (s.status == LRP_ENONFINITE || s.r == 0) {
      s.R = 0;
    } else if (s.R > s.rmax) {
      s.status = LRP_ERANKCAP;
    } else {
      done[r.group].push_back(r.group_slot);
    }
    finished.push_back(kv.first);
  }
  for (auto &kv : done)
    if ((e = kv.first->inverse(kv.second, kv.first->stream())) != LRP_OK) return e;
  for (auto &kv : done3)
    if ((e = kv.first->finish(kv.second, kv.first->stream())) != LRP_OK) return e;
  for (auto &kv : done)
    if (hipStreamSynchronize(kv.first->stream()) != hipSuccess) return LRP_EDEVICE;
  for (auto &kv : done3)
    if (hipStreamSynchronize(kv.first->stream()) != hipSuccess) return LRP_EDEVICE;
  for (uint64_t t : finished) {
    ServeReq r = ctx->running[t];
    ctx->running.erase(t);
    r.state = 2;
    if (r.group3) {
      Group3D *g = r.group3;
      fill_info3d(*g, r.group_slot, r.rank_out, &r.info);
      r.status = r.info.status;
      g->host(r.group_slot).phase = P3_IDLE;
      g->free_slots.push_back(r.group_slot);
    } else {
      Solve2D &s = r.group->host(r.group_slot);
      r.status = s.status;
      r.rank_out[0] = s.R;
      r.info.status = s.status;
      r.info.sweeps = s.sweep;
      r.info.k = s.k;
      r.info.rank = s.R;
      r.info.fwd_prec = r.group->plan(r.group_slot).fwd_prec;
      r.info.inv_prec = r.group->plan(r.group_slot).inv_prec;
      r.info.change = s.change;
      r.group->free_slots.push_back(r.group_slot);
    }
    ctx->finished[t] = r;
  }
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

}  // extern "C"
