"""Drive the library's continuous-batching request loop with a timed stream.

Requests arrive on a wall clock (Poisson arrivals from
``inputs.serving_stream``); each pass submits every request whose arrival
time has passed, calls the library's non-blocking scheduling step
(``lrp_serve_step``: every group whose previous work completed retires,
admits and enqueues its next sweep) and polls the outstanding tickets.  Latency is
completion time minus arrival time.  The right-hand sides are uploaded to the
device before the clock starts (factors resident on the device).
"""
from __future__ import annotations

import time

import numpy as np

from . import binding, inputs


def prepare(requests, device="cuda"):
    """Upload every request's RHS: (U, V) for 2D, (U1, U2, U3, G) for 3D with
    G as a Fortran-ordered flat tensor."""
    out = []
    for q in requests:
        f = q.rhs()
        if q.dim == 2:
            out.append((binding.colmajor(f[0], device), binding.colmajor(f[1], device)))
        else:
            out.append(tuple(binding.colmajor(u, device) for u in f[:3]) +
                       (binding.fortran_core(f[3], device),))
    return out


def run_stream(ctx: binding.Context, requests, factors, prec="auto",
               warmup: int = 0, time_scale: float = 1.0):
    """Serve ``requests`` (2D and 3D) against the wall clock.

    Returns dict with latencies (s) of the measured requests (after
    ``warmup``), solves/s over the measured window and per-request records.
    """
    import torch

    n_req = len(requests)
    order = sorted(range(n_req), key=lambda i: requests[i].arrival_s)
    t0 = time.perf_counter()
    nxt = 0
    pending = {}
    done = {}
    ticks = 0
    while len(done) < n_req:
        now = time.perf_counter() - t0
        while nxt < n_req and requests[order[nxt]].arrival_s * time_scale <= now:
            i = order[nxt]
            q = requests[i]
            if q.dim == 2:
                U, V = factors[i]
                ticket, outs = ctx.submit(U, V, q.eps, prec=prec)
            else:
                U1, U2, U3, G = factors[i]
                ticket, outs = ctx.submit3d(U1, U2, U3, G, q.eps, prec=prec)
            pending[ticket] = (i, outs)
            nxt += 1
        if not pending:
            # idle until the next arrival
            wait = requests[order[nxt]].arrival_s * time_scale - now
            if wait > 0:
                time.sleep(min(wait, 0.002))
            continue
        ctx.serve_step()
        ticks += 1
        tdone = time.perf_counter() - t0
        for ticket in list(pending):
            r = ctx.poll(ticket)
            if r is None:
                continue
            i, outs = pending.pop(ticket)
            status, ranks, info = r
            done[i] = dict(rid=i, arrival=requests[i].arrival_s * time_scale,
                           finish=tdone, latency=tdone - requests[i].arrival_s * time_scale,
                           status=status, rank=ranks[0], ranks=tuple(ranks),
                           sweeps=info["sweeps"], dim=requests[i].dim,
                           n=requests[i].n, r=requests[i].r, eps=requests[i].eps,
                           outs=outs)
    torch.cuda.synchronize()
    meas = [done[i] for i in range(warmup, n_req)]
    lat = np.array([d["latency"] for d in meas])
    t_first = min(d["arrival"] for d in meas)
    t_last = max(d["finish"] for d in meas)
    by_dim = {}
    for dim in sorted(set(d["dim"] for d in meas)):
        ld = np.array([d["latency"] for d in meas if d["dim"] == dim])
        by_dim[f"{dim}d"] = dict(count=int(ld.size),
                                 p50_ms=float(np.percentile(ld, 50) * 1e3),
                                 p99_ms=float(np.percentile(ld, 99) * 1e3))
    return dict(
        by_dim=by_dim,
        p50_ms=float(np.percentile(lat, 50) * 1e3),
        p99_ms=float(np.percentile(lat, 99) * 1e3),
        mean_ms=float(lat.mean() * 1e3),
        solves_per_s=len(meas) / (t_last - t_first),
        measured=len(meas), warmup=warmup, ticks=ticks,
        statuses=sorted(set(d["status"] for d in meas)),
        records=[done[i] for i in range(n_req)],
    )


def default_stream(count: int, seed: int = 5000, dims=(2, 3)):
    return inputs.serving_stream(count, 200.0, seed, dims=dims)


def check_sample(requests, records, per_shape=1, workers=None):
    """Relative error of served results against the float64 full-grid
    solution: the first ``per_shape`` finished requests of every (dim, n)
    shape (in request order) whose status is LRP_OK.  Returns a list of
    dicts (rid, dim, n, r, eps, rel_err).  Uses the CPU oracle (test and
    measurement infrastructure), never the solver."""
    from oracle import metrics, poisson
    seen = {}
    out = []
    for d in sorted(records, key=lambda d: d["rid"]):
        key = (d["dim"], d["n"])
        if d["status"] != binding.LRP_OK or seen.get(key, 0) >= per_shape:
            continue
        seen[key] = seen.get(key, 0) + 1
        q = requests[d["rid"]]
        outs, R = d["outs"], d["ranks"]
        if q.dim == 2:
            U, V = q.rhs()
            X = poisson.full_solve2d_factors(U, V, workers=workers)
            e = metrics.rel_err_factored(outs[0][:, :R[0]].cpu().numpy(),
                                         outs[1][:, :R[0]].cpu().numpy(), X)
        else:
            U1, U2, U3, G0 = q.rhs()
            X = poisson.full_solve3d_tucker(U1, U2, U3, np.asarray(G0), workers=workers)
            G = outs[3][:R[0] * R[1] * R[2]].view(R[2], R[1], R[0]).permute(2, 1, 0)
            Us = [outs[t][:, :R[t]].cpu().numpy() for t in range(3)]
            e = metrics.rel_err_tucker(Us[0], Us[1], Us[2], G.cpu().numpy(), X)
        del X
        out.append(dict(rid=int(d["rid"]), dim=q.dim, n=q.n, r=q.r, eps=q.eps,
                        ranks=list(R), rel_err=float(e)))
    return out
