"""GPU tests of the continuous-batching loop (lrp_submit / lrp_serve_step /
lrp_poll): requests of mixed dimension, grid size, rank and tolerance are
admitted while others run, share launches, and each result must equal the
same request solved alone through the synchronous entry points (relative
difference of the assembled solutions <= 1e-12) and match the oracle's full
solution to 10 eps."""
import numpy as np
import pytest

from oracle import metrics, poisson
from paper_1306_2150_amd import binding, inputs

from gpu_util import ctx, dev, host, log, rel

pytestmark = pytest.mark.gpu

MIX = [  # (dim, n, r, eps)
    (2, 512, 12, 1e-8), (3, 48, 6, 1e-6), (2, 1024, 30, 1e-6), (2, 256, 4, 1e-8),
    (3, 64, 10, 1e-8), (2, 512, 50, 1e-8), (3, 32, 4, 1e-6), (2, 1024, 8, 1e-8),
    (3, 48, 12, 1e-8), (2, 256, 64, 1e-6), (3, 64, 5, 1e-6), (2, 512, 20, 1e-6),
]


def mix_requests():
    return [inputs.Request(rid=i, arrival_s=0.0, dim=d, n=n, r=r, eps=e, seed=7000 + i)
            for i, (d, n, r, e) in enumerate(MIX)]


def assemble(dim, res):
    if dim == 2:
        Ux, Vx = res
        return host(Ux) @ host(Vx).T
    Xs, G = res
    Us = [host(x) for x in Xs]
    return poisson.tucker_full(np.asarray(host(G)), *Us)


def served_result(dim, outs, ranks):
    if dim == 2:
        return (outs[0][:, :ranks[0]], outs[1][:, :ranks[0]])
    R = ranks
    G = outs[3][:R[0] * R[1] * R[2]].view(R[2], R[1], R[0]).permute(2, 1, 0)
    return ([outs[d][:, :R[d]] for d in range(3)], G)


def serve_all(reqs, facs, prec, per_tick, gap_s=0.004):
    """Submit ``per_tick`` requests every ``gap_s`` seconds while calling the
    (non-blocking) scheduling step, so that requests arrive while others are
    on the device; step until all are done."""
    import time
    c = ctx()
    pending, done = {}, {}
    nxt, ticks = 0, 0
    t0 = time.time()
    while nxt < len(reqs) or pending:
        due = nxt < len(reqs) and time.time() - t0 >= gap_s * (nxt // per_tick)
        for _ in range(per_tick if due else 0):
            if nxt < len(reqs):
                q = reqs[nxt]
                if q.dim == 2:
                    t, outs = c.submit(facs[nxt][0], facs[nxt][1], q.eps, prec=prec)
                else:
                    t, outs = c.submit3d(*facs[nxt], q.eps, prec=prec)
                pending[t] = (nxt, outs)
                nxt += 1
        c.serve_step()
        ticks += 1
        assert time.time() - t0 < 60, "serving loop made no progress"
        for t in list(pending):
            r = c.poll(t)
            if r is not None:
                i, outs = pending.pop(t)
                done[i] = (r, outs)
    return done, ticks


@pytest.mark.parametrize("prec", ["fp64", "auto"])
def test_served_equals_alone(prec):
    from paper_1306_2150_amd import serving
    reqs = mix_requests()
    facs = serving.prepare(reqs)
    log("serve mix", prec, len(reqs))
    done, ticks = serve_all(reqs, facs, prec, per_tick=2)
    log("  ticks", ticks)
    c = ctx()
    nbit = 0
    for i, q in enumerate(reqs):
        (status, ranks, info), outs = done[i]
        assert status == binding.LRP_OK, (i, status)
        mine = assemble(q.dim, served_result(q.dim, outs, ranks))
        if q.dim == 2:
            Ux, Vx, _ = c.solve2d(facs[i][0], facs[i][1], q.eps, prec=prec)
            alone = assemble(2, (Ux, Vx))
            U, V = q.rhs()
            full = poisson.full_solve2d_factors(U, V)
        else:
            Xs, G, _ = c.solve3d(*facs[i], q.eps, prec=prec)
            alone = assemble(3, (Xs, G))
            U1, U2, U3, G0 = q.rhs()
            full = poisson.full_solve3d_tucker(U1, U2, U3, np.asarray(G0))
        d = rel(mine, alone)
        nbit += int(np.array_equal(mine, alone))
        e = rel(mine, full)
        log("  req", i, q.dim, q.n, q.r, q.eps, "ranks", ranks, "alone diff", d, "err", e)
        assert d <= 1e-12, (i, d)
        assert e <= 10 * q.eps, (i, e)
    log("  bitwise equal:", nbit, "of", len(reqs))


def test_served_errors_do_not_disturb_others():
    reqs = mix_requests()[:4]
    from paper_1306_2150_amd import serving
    facs = serving.prepare(reqs)
    log("serve errors")
    c = ctx()
    # a NaN right-hand side and a zero-rank 3D request among good ones
    bad = dev(np.full((512, 3), np.nan))
    tb, _ = c.submit(bad, bad, 1e-8)
    z = dev(np.zeros((48, 0)))
    tz, _ = c.submit3d(z, z, z, binding.fortran_core(np.zeros((0, 0, 0))), 1e-6)
    done, _ = serve_all(reqs, facs, "fp64", per_tick=4)
    import time
    res = {}
    t0 = time.time()
    while len(res) < 2 and time.time() - t0 < 30:
        for t in (tb, tz):
            if t not in res:
                r = c.poll(t)
                if r is not None:
                    res[t] = r
        c.serve_step()
    assert res[tb][0] == binding.LRP_ENONFINITE
    assert res[tz][0] == binding.LRP_OK and res[tz][1] == [0, 0, 0]
    for i in range(len(reqs)):
        assert done[i][0][0] == binding.LRP_OK
    with pytest.raises(binding.LrpError):
        c.submit(bad, bad, 0.0)


def _serve_until_done(c, tickets, limit_s=60):
    import time
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        assert time.time() - t0 < limit_s, "serving loop made no progress"
        c.serve_step()
        for t in tickets:
            if t not in res:
                r = c.poll(t)
                if r is not None:
                    res[t] = r
    return res


def test_served_group_over_budget_reports_enomem():
    """A request whose slot group can never fit the context's budget finishes
    with LRP_ENOMEM instead of staying queued."""
    log("serve over budget")
    c = binding.Context(0, workspace_bytes=64 << 20)
    try:
        rng = np.random.default_rng(5)
        U = dev(rng.standard_normal((1024, 4)))
        V = dev(rng.standard_normal((1024, 4)))
        t, _ = c.submit(U, V, 1e-8, prec="fp64")
        res = _serve_until_done(c, [t])
        assert res[t][0] == binding.LRP_ENOMEM, res[t]
    finally:
        c.close()


def test_served_frees_cached_batch_groups():
    """Serving a shape whose slot group does not fit beside the group that a
    synchronous batch call left cached frees that cache and then runs, with
    the batch's result."""
    n, count, eps = 1024, 256, 1e-8
    rng = np.random.default_rng(6)
    x = np.linspace(0.0, 1.0, n + 2)[1:-1]
    U = dev(np.stack([np.exp(-(x - a) ** 2 / 0.01) for a in (0.3, 0.5, 0.7)], 1))
    V = dev(np.stack([np.exp(-(x - a) ** 2 / 0.02) * w for a, w in
                      ((0.4, 1.0), (0.6, -0.5), (0.2, 0.3))], 1))
    problems = [(U, V, eps)] * count

    def batch_fits(budget):
        c = binding.Context(0, workspace_bytes=budget)
        try:
            c.batch2d(problems, prec="fp64").run(results=False)
            return True
        except binding.LrpError as e:
            assert e.status == binding.LRP_ENOMEM, e
            return False
        finally:
            c.close()

    # the smallest budget that holds the batch's group, to 1/64 of it
    lo, hi = 16 << 20, 8 << 30
    assert batch_fits(hi)
    while hi - lo > hi >> 6:
        mid = (lo + hi) // 2
        if batch_fits(mid):
            hi = mid
        else:
            lo = mid
    log("serve after batch: batch needs <=", hi >> 20, "MiB")
    # room for the batch's group, not for a 32-slot group beside it
    c = binding.Context(0, workspace_bytes=hi + (hi >> 5))
    try:
        (Ub, Vb, _), = c.batch2d(problems[:1] * count, prec="fp64").run()[:1]
        want = host(Ub) @ host(Vb).T
        t, outs = c.submit(U, V, eps, prec="fp64")
        status, ranks, _ = _serve_until_done(c, [t])[t]
        assert status == binding.LRP_OK, status
        got = assemble(2, served_result(2, outs, ranks))
        d = rel(got, want)
        log("  served vs batch", d)
        assert d <= 1e-12, d
    finally:
        c.close()


# The served stream's largest shapes (2D n = 8192 with rank 64 at eps = 1e-8;
# 3D n = 256 with Tucker ranks 64 and n = 512), in the AUTO plan the
# benchmark serves, submitted together so that they share the device.
BIG = [(2, 8192, 64, 1e-8), (3, 256, 64, 1e-6), (3, 512, 40, 1e-6), (2, 8192, 7, 1e-6),
       (3, 256, 9, 1e-8)]


def test_served_stream_largest_shapes():
    from paper_1306_2150_amd import serving
    reqs = [inputs.Request(rid=i, arrival_s=0.0, dim=d, n=n, r=r, eps=e, seed=5600 + i)
            for i, (d, n, r, e) in enumerate(BIG)]
    facs = serving.prepare(reqs)
    log("serve largest shapes", len(reqs))
    done, _ = serve_all(reqs, facs, "auto", per_tick=len(reqs))
    for i, q in enumerate(reqs):
        (status, ranks, info), outs = done[i]
        log("  req", i, q.dim, q.n, q.r, q.eps, "status", status, "ranks", ranks,
            "sweeps", info["sweeps"])
        assert status == binding.LRP_OK, (i, status)
        if q.dim == 2:
            Ux, Vx = served_result(2, outs, ranks)
            U, V = q.rhs()
            X = poisson.full_solve2d_factors(U, V, workers=16)
            e = metrics.rel_err_factored(host(Ux), host(Vx), X)
        else:
            Xs, G = served_result(3, outs, ranks)
            U1, U2, U3, G0 = q.rhs()
            X = poisson.full_solve3d_tucker(U1, U2, U3, np.asarray(G0), workers=16)
            Us = [host(x) for x in Xs]
            e = metrics.rel_err_tucker(Us[0], Us[1], Us[2], np.asarray(host(G)), X)
            del X
        log("    err", e)
        assert e <= 10 * q.eps, (i, e)
