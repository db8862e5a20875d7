"""Graph replay of the cross sweep steps (lrp_set_graph_replay): every
replay gives the bits of the plain launches.  The graphs are replayed many
times, with the program's own eager work (other solves, transforms, torch
kernels and synchronisations) between the replays, across batches whose
live-slot counts and rank buckets change, and in the served loop."""
import numpy as np
import pytest
import torch

from oracle import metrics, poisson
from paper_1306_2150_amd import binding, inputs

from gpu_util import ctx, dev, host, log

pytestmark = pytest.mark.gpu


def batch_problems(n, specs):
    out = []
    for inst, eps in specs:
        U, V = inputs.workload_rhs(2, inst, n=n)
        out.append((dev(U), dev(V), eps))
    return out


def snapshot(res):
    return [(host(Ux).copy(), host(Vx).copy(), i["rank"], i["sweeps"]) for Ux, Vx, i in res]


def test_graph_replay_matches_plain_launches():
    n = 1024
    specs = [(1, 1e-8), (2, 1e-6), (3, 1e-10), (4, 1e-8), (5, 1e-12), (6, 1e-7)]
    probs = batch_problems(n, specs)
    c = ctx()
    c.set_graph_replay(False)
    try:
        plain = snapshot(c.solve2d_batch(probs, prec="auto"))
        plain_sub = snapshot(c.solve2d_batch(probs[:3], prec="auto"))
    finally:
        c.set_graph_replay(True)
    other = torch.randn(512, 512, dtype=torch.float64, device="cuda")
    for rep in range(4):
        log("graph replay", rep)
        got = snapshot(c.solve2d_batch(probs, prec="auto"))
        for (Ua, Va, ra, sa), (Ub, Vb, rb, sb) in zip(plain, got):
            assert ra == rb and sa == sb
            assert np.array_equal(Ua, Ub) and np.array_equal(Va, Vb)
        # eager work between replays: a smaller batch (other live-slot
        # counts), a transform, a torch product, a synchronisation
        sub = snapshot(c.solve2d_batch(probs[:3], prec="auto"))
        for (Ua, Va, ra, _), (Ub, Vb, rb, _) in zip(plain_sub, sub):
            assert ra == rb and np.array_equal(Ua, Ub) and np.array_equal(Va, Vb)
        c.sine_transform(probs[0][0], prec="fp64")
        other = other @ other.T / 512.0
        torch.cuda.synchronize()
    U, V = inputs.workload_rhs(2, 1, n=n)
    X = poisson.full_solve2d_factors(U, V)
    assert metrics.rel_err_factored(got[0][0], got[0][1], X) <= 1e-7


def test_graph_replay_served_and_3d_match_plain():
    """A synchronous 2D solve, a 3D solve (its mode crosses replay the inner
    group's graphs) and a served 2D request: graphs on, twice, give the
    bits of graphs off."""
    c = ctx()
    n = 256
    U, V = inputs.workload_rhs(2, 7, n=n)
    U1, U2, U3, G = inputs.workload_rhs(3, 2, n=64)
    d3 = [binding.colmajor(x) for x in (U1, U2, U3)] + [binding.fortran_core(G)]

    def run():
        Ux, Vx, _ = c.solve2d(dev(U), dev(V), 1e-8, prec="auto")
        Xs, Gx, _ = c.solve3d(*d3, 1e-6, prec="auto")
        t, (Sx, Sy) = c.submit(dev(U), dev(V), 1e-8, prec="auto")
        status, ranks, _ = c.wait(t)
        assert status == binding.LRP_OK
        R = ranks[0]
        return [host(Ux).copy(), host(Vx).copy(), host(Gx).copy()] + \
            [host(x).copy() for x in Xs] + [host(Sx[:, :R]).copy(), host(Sy[:, :R]).copy()]

    c.set_graph_replay(False)
    try:
        plain = run()
    finally:
        c.set_graph_replay(True)
    for rep in range(2):
        log("graph replay served/3d", rep)
        got = run()
        assert len(got) == len(plain)
        for a, b in zip(plain, got):
            assert a.shape == b.shape and np.array_equal(a, b)
