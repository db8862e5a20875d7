"""GPU parity of the Stokes-consistent Laplacian (the operator of Section 2,
sum_d B_d B_d^T with the discrete gradients built from the shift difference
and shift sum; its Kronecker form is A1 (x) A2 + A2 (x) A1, Section 4.1)
against the CPU oracle (``poisson.full_solve2d`` / ``full_solve3d`` with
op = "stokes"), through the C-ABI.  The sine modes are its eigenvectors, so
the same transform diagonalises it; only the eigenvalue dividing the
transformed right-hand side differs.  Bar: 10 eps relative Frobenius."""
import numpy as np
import pytest

from oracle import metrics, poisson
from paper_1306_2150_amd import binding, inputs

from gpu_util import ctx, dev, host, log

pytestmark = pytest.mark.gpu


def sine_mode(n, p):
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.sin(p * np.pi * i / (n + 1))


@pytest.mark.parametrize("n,inst,eps,prec", [
    (256, 1, 1e-10, "fp64"), (1000, 2, 1e-8, "fp64"), (2049, 3, 1e-8, "auto"),
    (4096, 1, 1e-8, "auto"), (4096, 2, 1e-6, "fp64"), (3, 1, 1e-12, "fp64")])
def test_stokes_solve2d_matches_oracle(n, inst, eps, prec):
    log("stokes 2d", n, inst, eps, prec)
    U, V = inputs.workload_rhs(2, inst, n=n)
    Ux, Vx, info = ctx().solve2d(dev(U), dev(V), eps, prec=prec, op="stokes")
    X = poisson.full_solve2d_factors(U, V, op="stokes")
    e = metrics.rel_err_factored(host(Ux), host(Vx), X)
    log("  rank", info["rank"], "sweeps", info["sweeps"], "err", e)
    assert info["status_code"] == binding.LRP_OK
    assert e <= 10 * eps, e
    # the two operators' solutions differ by O(h^2) (relative); where that
    # difference is well above the tolerance, the result is the Stokes one
    XL = poisson.full_solve2d_factors(U, V)
    gap = float(np.linalg.norm(X - XL) / np.linalg.norm(XL))
    if gap > 100 * eps:
        assert metrics.rel_err_factored(host(Ux), host(Vx), XL) > 0.5 * gap


@pytest.mark.parametrize("p,q", [(5, 40), (4093, 4086), (4096, 4095)])
def test_stokes_single_mode_closed_form(p, q):
    """F = s_p s_q^T gives X = F / D_pq exactly, D the Stokes eigenvalue
    4 (s_p c_q + c_p s_q)/h^2 (half-angle sin^2, cos^2).  The operator's
    smallest eigenvalues sit at both corners of the spectrum (the smooth
    modes and the checkerboard-like modes near p = q = n), so the modes
    chosen here have eigenvalues of the same order as the smallest: the
    rounding noise of the transforms, divided by the smallest eigenvalue,
    stays small against the solution (a mode with D_pq ~ 1e7 D_min would
    carry ~1e-9 of such noise, in any float64 solver)."""
    log("stokes single mode", p, q)
    n = 4096
    u, v = sine_mode(n, p), sine_mode(n, q)
    Ux, Vx, info = ctx().solve2d(dev(u[:, None]), dev(v[:, None]), 1e-10, op="stokes")
    assert info["rank"] == 1
    h = 1.0 / (n + 1)
    sp, cp = np.sin(np.pi * p * h / 2) ** 2, np.cos(np.pi * p * h / 2) ** 2
    sq, cq = np.sin(np.pi * q * h / 2) ** 2, np.cos(np.pi * q * h / 2) ** 2
    X = np.outer(u, v) / (4.0 * (sp * cq + cp * sq) / h ** 2)
    assert metrics.rel_err_factored(host(Ux), host(Vx), X) < 1e-11


def test_stokes_batch_mixed_with_laplace_served():
    """Served Stokes and Laplace requests of one grid size share a slot
    group; each result matches its own operator's oracle."""
    log("stokes served mix")
    c = ctx()
    n = 1024
    jobs = []
    for i, op in enumerate(["stokes", "laplace", "stokes", "laplace"]):
        U, V = inputs.rhs2d_bumps(n, 8 + 4 * i, 9100 + i)
        Ud, Vd = dev(U), dev(V)       # inputs stay alive until the request finished
        t, outs = c.submit(Ud, Vd, 1e-8, prec="auto", op=op)
        jobs.append((t, outs, U, V, op, Ud, Vd))
    for t, outs, U, V, op, _, _ in jobs:
        status, ranks, _ = c.wait(t)
        assert status == binding.LRP_OK
        R = ranks[0]
        X = poisson.full_solve2d_factors(U, V, op={"laplace": "poisson"}.get(op, op))
        e = metrics.rel_err_factored(host(outs[0][:, :R]), host(outs[1][:, :R]), X)
        log("  ", op, "rank", R, "err", e)
        assert e <= 1e-7, (op, e)


@pytest.mark.parametrize("n,ranks,eps,seed", [
    (24, (3, 4, 5), 1e-8, 21), (64, (8, 8, 8), 1e-6, 22), (128, (16, 16, 16), 1e-6, 23)])
def test_stokes_solve3d_matches_oracle(n, ranks, eps, seed):
    log("stokes 3d", n, ranks, eps)
    U1, U2, U3, G = inputs.rhs3d_tucker(n, ranks, seed)
    Xs, Gx, info = ctx().solve3d(dev(U1), dev(U2), dev(U3), binding.fortran_core(G), eps,
                                 op="stokes")
    X = poisson.full_solve3d_tucker(U1, U2, U3, np.asarray(G), op="stokes")
    Us = [host(x) for x in Xs]
    e = metrics.rel_err_tucker(Us[0], Us[1], Us[2], np.asarray(host(Gx)), X)
    log("  ranks", info["ranks"], "sweeps", info["sweeps"], "err", e)
    assert info["status_code"] == binding.LRP_OK
    assert e <= 10 * eps, e
