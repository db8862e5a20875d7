"""GPU parity of the 3D (Tucker) path against the CPU oracle (through the C-ABI).

The oracle is the full-grid float64 solve of the 7-point problem (sine
transform along the three modes, division by lambda_i + lambda_j + lambda_k,
transform back).  A solve at tolerance eps must match it to 10 eps in the
relative Frobenius norm; the output factors must have orthonormal columns.
Tucker factors and ranks are not unique, so only the assembled tensor is
compared.
"""
import numpy as np
import pytest

from oracle import metrics, poisson
from paper_1306_2150_amd import binding, inputs

from gpu_util import ctx, dev, host, log

pytestmark = pytest.mark.gpu


def run3d(U1, U2, U3, G, eps, prec="fp64", rmax=None, check=True):
    return ctx().solve3d(dev(U1), dev(U2), dev(U3), binding.fortran_core(G), eps,
                         prec=prec, rmax=rmax, check=check)


def err_vs_full(Xs, Gx, X):
    Us = [host(x) for x in Xs]
    G = host(Gx) if Gx.numel() else np.zeros([u.shape[1] for u in Us])
    return metrics.rel_err_tucker(Us[0], Us[1], Us[2], np.asarray(G), X)


ORTH_TOL = {"fp64": 1e-12, "int8": 1e-10, "fp32": 1e-6, "bf16x3": 1e-4}


def orth_err(Xs):
    e = 0.0
    for x in Xs:
        Q = host(x)
        if Q.shape[1]:
            e = max(e, float(np.abs(Q.T @ Q - np.eye(Q.shape[1])).max()))
    return e


@pytest.mark.parametrize("n,ranks,eps,seed", [
    (16, (2, 3, 4), 1e-8, 11),
    (33, (5, 5, 5), 1e-6, 12),
    (64, (16, 16, 16), 1e-8, 13),
    (100, (8, 12, 4), 1e-10, 14),
    (257, (7, 9, 11), 1e-7, 15),
])
def test_solve3d_matches_full_oracle(n, ranks, eps, seed):
    log("solve3d", n, ranks, eps, seed)
    U1, U2, U3, G = inputs.rhs3d_tucker(n, ranks, seed)
    Xs, Gx, info = run3d(U1, U2, U3, G, eps)
    X = poisson.full_solve3d_tucker(U1, U2, U3, np.asarray(G))
    e = err_vs_full(Xs, Gx, X)
    log("  ranks", info["ranks"], "k", info["k"], "sweeps", info["sweeps"], "err", e)
    assert info["status_code"] == binding.LRP_OK
    assert e <= 10 * eps, e
    assert orth_err(Xs) <= 1e-12


def test_solve3d_workload_scaled_down():
    """The 3D workload's recipe (r = 16 per mode, eps = 1e-6) at n = 128."""
    log("solve3d workload n=128")
    U1, U2, U3, G = inputs.workload_rhs(3, 1, n=128)
    Xs, Gx, info = run3d(U1, U2, U3, G, 1e-6)
    X = poisson.full_solve3d_tucker(U1, U2, U3, np.asarray(G))
    e = err_vs_full(Xs, Gx, X)
    log("  ranks", info["ranks"], "err", e)
    assert e <= 1e-5, e


@pytest.mark.parametrize("inst,prec", [(1, "fp64"), (1, "auto"), (2, "auto"), (3, "fp64"),
                                       (4, "auto")])
def test_solve3d_workload_full_size(inst, prec):
    """n = 512, Tucker ranks (16, 16, 16), eps = 1e-6, against the full
    512^3 float64 solve, for four seeded instances, in the float64 plan and
    the AUTO plan (int8 transforms)."""
    log("solve3d workload n=512", inst, prec)
    U1, U2, U3, G = inputs.workload_rhs(3, inst)
    Xs, Gx, info = run3d(U1, U2, U3, G, 1e-6, prec=prec)
    X = poisson.full_solve3d_tucker(U1, U2, U3, np.asarray(G), workers=16)
    e = err_vs_full(Xs, Gx, X)
    log("  ranks", info["ranks"], "k", info["k"], "sweeps", info["sweeps"], "err", e,
        "fwd", info["fwd_prec"], "inv", info["inv_prec"])
    assert info["status_code"] == binding.LRP_OK
    assert e <= 1e-5, e
    # orthonormal to the precision of the inverse transform
    assert orth_err(Xs) <= ORTH_TOL[info["inv_prec"]]


@pytest.mark.parametrize("prec,eps", [("auto", 1e-6), ("fp32", 1e-6), ("bf16x3", 1e-5)])
def test_solve3d_reduced_precision(prec, eps):
    log("solve3d", prec, eps)
    U1, U2, U3, G = inputs.rhs3d_tucker(96, (10, 10, 10), 21)
    Xs, Gx, info = run3d(U1, U2, U3, G, eps, prec=prec)
    X = poisson.full_solve3d_tucker(U1, U2, U3, np.asarray(G))
    e = err_vs_full(Xs, Gx, X)
    log("  fwd", info["fwd_prec"], "inv", info["inv_prec"], "err", e)
    assert e <= 10 * eps, e


def test_solve3d_single_sine_mode_exact():
    """F = c s_p x s_q x s_w (sine modes) has the solution F / (lambda_p +
    lambda_q + lambda_w): Tucker rank (1, 1, 1)."""
    n, modes = 50, (1, 3, 7)
    log("solve3d sine mode", n, modes)
    i = np.arange(1, n + 1, dtype=np.float64)
    Us = [np.sin(p * np.pi * i / (n + 1))[:, None] for p in modes]
    G = np.full((1, 1, 1), 2.0)
    Xs, Gx, info = run3d(Us[0], Us[1], Us[2], G, 1e-10)
    lam = poisson.eigenvalues(n)
    X = poisson.tucker_full(G, *Us) / (lam[modes[0] - 1] + lam[modes[1] - 1] + lam[modes[2] - 1])
    assert info["ranks"] == (1, 1, 1)
    assert err_vs_full(Xs, Gx, X) <= 1e-12


def test_solve3d_small_grids():
    for n in (1, 2, 3):
        log("solve3d tiny", n)
        rng = np.random.default_rng(n)
        Us = [rng.standard_normal((n, 1)) for _ in range(3)]
        G = np.ones((1, 1, 1))
        Xs, Gx, info = run3d(Us[0], Us[1], Us[2], G, 1e-10)
        X = poisson.full_solve3d_tucker(Us[0], Us[1], Us[2], G)
        assert err_vs_full(Xs, Gx, X) <= 1e-9


def test_solve3d_zero_rhs():
    log("solve3d zero core")
    U1, U2, U3, G = inputs.rhs3d_tucker(40, (3, 3, 3), 31)
    Xs, Gx, info = run3d(U1, U2, U3, np.zeros_like(np.asarray(G)), 1e-8)
    assert info["status_code"] == binding.LRP_OK
    assert info["ranks"] == (0, 0, 0)


def test_solve3d_nonfinite():
    log("solve3d nan")
    U1, U2, U3, G = inputs.rhs3d_tucker(40, (3, 3, 3), 32)
    U2 = U2.copy()
    U2[5, 1] = np.nan
    Xs, Gx, info = run3d(U1, U2, U3, G, 1e-8, check=False)
    assert info["status_code"] == binding.LRP_ENONFINITE


def test_solve3d_rank_capacity():
    log("solve3d rmax")
    U1, U2, U3, G = inputs.rhs3d_tucker(64, (8, 8, 8), 33)
    Xs, Gx, info = run3d(U1, U2, U3, G, 1e-8, rmax=(2, 2, 2), check=False)
    assert info["status_code"] == binding.LRP_ERANKCAP
    assert max(info["ranks"]) > 2


def sine_modes(n, ps):
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.stack([np.sin(p * np.pi * i / (n + 1)) for p in ps], axis=1)


def tucker_diff_rel(G1, Us1, G2, Us2):
    """||[[G1; Us1]] - [[G2; Us2]]||_F / ||[[G2; Us2]]||_F without forming
    either tensor: QR of the stacked factors per mode, then the norm of the
    block-diagonal core difference transformed by the R factors."""
    shapes1, shapes2 = G1.shape, G2.shape
    big = np.zeros(tuple(shapes1[d] + shapes2[d] for d in range(3)))
    big[:shapes1[0], :shapes1[1], :shapes1[2]] = G1
    big[shapes1[0]:, shapes1[1]:, shapes1[2]:] = -G2
    ref = G2.copy()
    for d in range(3):
        _, R = np.linalg.qr(np.hstack([Us1[d], Us2[d]]))
        big = np.moveaxis(np.tensordot(R, np.moveaxis(big, d, 0), axes=(1, 0)), 0, d)
        _, R2 = np.linalg.qr(Us2[d])
        ref = np.moveaxis(np.tensordot(R2, np.moveaxis(ref, d, 0), axes=(1, 0)), 0, d)
    return float(np.linalg.norm(big) / np.linalg.norm(ref))


@pytest.mark.parametrize("n,eps", [(2048, 1e-8), (6000, 1e-7)])
def test_solve3d_large_grid_semi_analytic(n, eps):
    """Beyond the grids a full 3D oracle solve can check: a right-hand side
    F = sum_m s_(p_m) x s_(q_m) x w_m (sine modes in the first two modes, any
    w_m) has the solution sum_m s_(p_m) x s_(q_m) x z_m with
    (T + (lambda_p_m + lambda_q_m) I) z_m = w_m, a tridiagonal solve; the
    GPU's Tucker result is compared with it in factored form."""
    import scipy.linalg
    log("solve3d large grid", n, eps)
    rng = np.random.default_rng(n)
    ps, qs = [3, 40], [7, 11]
    U1, U2 = sine_modes(n, ps), sine_modes(n, qs)
    x = np.arange(1, n + 1) / (n + 1)
    W = np.stack([np.exp(-(x - 0.3) ** 2 / 0.01), np.exp(-(x - 0.7) ** 2 / 0.05) * x], 1)
    G = np.zeros((2, 2, 2))
    G[0, 0, 0], G[1, 1, 1] = 1.0, -0.5
    lam = poisson.eigenvalues(n)
    h2 = (n + 1.0) ** 2
    Z = np.empty_like(W)
    for m in range(2):
        shift = lam[ps[m] - 1] + lam[qs[m] - 1]
        ab = np.zeros((3, n))
        ab[0, 1:] = -h2
        ab[1, :] = 2 * h2 + shift
        ab[2, :-1] = -h2
        Z[:, m] = scipy.linalg.solve_banded((1, 1), ab, W[:, m])
    Xs, Gx, info = run3d(U1, U2, W, G, eps)
    log("  ranks", info["ranks"], "sweeps", info["sweeps"])
    assert info["status_code"] == binding.LRP_OK
    e = tucker_diff_rel(np.asarray(host(Gx)), [host(x) for x in Xs], G, [U1, U2, Z])
    log("  err", e)
    assert e <= 10 * eps, e


def test_solve3d_workspace_linear_in_n():
    """The 3D workspace no longer holds n x n^2 unfoldings: a 2048-point
    solve runs inside a 2 GiB context budget."""
    log("solve3d budget")
    c = binding.Context(0, workspace_bytes=2 << 30)
    try:
        U1, U2, U3, G = inputs.rhs3d_tucker(2048, (6, 6, 6), 51)
        Xs, Gx, info = c.solve3d(dev(U1), dev(U2), dev(U3), binding.fortran_core(G), 1e-6)
        assert info["status_code"] == binding.LRP_OK
    finally:
        c.close()


def test_solve3d_invalid_arguments():
    log("solve3d einval")
    n = binding.MAX_N3 + 1
    U = np.ones((n, 1))
    G = np.ones((1, 1, 1))
    with pytest.raises(binding.LrpError) as ei:
        run3d(U, U, U, G, 1e-6)
    assert ei.value.status == binding.LRP_EINVAL
    with pytest.raises(binding.LrpError):
        run3d(U[:8], U[:8], U[:8], G, 0.0)


def test_solve3d_repeatable():
    log("solve3d repeat")
    U1, U2, U3, G = inputs.rhs3d_tucker(48, (6, 5, 4), 41)
    a = run3d(U1, U2, U3, G, 1e-8)
    b = run3d(U1, U2, U3, G, 1e-8)
    for x, y in zip(a[0], b[0]):
        assert np.array_equal(host(x), host(y))
    assert np.array_equal(host(a[1]), host(b[1]))
