"""Pins of the exponential-sum comparator's oracle (oracle/expsum.py).

The quadrature is pinned to the function it approximates: the relative
error |x sum w e^(-p x) - 1| is checked on a grid far denser than the one the
construction used and at random points, and a planted mistake (weights
without the Jacobian e^t of the substitution p = e^t) must fail that check.
The solver is pinned to the full-grid solve (10 eps) and to the single-mode
closed form; a planted mistake (the exponential sum without its weights)
must fail."""
import numpy as np
import pytest

from oracle import expsum, metrics, poisson
from paper_1306_2150_amd import inputs


def dense_check(w, p, a, b, seed=0):
    x = np.concatenate([np.geomspace(a, b, 50000),
                        np.exp(np.random.default_rng(seed).uniform(np.log(a), np.log(b), 5000))])
    return float(np.max(np.abs(x * (np.exp(-np.outer(x, p)) @ w) - 1.0)))


@pytest.mark.parametrize("a,b,eps", [(1.0, 10.0, 1e-6), (1.0, 1e6, 1e-8),
                                     (19.7, 8.39e6, 1e-7), (0.5, 2.0, 1e-12)])
def test_expsum_relative_error(a, b, eps):
    w, p = expsum.expsum_1x(a, b, eps)
    assert dense_check(w, p, a, b) <= eps * 1.05
    assert np.all(w > 0) and np.all(p > 0)


def test_expsum_terms_grow_with_accuracy_and_range():
    r1 = len(expsum.expsum_1x(1.0, 1e4, 1e-6)[1])
    r2 = len(expsum.expsum_1x(1.0, 1e4, 1e-10)[1])
    r3 = len(expsum.expsum_1x(1.0, 1e8, 1e-6)[1])
    assert r1 < r2 and r1 < r3


def test_expsum_mutant_missing_jacobian_is_caught():
    a, b, eps = 1.0, 1e4, 1e-7
    w, p = expsum.expsum_1x(a, b, eps)
    h = np.log(p[1] / p[0])
    assert dense_check(np.full_like(w, h), p, a, b) > 1e-2


def test_expsum_paper_setting_term_count():
    """n = 1024, eps = 1e-7 (the paper's comparison, which reports a rank of
    35 for the inverse with a node construction it does not give): the sinc
    rule here takes about twice that; the eps-rank of the matrix
    1/(lambda_i + lambda_j) itself (a lower bound for any sum of rank-1
    Kronecker terms in the Frobenius sense) is 19."""
    from oracle.lowrank import truncation_rank
    a, b = expsum.operator_range(1024)
    w, p = expsum.expsum_1x(a, b, 1e-7)
    assert 30 <= len(p) <= 80
    lam = poisson.eigenvalues(1024)
    s = np.linalg.svd(1.0 / (lam[:, None] + lam[None, :]), compute_uv=False)
    assert truncation_rank(s, 1e-7) <= len(p)


@pytest.mark.parametrize("n,inst,eps", [(256, 1, 1e-7), (500, 2, 1e-6), (300, 3, 1e-9)])
def test_expsum_solve2d_vs_full(n, inst, eps):
    U, V = inputs.workload_rhs(2, inst, n=n)
    Ux, Vx, info = expsum.expsum_solve2d(U, V, eps)
    X = poisson.full_solve2d_factors(U, V)
    assert metrics.rel_err_factored(Ux, Vx, X) <= 10 * eps
    assert info["Rr"] == info["R"] * U.shape[1]


def test_expsum_solve2d_single_mode():
    n, p, q = 400, 3, 250
    i = np.arange(1, n + 1)
    u = np.sin(p * np.pi * i / (n + 1))[:, None]
    v = np.sin(q * np.pi * i / (n + 1))[:, None]
    lam = poisson.eigenvalues(n)
    Ux, Vx, info = expsum.expsum_solve2d(u, v, 1e-9)
    X = (u @ v.T) / (lam[p - 1] + lam[q - 1])
    assert info["rank"] == 1
    assert metrics.rel_err_factored(Ux, Vx, X) <= 1e-8


def test_expsum_solve2d_mutant_unweighted_is_caught(monkeypatch):
    real = expsum.expsum_1x
    monkeypatch.setattr(expsum, "expsum_1x",
                        lambda a, b, eps: (np.ones_like(real(a, b, eps)[0]), real(a, b, eps)[1]))
    U, V = inputs.workload_rhs(2, 1, n=256)
    Ux, Vx, _ = expsum.expsum_solve2d(U, V, 1e-7)
    X = poisson.full_solve2d_factors(U, V)
    assert metrics.rel_err_factored(Ux, Vx, X) > 1e-3


def test_expsum_nodes_are_a_trapezoidal_rule_of_the_integral():
    """The nodes discretise 1/x = int exp(t - x e^t) dt (which scipy's
    adaptive quadrature confirms at a few x): t_k = log p_k equally spaced by
    h, w_k = h p_k, and the tails cut where the bounds put them."""
    from scipy import integrate
    for x in (0.3, 7.0, 1234.5):
        val, _ = integrate.quad(lambda t: np.exp(t - x * np.exp(t)), -60.0, 10.0, limit=400,
                                epsabs=0.0, epsrel=1e-13)
        assert abs(val * x - 1.0) < 1e-10
    a, b, eps = 19.7, 8.39e6, 1e-7
    w, p = expsum.expsum_1x(a, b, eps)
    t = np.log(p)
    h = np.diff(t)
    assert np.allclose(h, h[0], rtol=1e-12, atol=0.0)
    assert np.allclose(w, h[0] * p, rtol=1e-13, atol=0.0)
    assert abs(t[0] - np.log(eps / (3 * b))) < 1e-12
    assert t[-1] >= np.log(np.log(3 / eps) / a) - 1e-12


def test_expsum_kronecker_form_entry_by_entry():
    """sum_k w_k exp(-p_k lambda_i) exp(-p_k lambda_j) against
    1/(lambda_i + lambda_j) on every (i, j) of a 64-point grid."""
    n, eps = 64, 1e-9
    lam = poisson.eigenvalues(n)
    w, p = expsum.expsum_1x(*expsum.operator_range(n), eps)
    E = np.exp(-np.outer(lam, p))
    L = (E * w) @ E.T
    exact = 1.0 / (lam[:, None] + lam[None, :])
    assert np.max(np.abs(L / exact - 1.0)) <= eps * 1.05


@pytest.mark.parametrize("cut", ["left", "right"])
def test_expsum_mutant_tail_cut_early_is_caught(cut):
    """Cutting either tail of the integral short (two nodes fewer at that
    end) breaks the bar the rule is held to (eps, 5 % slack) somewhere in
    the range."""
    a, b, eps = 1.0, 1e6, 1e-8
    w, p = expsum.expsum_1x(a, b, eps)
    sl = slice(2, None) if cut == "left" else slice(None, -2)
    assert dense_check(w[sl], p[sl], a, b) > 1.05 * eps


@pytest.mark.parametrize("mutant", ["weights_both_sides", "reversed_spectrum"])
def test_expsum_solve2d_planted_mistakes_are_caught(mutant, monkeypatch):
    """A weight applied on both factors (w^2 instead of w), or the
    exponentials taken of the reversed spectrum (an index mistake), must fail
    the full-solve bar."""
    real = expsum.expsum_1x
    if mutant == "weights_both_sides":
        monkeypatch.setattr(expsum, "expsum_1x",
                            lambda a, b, eps: (real(a, b, eps)[0] ** 2, real(a, b, eps)[1]))
    else:
        real_eig, rng = expsum.eigenvalues, expsum.operator_range(256)
        monkeypatch.setattr(expsum, "operator_range", lambda n: rng)
        monkeypatch.setattr(expsum, "eigenvalues", lambda n: real_eig(n)[::-1].copy())
    U, V = inputs.workload_rhs(2, 1, n=256)
    Ux, Vx, _ = expsum.expsum_solve2d(U, V, 1e-7)
    monkeypatch.undo()
    X = poisson.full_solve2d_factors(U, V)
    assert metrics.rel_err_factored(Ux, Vx, X) > 1e-3
