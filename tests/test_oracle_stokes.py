"""Pins of the Stokes oracle (oracle/stokes.py) against what Section 2 and
the mathematics fix:
  - the gradients and the Laplacian in matrix form against dense Kronecker
    products assembled entry by entry from G = E - Z and H = E + Z;
  - Delta^-1 (the sine-transform solve) against a dense solve;
  - the Schur complement's spectrum as Section 2 states it: two zero
    eigenvalues (the constant and the checkerboard pressure), (n-2)^2
    eigenvalues equal to 1, the rest in (0, 1] bounded away from 0 as h
    falls;
  - the Uzawa solve: exact recovery of a discrete solution, second-order
    convergence to the prescribed solution of eq. "ansin2d" (the error
    ratio per halving of h near 4, magnitudes of the order Table 1
    prints), an iteration count that does not grow like 1/h;
  - planted mistakes that must fail: G and H swapped in one gradient, the
    factor 4 of the Laplacian's inverse dropped, the divergence's sign
    flipped."""
import numpy as np
import pytest

from oracle import poisson, stokes


def dense(n):
    G, H = stokes.shift_matrices(n)
    h = 1.0 / n
    # column-major vec: vec(A X B^T) = kron(B, A) vec(X)
    Bx = np.kron(H, G) / (4 * h)
    By = np.kron(G, H) / (4 * h)
    return Bx, By


def vec(X):
    return X.reshape(-1, order="F")


def test_shift_matrices_entrywise():
    G, H = stokes.shift_matrices(5)
    x = np.arange(5.0) ** 2
    assert np.allclose(G @ x, x[1:] - x[:-1]) and np.allclose(H @ x, x[1:] + x[:-1])
    assert G.shape == (4, 5)


@pytest.mark.parametrize("n", [4, 7])
def test_matrix_form_against_dense_kronecker(n):
    rng = np.random.default_rng(n)
    Bx, By = dense(n)
    P = rng.standard_normal((n, n))
    U, V = rng.standard_normal((2, n - 1, n - 1))
    gx, gy = stokes.grad(P)
    assert np.allclose(vec(gx), Bx @ vec(P)) and np.allclose(vec(gy), By @ vec(P))
    assert np.allclose(vec(stokes.grad_t(U, V)), Bx.T @ vec(U) + By.T @ vec(V))
    D = Bx @ Bx.T + By @ By.T
    assert np.allclose(vec(stokes.laplace(U)), D @ vec(U))
    assert np.allclose(vec(stokes.laplace_solve(U)), np.linalg.solve(D, vec(U)))


@pytest.mark.parametrize("n", [6, 8, 10])
def test_schur_spectrum_as_section_2_states(n):
    Bx, By = dense(n)
    D = Bx @ Bx.T + By @ By.T
    B = np.vstack([Bx, By])
    S = B.T @ np.linalg.solve(np.kron(np.eye(2), D), B)
    assert np.allclose(S, S.T)
    ev = np.linalg.eigvalsh((S + S.T) / 2)
    assert np.sum(np.abs(ev) < 1e-10) == 2
    assert np.sum(np.abs(ev - 1.0) < 1e-10) == (n - 2) ** 2
    rest = ev[np.abs(ev) >= 1e-10]
    assert rest.min() > 0.2 and rest.max() < 1.0 + 1e-12
    # the kernel: constant and checkerboard, mapped to zero by B
    for K in stokes.kernel_basis(n):
        gx, gy = stokes.grad(K)
        assert np.abs(gx).max() < 1e-12 and np.abs(gy).max() < 1e-12


def test_schur_matrix_free_against_dense():
    n = 7
    rng = np.random.default_rng(3)
    Bx, By = dense(n)
    D = Bx @ Bx.T + By @ By.T
    B = np.vstack([Bx, By])
    S = B.T @ np.linalg.solve(np.kron(np.eye(2), D), B)
    P = rng.standard_normal((n, n))
    assert np.allclose(vec(stokes.schur(P)), S @ vec(P))


def test_uzawa_recovers_a_discrete_solution():
    """Right-hand sides made by the discrete operators from a known (u, v, p)
    give back that p (off the kernel) and that (u, v)."""
    n = 24
    rng = np.random.default_rng(5)
    p = stokes.project(rng.standard_normal((n, n)))
    u, v = rng.standard_normal((2, n - 1, n - 1))
    gx, gy = stokes.grad(p)
    fu, fv = stokes.laplace(u) + gx, stokes.laplace(v) + gy
    g = stokes.grad_t(u, v)
    ps, us, vs, it = stokes.uzawa_cg(fu, fv, g, tol=1e-13)
    assert np.linalg.norm(stokes.project(ps) - p) <= 1e-9 * np.linalg.norm(p)
    assert np.linalg.norm(us - u) <= 1e-9 * np.linalg.norm(u)
    assert np.linalg.norm(vs - v) <= 1e-9 * np.linalg.norm(v)


def ansin_error(n):
    fu, fv, g, u, v, p = stokes.ansin2d(n)
    ps, us, vs, it = stokes.uzawa_cg(fu, fv, g, tol=1e-12)
    pe = stokes.project(p)
    return (np.linalg.norm(stokes.project(ps) - pe) / np.linalg.norm(pe),
            np.linalg.norm(us - u) / np.linalg.norm(u), it)


def test_ansin2d_second_order_and_table1_magnitude():
    errs = {n: ansin_error(n) for n in (32, 64, 128)}
    r1 = errs[32][0] / errs[64][0]
    r2 = errs[64][0] / errs[128][0]
    assert 3.7 < r1 < 4.3 and 3.7 < r2 < 4.3, (r1, r2)
    # Table 1 prints 1.2e-3 at n = 64 and 2.9e-4 at n = 128 for its setting
    assert 5e-4 < errs[64][0] < 5e-3 and 1e-4 < errs[128][0] < 1.5e-3
    assert errs[128][1] < errs[64][1] < errs[32][1]
    # iterations independent of h up to the tolerance's slow growth
    assert errs[128][2] <= 2 * errs[32][2]


def test_ansin2d_factors_match_dense_right_hand_sides():
    n = 20
    fu, fv, g, *_ = stokes.ansin2d(n)
    (Uu, Vu), (Uv, Vv), (Ug, Vg) = stokes.ansin2d_factors(n)
    assert np.allclose(Uu @ Vu.T, fu) and np.allclose(Uv @ Vv.T, fv)
    assert np.allclose(Ug @ Vg.T, g)
    for K in stokes.kernel_basis(n):
        assert abs(np.sum(g * K)) < 1e-13


@pytest.mark.parametrize("mutant", ["gh_swapped", "no_factor_4", "div_sign"])
def test_planted_mistakes_are_caught(mutant, monkeypatch):
    if mutant == "gh_swapped":
        real = stokes.grad

        def bad_grad(P):
            n = P.shape[0]
            G, H = stokes.shift_matrices(n)
            gx, gy = real(P)
            return G @ P @ G.T / (4.0 / n), gy
        monkeypatch.setattr(stokes, "grad", bad_grad)
    elif mutant == "no_factor_4":
        monkeypatch.setattr(stokes, "laplace_solve", lambda F: poisson.full_solve2d(F, op="stokes"))
    else:
        real_t = stokes.grad_t
        monkeypatch.setattr(stokes, "grad_t", lambda U, V: -real_t(U, V))
    caught = False
    try:
        e = ansin_error(64)[0]
        caught = not (e < 5e-3)
    except (ZeroDivisionError, FloatingPointError, ValueError):
        caught = True
    if mutant == "gh_swapped":
        n = 6
        P = np.random.default_rng(0).standard_normal((n, n))
        K = stokes.kernel_basis(n)[1]
        gx, _ = stokes.grad(K)
        caught = caught or np.abs(gx).max() > 1e-8
    assert caught
