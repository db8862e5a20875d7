"""The discrete 2D Stokes problem and its Uzawa (Schur complement) solve in
full format, float64 -- test infrastructure only (the CPU oracle of the
low-rank Stokes driver; nothing here is imported by the library).

Section 2: pressure at the n x n cell centres of [0, 1]^2, h = 1/n, the two
velocity components at the (n-1) x (n-1) interior vertices (zero on the
boundary).  With the (n-1) x n shift matrices E (drops the first entry) and
Z (drops the last), G = E - Z and H = E + Z, i.e. (G x)_i = x_{i+1} - x_i
and (H x)_i = x_{i+1} + x_i, the discrete gradients are
    B_x = (G (x) H) / (4h),   B_y = (H (x) G) / (4h),
written here on matrices whose first index runs along x:
    B_x(P) = G P H^T / (4h),  B_y(P) = H P G^T / (4h),
    B_x^T(U) = G^T U H / (4h), B_y^T(V) = H^T V G / (4h),
and the Laplacian consistent with them is Delta = B_x B_x^T + B_y B_y^T.
The system is  Delta u + B_x p = f_u,  Delta v + B_y p = f_v,
B_x^T u + B_y^T v = g  (eq. "stprob", A = I_2 (x) Delta), and the Uzawa
method solves the Schur system (eq. "schur")
    S p = B^T A^-1 B p = B^T A^-1 f - g
for the pressure, then u = Delta^-1 (f_u - B_x p), v likewise.  S is
symmetric positive semidefinite with a two-dimensional kernel (the constant
and the checkerboard pressure, which B maps to zero), (n-2)^2 eigenvalues
equal to 1 and the rest in an interval bounded away from 0 independently of
h (Section 2), so CG on the complement of the kernel converges in a number
of steps independent of h.

Delta is diagonalised by the sine transform of the velocity grid: it is a
quarter of the Stokes-consistent operator of ``poisson.denominators2d``
(op "stokes", which carries a factor 4 so that smooth modes see the
-Laplacian), hence Delta^-1 F = 4 full_solve2d(F, op="stokes").

The test problem (Section 6, eq. "ansin2d") prescribes
    u = sin 2 pi x (1 - cos 2 pi y) / (4 pi^2),
    v = (1 - cos 2 pi x) sin 2 pi y / (4 pi^2),
    p = sin 2 pi x sin 2 pi y / pi,
and prints right-hand sides that these functions do not satisfy; here the
right-hand sides are derived from them through the continuous operators
that B and Delta approximate: B ~ grad/2 and Delta ~ -Laplacian/4 (G x ~ h
x', H x ~ 2 x), so
    f = -Lap(u)/4 + grad(p)/2  at the vertices,   g = -div(u)/2  at the
cell centres, with g's components along the kernel removed (the discrete
system is solvable only for g orthogonal to it).
"""
from __future__ import annotations

import numpy as np

from .poisson import full_solve2d


def shift_matrices(n: int):
    """G = E - Z and H = E + Z, (n-1) x n (Section 2)."""
    G = np.zeros((n - 1, n))
    H = np.zeros((n - 1, n))
    for i in range(n - 1):
        G[i, i + 1], G[i, i] = 1.0, -1.0
        H[i, i + 1], H[i, i] = 1.0, 1.0
    return G, H


def grad(P: np.ndarray):
    """(B_x P, B_y P) for an n x n pressure P: (n-1) x (n-1) each."""
    n = P.shape[0]
    G, H = shift_matrices(n)
    h = 1.0 / n
    return G @ P @ H.T / (4 * h), H @ P @ G.T / (4 * h)


def grad_t(U: np.ndarray, V: np.ndarray) -> np.ndarray:
    """B_x^T U + B_y^T V for (n-1) x (n-1) velocity components: n x n."""
    n = U.shape[0] + 1
    G, H = shift_matrices(n)
    h = 1.0 / n
    return (G.T @ U @ H + H.T @ V @ G) / (4 * h)


def laplace(U: np.ndarray) -> np.ndarray:
    """Delta U = B_x B_x^T U + B_y B_y^T U on the velocity grid."""
    n = U.shape[0] + 1
    G, H = shift_matrices(n)
    h = 1.0 / n
    return (G @ G.T @ U @ H @ H.T + H @ H.T @ U @ G @ G.T) / (16 * h * h)


def laplace_solve(F: np.ndarray) -> np.ndarray:
    """Delta^-1 F (sine transform, divide, transform back)."""
    return 4.0 * full_solve2d(F, op="stokes")


def schur(P: np.ndarray) -> np.ndarray:
    """S P = B_x^T Delta^-1 B_x P + B_y^T Delta^-1 B_y P."""
    Bx, By = grad(P)
    return grad_t(laplace_solve(Bx), laplace_solve(By))


def kernel_basis(n: int):
    """The constant and the checkerboard pressure, unit Frobenius norm."""
    c = (-1.0) ** np.arange(n)
    return np.ones((n, n)) / n, np.outer(c, c) / n


def project(P: np.ndarray) -> np.ndarray:
    """P without its components along the kernel of B."""
    out = P.copy()
    for K in kernel_basis(P.shape[0]):
        out -= np.sum(P * K) * K
    return out


def ansin2d(n: int):
    """Right-hand sides and the prescribed solution of the test problem on
    grid n: (f_u, f_v, g, u, v, p), g projected off the kernel."""
    h = 1.0 / n
    xv = np.arange(1, n) * h
    xc = (np.arange(n) + 0.5) * h
    t = 2 * np.pi
    sv, cv = np.sin(t * xv), np.cos(t * xv)
    sc, cc = np.sin(t * xc), np.cos(t * xc)
    ov, oc = np.ones(n - 1), np.ones(n)
    # -Lap(u) = sin 2pi x - 2 sin 2pi x cos 2pi y; p_x = 2 cos 2pi x sin 2pi y
    fu = 0.25 * (np.outer(sv, ov) - 2 * np.outer(sv, cv)) + np.outer(cv, sv)
    fv = 0.25 * (np.outer(ov, sv) - 2 * np.outer(cv, sv)) + np.outer(sv, cv)
    # div u = (cos 2pi x + cos 2pi y - 2 cos 2pi x cos 2pi y) / (2 pi)
    g = -(np.outer(cc, oc) + np.outer(oc, cc) - 2 * np.outer(cc, cc)) / (4 * np.pi)
    u = np.outer(sv, 1 - cv) / (4 * np.pi ** 2)
    v = np.outer(1 - cv, sv) / (4 * np.pi ** 2)
    p = np.outer(sc, sc) / np.pi
    return fu, fv, project(g), u, v, p


def ansin2d_factors(n: int):
    """The same right-hand sides as rank-3 factor pairs (U, V) with
    F = U V^T, g's two kernel components appended as two more columns."""
    h = 1.0 / n
    xv = np.arange(1, n) * h
    xc = (np.arange(n) + 0.5) * h
    t = 2 * np.pi
    sv, cv = np.sin(t * xv), np.cos(t * xv)
    cc = np.cos(t * xc)
    ov, oc = np.ones(n - 1), np.ones(n)
    fu = (np.column_stack([0.25 * sv, -0.5 * sv, cv]), np.column_stack([ov, cv, sv]))
    fv = (np.column_stack([0.25 * ov, -0.5 * cv, sv]), np.column_stack([sv, sv, cv]))
    gU = np.column_stack([-cc, -oc, 2 * cc]) / (4 * np.pi)
    gV = np.column_stack([oc, cc, cc])
    G = gU @ gV.T
    K1, K2 = kernel_basis(n)
    c = (-1.0) ** np.arange(n)
    a1, a2 = np.sum(G * K1), np.sum(G * K2)
    gU = np.column_stack([gU, -a1 * oc / n, -a2 * c / n])
    gV = np.column_stack([gV, oc, c])
    return fu, fv, (gU, gV)


def uzawa_cg(fu: np.ndarray, fv: np.ndarray, g: np.ndarray, tol: float = 1e-12,
             maxit: int = 1000):
    """Full-format Uzawa: CG on S p = B^T Delta^-1 f - g from p = 0 (the
    iterates stay off the kernel), stopped at ||r|| <= tol ||b||; then the
    velocity.  Returns (p, u, v, iterations)."""
    b = grad_t(laplace_solve(fu), laplace_solve(fv)) - g
    p = np.zeros_like(b)
    r = b.copy()
    d = r.copy()
    rr = float(np.sum(r * r))
    nb = np.sqrt(rr)
    it = 0
    while np.sqrt(rr) > tol * nb and it < maxit:
        Sd = schur(d)
        al = rr / float(np.sum(d * Sd))
        p += al * d
        r -= al * Sd
        rn = float(np.sum(r * r))
        d = r + (rn / rr) * d
        rr = rn
        it += 1
    Bx, By = grad(p)
    return p, laplace_solve(fu - Bx), laplace_solve(fv - By), it
