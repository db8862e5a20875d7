"""Plain definitions of the discrete Poisson problem and its full-grid solver.

Test infrastructure only (see the package docstring).

Problem (paper Section 4.1, eq. "pois"; readings):
  * n interior unknowns per axis, h = 1/(n+1), zero Dirichlet boundary
    (the paper writes h = 1/n with n-1 unknowns, Sections 2-3; only the
    counting differs).
  * 1D operator T = h^-2 tridiag(-1, 2, -1) (positive definite); the 2D
    operator is T (x) I + I (x) T, the 3D one the three-term sum.  The
    paper says the scale is immaterial (Section 4.1); this scale makes the
    discrete solution approximate the continuous -Lap u = f.
  * 2D unknown stored as an n x n matrix X with X[i, j] = u(x_i, y_j); the
    equation is T X + X T = F (Kronecker form (T(x)I + I(x)T) vec X = vec F).

The paper's Section 4.1 diagonalises the operator with the discrete sine
transform (eq. "diag"): S T S = diag(lambda), S = S^T = S^-1 with
S[j, k] = sqrt(2/(n+1)) sin(pi j k/(n+1)), j, k = 1..n, and
lambda_k = 4/h^2 sin^2(pi k h / 2).  The full-format solve is then:
transform, divide by lambda_i + lambda_j (+ lambda_l), transform back.
"""
from __future__ import annotations

import numpy as np
import scipy.fft


def mesh_h(n: int) -> float:
    """Mesh size h = 1/(n+1) for n interior points."""
    return 1.0 / (n + 1)


def laplacian_1d(n: int) -> np.ndarray:
    """Dense T = h^-2 tridiag(-1, 2, -1) of order n (positive definite)."""
    h = mesh_h(n)
    T = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    return T / (h * h)


def eigenvalues(n: int) -> np.ndarray:
    """lambda_k = 4/h^2 sin^2(pi k h/2), k = 1..n (eq. "diag").

    Evaluated in the sin^2 form; 2 - 2cos loses relative accuracy at small k.
    Pin: equals numpy.linalg.eigvalsh(laplacian_1d(n)).
    """
    h = mesh_h(n)
    k = np.arange(1, n + 1, dtype=np.float64)
    s = np.sin(np.pi * k * h / 2.0)
    return 4.0 / (h * h) * s * s


def sine_matrix(n: int) -> np.ndarray:
    """Explicit orthonormal DST-I matrix S[j,k] = sqrt(2/(n+1)) sin(pi jk/(n+1)).

    Pin: S^T S = I and S T S = diag(lambda) (eq. "diag").
    """
    N = n + 1
    j = np.arange(1, n + 1, dtype=np.float64)
    return np.sqrt(2.0 / N) * np.sin(np.pi * np.outer(j, j) / N)


def dst(X: np.ndarray, axis: int = 0) -> np.ndarray:
    """Apply S along ``axis`` (library DST-I with orthonormal scaling).

    Pin: equals sine_matrix(n) @ X.
    """
    return scipy.fft.dst(np.asarray(X, dtype=np.float64), type=1,
                         norm="ortho", axis=axis)


def full_solve2d(F: np.ndarray, workers: int | None = None) -> np.ndarray:
    """Full-grid 2D solve X = S[(S F S) / (lambda_i + lambda_j)]S.

    Section 4.1: "applying the DST, inverting the diagonal matrix, and then
    applying the DST back".  Pins: scipy.linalg.solve_sylvester, dense
    Kronecker solve, residual, single sine mode.
    """
    F = np.asarray(F, dtype=np.float64)
    n1, n2 = F.shape
    Fh = scipy.fft.dstn(F, type=1, norm="ortho", workers=workers)
    lam1 = eigenvalues(n1)
    lam2 = eigenvalues(n2)
    Fh /= (lam1[:, None] + lam2[None, :])
    return scipy.fft.idstn(Fh, type=1, norm="ortho", workers=workers)


def full_solve2d_factors(U: np.ndarray, V: np.ndarray,
                         workers: int | None = None) -> np.ndarray:
    """Full-grid solve for F = U V^T (forms F, then ``full_solve2d``)."""
    return full_solve2d(np.asarray(U) @ np.asarray(V).T, workers=workers)


def full_solve3d(F: np.ndarray, workers: int | None = None) -> np.ndarray:
    """Full-grid 3D solve: S along each mode, divide by the three-term sum,
    S back along each mode (the 3D analogue of eq. "diag").

    Pins: dense Kronecker solve at tiny n; single sine mode.
    """
    F = np.asarray(F, dtype=np.float64)
    n1, n2, n3 = F.shape
    Fh = scipy.fft.dstn(F, type=1, norm="ortho", workers=workers)
    l1, l2, l3 = eigenvalues(n1), eigenvalues(n2), eigenvalues(n3)
    Fh /= (l1[:, None, None] + l2[None, :, None] + l3[None, None, :])
    return scipy.fft.idstn(Fh, type=1, norm="ortho", workers=workers)


def tucker_full(G: np.ndarray, U1: np.ndarray, U2: np.ndarray,
                U3: np.ndarray) -> np.ndarray:
    """Expand a Tucker tensor A(i1,i2,i3) = sum G(a1,a2,a3) U1 U2 U3
    (paper Section 3, eq. "tucker")."""
    return np.einsum("abc,ia,jb,kc->ijk", G, U1, U2, U3, optimize=True)


def full_solve3d_tucker(U1, U2, U3, G, workers: int | None = None):
    """Full-grid 3D solve for a Tucker RHS (forms F, then ``full_solve3d``)."""
    return full_solve3d(tucker_full(G, U1, U2, U3), workers=workers)
