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


def stokes_half_angles(n: int):
    """sin^2 and cos^2 of pi k/(2(n+1)), k = 1..n, and h.

    The Stokes-consistent Laplacian of Section 2 is built from G = E - Z and
    H = E + Z (shift difference and shift sum from the n+1 cell values to the
    n interior vertices); A1 = G G^T = tridiag(-1, 2, -1) and A2 = H H^T =
    tridiag(1, 2, 1) are diagonalised by the same sine transform (Section
    4.1) with eigenvalues 4 sin^2 and 4 cos^2 of these half angles.
    Pin: A1, A2 built from G, H and compared with eigvalsh.
    """
    N = n + 1
    k = np.arange(1, n + 1, dtype=np.float64)
    t = np.pi * k / (2.0 * N)
    return np.sin(t) ** 2, np.cos(t) ** 2, 1.0 / N


def denominators2d(n1: int, n2: int, op: str = "poisson") -> np.ndarray:
    """Eigenvalue of the 2D operator at sine mode (i, j), an n1 x n2 array.

    poisson: lambda_i + lambda_j (5-point, eq. "div").
    stokes:  4 (B_x B_x^T + B_y B_y^T) with B_x = (G (x) H)/(4h),
             B_y = (H (x) G)/(4h) (Section 2), i.e. the Kronecker form
             A1 (x) A2 + A2 (x) A1 of Section 4.1 scaled by 1/(4 h^2):
             (4 s_i c_j + 4 c_i s_j) / h^2 with s = sin^2, c = cos^2 of the
             half angles.  (The scale 4 makes smooth modes see -Laplacian,
             like the 5-point operator; Section 4.1 leaves the scale free.)
    Pins: dense Kronecker operators built from G and H.
    """
    if op == "poisson":
        return eigenvalues(n1)[:, None] + eigenvalues(n2)[None, :]
    if op != "stokes":
        raise ValueError(op)
    s1, c1, h1 = stokes_half_angles(n1)
    s2, c2, h2 = stokes_half_angles(n2)
    if n1 != n2:
        raise ValueError("the Stokes operator is defined on square grids")
    return 4.0 * (s1[:, None] * c2[None, :] + c1[:, None] * s2[None, :]) / (h1 * h1)


def denominators3d(n: int, op: str = "poisson") -> np.ndarray:
    """Eigenvalue of the 3D operator at sine mode (i, j, l), n x n x n.

    poisson: lambda_i + lambda_j + lambda_l (7-point).
    stokes:  B_x B_x^T + B_y B_y^T + B_z B_z^T with B_x = (G (x) H (x) H)/(4h)
             and its permutations (Section 2):
             4 (s_i c_j c_l + c_i s_j c_l + c_i c_j s_l) / h^2.
    Pins: dense Kronecker operators built from G and H.
    """
    if op == "poisson":
        lam = eigenvalues(n)
        return lam[:, None, None] + lam[None, :, None] + lam[None, None, :]
    if op != "stokes":
        raise ValueError(op)
    s, c, h = stokes_half_angles(n)
    S_, C_ = s[:, None, None], c[:, None, None]
    Sj, Cj = s[None, :, None], c[None, :, None]
    Sl, Cl = s[None, None, :], c[None, None, :]
    return 4.0 * (S_ * Cj * Cl + C_ * Sj * Cl + C_ * Cj * Sl) / (h * h)


def full_solve2d(F: np.ndarray, workers: int | None = None,
                 op: str = "poisson") -> np.ndarray:
    """Full-grid 2D solve X = S[(S F S) / D]S, D = ``denominators2d``.

    Section 4.1's direct method: the sine transform on both sides, a
    division by the operator's eigenvalues, the sine transform back.  Pins: scipy.linalg.solve_sylvester, dense
    Kronecker solve, residual, single sine mode (Stokes operator: dense
    Kronecker solve from G and H).
    """
    F = np.asarray(F, dtype=np.float64)
    n1, n2 = F.shape
    Fh = scipy.fft.dstn(F, type=1, norm="ortho", workers=workers)
    Fh /= denominators2d(n1, n2, op)
    return scipy.fft.idstn(Fh, type=1, norm="ortho", workers=workers)


def full_solve2d_factors(U: np.ndarray, V: np.ndarray,
                         workers: int | None = None, op: str = "poisson") -> np.ndarray:
    """Full-grid solve for F = U V^T (forms F, then ``full_solve2d``)."""
    return full_solve2d(np.asarray(U) @ np.asarray(V).T, workers=workers, op=op)


def full_solve3d(F: np.ndarray, workers: int | None = None,
                 op: str = "poisson") -> np.ndarray:
    """Full-grid 3D solve: S along each mode, divide by the operator's
    eigenvalue (``denominators3d``; for the 7-point Laplacian the three-term
    sum), S back along each mode (the 3D analogue of eq. "diag").

    Pins: dense Kronecker solve at tiny n; single sine mode.
    """
    F = np.asarray(F, dtype=np.float64)
    n1, n2, n3 = F.shape
    Fh = scipy.fft.dstn(F, type=1, norm="ortho", workers=workers)
    if op == "poisson":
        l1, l2, l3 = eigenvalues(n1), eigenvalues(n2), eigenvalues(n3)
        Fh /= (l1[:, None, None] + l2[None, :, None] + l3[None, None, :])
    else:
        if not n1 == n2 == n3:
            raise ValueError("the Stokes operator is defined on cubic grids")
        Fh /= denominators3d(n1, op)
    return scipy.fft.idstn(Fh, type=1, norm="ortho", workers=workers)


def tucker_full(G: np.ndarray, U1: np.ndarray, U2: np.ndarray,
                U3: np.ndarray) -> np.ndarray:
    """Expand a Tucker tensor A(i1,i2,i3) = sum G(a1,a2,a3) U1 U2 U3
    (paper Section 3, eq. "tucker")."""
    return np.einsum("abc,ia,jb,kc->ijk", G, U1, U2, U3, optimize=True)


def full_solve3d_tucker(U1, U2, U3, G, workers: int | None = None,
                        op: str = "poisson"):
    """Full-grid 3D solve for a Tucker RHS (forms F, then ``full_solve3d``)."""
    return full_solve3d(tucker_full(G, U1, U2, U3), workers=workers, op=op)
