"""Exponential-sum comparator, float64 -- test infrastructure only.

The approach the paper's Section 4.1 compares against (eqs. "int" and
"expsum"): approximate 1/x on the range of the operator's eigenvalues by a
sum of exponentials, 1/x ~ sum_k w_k exp(-p_k x); then, because the 2D
eigenvalue is a sum lambda_i + lambda_j, the inverse of the diagonal matrix
is approximated by a sum of R rank-1 Kronecker products,
    Lambda^-1 ~ sum_k w_k diag(exp(-p_k lambda)) (x) diag(exp(-p_k lambda)),
and Lambda^-1 Fh = Fh / (lambda_i + lambda_j) becomes the Hadamard product of
the rank-r transformed right-hand side with that rank-R matrix: a matrix of
rank R r, rounded by QR + SVD to the tolerance (Section 3).  Section 4.2
notes that R r is large (R and r of order 30), which is the reason for the
cross method; Section 6.1 compares the two at n = 1024, eps = 1e-7.

The quadrature (the paper gives eq. "int" only; its eq. "expsum" is garbled
in its indices and Kronecker factors): with p = e^t,
    1/x = int_0^inf e^(-p x) dp = int_R exp(t - x e^t) dt,
an integrand analytic in the strip |Im t| < pi/2 that decays like e^t as
t -> -inf and doubly exponentially as t -> +inf, so the trapezoidal (sinc)
rule with step h on t_k = t0 + k h converges exponentially:
    1/x ~ h sum_k e^(t_k) exp(-x e^(t_k)),   p_k = e^(t_k), w_k = h e^(t_k).
The nodes here are chosen from the error terms (truncation of both tails and
the discretisation error of the sinc rule) and checked on a dense grid.
"""
from __future__ import annotations

import numpy as np

from .lowrank import truncation_rank
from .poisson import dst, eigenvalues


def relative_error(w, p, a, b, points: int = 4000) -> float:
    """max over x in [a, b] (log-spaced, both ends) of |x sum w e^(-p x) - 1|."""
    x = np.geomspace(a, b, points)
    approx = np.exp(-np.outer(x, p)) @ w
    return float(np.max(np.abs(x * approx - 1.0)))


def expsum_1x(a: float, b: float, eps: float):
    """Weights w and exponents p with |1/x - sum w_k exp(-p_k x)| <= eps / x
    for x in [a, b] (relative accuracy eps), as few terms as the sinc rule
    with the tails cut at the tolerance allows.

    The tails: int_{-inf}^{t0} e^t e^(-x e^t) dt <= e^(t0), relative x e^(t0);
    int_{t1}^{inf} = e^(-x e^(t1))/x, relative e^(-x e^(t1)).  Each gets a
    third of eps (t0 = log(eps/(3 b)), t1 = log(log(3/eps)/a)); the step h is
    the largest on a fine grid of steps whose rule meets eps on [a, b].
    Pins: the relative error on a dense grid and at random points; the
    integral it discretises.
    """
    if not (0.0 < a <= b) or not (0.0 < eps < 1.0):
        raise ValueError((a, b, eps))
    t0 = np.log(eps / (3.0 * b))
    t1 = np.log(np.log(3.0 / eps) / a)
    best = None
    for h in np.linspace(1.5, 0.05, 300):
        K = int(np.ceil((t1 - t0) / h)) + 1
        t = t0 + h * np.arange(K)
        p = np.exp(t)
        w = h * p
        if relative_error(w, p, a, b) <= eps:
            best = (w, p)
            break
    if best is None:
        raise RuntimeError("no step met the tolerance")
    return best


def operator_range(n: int):
    """Range of the 5-point eigenvalue lambda_i + lambda_j: [2 lambda_1, 2 lambda_n]."""
    lam = eigenvalues(n)
    return 2.0 * lam[0], 2.0 * lam[-1]


def expsum_solve2d(U: np.ndarray, V: np.ndarray, eps: float, eps_q: float | None = None):
    """Solve T X + X T = U V^T by the exponential-sum inverse (returns Ux, Vx,
    info): transform the factors, Hadamard product with the rank-R
    exponential sum (quadrature to eps_q, default eps), round by QR of both
    stacked factors and SVD of the product of their R factors to eps
    (relative Frobenius tail), transform back.  info: R (terms), Rr (rank
    before rounding), rank.
    Pins: the full-grid solve, the single-mode closed form."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    n, r = U.shape
    lam = eigenvalues(n)
    w, p = expsum_1x(*operator_range(n), eps if eps_q is None else eps_q)
    Uh, Vh = dst(U), dst(V)
    E = np.exp(-np.outer(lam, p))                    # n x R: exp(-p_k lambda_i)
    A = np.hstack([(w[k] * E[:, k])[:, None] * Uh for k in range(len(p))])
    B = np.hstack([E[:, k][:, None] * Vh for k in range(len(p))])
    Qa, Ra = np.linalg.qr(A)
    Qb, Rb = np.linalg.qr(B)
    W, s, Zt = np.linalg.svd(Ra @ Rb.T)
    R = truncation_rank(s, eps)
    Ux = dst(Qa @ (W[:, :R] * s[:R]))
    Vx = dst(Qb @ Zt[:R].T)
    return Ux, Vx, dict(R=len(p), Rr=A.shape[1], rank=R)
