"""Naive float64 low-rank 2D Poisson solver -- test infrastructure only.

The paper's method (Section 4.2, with the transform of Section 4.1 and the
rounding of Section 3), step by step and in its order:

  1. lambda_k (eq. "diag"),
  2. transform the factors: Uh = S U, Vh = S V (Section 4.1; the rank does
     not change),
  3. any entry of the divided spectrum Xh_ij = (Uh_i . Vh_j)/(lambda_i +
     lambda_j) costs O(r) (eq. "div"),
  4. approximate Xh by a cross (skeleton) built from k rows and k columns
     picked by maxvol (Section 4.2, refs. gt-maxvol-2001, gostz-maxvol-2010),
  5. round the skeleton to accuracy eps by QR of the factors plus SVD of the
     small core (Section 3, "rounding"),
  6. transform the factors back.

The paper gives steps 4-5 as prose plus citations only.  The reading used
here (the same one the GPU solver implements; listed in the design notes):

  * maxvol: initial rows = pivot rows of Gaussian elimination with partial
    pivoting; B = A A[I,:]^-1; while max|B| > tau swap the argmax row in
    (ties: lowest row, then lowest column); tau = 1.05.
  * sweep with column set J: C = Xh[:, J]; Qc = qr(C); I = maxvol(Qc);
    Rm = Xh[I, :]; Qr = qr(Rm^T); J' = maxvol(Qr).  Skeleton
    X~ = Qc (Qc[I,:])^-1 Rm.  Compress: M = (Qc[I,:])^-1 Rm, M^T = Qm Rm',
    SVD Rm'^T = W S Z^T, so X~ = (Qc W) S (Qm Z)^T.
  * truncation rank: smallest R with ||s[R:]||_2 <= eps ||s||_2.
  * rank control: k0 = min(n, r + kick, k_max), kick = 8; J0 = maxvol(qr(Vh))
    padded with evenly spaced unused indices.  If the truncation leaves fewer
    than ``min_slack`` = kick/2 = 4 unused columns (R > k - 4) and k can grow,
    k += kick and the kick new columns are those with the largest residual
    |Xh - X~| on kick evenly spaced probe rows outside I.  (With a slack of
    one column the 256-point eps = 1e-10 case ends at 7.3 eps on seed 1001;
    with four, every tested seed ends at or below 1.05 eps.)
    Otherwise stop once ||X~_t - X~_{t-1}||_F <= eps ||X~_t||_F (skeletons
    before truncation; the difference is measured through QR of the stacked
    factors).  At most ``max_sweeps`` sweeps.
  * output Ux = S (Qc W S)[:, :R] (carries the scale), Vx = S (Qm Z)[:, :R]
    (orthonormal columns).
"""
from __future__ import annotations

import numpy as np

from .poisson import dst, eigenvalues, stokes_half_angles


def gepp_rows(A: np.ndarray) -> np.ndarray:
    """Pivot rows of Gaussian elimination with partial pivoting on A (n x k).

    Returns k row indices in pivot order.  A zero pivot column (rank
    deficiency) takes the first remaining row and eliminates nothing.
    Pin: for k = 1 it is argmax |A|; the rows give a nonsingular A[I,:]
    whenever A has full column rank.
    """
    W = np.array(A, dtype=np.float64, copy=True)
    n, k = W.shape
    perm = np.arange(n)
    for j in range(min(n, k)):
        p = j + int(np.argmax(np.abs(W[j:, j])))
        if p != j:
            W[[j, p]] = W[[p, j]]
            perm[[j, p]] = perm[[p, j]]
        piv = W[j, j]
        if piv != 0.0:
            lcol = W[j + 1:, j] / piv
            W[j + 1:, j + 1:] -= np.outer(lcol, W[j, j + 1:])
            W[j + 1:, j] = lcol
    return perm[:min(n, k)].copy()


def maxvol(A: np.ndarray, tau: float = 1.05, max_swaps: int | None = None):
    """Row maxvol (Goreinov, Oseledets, Savostyanov, Tyrtyshnikov, Zamarashkin).

    Returns (I, B, swaps): I has k rows such that B = A A[I,:]^-1 satisfies
    B[I,:] = identity and max|B| <= tau (unless the swap cap is hit).
    Pins: the exit invariants; every swap multiplies |det A[I,:]| by the
    swapped entry (> tau); brute-force maximum volume is at most
    (tau sqrt(k))^k times the returned volume (Hadamard bound).
    """
    A = np.asarray(A, dtype=np.float64)
    n, k = A.shape
    if k == 0:
        return np.zeros(0, dtype=np.int64), np.zeros((n, 0)), 0
    I = gepp_rows(A)
    B = np.linalg.solve(A[I, :].T, A.T).T
    if max_swaps is None:
        max_swaps = 100 * k
    swaps = 0
    while swaps < max_swaps:
        flat = int(np.argmax(np.abs(B)))        # row-major: lowest row, then col
        i, j = divmod(flat, k)
        if abs(B[i, j]) <= tau:
            break
        I[j] = i
        bij = B[i, j]
        row = B[i, :].copy()
        row[j] -= 1.0
        B -= np.outer(B[:, j], row) / bij
        swaps += 1
    return I, B, swaps


def truncation_rank(s: np.ndarray, eps: float) -> int:
    """Smallest R with sqrt(sum_{i>=R} s_i^2) <= eps * ||s||_2 (s descending)."""
    s = np.asarray(s, dtype=np.float64)
    if s.size == 0:
        return 0
    tail = np.sqrt(np.cumsum((s * s)[::-1]))[::-1]   # tail[i] = ||s[i:]||
    tot = tail[0]
    if tot == 0.0:
        return 0
    for R in range(s.size + 1):
        t = tail[R] if R < s.size else 0.0
        if t <= eps * tot:
            return R
    return s.size


def spread_indices(n: int, count: int, used, offset: int = 0) -> np.ndarray:
    """``count`` evenly spaced indices in [0, n) avoiding ``used``.

    Candidate i is (floor((2i+1) n / (2 count)) + offset) mod n; a taken
    candidate moves to the next free index (cyclically).  Deterministic.
    """
    taken = set(int(u) for u in used)
    out = []
    for i in range(count):
        if len(taken) >= n:
            break
        j = (((2 * i + 1) * n) // (2 * count) + offset) % n
        while j in taken:
            j = (j + 1) % n
        taken.add(j)
        out.append(j)
    return np.asarray(out, dtype=np.int64)


def _stacked_change(A, B, Ap, Bp) -> float:
    """||A B^T - Ap Bp^T||_F via QR of the stacked factors."""
    _, Ra = np.linalg.qr(np.hstack([A, -Ap]))
    _, Rb = np.linalg.qr(np.hstack([B, Bp]))
    return float(np.linalg.norm(Ra @ Rb.T))


def operator_factors(n: int, op: str = "poisson"):
    """Per-axis factors of the 2D operator's eigenvalue at mode (i, j).

    5-point Laplacian: returns (lambda, None); the eigenvalue is
    lambda_i + lambda_j (eq. "div").  Stokes-consistent operator: returns
    (p, q) = (2 sin^2 / h, 2 cos^2 / h) of the half angles; the eigenvalue is
    p_i q_j + q_i p_j (``poisson.denominators2d``)."""
    if op == "poisson":
        return eigenvalues(n), None
    s, c, h = stokes_half_angles(n)
    return 2.0 * s / h, 2.0 * c / h


def lr_solve2d(U: np.ndarray, V: np.ndarray, eps: float, kick: int = 8,
               k_max: int = 64, tau: float = 1.05, max_sweeps: int = 10,
               min_slack: int = 4, k0_extra: int = 0, seed: int = 0,
               op: str = "poisson"):
    """Low-rank solution of T X + X T = U V^T (returns Ux, Vx, info).

    See the module docstring for the steps and the reading of the paper.
    ``op`` = "stokes" solves with the Stokes-consistent Laplacian of
    Section 2 instead (denominators p_i q_j + q_i p_j, ``operator_factors``);
    ``seed`` offsets the deterministic index sequences (padding of the first
    column set, probe rows) by seed mod n.
    ``info`` has keys status ('ok' | 'rankcap' | 'noconv'), sweeps, k, rank,
    ranks (per sweep) and change (last measured change / ||X~||).
    """
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    n, r = U.shape
    info = dict(status="ok", sweeps=0, k=0, rank=0, ranks=[], change=None)
    if r == 0 or not np.any(U) or not np.any(V):
        return np.zeros((n, 0)), np.zeros((n, 0)), info

    lam, q = operator_factors(n, op)
    off = int(seed % n)
    Uh = dst(U)                   # Section 4.1: transform of the factors
    Vh = dst(V)

    def den(I, J):                # the operator's eigenvalue at modes (I, J)
        if q is None:
            return lam[I][:, None] + lam[J][None, :]
        return lam[I][:, None] * q[J][None, :] + q[I][:, None] * lam[J][None, :]

    def xh_cols(J):               # eq. "div", columns J
        return (Uh @ Vh[J].T) / den(np.arange(n), J)

    def xh_rows(I):               # eq. "div", rows I
        return (Uh[I] @ Vh.T) / den(I, np.arange(n))

    k_cap = min(n, k_max)
    k = min(n, r + kick + k0_extra, k_max)
    Qv, _ = np.linalg.qr(Vh)
    J, _, _ = maxvol(Qv, tau)
    J = J[:k]
    if J.size < k:
        J = np.concatenate([J, spread_indices(n, k - J.size, J, off)])

    prev = None
    A = B = None
    R = 0
    for sweep in range(max_sweeps):
        info["sweeps"] = sweep + 1
        k = J.size
        C = xh_cols(J)
        Qc, _ = np.linalg.qr(C)
        I, _, _ = maxvol(Qc, tau)
        Rm = xh_rows(I)
        Qr, _ = np.linalg.qr(Rm.T)
        Jn, _, _ = maxvol(Qr, tau)
        M = np.linalg.solve(Qc[I, :], Rm)          # skeleton core times rows
        Qm, RM = np.linalg.qr(M.T)
        W, s, Zt = np.linalg.svd(RM.T)
        A = (Qc @ W) * s[None, :]
        B = Qm @ Zt.T
        R = truncation_rank(s, eps)
        info["ranks"].append(R)
        nrm = float(np.linalg.norm(s))
        change = None
        if prev is not None:
            change = _stacked_change(A, B, prev[0], prev[1])
            info["change"] = change / nrm if nrm > 0 else 0.0
        no_slack = (R > k - min_slack) and (k < n)
        if no_slack and k < k_cap:
            grow = min(kick, k_cap - k)
            probe = spread_indices(n, kick, I, off)
            res = xh_rows(probe) - A[probe, :] @ B.T
            score = np.max(np.abs(res), axis=0)
            score[Jn] = -1.0
            order = np.argsort(-score, kind="stable")
            J = np.concatenate([Jn, order[:grow]])
            prev = (A, B)
            continue
        if change is not None and change <= eps * nrm:
            if no_slack:
                info["status"] = "rankcap"
            break
        J = Jn
        prev = (A, B)
    else:
        info["status"] = "noconv"

    info["k"] = int(k)
    info["rank"] = int(R)
    Ux = dst(A[:, :R])            # back transform (S = S^-1)
    Vx = dst(B[:, :R])
    return Ux, Vx, info
