"""Error measures for factored results -- test infrastructure only.

The acceptance measure is the relative Frobenius error of the assembled
low-rank result against the full-grid solution,
``||Ux Vx^T - X||_F / ||X||_F``.  It is accumulated blockwise as a direct
difference (never as ||a||^2 - 2<a,b> + ||b||^2, which cancels at the 1e-10
level).
"""
from __future__ import annotations

import numpy as np


def rel_err_factored(Ux: np.ndarray, Vx: np.ndarray, X: np.ndarray,
                     block: int = 1024) -> float:
    """||Ux Vx^T - X||_F / ||X||_F computed in row blocks in float64."""
    n = X.shape[0]
    num = 0.0
    den = 0.0
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        blk = Ux[i0:i1] @ Vx.T
        d = blk - X[i0:i1]
        num += float(np.sum(d * d))
        den += float(np.sum(X[i0:i1] * X[i0:i1]))
    if den == 0.0:
        return float(np.sqrt(num))
    return float(np.sqrt(num / den))


def rel_err_tucker(U1, U2, U3, G, X: np.ndarray, step: int | None = None) -> float:
    """||[[G; U1, U2, U3]] - X||_F / ||X||_F, slab by slab along mode 1.

    ``step`` is the slab height (rows of mode 1 per slab); by default slabs
    hold about 4M entries.  Pins: equals the norm of the expanded difference
    (``poisson.tucker_full``) and an element-by-element brute-force sum at
    small non-cubic shapes, for every slab height.
    """
    num = 0.0
    den = 0.0
    # T[a, j, k] = sum_bc G[a,b,c] U2[j,b] U3[k,c]
    T = np.einsum("abc,jb,kc->ajk", G, U2, U3, optimize=True)
    n1 = X.shape[0]
    if step is None:
        step = max(1, 2 ** 22 // max(1, X.shape[1] * X.shape[2]))
    for i0 in range(0, n1, step):
        i1 = min(n1, i0 + step)
        blk = np.tensordot(U1[i0:i1], T, axes=(1, 0))
        d = blk - X[i0:i1]
        num += float(np.sum(d * d))
        den += float(np.sum(X[i0:i1] * X[i0:i1]))
    if den == 0.0:
        return float(np.sqrt(num))
    return float(np.sqrt(num / den))
