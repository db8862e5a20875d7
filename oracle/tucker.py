"""Naive float64 low-rank 3D (Tucker) Poisson solver -- test infrastructure only.

The paper states the method for 2D, promises the 3D generalisation
(Section 4.1) and leaves it as future work (Section 7); it cites Tucker cross
approximation for tensors (Section 4.2, refs. ost-tucker-2008,
ot-ttcross-2010) and the Tucker format with linear-in-n rounding (Section 3,
eq. "tucker").  The reading implemented here:

  * transform the three factors, Uh_d = S U_d (eq. "diag" applied per mode);
  * any entry Xh(i,j,l) = G x1 Uh1[i] x2 Uh2[j] x3 Uh3[l] /
    (lambda_i + lambda_j + lambda_l) costs O(r1 r2 r3);
  * Tucker cross: index sets I_1, I_2, I_3 start from maxvol(qr(Uh_d))
    padded with evenly spaced unused indices (k_d = min(n, r_d + kick,
    k_max)); a sweep visits d = 1, 2, 3: the mode-d fiber matrix
    C_d = Xh(:, I_d', I_d'') unfolded to n x (k_d' k_d''), its leading left
    singular vectors Q_d (ranks: truncation at eps/sqrt(3) plus kick slack),
    I_d = maxvol(Q_d);
  * core Xh(I_1, I_2, I_3) x_d (Q_d[I_d,:])^-1, so X~ = core x_d Q_d;
  * HOSVD truncation of the core at eps/sqrt(3) per mode, rotate factors;
  * stop after a sweep (not the first) whose mode sizes did not grow and
    whose change ||X~_t - X~_{t-1}||_F <= eps ||X~_t||_F (untruncated,
    measured through QR of stacked factors);
  * output factors S (Q_d W_d) (orthonormal columns) and the core.
"""
from __future__ import annotations

import numpy as np

from .lowrank import maxvol, spread_indices, truncation_rank
from .poisson import dst, eigenvalues, stokes_half_angles


def mode_product(T: np.ndarray, M: np.ndarray, d: int) -> np.ndarray:
    """T x_d M : contracts mode d of T with the columns of M (M is m x T.shape[d])."""
    Tm = np.moveaxis(T, d, 0)
    sh = Tm.shape
    out = M @ Tm.reshape(sh[0], -1)
    return np.moveaxis(out.reshape((M.shape[0],) + sh[1:]), 0, d)


def unfold(T: np.ndarray, d: int) -> np.ndarray:
    """Mode-d unfolding (mode d becomes rows)."""
    return np.moveaxis(T, d, 0).reshape(T.shape[d], -1)


def _tucker_change(core, Q, core_p, Q_p) -> float:
    """||[[core; Q]] - [[core_p; Q_p]]||_F via QR of stacked factors."""
    k = core.shape
    kp = core_p.shape
    big = np.zeros(tuple(k[d] + kp[d] for d in range(3)))
    big[:k[0], :k[1], :k[2]] = core
    big[k[0]:, k[1]:, k[2]:] = -core_p
    for d in range(3):
        _, Rd = np.linalg.qr(np.hstack([Q[d], Q_p[d]]))
        big = mode_product(big, Rd, d)
    return float(np.linalg.norm(big))


def lr_solve3d(U1, U2, U3, G, eps: float, kick: int = 8, k_max: int = 64,
               tau: float = 1.05, max_sweeps: int = 10, op: str = "poisson"):
    """Low-rank Tucker solution of the 7-point Dirichlet Poisson problem
    (``op`` = "stokes": the Stokes-consistent Laplacian of Section 2, whose
    eigenvalue at mode (i, j, l) is 4 (s_i c_j c_l + c_i s_j c_l +
    c_i c_j s_l) / h^2 with s, c the squared sine and cosine of the half
    angles, ``poisson.denominators3d``).

    Returns (factors [V1, V2, V3], core, info).  See the module docstring.
    """
    Us = [np.asarray(u, dtype=np.float64) for u in (U1, U2, U3)]
    G = np.asarray(G, dtype=np.float64)
    n = Us[0].shape[0]
    info = dict(status="ok", sweeps=0, ranks=[], change=None)
    if G.size == 0 or not np.any(G) or any(not np.any(u) for u in Us):
        z = np.zeros((n, 0))
        return [z, z.copy(), z.copy()], np.zeros((0, 0, 0)), info
    lam = eigenvalues(n)
    sq, cq, h = stokes_half_angles(n)
    Uh = [dst(u) for u in Us]
    eps_d = eps / np.sqrt(3.0)

    def entries(I1, I2, I3):
        num = np.einsum("abc,ia,jb,kc->ijk", G, Uh[0][I1], Uh[1][I2],
                        Uh[2][I3], optimize=True)
        if op == "poisson":
            den = (lam[I1][:, None, None] + lam[I2][None, :, None]
                   + lam[I3][None, None, :])
        else:
            s1, c1 = sq[I1][:, None, None], cq[I1][:, None, None]
            s2, c2 = sq[I2][None, :, None], cq[I2][None, :, None]
            s3, c3 = sq[I3][None, None, :], cq[I3][None, None, :]
            den = 4.0 * (s1 * c2 * c3 + c1 * s2 * c3 + c1 * c2 * s3) / (h * h)
        return num / den

    idx = []
    for d in range(3):
        kd = min(n, G.shape[d] + kick, k_max)
        Qd, _ = np.linalg.qr(Uh[d])
        Id, _, _ = maxvol(Qd, tau)
        Id = Id[:kd]
        if Id.size < kd:
            Id = np.concatenate([Id, spread_indices(n, kd - Id.size, Id)])
        idx.append(Id)

    prev = None
    Q = [None, None, None]
    core = None
    for sweep in range(max_sweeps):
        info["sweeps"] = sweep + 1
        grew = False
        for d in range(3):
            sets = list(idx)
            sets[d] = np.arange(n)
            Cd = unfold(entries(*sets), d)
            Ud, s, _ = np.linalg.svd(Cd, full_matrices=False)
            Rd = truncation_rank(s, eps_d)
            kd = max(1, min(Rd + kick, n, k_max, Cd.shape[1]))
            if kd > idx[d].size:
                grew = True
            Q[d] = Ud[:, :kd]
            idx[d], _, _ = maxvol(Q[d], tau)
        core = entries(*idx)
        for d in range(3):
            core = mode_product(core, np.linalg.inv(Q[d][idx[d], :]), d)
        nrm = float(np.linalg.norm(core))
        info["ranks"].append(tuple(q.shape[1] for q in Q))
        done = False
        if prev is not None:
            ch = _tucker_change(core, Q, prev[0], prev[1])
            info["change"] = ch / nrm if nrm > 0 else 0.0
            done = (not grew) and ch <= eps * nrm
        prev = (core.copy(), [q.copy() for q in Q])
        if done:
            break
    else:
        info["status"] = "noconv"

    # HOSVD truncation of the core, eps/sqrt(3) per mode
    Ws = []
    for d in range(3):
        W, s, _ = np.linalg.svd(unfold(core, d), full_matrices=False)
        Rd = truncation_rank(s, eps_d)
        Ws.append(W[:, :Rd])
    out_core = core
    for d in range(3):
        out_core = mode_product(out_core, Ws[d].T, d)
    facs = [dst(Q[d] @ Ws[d]) for d in range(3)]
    info["rank"] = tuple(w.shape[1] for w in Ws)
    return facs, out_core, info
