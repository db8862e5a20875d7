"""Seeded synthetic right-hand sides for the low-rank Poisson solve.

This module only draws random numbers and evaluates Gaussian bumps on the
grid; it contains none of the solver's arithmetic (no transform, no
eigenvalues, no cross approximation).  It is the one piece shared by the
CPU oracle tests, the GPU parity tests and the benchmark, so that both sides
see bit-identical inputs.

Grid convention (the paper's Section 2 uses h = 1/n with n-1 unknowns; here
n counts interior unknowns): x_i = i/(n+1), i = 1..n.

Every draw uses ``numpy.random.default_rng(seed)`` (PCG64) and vector draws in
the order written below.  Factors are float64, column-major (Fortran order),
shape (n, r), which is the layout the C interface expects.
"""
from __future__ import annotations

import dataclasses

import numpy as np


def grid(n: int) -> np.ndarray:
    """Interior grid points x_i = i/(n+1), i = 1..n (float64)."""
    return np.arange(1, n + 1, dtype=np.float64) / float(n + 1)


def _bumps(x: np.ndarray, centre: np.ndarray, width: np.ndarray) -> np.ndarray:
    # column alpha = exp(-(x - centre_alpha)^2 / width_alpha^2)
    d = x[:, None] - centre[None, :]
    return np.asfortranarray(np.exp(-(d * d) / (width * width)[None, :]))


def rhs2d_single_bumps(n: int = 256, r: int = 4, seed: int = 1001):
    """Low-rank RHS F = U V^T with independent bumps on each side.

    Draw order: aU ~ U(0.2,0.8)^r, sU ~ U(0.05,0.3)^r, aV ~ U(0.2,0.8)^r,
    sV ~ U(0.05,0.3)^r, c ~ N(0,1)^r.  U_a = c_a exp(-(x-aU_a)^2/sU_a^2),
    V_a = exp(-(x-aV_a)^2/sV_a^2).  (The small 256-point, rank-4 case.)
    """
    rng = np.random.default_rng(seed)
    aU = rng.uniform(0.2, 0.8, r)
    sU = rng.uniform(0.05, 0.3, r)
    aV = rng.uniform(0.2, 0.8, r)
    sV = rng.uniform(0.05, 0.3, r)
    c = rng.standard_normal(r)
    x = grid(n)
    U = _bumps(x, aU, sU) * c[None, :]
    V = _bumps(x, aV, sV)
    return np.asfortranarray(U), np.asfortranarray(V)


def rhs2d_bumps(n: int = 4096, r: int = 16, seed: int = 2001):
    """Sum of r separable 2D Gaussian bumps, F = sum_a w_a g_a(x) g'_a(y).

    Draw order: a ~ U(0.1,0.9)^r, b ~ U(0.1,0.9)^r, s ~ U(0.02,0.2)^r,
    w ~ N(0,1)^r.  U_a = w_a exp(-(x-a_a)^2/s_a^2), V_a = exp(-(y-b_a)^2/s_a^2).
    Used for the 4096-point rank-16 case, the 16384-point rank-32 case and
    the 2D requests of the served stream.
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.1, 0.9, r)
    b = rng.uniform(0.1, 0.9, r)
    s = rng.uniform(0.02, 0.2, r)
    w = rng.standard_normal(r)
    x = grid(n)
    U = _bumps(x, a, s) * w[None, :]
    V = _bumps(x, b, s)
    return np.asfortranarray(U), np.asfortranarray(V)


def rhs3d_tucker(n: int = 512, ranks=(16, 16, 16), seed: int = 3001):
    """Tucker RHS: factors U1, U2, U3 (n x r_d) and core G (r1 x r2 x r3).

    Draw order: for d = 1..3: a_d ~ U(0.1,0.9)^{r_d}, s_d ~ U(0.02,0.2)^{r_d};
    then G ~ N(0,1) of shape (r1, r2, r3) in C order, scaled by
    2^{-(i+j+k)/4} with 0-based i, j, k.  U_d[:, a] = exp(-(x-a_da)^2/s_da^2).
    Returns (U1, U2, U3, G) with G stored Fortran-ordered (i1 fastest), the
    layout of the C interface.
    """
    rng = np.random.default_rng(seed)
    x = grid(n)
    facs = []
    for d in range(3):
        a = rng.uniform(0.1, 0.9, ranks[d])
        s = rng.uniform(0.02, 0.2, ranks[d])
        facs.append(_bumps(x, a, s))
    G = rng.standard_normal(tuple(ranks))
    i, j, k = np.meshgrid(*[np.arange(q) for q in ranks], indexing="ij")
    G = G * np.power(2.0, -(i + j + k) / 4.0)
    return facs[0], facs[1], facs[2], np.asfortranarray(G)


# The five named workloads.  Seeds are 1000 * workload + instance.
WORKLOADS = {
    1: dict(dim=2, n=256, r=4, eps=1e-10, gen="single"),
    2: dict(dim=2, n=4096, r=16, eps=1e-8, gen="bumps"),
    3: dict(dim=3, n=512, r=16, eps=1e-6, gen="tucker"),
    4: dict(dim=2, n=16384, r=32, eps=1e-7, gen="bumps"),
}


def workload_rhs(w: int, instance: int = 1, n: int | None = None):
    """RHS of named workload ``w`` (1..4), instance ``instance``.

    ``n`` overrides the grid size (same recipe, same seed) for scaled-down
    parity cases.
    """
    cfg = WORKLOADS[w]
    nn = cfg["n"] if n is None else n
    seed = 1000 * w + instance
    if cfg["gen"] == "single":
        return rhs2d_single_bumps(nn, cfg["r"], seed)
    if cfg["gen"] == "bumps":
        return rhs2d_bumps(nn, cfg["r"], seed)
    return rhs3d_tucker(nn, (cfg["r"],) * 3, seed)


@dataclasses.dataclass
class Request:
    """One request of the served stream."""
    rid: int
    arrival_s: float
    dim: int
    n: int
    r: int
    eps: float
    seed: int

    def rhs(self):
        if self.dim == 2:
            return rhs2d_bumps(self.n, self.r, self.seed)
        return rhs3d_tucker(self.n, (self.r,) * 3, self.seed)


SERVE_SHAPES = [(2, 512), (2, 1024), (2, 2048), (2, 4096), (2, 8192),
                (3, 128), (3, 256), (3, 512)]


def serving_stream(count: int, rate_per_s: float = 200.0, seed: int = 5000,
                   dims=(2, 3), max_rank: int = 64):
    """Poisson arrival stream of mixed solves (the served workload).

    Inter-arrival ~ Exp(mean 1/rate).  Per request: (dim, n) uniform over
    SERVE_SHAPES (restricted to ``dims``), r ~ U{4..max_rank}, eps uniform over
    {1e-6, 1e-8}; request id i uses RHS seed 5000 + i.  The stream itself is
    drawn from ``seed``.
    """
    rng = np.random.default_rng(seed)
    shapes = [s for s in SERVE_SHAPES if s[0] in dims]
    gaps = rng.exponential(1.0 / rate_per_s, count)
    pick = rng.integers(0, len(shapes), count)
    ranks = rng.integers(4, max_rank + 1, count)
    epss = rng.integers(0, 2, count)
    t = np.cumsum(gaps)
    out = []
    for i in range(count):
        dim, n = shapes[int(pick[i])]
        out.append(Request(rid=i, arrival_s=float(t[i]), dim=dim, n=n,
                           r=int(ranks[i]), eps=(1e-6, 1e-8)[int(epss[i])],
                           seed=5000 + i))
    return out

