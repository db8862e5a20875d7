"""GPU parity of the 2D path against the CPU oracle (through the C-ABI).

Tolerances: the float64 sine transform must match the oracle's library DST to
1e-13 (relative Frobenius; both are O(u log n)-accurate); a solve at
tolerance eps must match the oracle's full-grid solution to 10 eps (relative
Frobenius), the acceptance bar of the method.  Pivots, ranks and factors are
not unique, so only the assembled solution and the orthonormality of Vx are
compared.
"""
import numpy as np
import pytest

from oracle import metrics, poisson
from paper_1306_2150_amd import binding, inputs

from gpu_util import ctx, dev, host, log, rel

pytestmark = pytest.mark.gpu


def sine_mode(n, p):
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.sin(p * np.pi * i / (n + 1))


# ---------------------------------------------------------- sine transform
@pytest.mark.parametrize("n,c", [(1, 1), (2, 3), (3, 1), (63, 5), (64, 32),
                                 (65, 33), (257, 17), (1000, 40), (4096, 32),
                                 (4096, 100), (16384, 8)])
def test_dst_fp64_matches_oracle(n, c):
    log("dst fp64", n, c)
    rng = np.random.default_rng(n * 7 + c)
    X = rng.standard_normal((n, c))
    Y = host(ctx().sine_transform(dev(X), "fp64"))
    assert rel(Y, poisson.dst(X)) <= 1e-13


@pytest.mark.parametrize("n,c", [(1, 1), (2, 3), (3, 2), (4, 1), (63, 5), (64, 32), (65, 33),
                                 (1000, 40), (2047, 7), (2048, 9), (2049, 300), (3001, 70),
                                 (4095, 11), (4096, 1100)])
def test_dst_fft64_matches_oracle(n, c):
    """The chirp-z FFT transform (float64): every column within 1e-14 of the
    oracle's library DST, odd and even n (with and without the middle point
    of the fold), one- to four-point grids, the largest supported n."""
    log("dst fft64", n, c)
    rng = np.random.default_rng(n * 17 + c)
    X = rng.standard_normal((n, c))
    X[:, 0] *= 1e-250              # column scales are independent
    Y = host(ctx().sine_transform(dev(X), "fft64"))
    R = poisson.dst(X)
    worst = max(rel(Y[:, j], R[:, j]) for j in range(c))
    log("  worst column", worst)
    assert worst <= 1e-14, worst


def test_dst_fft64_limits_and_nonfinite():
    log("dst fft64 limits")
    from paper_1306_2150_amd import binding
    with pytest.raises(binding.LrpError) as ei:
        ctx().sine_transform(dev(np.ones((4097, 1))), "fft64")
    assert ei.value.status == binding.LRP_EINVAL
    # a NaN in a solve's factor is reported by the forward transform
    U, V = inputs.workload_rhs(2, 1, n=4000)
    U = U.copy()
    U[3999, 2] = np.nan
    _, _, info = ctx().solve2d(dev(U), dev(V), 1e-8, prec="fft64", check=False)
    assert info["status_code"] == binding.LRP_ENONFINITE


def test_dst_leading_dimension_and_involution():
    log("dst ld")
    import torch
    n, c = 300, 7
    rng = np.random.default_rng(1)
    X = rng.standard_normal((n, c))
    big = torch.zeros((c, n + 13), dtype=torch.float64, device="cuda").T
    big[:n].copy_(torch.from_numpy(X).cuda())
    Xd = big[:n]
    Y = ctx().sine_transform(Xd, "fp64")
    Z = ctx().sine_transform(Y, "fp64")           # S S = I
    assert rel(host(Z), X) <= 1e-13


@pytest.mark.parametrize("n,c", [(1, 1), (2, 3), (63, 5), (100, 70), (257, 17), (1000, 40),
                                 (4096, 32), (4096, 200), (8191, 9), (12000, 3)])
def test_dst_int8_slices_match_oracle(n, c):
    """Exact-integer slice transform: the only errors are the six-slice
    representations of the sines and of x (2^-42 of their largest entries)
    and the dropped slice levels >= 6 (about 2^-42 each); a few 1e-13 to
    2e-12 in the relative Frobenius norm of a column."""
    log("dst int8", n, c)
    rng = np.random.default_rng(n * 11 + c)
    X = rng.standard_normal((n, c))
    X[:, 0] *= 1e-30               # column scales are independent
    Y = host(ctx().sine_transform(dev(X), "int8"))
    R = poisson.dst(X)
    for j in range(c):
        assert rel(Y[:, j], R[:, j]) <= 1e-11, (j, rel(Y[:, j], R[:, j]))


def test_dst_int8_columns_independent_of_batch():
    log("dst int8 batch")
    n = 3000
    rng = np.random.default_rng(5)
    X = rng.standard_normal((n, 300))
    # 12 row tiles x 2 parities x 5 column tiles = 120 < 256: 32-column tiles
    big = host(ctx().sine_transform(dev(X), "int8"))        # narrow tiles, no K split
    small = host(ctx().sine_transform(dev(X[:, 7:9]), "int8"))   # K split
    assert np.array_equal(big[:, 7:9], small)


# (n, columns): row tiles R = ceil(ceil(n/2)/128); a launch takes the
# 64-column tiles when R * 2 * ceil(columns/64) >= 256.
@pytest.mark.parametrize("n,c", [
    (4096, 1024),   # 16 * 2 * 16 = 512: 64-point stages, whole-period table
    (4096, 460),    # 16 * 2 * 8 = 256: the smallest wide launch at this n
    (8192, 256),    # 32 * 2 * 4 = 256
    (8192, 1024),   # 32 * 2 * 16 = 1024
    (12000, 300),   # 47 * 2 * 5 = 470: quarter-wave table
    (16384, 200),   # 64 * 2 * 4 = 512: quarter table, 32-point stages
])
def test_dst_int8_wide_tiles_match_oracle_and_narrow(n, c):
    """The 64-column tile kernels (the ones large batched launches run):
    every column within 1e-11 of the oracle's DST, and bit-identical to the
    32-column tiles of a small launch of the same columns (the exact int32
    level sums do not depend on the tiling)."""
    log("dst int8 wide", n, c)
    rng = np.random.default_rng(n + c)
    X = rng.standard_normal((n, c))
    X[:, 1] *= 1e-200              # column scales are independent
    X[:, 2] = 0.0
    Y = host(ctx().sine_transform(dev(X), "int8"))
    R = poisson.dst(X)
    for j in range(c):
        if j == 2:
            assert not np.any(Y[:, j])
            continue
        assert rel(Y[:, j], R[:, j]) <= 1e-11, (j, rel(Y[:, j], R[:, j]))
    # 40 columns: R * 2 * 1 < 256, narrow tiles (and a K split)
    sub = [0, 1, 2, 3, c // 2, c - 1]
    Ys = host(ctx().sine_transform(dev(X[:, sub]), "int8"))
    assert np.array_equal(Ys, Y[:, sub])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_dst_columns_independent_of_batch(prec):
    """The folded transform's K chunks depend on n only: a column's result is
    the same bits whether its launch splits K over workgroups (few columns)
    or not (many columns)."""
    log("dst batch", prec)
    n = 3001
    rng = np.random.default_rng(6)
    X = rng.standard_normal((n, 300))
    big = host(ctx().sine_transform(dev(X), prec))
    small = host(ctx().sine_transform(dev(X[:, 7:9]), prec))
    assert np.array_equal(big[:, 7:9], small)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("bf16x3", 5e-5), ("bf16x6", 1e-6)])
@pytest.mark.parametrize("n,c", [(1, 1), (2, 3), (3, 2), (64, 5), (65, 40), (1001, 33)])
def test_dst_reduced_precision_odd_even_sizes(prec, tol, n, c):
    """Both parities of the folded transform, odd and even n (with and
    without the middle point), one- and two-point grids."""
    log("dst", prec, n, c)
    rng = np.random.default_rng(n * 13 + c)
    X = rng.standard_normal((n, c))
    Y = host(ctx().sine_transform(dev(X), prec))
    e = rel(Y, poisson.dst(X))
    assert e <= tol, e


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("bf16x3", 5e-5), ("bf16x6", 3e-7)])
def test_dst_reduced_precision_error_bound(prec, tol):
    log("dst", prec)
    n, c = 4096, 32
    U, V = inputs.rhs2d_bumps(n, 16, 2001)
    X = np.hstack([U, V])
    Y = host(ctx().sine_transform(dev(X), prec))
    e = rel(Y, poisson.dst(X))
    assert e <= tol, e


# ------------------------------------------------------------- 2D solves
def solve_and_check(U, V, eps, prec="fp64", bar=None, **kw):
    Ux, Vx, info = ctx().solve2d(dev(U), dev(V), eps, prec=prec, **kw)
    Ux, Vx = host(Ux), host(Vx)
    X = poisson.full_solve2d_factors(U, V)
    e = metrics.rel_err_factored(Ux, Vx, X)
    bar = 10 * eps if bar is None else bar
    assert info["status"] == binding.LRP_OK, info
    assert e <= bar, (e, info)
    if Vx.shape[1]:
        # orthonormal to the precision of the inverse transform
        otol = {"fp64": 1e-10, "int8": 1e-10, "fft64": 1e-10, "fp32": 1e-6,
                "bf16x6": 1e-6, "bf16x3": 1e-4}[info["inv_prec"]]
        assert np.max(np.abs(Vx.T @ Vx - np.eye(Vx.shape[1]))) < otol
    return e, info


@pytest.mark.parametrize("inst", [1, 2, 3, 4])
def test_solve2d_n256_eps1e10(inst):
    log("solve2d n256 inst", inst)
    U, V = inputs.workload_rhs(1, inst)
    solve_and_check(U, V, 1e-10)


@pytest.mark.parametrize("n,inst", [(1024, 1), (1024, 2), (1000, 3), (2049, 4)])
def test_solve2d_bumps_eps1e8(n, inst):
    log("solve2d bumps", n, inst)
    U, V = inputs.workload_rhs(2, inst, n=n)
    solve_and_check(U, V, 1e-8)


def test_solve2d_n4096_r16_eps1e8():
    log("solve2d n4096 r16")
    U, V = inputs.workload_rhs(2, 1)
    e, info = solve_and_check(U, V, 1e-8, bar=1e-7)
    assert 15 <= info["rank"] <= 40


@pytest.mark.parametrize("prec", ["auto", "fp64"])
def test_solve2d_n4096_sixteen_seeds_batched(prec):
    """The 4096-point rank-16 workload at eps = 1e-8, sixteen seeded
    instances solved in one batched call (the launch shape the benchmark
    times), each against its own full-grid oracle solution (bar 1e-7)."""
    log("solve2d n4096 16 seeds", prec)
    rhs = [inputs.workload_rhs(2, inst) for inst in range(1, 17)]
    res = ctx().solve2d_batch([(dev(U), dev(V), 1e-8) for U, V in rhs], prec=prec)
    worst = 0.0
    for (U, V), (Ux, Vx, info) in zip(rhs, res):
        assert info["status"] == binding.LRP_OK, info
        X = poisson.full_solve2d_factors(U, V, workers=16)
        e = metrics.rel_err_factored(host(Ux), host(Vx), X)
        worst = max(worst, e)
        assert e <= 1e-7, e
    log("  worst", worst)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 20])
def test_solve2d_tiny_grids(n):
    log("solve2d tiny", n)
    rng = np.random.default_rng(n)
    U, V = rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
    solve_and_check(U, V, 1e-12)


def test_solve2d_single_mode_closed_form():
    log("solve2d single mode")
    n = 4096
    u, v = sine_mode(n, 3), sine_mode(n, 77)
    lam = poisson.eigenvalues(n)
    Ux, Vx, info = ctx().solve2d(dev(u[:, None]), dev(v[:, None]), 1e-10)
    Ux, Vx = host(Ux), host(Vx)
    assert info["rank"] == 1
    X = np.outer(u, v) / (lam[2] + lam[76])
    assert metrics.rel_err_factored(Ux, Vx, X) < 1e-11


def test_solve2d_exact_rank_q():
    log("solve2d exact rank")
    n, ps = 3000, [2, 11, 40, 151, 999]
    rng = np.random.default_rng(14)
    U = np.stack([sine_mode(n, p) for p in ps], axis=1)
    V = rng.standard_normal((n, len(ps)))
    Ux, Vx, info = ctx().solve2d(dev(U), dev(V), 1e-13)
    assert info["rank"] == len(ps)
    X = poisson.full_solve2d_factors(U, V)
    assert metrics.rel_err_factored(host(Ux), host(Vx), X) < 1e-11


def test_solve2d_zero_rhs():
    log("solve2d zero")
    U = np.zeros((500, 4))
    V = np.ones((500, 4))
    Ux, Vx, info = ctx().solve2d(dev(U), dev(V), 1e-8)
    assert info["rank"] == 0 and info["status"] == binding.LRP_OK


def test_solve2d_nonfinite_rejected():
    log("solve2d nonfinite")
    U, V = inputs.workload_rhs(2, 1, n=512)
    U = U.copy()
    U[100, 3] = np.nan
    Ux, Vx, info = ctx().solve2d(dev(U), dev(V), 1e-8, check=False)
    assert info["status_code"] == binding.LRP_ENONFINITE


def test_solve2d_rank_cap_and_rmax():
    log("solve2d caps")
    U, V = inputs.workload_rhs(2, 2, n=1024)
    # a cross capped at 8 columns cannot reach 1e-8 (the solution has rank ~25)
    Ux, Vx, info = ctx().solve2d(dev(U), dev(V), 1e-8, check=False, rank_cap=8)
    assert info["status_code"] in (binding.LRP_ERANKCAP, binding.LRP_ENOCONV)
    # output capacity smaller than the rank: ERANKCAP with the needed rank
    Ux, Vx, info = ctx().solve2d(dev(U), dev(V), 1e-8, rmax=4, check=False)
    assert info["status_code"] == binding.LRP_ERANKCAP
    assert info["rank"] > 4
    # one sweep cannot show convergence
    Ux, Vx, info = ctx().solve2d(dev(U), dev(V), 1e-8, check=False, max_sweeps=1)
    assert info["status_code"] == binding.LRP_ENOCONV


def test_solve2d_invalid_arguments():
    log("solve2d einval")
    c = ctx()
    import torch
    buf = torch.zeros((64, 8), dtype=torch.float64, device="cuda")
    p = buf.data_ptr()
    assert c.raw_solve2d(0, 2, p, p, 64, 1e-8, p, p, 64, 8)[0] == binding.LRP_EINVAL
    assert c.raw_solve2d(64, 65, p, p, 64, 1e-8, p, p, 64, 8)[0] == binding.LRP_EINVAL
    assert c.raw_solve2d(64, 2, p, p, 63, 1e-8, p, p, 64, 8)[0] == binding.LRP_EINVAL
    assert c.raw_solve2d(64, 2, p, p, 64, 0.0, p, p, 64, 8)[0] == binding.LRP_EINVAL
    assert c.raw_solve2d(64, 2, p, p, 64, 1.5, p, p, 64, 8)[0] == binding.LRP_EINVAL
    assert c.raw_solve2d(64, 2, 0, p, 64, 1e-8, p, p, 64, 8)[0] == binding.LRP_EINVAL
    assert c.raw_solve2d(64, 2, p, p, 64, 1e-8, p, p, 32, 8)[0] == binding.LRP_EINVAL


def test_solve2d_batch_same_as_alone():
    log("solve2d batch")
    n = 2048
    probs = []
    for inst, eps in [(1, 1e-8), (2, 1e-6), (3, 1e-8), (4, 1e-10)]:
        U, V = inputs.workload_rhs(2, inst, n=n)
        probs.append((U, V, eps))
    res_b = ctx().solve2d_batch([(dev(U), dev(V), eps) for U, V, eps in probs])
    for (U, V, eps), (Uxb, Vxb, ib) in zip(probs, res_b):
        Uxa, Vxa, ia = ctx().solve2d(dev(U), dev(V), eps)
        A = host(Uxa) @ host(Vxa).T
        B = host(Uxb) @ host(Vxb).T
        assert ia["rank"] == ib["rank"]
        assert rel(B, A) <= 1e-12
        X = poisson.full_solve2d_factors(U, V)
        assert metrics.rel_err_factored(host(Uxb), host(Vxb), X) <= 10 * eps


def test_solve2d_batch_mixed_rank_buckets():
    """A batch whose slots sit in three rank buckets (the leaf-level sweep
    kernels run once per bucket, each on its own slots; the tree nodes,
    maxvol inverse and swaps and the core once at the largest): every
    problem gives the rank and, to 1e-12, the result it gives alone, and is
    within 10 eps of the float64 full solve."""
    n = 1024
    probs = [(*inputs.rhs2d_single_bumps(n, 1, 77), 1e-4),     # k <= 16
             (*inputs.workload_rhs(2, 5, n=n), 1e-8),            # k about 32
             (*inputs.workload_rhs(2, 6, n=n), 1e-12),           # k above 32
             (*inputs.rhs2d_single_bumps(n, 1, 79), 1e-5)]
    log("solve2d batch buckets", [(U.shape[1], eps) for U, V, eps in probs])
    res_b = ctx().solve2d_batch([(dev(U), dev(V), eps) for U, V, eps in probs])
    ks = []
    for (U, V, eps), (Uxb, Vxb, ib) in zip(probs, res_b):
        Uxa, Vxa, ia = ctx().solve2d(dev(U), dev(V), eps)
        ks.append(ib["k"])
        assert ia["rank"] == ib["rank"] and ia["k"] == ib["k"]
        assert rel(host(Uxb) @ host(Vxb).T, host(Uxa) @ host(Vxa).T) <= 1e-12
        X = poisson.full_solve2d_factors(U, V)
        assert metrics.rel_err_factored(host(Uxb), host(Vxb), X) <= 10 * eps
    log("  k", ks)
    assert min(ks) <= 16 and max(ks) > 32, ks


def test_prepared_batch_reruns_identically():
    """A prepared batch (argument array and outputs built once) solves every
    problem again on each run: equal bits on a second run, and equal to a
    fresh batch call."""
    log("solve2d prepared batch")
    n = 1024
    probs = []
    for inst, eps in [(1, 1e-8), (2, 1e-6), (3, 1e-10)]:
        U, V = inputs.workload_rhs(2, inst, n=n)
        probs.append((dev(U), dev(V), eps))
    b = ctx().batch2d(probs, prec="auto")
    first = [(host(Ux).copy(), host(Vx).copy(), i["rank"]) for Ux, Vx, i in b.run()]
    # overwrite the outputs, then run again
    for Ux, Vx in b.outs:
        Ux.fill_(float("nan"))
        Vx.fill_(float("nan"))
    second = b.run()
    fresh = ctx().solve2d_batch(probs, prec="auto")
    for (Ua, Va, ra), (Ub, Vb, ib), (Uc, Vc, ic) in zip(first, second, fresh):
        assert ra == ib["rank"] == ic["rank"]
        assert np.array_equal(Ua, host(Ub)) and np.array_equal(Va, host(Vb))
        assert np.array_equal(Ua, host(Uc)) and np.array_equal(Va, host(Vc))


@pytest.mark.parametrize("prec,eps,bar", [("fft64", 1e-8, 1e-7), ("fft64", 1e-12, 1e-11),
                                          ("bf16x6", 1e-7, 1e-6),
                                          ("fp32", 1e-7, 1e-6), ("auto", 1e-8, 1e-7),
                                          ("auto", 1e-7, 1e-6), ("auto", 1e-6, 1e-5),
                                          ("bf16x3", 1e-5, 1e-4), ("int8", 1e-8, 1e-7),
                                          ("int8", 1e-10, 1e-9)])
def test_solve2d_mixed_precision(prec, eps, bar):
    log("solve2d mixed", prec, eps)
    U, V = inputs.workload_rhs(2, 1, n=4096)
    solve_and_check(U, V, eps, prec=prec, bar=bar)


# ---------------------------------------------- precision workload, n = 16384
@pytest.fixture(scope="module")
def n16384_case():
    """The 16384-point rank-32 bump workload at eps = 1e-7 and its float64
    full-grid solution (2 GiB, computed once)."""
    U, V = inputs.workload_rhs(4, 1)
    X = poisson.full_solve2d_factors(U, V, workers=16)
    return U, V, X


@pytest.mark.parametrize("prec", ["fp64", "auto", "int8", "fp32", "bf16x6"])
def test_precision_workload_n16384(n16384_case, prec):
    """Error of every transform precision against the float64 full solve at
    n = 16384, r = 32, eps = 1e-7, held to the acceptance bar 10 eps = 1e-6:
    float64, int8 slices, FP32 and the split-BF16 plan with three pieces and
    six products."""
    U, V, X = n16384_case
    log("precision n=16384", prec)
    Ux, Vx, info = ctx().solve2d(dev(U), dev(V), 1e-7, prec=prec)
    e = metrics.rel_err_factored(host(Ux), host(Vx), X)
    log("  fwd", info["fwd_prec"], "inv", info["inv_prec"], "rank", info["rank"],
        "sweeps", info["sweeps"], "err", e)
    assert info["status_code"] == binding.LRP_OK
    if prec != "auto":
        assert info["fwd_prec"] == prec and info["inv_prec"] == prec, info
    assert e <= 1e-6, e


def test_precision_workload_n16384_bf16x3_floor(n16384_case):
    """The two-piece split-BF16 plan (three products) cannot meet 10 eps =
    1e-6 here: its transforms carry a relative error floor of a few 1e-6
    that the inverse transform passes straight to the result.  Not a pass of
    the acceptance bar: the test records the floor and checks that it stays
    in its measured band (above the bar, below 1e-5)."""
    U, V, X = n16384_case
    log("precision n=16384 bf16x3 floor")
    Ux, Vx, info = ctx().solve2d(dev(U), dev(V), 1e-7, prec="bf16x3")
    e = metrics.rel_err_factored(host(Ux), host(Vx), X)
    log("  bf16x3 floor err", e)
    assert 1e-6 < e < 1e-5, e


def test_int8_plan_limits():
    """An explicit INT8 plan runs the int8 transforms both ways, and a grid
    too large for its sine record table is refused (LRP_EINVAL) rather than
    solved another way."""
    log("int8 plan")
    U, V = inputs.workload_rhs(2, 1, n=1000)
    Ux, Vx, info = ctx().solve2d(dev(U), dev(V), 1e-8, prec="int8")
    assert info["fwd_prec"] == "int8" and info["inv_prec"] == "int8"
    n = 20000
    big = dev(np.ones((n, 1)))
    with pytest.raises(binding.LrpError) as ei:
        ctx().solve2d(big, big, 1e-6, prec="int8")
    assert ei.value.status == binding.LRP_EINVAL
