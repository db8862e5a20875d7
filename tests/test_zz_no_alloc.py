"""The sine transform entry point that allocates nothing
(lrp_sine_transform_noalloc, for callers that cannot allocate), through the
C-ABI: its results equal those of lrp_sine_transform (same kernels, same
tables: bit for bit) and the oracle's DST (1e-13 float64, 1e-11 int8 per
column), on calls in a row whose second input is smaller, and across grid
sizes and precisions (the static array keeps the last call's tables)."""
import numpy as np
import pytest

from oracle import poisson

from gpu_util import ctx, dev, host, log, rel

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-13, "int8": 1e-11, "fft64": 1e-14, "fp32": 1e-6, "bf16x3": 5e-5,
       "bf16x6": 1e-6}


def check(n, c, prec, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, c))
    Xd = dev(X)
    got = host(ctx().sine_transform_noalloc(Xd, prec))
    want = host(ctx().sine_transform(Xd, prec))
    assert np.array_equal(got, want), (n, c, prec)
    R = poisson.dst(X)
    worst = max(rel(got[:, j], R[:, j]) for j in range(c))
    log("  noalloc", n, c, prec, "worst column err", worst)
    assert worst <= TOL[prec], worst


@pytest.mark.parametrize("prec", ["fp64", "int8"])
def test_noalloc_two_calls_second_smaller(prec):
    log("noalloc", prec)
    check(4096, 1500, prec, 1)      # more columns than one launch takes
    check(4096, 37, prec, 2)        # smaller: split-K launch, same tables


def test_noalloc_grid_sizes_and_precisions():
    log("noalloc sizes")
    for i, (n, c, prec) in enumerate([(1000, 200, "fp64"), (1, 3, "fp64"), (12000, 90, "int8"),
                                      (3001, 64, "fp32"), (3001, 5, "bf16x3"),
                                      (16384, 600, "int8"), (257, 9, "int8"),
                                      (4096, 300, "fft64"), (2049, 3, "fft64"),
                                      (20000, 70, "bf16x6")]):
        check(n, c, prec, 10 + i)


def test_noalloc_limits():
    from paper_1306_2150_amd import binding
    log("noalloc limits")
    Xd = dev(np.ones((20000, 1)))
    with pytest.raises(binding.LrpError) as ei:
        ctx().sine_transform_noalloc(Xd, "int8")       # beyond the int8 table limit
    assert ei.value.status == binding.LRP_EINVAL
    with pytest.raises(binding.LrpError) as ei:
        ctx().sine_transform_noalloc(Xd, "auto")
    assert ei.value.status == binding.LRP_EINVAL
