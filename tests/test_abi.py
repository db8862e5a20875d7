"""The C-ABI library loads and exports every entry point the header declares,
and argument validation rejects bad calls before touching a device.  No GPU
work is done here."""
import ctypes
import os
import re

import pytest

from paper_1306_2150_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lrpoisson.h")
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_functions():
    names = []
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(",
                            src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("liblrpoisson.so is not built (run __graft_entry__.build())")
    return binding.load()


def test_header_declares_expected_api():
    names = declared_functions()
    assert set(names) == set(binding.EXPORTS), names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror_is_host_only(lib):
    assert binding.strerror(binding.LRP_OK) == "ok"
    assert "invalid" in binding.strerror(binding.LRP_EINVAL)
    assert binding.strerror(12345) == "unknown status"


def test_null_context_rejected(lib):
    P = ctypes.c_void_p
    rank = ctypes.c_int32(0)
    st = lib.lrpoisson_solve2d(None, 16, 2, P(1), P(1), 16, 1e-8, None, P(1),
                               P(1), 16, 8, ctypes.byref(rank), None, None)
    assert st == binding.LRP_EINVAL
    assert lib.lrp_create(None, 0, 0) == binding.LRP_EINVAL
    assert lib.lrp_destroy(None) == binding.LRP_EINVAL
    assert lib.lrp_serve_step(None, None) == binding.LRP_EINVAL
    assert lib.lrp_sine_transform(None, 16, 1, P(1), 16, P(1), 16, 0, None) == binding.LRP_EINVAL
    res = ctypes.c_int32(0)
    assert lib.lrp_wait(None, 1, ctypes.byref(res), None, None) == binding.LRP_EINVAL
    assert lib.lrp_poll(None, 1, ctypes.byref(res), None, None) == binding.LRP_EINVAL
    probs = (binding.LrpProblem2D * 1)()
    assert lib.lrp_expsum_solve2d_batch(None, 1024, 1, probs, None, None) == binding.LRP_EINVAL
    conv = ctypes.c_int32(0)
    rows = (ctypes.c_int32 * 4)()
    assert lib.lrp_kernel_qr_maxvol(None, 16, 4, P(1), 16, 0.0, P(1), 16, P(1), 4, rows,
                                    ctypes.byref(conv), None) == binding.LRP_EINVAL
    assert lib.lrp_kernel_core_svd(None, 4, P(1), 4, P(1), P(1), P(1), None) == binding.LRP_EINVAL
    sp = binding.LrpStokes2DProblem()
    assert lib.lrp_stokes2d(None, ctypes.byref(sp), None) == binding.LRP_EINVAL
    assert lib.lrp_set_graph_replay(None, 1) == binding.LRP_EINVAL


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the public structs have the C compiler's layout."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "lrpoisson.h"
int main(void) {
  printf("%zu %zu %zu %zu\\n", sizeof(lrp_opts), sizeof(lrp_info),
         sizeof(lrp_problem2d), sizeof(lrp_request));
  printf("%zu %zu %zu %zu\\n", offsetof(lrp_problem2d, eps),
         offsetof(lrp_problem2d, info), offsetof(lrp_request, eps),
         offsetof(lrp_request, Gx));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(lrp_opts, op), offsetof(lrp_opts, seed),
         offsetof(lrp_info, err_est), offsetof(lrp_info, us_phase),
         offsetof(lrp_request, op));
  printf("%zu %zu %zu %zu %zu\\n", sizeof(lrp_stokes2d_problem),
         offsetof(lrp_stokes2d_problem, eps), offsetof(lrp_stokes2d_problem, p_U),
         offsetof(lrp_stokes2d_problem, rank_out), offsetof(lrp_stokes2d_problem, true_residual));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True,
                         text=True).stdout.split()
    got = [int(v) for v in out]
    want = [ctypes.sizeof(binding.LrpOpts), ctypes.sizeof(binding.LrpInfo),
            ctypes.sizeof(binding.LrpProblem2D), ctypes.sizeof(binding.LrpRequest),
            binding.LrpProblem2D.eps.offset, binding.LrpProblem2D.info.offset,
            binding.LrpRequest.eps.offset, binding.LrpRequest.Gx.offset,
            binding.LrpOpts.op.offset, binding.LrpOpts.seed.offset,
            binding.LrpInfo.err_est.offset, binding.LrpInfo.us_phase.offset,
            binding.LrpRequest.op.offset,
            ctypes.sizeof(binding.LrpStokes2DProblem), binding.LrpStokes2DProblem.eps.offset,
            binding.LrpStokes2DProblem.p_U.offset, binding.LrpStokes2DProblem.rank_out.offset,
            binding.LrpStokes2DProblem.true_residual.offset]
    assert got == want


def test_header_constants_match_binding():
    src = open(HEADER).read()
    defs = dict(re.findall(r"#define\s+(LRP_[A-Z0-9_]+)\s+(\d+)", src))
    assert int(defs["LRP_MAX_N"]) == binding.MAX_N
    assert int(defs["LRP_MAX_N3"]) == binding.MAX_N3
    assert int(defs["LRP_MAX_RANK"]) == binding.MAX_RANK
    assert int(defs["LRP_MAX_SWEEPS"]) == binding.MAX_SWEEPS
    codes = dict(re.findall(r"(LRP_E[A-Z]+|LRP_OK)\s*=\s*(-?\d+)", src))
    for name, val in codes.items():
        assert getattr(binding, name) == int(val), name
    ops = dict(re.findall(r"LRP_OP_([A-Z]+)\s*=\s*(\d+)", src))
    assert {k.lower(): int(v) for k, v in ops.items()} == binding.OP
    precs = dict(re.findall(r"LRP_PREC_([A-Z0-9]+)\s*=\s*(\d+)", src))
    assert {k.lower(): int(v) for k, v in precs.items()} == binding.PREC


def test_solve3d_null_context_rejected(lib):
    P = ctypes.c_void_p
    rank = (ctypes.c_int32 * 3)(2, 2, 2)
    rmax = (ctypes.c_int32 * 3)(4, 4, 4)
    out = (ctypes.c_int32 * 3)()
    st = lib.lrpoisson_solve3d(None, 16, rank, P(1), P(1), P(1), 16, P(1), 1e-6,
                               None, P(1), P(1), P(1), 16, P(1), rmax, out, None,
                               None)
    assert st == binding.LRP_EINVAL
