"""ctypes binding of ``liblrpoisson.so`` (declared in ``include/lrpoisson.h``).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Device buffers are torch CUDA (HIP) float64 tensors in column-major
layout (a tensor ``t`` of shape (n, r) with ``t.stride() == (1, ld)``, e.g.
``torch.empty(r, n).T`` or ``x.T.contiguous().T``); the stream is torch's
current stream unless one is given.  There is no CPU fallback: a missing
library raises.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "liblrpoisson.so")

LRP_OK = 0
LRP_EINVAL = -1
LRP_ENONFINITE = -2
LRP_ERANKCAP = -3
LRP_ENOCONV = -4
LRP_ENOMEM = -5
LRP_EDEVICE = -6
LRP_EBUSY = -7
LRP_ENOTREADY = -8
STATUS_NAME = {0: "ok", -1: "einval", -2: "enonfinite", -3: "erankcap", -4: "enoconv",
               -5: "enomem", -6: "edevice", -7: "ebusy", -8: "enotready"}

PREC = {"fp64": 0, "auto": 1, "fp32": 2, "bf16x3": 3, "int8": 4, "fft64": 5, "bf16x6": 6}
PREC_NAME = {v: k for k, v in PREC.items()}
OP = {"laplace": 0, "stokes": 1}

MAX_RANK = 64
MAX_N = 32767
MAX_N3 = 32767
MAX_SWEEPS = 64
PHASES = ("forward", "cross", "inverse")

# every symbol the header declares
EXPORTS = ["lrp_create", "lrp_destroy", "lrp_strerror", "lrpoisson_solve2d",
           "lrpoisson_solve2d_batch", "lrpoisson_solve3d", "lrp_submit",
           "lrp_serve_step", "lrp_poll", "lrp_wait", "lrp_sine_transform",
           "lrp_sine_transform_noalloc", "lrp_expsum_solve2d_batch",
           "lrp_kernel_qr_maxvol", "lrp_kernel_core_svd", "lrp_stokes2d",
           "lrp_lowrank_round",
           "lrp_set_kernel_timing", "lrp_kernel_stats", "lrp_set_graph_replay"]


class LrpOpts(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("rank_cap", ctypes.c_int32), ("kick", ctypes.c_int32),
                ("maxvol_tau", ctypes.c_double), ("op", ctypes.c_int32),
                ("k0", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class LrpInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("k", ctypes.c_int32), ("rank", ctypes.c_int32),
                ("fwd_prec", ctypes.c_int32), ("inv_prec", ctypes.c_int32),
                ("change", ctypes.c_double), ("err_est", ctypes.c_double),
                ("us_phase", ctypes.c_float * 3), ("pad", ctypes.c_int32)]

    def as_dict(self):
        return dict(status=self.status, sweeps=self.sweeps, k=self.k,
                    rank=self.rank, fwd_prec=PREC_NAME.get(self.fwd_prec),
                    inv_prec=PREC_NAME.get(self.inv_prec), change=self.change,
                    err_est=self.err_est,
                    us_phase=dict(zip(PHASES, (float(x) for x in self.us_phase))))


class LrpKernelStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("columns", ctypes.c_int64),
                ("ms", ctypes.c_double), ("flops", ctypes.c_double)]


class LrpProblem2D(ctypes.Structure):
    _fields_ = [("U", ctypes.c_void_p), ("V", ctypes.c_void_p),
                ("ld", ctypes.c_int64), ("rank", ctypes.c_int32),
                ("rmax", ctypes.c_int32), ("eps", ctypes.c_double),
                ("Ux", ctypes.c_void_p), ("Vx", ctypes.c_void_p),
                ("ldx", ctypes.c_int64), ("rank_out", ctypes.c_int32),
                ("info", LrpInfo)]


class LrpStokes2DProblem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("rank_fu", ctypes.c_int32),
                ("rank_fv", ctypes.c_int32), ("rank_g", ctypes.c_int32),
                ("prec", ctypes.c_int32),
                ("fu_U", ctypes.c_void_p), ("fu_V", ctypes.c_void_p),
                ("fv_U", ctypes.c_void_p), ("fv_V", ctypes.c_void_p),
                ("g_U", ctypes.c_void_p), ("g_V", ctypes.c_void_p),
                ("ld", ctypes.c_int64), ("eps", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("p_U", ctypes.c_void_p), ("p_V", ctypes.c_void_p),
                ("u_U", ctypes.c_void_p), ("u_V", ctypes.c_void_p),
                ("v_U", ctypes.c_void_p), ("v_V", ctypes.c_void_p),
                ("ldx", ctypes.c_int64), ("rmax", ctypes.c_int32),
                ("rank_out", ctypes.c_int32 * 3), ("iterations", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("max_krylov_rank", ctypes.c_int32),
                ("status", ctypes.c_int32), ("residual", ctypes.c_double),
                ("true_residual", ctypes.c_double)]


class LrpRequest(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("n", ctypes.c_int64), ("rank", ctypes.c_int32 * 3),
                ("rmax", ctypes.c_int32 * 3), ("U", ctypes.c_void_p * 3),
                ("G", ctypes.c_void_p), ("ld", ctypes.c_int64),
                ("X", ctypes.c_void_p * 3), ("Gx", ctypes.c_void_p),
                ("ldx", ctypes.c_int64), ("eps", ctypes.c_double),
                ("op", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class LrpError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -m paper_1306_2150_amd.build` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I32, I64, F64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.lrp_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, ctypes.c_size_t]
    lib.lrp_destroy.argtypes = [P]
    lib.lrp_strerror.argtypes = [I32]
    lib.lrp_strerror.restype = ctypes.c_char_p
    lib.lrpoisson_solve2d.argtypes = [P, I64, I32, P, P, I64, F64,
                                      ctypes.POINTER(LrpOpts), P, P, I64, I32,
                                      ctypes.POINTER(I32), ctypes.POINTER(LrpInfo), P]
    lib.lrpoisson_solve2d_batch.argtypes = [P, I64, I32, ctypes.POINTER(LrpProblem2D),
                                            ctypes.POINTER(LrpOpts), P]
    lib.lrp_expsum_solve2d_batch.argtypes = [P, I64, I32, ctypes.POINTER(LrpProblem2D),
                                             ctypes.POINTER(LrpOpts), P]
    lib.lrp_kernel_qr_maxvol.argtypes = [P, I64, I32, P, I64, F64, P, I64, P, I64,
                                         ctypes.POINTER(I32), ctypes.POINTER(I32), P]
    lib.lrp_kernel_core_svd.argtypes = [P, I32, P, I64, P, P, P, P]
    lib.lrp_stokes2d.argtypes = [P, ctypes.POINTER(LrpStokes2DProblem), P]
    lib.lrp_lowrank_round.argtypes = [P, I64, I32, P, P, I64, F64, P, P, I64, I32,
                                      ctypes.POINTER(I32), P]
    lib.lrpoisson_solve3d.argtypes = [P, I64, ctypes.POINTER(I32), P, P, P, I64, P,
                                      F64, ctypes.POINTER(LrpOpts), P, P, P, I64, P,
                                      ctypes.POINTER(I32), ctypes.POINTER(I32),
                                      ctypes.POINTER(LrpInfo), P]
    lib.lrp_sine_transform.argtypes = [P, I64, I32, P, I64, P, I64, I32, P]
    lib.lrp_sine_transform_noalloc.argtypes = [I64, I32, P, I64, P, I64, I32, P]
    lib.lrp_set_kernel_timing.argtypes = [P, I32]
    lib.lrp_set_graph_replay.argtypes = [P, I32]
    lib.lrp_kernel_stats.argtypes = [P, I32, ctypes.POINTER(LrpKernelStat), I32]
    lib.lrp_submit.argtypes = [P, ctypes.POINTER(LrpRequest), ctypes.POINTER(ctypes.c_uint64)]
    lib.lrp_serve_step.argtypes = [P, ctypes.POINTER(I32)]
    lib.lrp_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(I32),
                             ctypes.POINTER(I32), ctypes.POINTER(LrpInfo)]
    lib.lrp_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(I32),
                             ctypes.POINTER(I32), ctypes.POINTER(LrpInfo)]
    for name in EXPORTS:
        f = getattr(lib, name)
        if name != "lrp_strerror":
            f.restype = ctypes.c_int32
    _lib = lib
    return lib


def strerror(status: int) -> str:
    if _lib is None:
        return f"status {status}"
    return _lib.lrp_strerror(status).decode()


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _ld(t) -> int:
    """Leading dimension of a column-major (n, r) float64 CUDA tensor."""
    import torch
    if t.dtype != torch.float64 or not t.is_cuda:
        raise ValueError("factors must be float64 tensors on the GPU")
    if t.dim() != 2 or t.stride(0) != 1:
        raise ValueError("factors must be column-major (stride(0) == 1)")
    return max(t.stride(1), t.shape[0])


def colmajor(a, device="cuda"):
    """Copy an (n, r) array / tensor to a column-major float64 GPU tensor."""
    import numpy as np
    import torch
    x = torch.as_tensor(np.asarray(a, dtype=np.float64))
    n, r = x.shape
    out = torch.empty((r, n), dtype=torch.float64, device=device).T
    out.copy_(x.to(device))
    return out


def fortran_core(G, device="cuda"):
    """Copy an (r0, r1, r2) core to a GPU tensor stored in Fortran order."""
    import numpy as np
    import torch
    g = np.asarray(G, dtype=np.float64)
    flat = torch.as_tensor(np.ascontiguousarray(g.reshape(-1, order="F")))
    return flat.to(device)


def empty_colmajor(n, r, device="cuda"):
    import torch
    return torch.empty((max(r, 1), n), dtype=torch.float64, device=device).T[:, :r]


def _opts(prec="fp64", max_sweeps=0, rank_cap=0, kick=0, tau=0.0, op="laplace",
          seed=0, k0=0):
    return LrpOpts(PREC[prec] if isinstance(prec, str) else int(prec),
                   max_sweeps, rank_cap, kick, tau,
                   OP[op] if isinstance(op, str) else int(op), k0, seed)


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(int(s.cuda_stream))


class Batch2D:
    """Arguments of one lrpoisson_solve2d_batch call (method "cross") or
    lrp_expsum_solve2d_batch call (method "expsum"), kept for repeated runs:
    problems (U, V, eps) on one grid size, one (Ux, Vx) output pair of rmax
    columns per problem (the views of the last run's results stay valid until
    the next run overwrites them)."""

    ENTRY = {"cross": "lrpoisson_solve2d_batch", "expsum": "lrp_expsum_solve2d_batch"}

    def __init__(self, ctx, problems, prec, rmax, kw, method="cross"):
        import torch
        self.ctx = ctx
        self.entry = self.ENTRY[method]
        self.n = n = problems[0][0].shape[0] if problems else 0
        self.rmax = rmax = MAX_RANK if rmax is None else rmax
        nb = len(problems)
        dev = problems[0][0].device if problems else "cuda"
        # all outputs in two allocations: Ux of problem i = columns
        # [i rmax, (i+1) rmax) of one n x (nb rmax) column-major block
        w = max(rmax, 1)
        self._ux = torch.empty((nb * w, max(n, 1)), dtype=torch.float64, device=dev)
        self._vx = torch.empty((nb * w, max(n, 1)), dtype=torch.float64, device=dev)
        self.outs = [(self._ux[i * w:i * w + rmax].T, self._vx[i * w:i * w + rmax].T)
                     for i in range(nb)]
        self.arr = (LrpProblem2D * nb)()
        for i, (U, V, eps) in enumerate(problems):
            Ux, Vx = self.outs[i]
            r = U.shape[1]
            self.arr[i] = LrpProblem2D(_ptr(U), _ptr(V), _ld(U) if r else n, r, rmax,
                                       eps, Ux.data_ptr(), Vx.data_ptr(), max(n, 1), 0,
                                       LrpInfo())
        self.opts = _opts(prec, **kw)
        self.inputs = problems            # keeps the inputs alive

    def run(self, stream=None, results=True):
        """Solve every problem; returns [(Ux, Vx, info)] (views of the
        reused outputs) or, with results=False, None (``results()`` builds
        the list later)."""
        nb = len(self.arr)
        if nb == 0:
            return []
        st = getattr(self.ctx.lib, self.entry)(self.ctx.h, self.n, nb, self.arr,
                                               ctypes.byref(self.opts), _stream(stream))
        if st in (LRP_EINVAL, LRP_EDEVICE, LRP_ENOMEM):
            raise LrpError(st, self.entry)
        return self.results() if results else None

    def results(self):
        """[(Ux, Vx, info)] of the last run (views of the reused outputs)."""
        res = []
        for i, (Ux, Vx) in enumerate(self.outs):
            R = self.arr[i].rank_out
            res.append((Ux[:, :R], Vx[:, :R], self.arr[i].info.as_dict()))
        return res


class Context:
    """Solver context on one GPU (owns tables and workspace)."""

    def __init__(self, device: int = 0, workspace_bytes: int = 0):
        self.lib = load()
        self.h = ctypes.c_void_p()
        st = self.lib.lrp_create(ctypes.byref(self.h), device, workspace_bytes)
        if st != LRP_OK:
            raise LrpError(st, "lrp_create")
        self.device = device

    def close(self):
        if self.h:
            self.lib.lrp_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- 2D
    def solve2d(self, U, V, eps, rmax=None, prec="fp64", stream=None, check=True,
                **kw):
        """Solve T X + X T = U V^T; returns (Ux, Vx, info) with X ~= Ux Vx^T."""
        n, r = U.shape
        rmax = MAX_RANK if rmax is None else rmax
        Ux = empty_colmajor(n, rmax, U.device)
        Vx = empty_colmajor(n, rmax, U.device)
        rank = ctypes.c_int32(0)
        info = LrpInfo()
        opts = _opts(prec, **kw)
        st = self.lib.lrpoisson_solve2d(
            self.h, n, r, _ptr(U), _ptr(V), _ld(U) if r else n, eps,
            ctypes.byref(opts), _ptr(Ux), _ptr(Vx), n, rmax, ctypes.byref(rank),
            ctypes.byref(info), _stream(stream))
        if check and st not in (LRP_OK,):
            raise LrpError(st, "lrpoisson_solve2d")
        R = rank.value
        d = info.as_dict()
        d["status_code"] = st
        return Ux[:, :R], Vx[:, :R], d

    def solve2d_batch(self, problems, prec="fp64", stream=None, rmax=None, **kw):
        """problems: list of (U, V, eps) on one grid size.  Returns a list of
        (Ux, Vx, info)."""
        if not problems:
            return []
        return self.batch2d(problems, prec=prec, rmax=rmax, **kw).run(stream)

    def batch2d(self, problems, prec="fp64", rmax=None, method="cross", **kw):
        """A prepared batch: the argument array and the output factors are
        built once and reused by every ``run()`` (each run solves every
        problem of the batch from its inputs).  method "expsum" runs the
        exponential-sum comparator instead of the cross."""
        return Batch2D(self, problems, prec, rmax, kw, method)

    def expsum_solve2d_batch(self, problems, prec="fp64", stream=None, rmax=None, **kw):
        """The exponential-sum comparator on problems (U, V, eps) of one grid
        size: a list of (Ux, Vx, info), info["k"] = the number of terms,
        info["sweeps"] = the rounding steps."""
        if not problems:
            return []
        return self.batch2d(problems, prec=prec, rmax=rmax, method="expsum", **kw).run(stream)

    # ---- the low-rank Uzawa-GMRES Stokes driver
    def stokes2d(self, fu, fv, g, eps, rmax=None, prec="fp64", max_iter=0, restart=0,
                 stream=None, check=True):
        """The 2D Stokes problem on n x n pressure cells: fu, fv = (U, V)
        factor pairs of the velocity right-hand sides ((n-1) rows), g = (U, V)
        of the pressure one (n rows), column-major float64 GPU tensors.
        Returns ((pU, pV), (uU, uV), (vU, vV), info)."""
        import torch
        n = g[0].shape[0]
        rmax = MAX_RANK if rmax is None else rmax
        dev = g[0].device
        # inputs share one leading dimension: copy them into n-row blocks
        ld = n

        def pad(t, rows):
            out = torch.zeros((max(t.shape[1], 1), ld), dtype=torch.float64, device=dev).T
            out[:rows, :t.shape[1]] = t
            return out[:, :t.shape[1]]
        ins = [pad(fu[0], n - 1), pad(fu[1], n - 1), pad(fv[0], n - 1), pad(fv[1], n - 1),
               pad(g[0], n), pad(g[1], n)]
        outs = [empty_colmajor(n, rmax, dev) for _ in range(6)]
        pr = LrpStokes2DProblem()
        pr.n = n
        pr.rank_fu, pr.rank_fv, pr.rank_g = fu[0].shape[1], fv[0].shape[1], g[0].shape[1]
        pr.prec = PREC[prec] if isinstance(prec, str) else int(prec)
        pr.fu_U, pr.fu_V, pr.fv_U, pr.fv_V, pr.g_U, pr.g_V = [_ptr(t) for t in ins]
        pr.ld = ld
        pr.eps = eps
        pr.max_iter = max_iter
        pr.restart = restart
        pr.p_U, pr.p_V, pr.u_U, pr.u_V, pr.v_U, pr.v_V = [_ptr(t) for t in outs]
        pr.ldx = n
        pr.rmax = rmax
        st = self.lib.lrp_stokes2d(self.h, ctypes.byref(pr), _stream(stream))
        if check and st != LRP_OK:
            raise LrpError(st, "lrp_stokes2d")
        rp, ru, rv = pr.rank_out[0], pr.rank_out[1], pr.rank_out[2]
        info = dict(status=st, iterations=pr.iterations, restarts=pr.restarts,
                    max_krylov_rank=pr.max_krylov_rank, residual=pr.residual,
                    true_residual=pr.true_residual, ranks=(rp, ru, rv))
        return ((outs[0][:, :rp], outs[1][:, :rp]),
                (outs[2][:n - 1, :ru], outs[3][:n - 1, :ru]),
                (outs[4][:n - 1, :rv], outs[5][:n - 1, :rv]), info)

    # ---- the cross's building blocks on caller data (lrpoisson_kernels.h)
    def kernel_qr_maxvol(self, A, tau=0.0, stream=None):
        """TSQR of A (n x k, column-major float64 on the GPU) and maxvol on
        its Q: returns (Q, R, rows, converged)."""
        import torch
        n, k = A.shape
        Q = empty_colmajor(n, k, A.device)
        R = empty_colmajor(k, k, A.device)
        rows = (ctypes.c_int32 * max(k, 1))()
        conv = ctypes.c_int32(0)
        st = self.lib.lrp_kernel_qr_maxvol(self.h, n, k, _ptr(A), _ld(A), float(tau), _ptr(Q),
                                           n, _ptr(R), k, rows, ctypes.byref(conv),
                                           _stream(stream))
        if st != LRP_OK:
            raise LrpError(st, "lrp_kernel_qr_maxvol")
        return Q, R, [rows[i] for i in range(k)], bool(conv.value)

    def lowrank_round(self, U, V, eps, rmax=MAX_RANK, stream=None):
        """Round U V^T (n x K factors on the GPU) to eps: returns (Ux, Vx)."""
        n, K = U.shape
        Ux = empty_colmajor(n, rmax, U.device)
        Vx = empty_colmajor(n, rmax, U.device)
        rank = ctypes.c_int32(0)
        st = self.lib.lrp_lowrank_round(self.h, n, K, _ptr(U), _ptr(V), _ld(U) if K else n,
                                        eps, _ptr(Ux), _ptr(Vx), n, rmax, ctypes.byref(rank),
                                        _stream(stream))
        if st != LRP_OK:
            raise LrpError(st, f"lrp_lowrank_round (rank {rank.value})")
        return Ux[:, :rank.value], Vx[:, :rank.value]

    def kernel_core_svd(self, M, stream=None):
        """Jacobi SVD of a k x k core (column-major float64 on the GPU):
        returns (W, sigma, Z) with M = W diag(sigma) Z^T."""
        import torch
        k = M.shape[0]
        W = empty_colmajor(k, k, M.device)
        Z = empty_colmajor(k, k, M.device)
        sig = torch.empty(k, dtype=torch.float64, device=M.device)
        st = self.lib.lrp_kernel_core_svd(self.h, k, _ptr(M), _ld(M), _ptr(W), _ptr(sig),
                                          _ptr(Z), _stream(stream))
        if st != LRP_OK:
            raise LrpError(st, "lrp_kernel_core_svd")
        return W, sig, Z

    def expsum_solve2d(self, U, V, eps, rmax=None, prec="fp64", stream=None, **kw):
        """One comparator solve; returns (Ux, Vx, info)."""
        return self.expsum_solve2d_batch([(U, V, eps)], prec=prec, stream=stream,
                                         rmax=rmax, **kw)[0]

    # ---- 3D
    def solve3d(self, U1, U2, U3, G, eps, rmax=None, prec="fp64", stream=None,
                check=True, **kw):
        """Solve the 7-point problem with the Tucker RHS [[G; U1, U2, U3]].

        U_d: column-major (n, r_d) float64 GPU tensors; G: (r0, r1, r2)
        float64 GPU tensor, contiguous in Fortran order (i0 fastest), e.g.
        ``fortran_core(G)``.  Returns (Xs, Gx, info) with Xs the three output
        factors (orthonormal columns) and Gx the output core as an
        (R0, R1, R2) tensor view in Fortran order.
        """
        import torch
        n = U1.shape[0]
        ranks = (ctypes.c_int32 * 3)(U1.shape[1], U2.shape[1], U3.shape[1])
        rm = [MAX_RANK] * 3 if rmax is None else list(rmax)
        rmx = (ctypes.c_int32 * 3)(*rm)
        Xs = [empty_colmajor(n, rm[d], U1.device) for d in range(3)]
        Gbuf = torch.empty(max(1, rm[0] * rm[1] * rm[2]), dtype=torch.float64,
                           device=U1.device)
        rank = (ctypes.c_int32 * 3)(0, 0, 0)
        info = LrpInfo()
        opts = _opts(prec, **kw)
        lds = [_ld(u) for u in (U1, U2, U3) if u.shape[1] > 0]
        if lds and any(x != lds[0] for x in lds):
            raise ValueError("U1, U2, U3 must share one leading dimension")
        ld = lds[0] if lds else n
        st = self.lib.lrpoisson_solve3d(
            self.h, n, ranks, _ptr(U1), _ptr(U2), _ptr(U3), ld, _ptr(G), eps,
            ctypes.byref(opts), _ptr(Xs[0]), _ptr(Xs[1]), _ptr(Xs[2]), n,
            _ptr(Gbuf), rmx, rank, ctypes.byref(info), _stream(stream))
        if check and st != LRP_OK:
            raise LrpError(st, "lrpoisson_solve3d")
        R = [rank[d] for d in range(3)]
        d = info.as_dict()
        d["status_code"] = st
        d["ranks"] = tuple(R)
        if any(R[i] > rm[i] for i in range(3)):
            # LRP_ERANKCAP: rank_out holds the ranks needed, nothing written
            return [Xs[i][:, :0] for i in range(3)], Gbuf[:0].view(0, 0, 0), d
        Gx = Gbuf[:R[0] * R[1] * R[2]].view(R[2], R[1], R[0]).permute(2, 1, 0)
        return [Xs[i][:, :R[i]] for i in range(3)], Gx, d

    # ---- sine transform
    def sine_transform(self, X, prec="fp64", out=None, stream=None):
        """S X for a column-major (n, c) float64 GPU tensor."""
        n, c = X.shape
        Y = empty_colmajor(n, c, X.device) if out is None else out
        st = self.lib.lrp_sine_transform(self.h, n, c, _ptr(X), _ld(X), _ptr(Y),
                                         _ld(Y) if c else n, PREC[prec],
                                         _stream(stream))
        if st != LRP_OK:
            raise LrpError(st, "lrp_sine_transform")
        return Y

    def sine_transform_noalloc(self, X, prec="fp64", out=None, stream=None):
        """S X through the entry point that allocates nothing (the output is
        allocated here, by torch, when not given)."""
        n, c = X.shape
        Y = empty_colmajor(n, c, X.device) if out is None else out
        st = self.lib.lrp_sine_transform_noalloc(n, c, _ptr(X), _ld(X), _ptr(Y),
                                                 _ld(Y) if c else n, PREC[prec],
                                                 _stream(stream))
        if st != LRP_OK:
            raise LrpError(st, "lrp_sine_transform_noalloc")
        return Y

    # ---- kernel timing
    def set_kernel_timing(self, on: bool):
        st = self.lib.lrp_set_kernel_timing(self.h, 1 if on else 0)
        if st != LRP_OK:
            raise LrpError(st, "lrp_set_kernel_timing")

    def set_graph_replay(self, on: bool):
        """Replay the cross sweep steps as captured HIP graphs (default on)."""
        st = self.lib.lrp_set_graph_replay(self.h, 1 if on else 0)
        if st != LRP_OK:
            raise LrpError(st, "lrp_set_graph_replay")

    def kernel_stats(self, prec="fp64", reset=False):
        k = LrpKernelStat()
        st = self.lib.lrp_kernel_stats(self.h, PREC[prec], ctypes.byref(k),
                                       1 if reset else 0)
        if st != LRP_OK:
            raise LrpError(st, "lrp_kernel_stats")
        return dict(launches=k.launches, columns=k.columns, ms=k.ms, flops=k.flops)

    # ---- serving
    def submit(self, U, V, eps, prec="auto", rmax=None, out=None, op="laplace"):
        """Queue a 2D request; returns (ticket, (Ux, Vx))."""
        n, r = U.shape
        rmax = MAX_RANK if rmax is None else rmax
        if out is None:
            out = (empty_colmajor(n, rmax, U.device), empty_colmajor(n, rmax, U.device))
        Ux, Vx = out
        q = LrpRequest()
        q.dim = 2
        q.prec = PREC[prec]
        q.n = n
        q.rank[0] = r
        q.rmax[0] = rmax
        q.U[0] = _ptr(U)
        q.U[1] = _ptr(V)
        q.ld = _ld(U) if r else n
        q.X[0] = _ptr(Ux)
        q.X[1] = _ptr(Vx)
        q.ldx = n
        q.eps = eps
        q.op = OP[op]
        t = ctypes.c_uint64(0)
        st = self.lib.lrp_submit(self.h, ctypes.byref(q), ctypes.byref(t))
        if st != LRP_OK:
            raise LrpError(st, "lrp_submit")
        return t.value, (Ux, Vx)

    def submit3d(self, U1, U2, U3, G, eps, prec="auto", rmax=None, out=None,
                 op="laplace"):
        """Queue a 3D request (G: Fortran-ordered flat GPU tensor, see
        ``fortran_core``); returns (ticket, (X1, X2, X3, Gbuf)).  The output
        core is Gbuf[:R0*R1*R2] in Fortran order."""
        import torch
        n = U1.shape[0]
        rm = [MAX_RANK] * 3 if rmax is None else list(rmax)
        if out is None:
            out = tuple(empty_colmajor(n, rm[d], U1.device) for d in range(3)) + (
                torch.empty(max(1, rm[0] * rm[1] * rm[2]), dtype=torch.float64,
                            device=U1.device),)
        q = LrpRequest()
        q.dim = 3
        q.prec = PREC[prec]
        q.n = n
        lds = []
        for d, u in enumerate((U1, U2, U3)):
            q.rank[d] = u.shape[1]
            q.rmax[d] = rm[d]
            q.U[d] = _ptr(u)
            q.X[d] = _ptr(out[d])
            if u.shape[1]:
                lds.append(_ld(u))
        q.G = _ptr(G)
        q.Gx = _ptr(out[3])
        q.ld = lds[0] if lds else n
        q.ldx = n
        q.eps = eps
        q.op = OP[op]
        t = ctypes.c_uint64(0)
        st = self.lib.lrp_submit(self.h, ctypes.byref(q), ctypes.byref(t))
        if st != LRP_OK:
            raise LrpError(st, "lrp_submit")
        return t.value, out

    def serve_step(self):
        pend = ctypes.c_int32(0)
        st = self.lib.lrp_serve_step(self.h, ctypes.byref(pend))
        if st != LRP_OK:
            raise LrpError(st, "lrp_serve_step")
        return pend.value

    def poll(self, ticket):
        """None while pending, else (status, ranks, info)."""
        res = ctypes.c_int32(0)
        ranks = (ctypes.c_int32 * 3)()
        info = LrpInfo()
        st = self.lib.lrp_poll(self.h, ticket, ctypes.byref(res), ranks,
                               ctypes.byref(info))
        if st == LRP_ENOTREADY:
            return None
        if st != LRP_OK:
            raise LrpError(st, "lrp_poll")
        return res.value, list(ranks), info.as_dict()

    def wait(self, ticket):
        """Block (running scheduling ticks) until the request has finished;
        returns (status, ranks, info)."""
        res = ctypes.c_int32(0)
        ranks = (ctypes.c_int32 * 3)()
        info = LrpInfo()
        st = self.lib.lrp_wait(self.h, ticket, ctypes.byref(res), ranks,
                               ctypes.byref(info))
        if st != LRP_OK:
            raise LrpError(st, "lrp_wait")
        return res.value, list(ranks), info.as_dict()

    # ---- raw call for argument-validation tests
    def raw_solve2d(self, n, r, U, V, ld, eps, Ux, Vx, ldx, rmax, prec=0, **kw):
        rank = ctypes.c_int32(-1)
        info = LrpInfo()
        opts = _opts(prec, **kw)
        return self.lib.lrpoisson_solve2d(self.h, n, r, U, V, ld, eps,
                                          ctypes.byref(opts), Ux, Vx, ldx, rmax,
                                          ctypes.byref(rank), ctypes.byref(info),
                                          None), rank.value
