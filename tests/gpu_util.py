"""Helpers for the GPU tests: device context, transfers, oracle comparisons."""
import sys

import numpy as np


def log(*a):
    """Name the case before each GPU step (flushed, so a crash still shows it)."""
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


_CTX = None


def ctx():
    global _CTX
    import torch
    from paper_1306_2150_amd import binding
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    if _CTX is None:
        _CTX = binding.Context(0, workspace_bytes=48 << 30)
    return _CTX


def dev(a):
    from paper_1306_2150_amd import binding
    return binding.colmajor(a)


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))
