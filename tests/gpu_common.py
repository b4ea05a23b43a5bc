"""Helpers shared by the GPU tests (no method arithmetic here)."""
import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def to_dev(x):
    torch = torch_cuda()
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda")


def gpu_matvec(pos, forces, a, eta=1.0, eps=1e-6, **kw):
    import paper_1711_02976_amd as R
    torch = torch_cuda()
    P = R.Plan(to_dev(pos), a, eta, eps, **kw)
    try:
        u = P.matvec(to_dev(forces))
        torch.cuda.synchronize()
        return u.cpu().numpy(), P.stats()
    finally:
        P.free()
