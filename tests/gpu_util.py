"""Shared helpers of the GPU tests (need torch with a visible MI355X and the built library)."""
import numpy as np
import torch

from paper_2508_18540_amd import torch_api as T

_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        assert torch.cuda.is_available(), "GPU tests need a visible GPU"
        _CTX = T.Context(0)
    return _CTX


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t if dtype is None else t.to(dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().float().cpu().numpy().astype(np.float64)


def psnr(a, b):
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10 * np.log10(1.0 / mse)


def announce(*args):
    print("[case]", *args, flush=True)
