"""Helpers shared by the GPU parity tests (device transfer, case banners)."""
import sys

import numpy as np


def banner(msg: str):
    """Name the case before a GPU step, flushed, so a failing run names it."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(x, dtype=None):
    import torch
    a = np.ascontiguousarray(x)
    if dtype is not None:
        a = a.astype(dtype)
    return torch.from_numpy(a).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def c64(x):
    return np.ascontiguousarray(np.asarray(x).astype(np.complex64))
