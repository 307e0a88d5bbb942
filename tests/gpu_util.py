"""Helpers shared by the GPU parity tests (no test functions here)."""
import sys

import numpy as np


def to_gpu(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(got - ref) / np.abs(ref)


def announce(*what):
    """Name the case on stdout before a GPU step (flushed), so a crash log
    says what ran."""
    print("[gpu case]", *what, flush=True)
    sys.stdout.flush()
