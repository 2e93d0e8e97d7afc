"""Shared helpers of the GPU parity tests (test infrastructure)."""
import numpy as np


def to_gpu(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).cuda()


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel_max(a, b):
    a, b = np.asarray(a).reshape(-1), np.asarray(b).reshape(-1)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def announce(msg):
    print(msg, flush=True)
