"""Helpers for the GPU parity tests: device tensors and a shared context."""
import numpy as np

_CTX = None


def ctx():
    global _CTX
    from paper_1603_09337_amd import hasf
    if _CTX is None:
        _CTX = hasf.Context(0)
    return _CTX


def dev(a, pitch=None):
    """uint8 numpy image -> CUDA tensor view with row pitch `pitch` (>= W)."""
    import torch
    a = np.ascontiguousarray(a, dtype=np.uint8)
    H, W = a.shape
    if pitch is None or pitch == W:
        return torch.from_numpy(a.copy()).to("cuda:0")
    buf = torch.full((H, pitch), 7, dtype=torch.uint8, device="cuda:0")
    buf[:, :W] = torch.from_numpy(a).to("cuda:0")
    return buf[:, :W]


def host(t):
    return t.cpu().numpy()


def say(*a):
    print(*a, flush=True)
