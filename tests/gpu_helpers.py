"""Small helpers for the GPU tests (device tensors, canary padding)."""

import numpy as np


def torch():
    import torch as t
    return t


def dev():
    return torch().device("cuda:0")


def to_dev(a: np.ndarray):
    return torch().from_numpy(np.ascontiguousarray(a)).to(dev())


def to_host(t) -> np.ndarray:
    torch().cuda.synchronize()
    return t.cpu().numpy()


def grid_host(g) -> np.ndarray:
    return to_host(g).view(np.uint32)


def padded(n_elems: int, dtype, pad: int, fill: int):
    """A device buffer with `pad` canary elements before and after the
    `n_elems` payload; returns (whole, payload view)."""
    t = torch()
    whole = t.full((n_elems + 2 * pad,), fill, dtype=dtype, device=dev())
    return whole, whole[pad:pad + n_elems]


def canaries_intact(whole, pad: int, fill: int) -> bool:
    h = to_host(whole)
    return bool(np.all(h[:pad] == fill) and np.all(h[-pad:] == fill))
