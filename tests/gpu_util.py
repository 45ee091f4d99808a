"""Helpers shared by the GPU tests: numpy <-> column-major device tensors."""
import numpy as np


def torch():
    import torch as t
    return t


def dev(x, device="cuda:0"):
    """numpy (n x k) -> column-major complex128 tensor on the GPU."""
    t = torch()
    a = np.asarray(x, dtype=np.complex128)
    if a.ndim == 1:
        a = a[:, None]
    h = t.from_numpy(np.ascontiguousarray(a.T))
    return h.to(device).transpose(0, 1)


def host(t_):
    """column-major (or any) device tensor -> numpy array."""
    return t_.detach().cpu().numpy()


def rel_col_err(got, ref):
    num = np.linalg.norm(got - ref, axis=0)
    den = np.maximum(np.linalg.norm(ref, axis=0), 1e-300)
    return num / den
