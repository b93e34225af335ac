"""Shared helpers for the GPU parity tests (layout conversion, tolerances)."""
import numpy as np
import torch

DEV = "cuda:0"


def to_gpu(oracle_vec, dtype=torch.float64):
    """Oracle layout (dof, b) -> device vector [b][slab][l][space]."""
    a = np.ascontiguousarray(np.asarray(oracle_vec).T)
    return torch.from_numpy(a.ravel()).to(device=DEV, dtype=dtype)


def to_oracle(gpu_vec, batch):
    a = gpu_vec.detach().to("cpu", torch.float64).numpy()
    return a.reshape(batch, -1).T.copy()


def nodal_to_gpu(arr, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(arr).ravel()).to(device=DEV, dtype=dtype)


def rel_err(a, b):
    """max |a - b| / max |b| (elementwise against the oracle's scale)."""
    a = np.asarray(a)
    b = np.asarray(b)
    scale = np.abs(b).max()
    return np.abs(a - b).max() / (scale if scale > 0 else 1.0)


def norm_rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
