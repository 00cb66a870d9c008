"""Shared helpers of the GPU parity tests (comparison only, no method code)."""
import numpy as np

# FP64 parity bar: normwise relative error per component
TOL_FP64 = 1e-10
# mixed precision (FP32 Newton matrix, FP64 residual): bar after Newton
TOL_MIXED = 1e-8


def rel_err_per_component(a, ref):
    """max_z |a - ref| / max_z |ref| for each leading-axis component."""
    a = np.asarray(a, dtype=np.float64).reshape(a.shape[0], -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(ref.shape[0], -1)
    scale = np.abs(ref).max(axis=1)
    scale = np.where(scale > 0, scale, 1.0)
    return np.abs(a - ref).max(axis=1) / scale


def to_gpu(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_np(t):
    return t.detach().cpu().numpy()
