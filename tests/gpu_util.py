"""Helpers shared by the GPU tests (host-side only: tensors in and out, error norms)."""

import math

import numpy as np

# Field floors for the field-relative error of a state [h, u, v, w, eta]:
# depth-like planes are measured against the still-water depth 1, velocity-like
# planes against the shallow-water speed sqrt(g * 1).
STATE_FLOORS = (1.0, math.sqrt(9.81), math.sqrt(9.81), math.sqrt(9.81), 1.0)


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda().contiguous()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def field_rel_err(got, ref, floors=None):
    """Per-field max|got - ref| / max(max|ref|, floor)."""
    out = []
    for f in range(ref.shape[0]):
        scale = np.abs(ref[f]).max()
        if floors is not None:
            scale = max(scale, floors[f])
        scale = scale if scale > 0 else 1.0
        out.append(float(np.abs(got[f] - ref[f]).max() / scale))
    return np.array(out)


def solver(grid, dtype=None, source=0):
    from paper_2601_02540_amd.binding import Solver
    return Solver(grid, dtype=dtype, source=source)
