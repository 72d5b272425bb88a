"""Helpers shared by the GPU tests (host-side only: tensors in and out, error norms)."""

import math

import numpy as np

# Field floors for the field-relative error of a state [h, u, v, w, eta]:
# depth-like planes are measured against the still-water depth 1, velocity-like
# planes against the shallow-water speed sqrt(g * 1).
STATE_FLOORS = (1.0, math.sqrt(9.81), math.sqrt(9.81), math.sqrt(9.81), 1.0)


# FP32 results are bounded by four times the error of the oracle evaluated in
# single precision, both measured field-relative against the FP64 oracle.
# Where the oracle's FP32 error is smaller than the rounding of the field
# itself to FP32 (a field that barely moves), the bound uses that rounding
# instead: half an FP32 ulp of the field scale, 2^-24.
FP32_FLOOR = 2.0 ** -24


def fp32_bound(oracle_f32_err):
    return 4.0 * np.maximum(oracle_f32_err, FP32_FLOOR)


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


# ---------------------------------------------------------------------------
# Exact checks of sampled windows of a large run (see test_gpu_fullsize.py):
# K RK4 steps at a node depend only on the initial state within 4K nodes, so
# the oracle steps a window widened by 4K nodes as a grid of its own and only
# the nodes at least 4K away from the window's artificial edges are compared.

def axis_window(kind, n, bc, reach, win, start=0):
    """Indices of a window along one axis, the window grid's boundary type and
    the slice of compared nodes.  kind: "in" (any start; wraps on a periodic
    axis), "wall_lo" or "wall_hi" (a reflecting axis's walls, kept as walls)."""
    per, ref = 0, 1
    if kind == "wall_lo":
        assert bc == ref
        return np.arange(0, win + reach), ref, slice(0, win)
    if kind == "wall_hi":
        assert bc == ref
        return np.arange(n - win - reach, n), ref, slice(reach, reach + win)
    idx = np.arange(start - reach, start + win + reach)
    if bc == per:
        idx = idx % n
    else:
        assert idx[0] >= 0 and idx[-1] < n
    return idx, per, slice(reach, reach + win)


def window_grid(grid, ny, nx, bcy, bcx):
    from paper_2601_02540_amd import workloads as W
    dx, dy = grid.spacing()
    lx = nx * dx if bcx == 0 else (nx - 1) * dx
    ly = ny * dy if bcy == 0 else (ny - 1) * dy
    return W.Grid(nx, ny, 0.0, lx, 0.0, ly, bcx, bcy, grid.g, grid.lam)


def check_windows(grid, q0, b, got, dt, steps, windows, win=32, f32=False):
    """Compare `got` (the GPU state after `steps` steps from q0) with the oracle
    on every window ((kind_y, start_y), (kind_x, start_x)); FP64 within 1e-12
    field-relative, FP32 within four times the oracle's own FP32 error."""
    import oracle
    reach = 4 * steps
    for (ky, sy), (kx, sx) in windows:
        ry, bcy, keep_y = axis_window(ky, grid.ny, grid.bc_y, reach, win, sy)
        rx, bcx, keep_x = axis_window(kx, grid.nx, grid.bc_x, reach, win, sx)
        wg = window_grid(grid, len(ry), len(rx), bcy, bcx)
        qw = q0[:, ry][:, :, rx]
        bw = b[ry][:, rx]
        ref = oracle.rk4(wg, qw, bw, dt, steps)[:, keep_y, keep_x]
        g = got[:, ry][:, :, rx][:, keep_y, keep_x]
        err = field_rel_err(g, ref, STATE_FLOORS)
        if f32:
            o32 = oracle.rk4_f32(wg, qw, bw, dt, steps).astype(np.float64)[:, keep_y, keep_x]
            bound = field_rel_err(o32, ref, STATE_FLOORS)
            assert np.all(err <= fp32_bound(bound)), ((ky, sy), (kx, sx), err, bound)
        else:
            assert np.all(err <= 1e-12), ((ky, sy), (kx, sx), err)
