"""Thin ctypes binding of the C ABI in ``include/sgn.h``.

Argument marshalling only: every step of the computation runs in the HIP
library ``libsgn.so``.  PyTorch supplies device memory (tensors) and the stream
(the current stream when a :class:`Solver` is created).  There is no CPU
fallback: without a GPU or without the built library every entry point raises.
"""

from __future__ import annotations

import ctypes
import os
import re
from typing import List, Optional, Tuple

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "libsgn.so")
HEADER_PATH = os.path.join(ROOT, "include", "sgn.h")

SGN_F64, SGN_F32 = 0, 1
SGN_SRC_NONE, SGN_SRC_MMS = 0, 1
SGN_OPT_STEP_PATH, SGN_OPT_TILE_Y, SGN_OPT_ADJOINT_STORE = 0, 1, 2
SGN_PATH_PAIRS, SGN_PATH_STAGES, SGN_PATH_FUSED = 0, 1, 2


class SgnError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_name(status)} ({status}): {message}")
        self.status = status


class SgnAdaptiveResult(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("h_next", ctypes.c_double), ("last_err", ctypes.c_double),
                ("attempts", ctypes.c_int64), ("accepted", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("reached_end", ctypes.c_int32)]


class SgnParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("xmin", ctypes.c_double), ("xmax", ctypes.c_double),
                ("ymin", ctypes.c_double), ("ymax", ctypes.c_double),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
                ("g", ctypes.c_double), ("lam", ctypes.c_double),
                ("dtype", ctypes.c_int32), ("source", ctypes.c_int32)]


_lib = None


def header_symbols() -> List[str]:
    """Every function declared in include/sgn.h."""
    text = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(sgn_[a-z0-9_]+)\s*\(", text, re.M)))


def load_library() -> ctypes.CDLL:
    """Loads libsgn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2601_02540_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, cvp = ctypes.c_void_p, ctypes.c_void_p
    d, dp = ctypes.c_double, ctypes.POINTER(ctypes.c_double)
    st = ctypes.c_int32
    sigs = {
        "sgn_create": ([ctypes.POINTER(SgnParams), vp, ctypes.POINTER(vp)], st),
        "sgn_destroy": ([vp], st),
        "sgn_set_stream": ([vp, vp], st),
        "sgn_set_option": ([vp, ctypes.c_int32, ctypes.c_int64], st),
        "sgn_set_bathymetry": ([vp, cvp], st),
        "sgn_init_aux": ([vp, vp], st),
        "sgn_rhs": ([vp, cvp, vp, d], st),
        "sgn_step": ([vp, vp, d, ctypes.c_int64, d], st),
        "sgn_prepare_step": ([vp, vp, d, ctypes.c_int64], st),
        "sgn_step_adaptive": ([vp, vp, d, d, d, d, d, ctypes.c_int32, ctypes.c_int64, dp, ctypes.c_int64,
                               ctypes.POINTER(SgnAdaptiveResult)], st),
        "sgn_mass": ([vp, cvp, dp], st),
        "sgn_energy": ([vp, cvp, dp], st),
        "sgn_mass_energy": ([vp, cvp, dp, dp], st),
        "sgn_mass_energy_noalloc": ([ctypes.POINTER(SgnParams), cvp, cvp, vp, dp], st),
        "sgn_rates": ([vp, cvp, dp, dp], st),
        "sgn_cfl_dt": ([vp, cvp, d, dp], st),
        "sgn_check": ([vp], st),
        "sgn_profile_stages": ([vp, vp, d, ctypes.c_int64, dp], st),
        "sgn_spacing": ([vp, dp, dp], st),
        "sgn_last_error": ([vp], ctypes.c_char_p),
        "sgn_rhs_vjp": ([vp, cvp, cvp, vp, vp], st),
        "sgn_step_vjp": ([vp, cvp, d, vp, vp], st),
        "sgn_gauge_series": ([vp, cvp, ctypes.c_int64, d, cvp, ctypes.c_int32, vp], st),
        "sgn_gauge_loss_grad": ([vp, cvp, ctypes.c_int64, d, cvp, ctypes.c_int32, cvp, ctypes.c_int64, dp, vp, vp],
                                st),
        "sgn_batch_create": ([ctypes.c_int32, ctypes.POINTER(SgnParams), vp, ctypes.POINTER(vp)], st),
        "sgn_batch_destroy": ([vp], st),
        "sgn_batch_set_bathymetry": ([vp, ctypes.c_int32, cvp], st),
        "sgn_batch_set_states": ([vp, ctypes.POINTER(vp)], st),
        "sgn_batch_init_aux": ([vp], st),
        "sgn_batch_step": ([vp, dp, ctypes.c_int64], st),
        "sgn_batch_mass_energy": ([vp, dp, dp], st),
        "sgn_batch_cfl_dt": ([vp, d, dp], st),
        "sgn_batch_set_tiling": ([vp, ctypes.c_int32, ctypes.c_int32], st),
        "sgn_step_relaxation": ([vp, vp, d, ctypes.c_int64, d, dp], st),
        "sgn_step_totals": ([vp, vp, d, ctypes.c_int64, vp], st),
        "sgn_batch_set_step_path": ([vp, ctypes.c_int32], st),
        "sgn_batch_autotune": ([vp, dp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), dp], st),
        "sgn_batch_check": ([vp, ctypes.POINTER(ctypes.c_int32)], st),
        "sgn_batch_total_nodes": ([vp, ctypes.POINTER(ctypes.c_int64)], st),
        "sgn_batch_last_error": ([vp], ctypes.c_char_p),
        "sgn_status_string": ([ctypes.c_int32], ctypes.c_char_p),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def status_name(status: int) -> str:
    try:
        return load_library().sgn_status_string(status).decode()
    except Exception:  # pragma: no cover - only when the library itself is unavailable
        return str(status)


def _torch():
    import torch
    return torch


def _require_gpu():
    torch = _torch()
    if not torch.cuda.is_available():
        raise RuntimeError("the SGN solver runs only on a ROCm GPU (torch.cuda.is_available() is False)")


def mass_energy_noalloc(grid, q, b, out, stream=None):
    """sgn_mass_energy_noalloc: mass and energy of state q (5 planes) over
    bathymetry b into the device tensor out (2 float64 values), asynchronously
    on `stream` (default: the current stream), without a context and without
    any allocation by the library."""
    torch = _torch()
    _require_gpu()
    lib = load_library()
    if q.dtype not in (torch.float64, torch.float32) or b.dtype != q.dtype:
        raise ValueError("q and b must share dtype float64 or float32")
    if tuple(q.shape) != (5, grid.ny, grid.nx) or tuple(b.shape) != (grid.ny, grid.nx):
        raise ValueError("q must be (5, ny, nx) and b (ny, nx)")
    if not (q.is_cuda and b.is_cuda and out.is_cuda and q.is_contiguous() and b.is_contiguous()):
        raise ValueError("q, b and out must be contiguous device tensors")
    if out.dtype != torch.float64 or out.numel() < 2 or not out.is_contiguous():
        raise ValueError("out must hold two contiguous float64 values")
    stream = torch.cuda.current_stream(q.device) if stream is None else stream
    p = SgnParams(grid.nx, grid.ny, grid.xmin, grid.xmax, grid.ymin, grid.ymax, grid.bc_x, grid.bc_y,
                  grid.g, grid.lam, SGN_F64 if q.dtype == torch.float64 else SGN_F32, SGN_SRC_NONE)
    s = lib.sgn_mass_energy_noalloc(ctypes.byref(p), ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(b.data_ptr()),
                                    ctypes.c_void_p(stream.cuda_stream),
                                    ctypes.cast(ctypes.c_void_p(out.data_ptr()), ctypes.POINTER(ctypes.c_double)))
    if s != 0:
        raise SgnError(s, lib.sgn_last_error(None).decode())
    return out


class Solver:
    """One C-ABI context for one grid, storage type and stream.

    ``grid`` is any object with nx, ny, xmin, xmax, ymin, ymax, bc_x, bc_y, g, lam
    (e.g. :class:`paper_2601_02540_amd.workloads.Grid`).
    """

    def __init__(self, grid, dtype=None, source: int = SGN_SRC_NONE, device: Optional[int] = None):
        torch = _torch()
        _require_gpu()
        self.lib = load_library()
        self.grid = grid
        self.dtype = torch.float64 if dtype is None else dtype
        if self.dtype not in (torch.float64, torch.float32):
            raise ValueError("dtype must be torch.float64 or torch.float32")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            p = SgnParams(grid.nx, grid.ny, grid.xmin, grid.xmax, grid.ymin, grid.ymax, grid.bc_x, grid.bc_y,
                          grid.g, grid.lam, SGN_F64 if self.dtype == torch.float64 else SGN_F32, source)
            ctx = ctypes.c_void_p()
            s = self.lib.sgn_create(ctypes.byref(p), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
            if s != 0:
                raise SgnError(s, self.lib.sgn_last_error(None).decode())
        self.ctx = ctx
        self.shape = (5, grid.ny, grid.nx)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.sgn_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -----------------------------------------------------------
    def _chk(self, s: int):
        if s != 0:
            raise SgnError(s, self.lib.sgn_last_error(self.ctx).decode())

    def _state(self, q, name="q"):
        if tuple(q.shape) != self.shape or q.dtype != self.dtype or not q.is_contiguous() or q.device != self.device:
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of shape {self.shape} on {self.device}")
        return ctypes.c_void_p(q.data_ptr())

    def _plane(self, b, name="b"):
        if tuple(b.shape) != self.shape[1:] or b.dtype != self.dtype or not b.is_contiguous() or b.device != self.device:
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of shape {self.shape[1:]} on {self.device}")
        return ctypes.c_void_p(b.data_ptr())

    def empty_state(self):
        return _torch().empty(self.shape, dtype=self.dtype, device=self.device)

    # -- API ---------------------------------------------------------------
    def spacing(self) -> Tuple[float, float]:
        dx, dy = ctypes.c_double(), ctypes.c_double()
        self._chk(self.lib.sgn_spacing(self.ctx, ctypes.byref(dx), ctypes.byref(dy)))
        return dx.value, dy.value

    def set_option(self, option: int, value: int):
        self._chk(self.lib.sgn_set_option(self.ctx, int(option), int(value)))

    def set_step_path(self, path: str):
        """'fused' (one kernel per step, default), 'pairs' (two fused stage pairs per step) or
        'stages' (four stage kernels)."""
        self.set_option(SGN_OPT_STEP_PATH,
                        {"pairs": SGN_PATH_PAIRS, "stages": SGN_PATH_STAGES, "fused": SGN_PATH_FUSED}[path])

    def set_tile_y(self, ty: int):
        self.set_option(SGN_OPT_TILE_Y, ty)

    def set_adjoint_store(self, nbytes: int):
        """Device memory the gauge-loss gradient may fill with the states and stage
        states of the rollout's last steps instead of recomputing them."""
        self.set_option(SGN_OPT_ADJOINT_STORE, nbytes)

    def set_bathymetry(self, b):
        self._chk(self.lib.sgn_set_bathymetry(self.ctx, self._plane(b)))
        self._b = b  # the copy is asynchronous: keep the source alive until the stream passes it

    def init_aux(self, q):
        self._chk(self.lib.sgn_init_aux(self.ctx, self._state(q)))
        return q

    def rhs(self, q, dq=None, t: float = 0.0):
        if dq is None:
            dq = self.empty_state()
        self._chk(self.lib.sgn_rhs(self.ctx, self._state(q), self._state(dq, "dq"), float(t)))
        return dq

    def step(self, q, dt: float, nsteps: int = 1, t0: float = 0.0):
        self._chk(self.lib.sgn_step(self.ctx, self._state(q), float(dt), int(nsteps), float(t0)))
        return q

    def prepare_step(self, q, dt: float, nsteps: int):
        """Instantiate the graphs step(q, dt, nsteps) replays; runs nothing."""
        self._chk(self.lib.sgn_prepare_step(self.ctx, self._state(q), float(dt), int(nsteps)))

    def step_adaptive(self, q, t0: float, t_end: float, dt0: float, rtol: float = 1e-6, atol: float = 1e-6,
                      adaptive: bool = True, max_attempts: int = 1_000_000, record: int = 0):
        """The adaptive five-stage third-order FSAL pair from t0 to t_end, q in
        place.  Returns a dict of the run (t, h_next, last_err, attempts,
        accepted, rejected, reached_end) and, with record > 0, a (record, 3)
        float64 device tensor of (h, err, accepted) per attempt."""
        torch = _torch()
        rec = None
        rp = None
        if record > 0:
            rec = torch.full((int(record), 3), float("nan"), dtype=torch.float64, device=self.device)
            rp = ctypes.cast(ctypes.c_void_p(rec.data_ptr()), ctypes.POINTER(ctypes.c_double))
        out = SgnAdaptiveResult()
        self._chk(self.lib.sgn_step_adaptive(self.ctx, self._state(q), float(t0), float(t_end), float(dt0),
                                             float(rtol), float(atol), 1 if adaptive else 0, int(max_attempts), rp,
                                             int(record), ctypes.byref(out)))
        res = {k: getattr(out, k) for k, _ in SgnAdaptiveResult._fields_}
        return (res, rec) if record > 0 else res

    def step_relaxation(self, q, dt: float, nsteps: int = 1, t0: float = 0.0) -> float:
        """Relaxation RK4 steps in place; returns the final time t0 + sum gam_n dt."""
        t_end = ctypes.c_double()
        self._chk(self.lib.sgn_step_relaxation(self.ctx, self._state(q), float(dt), int(nsteps), float(t0),
                                               ctypes.byref(t_end)))
        return t_end.value

    def step_totals(self, q, dt: float, nsteps: int = 1):
        """RK4 steps in place, recording mass and energy after every step;
        returns a (nsteps, 2) FP64 tensor on the device (asynchronous)."""
        torch = _torch()
        series = torch.empty((max(int(nsteps), 0), 2), dtype=torch.float64, device=self.device)
        self._chk(self.lib.sgn_step_totals(self.ctx, self._state(q), float(dt), int(nsteps),
                                           ctypes.c_void_p(series.data_ptr())))
        return series

    def mass_energy(self, q) -> Tuple[float, float]:
        m, e = ctypes.c_double(), ctypes.c_double()
        self._chk(self.lib.sgn_mass_energy(self.ctx, self._state(q), ctypes.byref(m), ctypes.byref(e)))
        return m.value, e.value

    def mass(self, q) -> float:
        m = ctypes.c_double()
        self._chk(self.lib.sgn_mass(self.ctx, self._state(q), ctypes.byref(m)))
        return m.value

    def energy(self, q) -> float:
        e = ctypes.c_double()
        self._chk(self.lib.sgn_energy(self.ctx, self._state(q), ctypes.byref(e)))
        return e.value

    def rates(self, q) -> Tuple[float, float]:
        mr, er = ctypes.c_double(), ctypes.c_double()
        self._chk(self.lib.sgn_rates(self.ctx, self._state(q), ctypes.byref(mr), ctypes.byref(er)))
        return mr.value, er.value

    def cfl_dt(self, q, cfl: float = 0.5) -> float:
        dt = ctypes.c_double()
        self._chk(self.lib.sgn_cfl_dt(self.ctx, self._state(q), float(cfl), ctypes.byref(dt)))
        return dt.value

    def profile_stages(self, q, dt: float, nsteps: int):
        """Mean kernel durations (ms) over nsteps steps: the four stage kernels, the two
        pair kernels (then two zeros) or the step kernel (then three zeros)."""
        ms = (ctypes.c_double * 4)()
        self._chk(self.lib.sgn_profile_stages(self.ctx, self._state(q), float(dt), int(nsteps), ms))
        return list(ms)

    def check(self):
        self._chk(self.lib.sgn_check(self.ctx))

    # -- discrete adjoint ------------------------------------------------------
    def rhs_vjp(self, q, a):
        """(qbar, bbar) = J^T a for the right-hand side's Jacobian at q."""
        qbar = self.empty_state()
        bbar = _torch().empty(self.shape[1:], dtype=self.dtype, device=self.device)
        self._chk(self.lib.sgn_rhs_vjp(self.ctx, self._state(q), self._state(a, "a"), self._state(qbar, "qbar"),
                                       self._plane(bbar, "bbar")))
        return qbar, bbar

    def step_vjp(self, q_n, dt: float, qbar, bbar):
        """In place: qbar (cotangent of q_{n+1}) becomes that of q_n; bbar accumulates."""
        self._chk(self.lib.sgn_step_vjp(self.ctx, self._state(q_n), float(dt), self._state(qbar, "qbar"),
                                        self._plane(bbar, "bbar")))

    def _gauges(self, gauges):
        torch = _torch()
        if gauges.dtype != torch.int64 or gauges.device != self.device or gauges.dim() != 1:
            raise ValueError("gauges must be a 1-D int64 tensor of row-major node indices on the solver's device")
        n = self.shape[1] * self.shape[2]
        if gauges.numel() == 0 or int(gauges.min()) < 0 or int(gauges.max()) >= n:
            raise ValueError("gauge indices out of range")
        return gauges.contiguous()

    def gauge_series(self, zeta0, nsteps: int, dt: float, gauges):
        """zeta = h + b at the gauges after each of nsteps steps from surface zeta0 (float64 [nsteps, ng])."""
        torch = _torch()
        gauges = self._gauges(gauges)
        series = torch.empty((int(nsteps), gauges.numel()), dtype=torch.float64, device=self.device)
        self._chk(self.lib.sgn_gauge_series(self.ctx, self._plane(zeta0, "zeta0"), int(nsteps), float(dt),
                                            ctypes.c_void_p(gauges.data_ptr()), gauges.numel(),
                                            ctypes.c_void_p(series.data_ptr())))
        return series

    def gauge_loss_grad(self, zeta0, nsteps: int, dt: float, gauges, target, checkpoint_every: int = 0):
        """(L, dL/dzeta0, dL/db) of the gauge misfit; target is float64 [nsteps, ng] on the device."""
        torch = _torch()
        gauges = self._gauges(gauges)
        if tuple(target.shape) != (int(nsteps), gauges.numel()) or target.dtype != torch.float64 or \
                target.device != self.device:
            raise ValueError("target must be a float64 [nsteps, ngauges] tensor on the solver's device")
        target = target.contiguous()
        gz = torch.empty(self.shape[1:], dtype=self.dtype, device=self.device)
        gb = torch.empty_like(gz)
        loss = ctypes.c_double()
        self._chk(self.lib.sgn_gauge_loss_grad(self.ctx, self._plane(zeta0, "zeta0"), int(nsteps), float(dt),
                                               ctypes.c_void_p(gauges.data_ptr()), gauges.numel(),
                                               ctypes.c_void_p(target.data_ptr()), int(checkpoint_every),
                                               ctypes.byref(loss), ctypes.c_void_p(gz.data_ptr()),
                                               ctypes.c_void_p(gb.data_ptr())))
        return loss.value, gz, gb


class Batch:
    """An ensemble of independent problems (C-ABI sgn_batch_*).

    ``grids`` is a list of grid objects (see :class:`Solver`); all instances share
    ``dtype``.  States are caller-owned tensors registered with :meth:`set_states`.
    """

    def __init__(self, grids, dtype=None):
        torch = _torch()
        _require_gpu()
        self.lib = load_library()
        self.grids = list(grids)
        self.n = len(self.grids)
        self.dtype = torch.float64 if dtype is None else dtype
        code = SGN_F64 if self.dtype == torch.float64 else SGN_F32
        arr = (SgnParams * self.n)(*[SgnParams(g.nx, g.ny, g.xmin, g.xmax, g.ymin, g.ymax, g.bc_x, g.bc_y, g.g,
                                               g.lam, code, SGN_SRC_NONE) for g in self.grids])
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        s = self.lib.sgn_batch_create(self.n, arr, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if s != 0:
            raise SgnError(s, self.lib.sgn_batch_last_error(None).decode())
        self.h = h
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            self.lib.sgn_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, s):
        if s != 0:
            raise SgnError(s, self.lib.sgn_batch_last_error(self.h).decode())

    def _dbl(self, vals):
        return (ctypes.c_double * self.n)(*[float(v) for v in vals])

    def set_bathymetry(self, i: int, b):
        g = self.grids[i]
        if tuple(b.shape) != (g.ny, g.nx) or b.dtype != self.dtype or not b.is_contiguous():
            raise ValueError(f"bathymetry {i} must be a contiguous {self.dtype} tensor of shape {(g.ny, g.nx)}")
        self._chk(self.lib.sgn_batch_set_bathymetry(self.h, i, ctypes.c_void_p(b.data_ptr())))
        self._keep.append(b)

    def set_states(self, qs):
        for i, (q, g) in enumerate(zip(qs, self.grids)):
            if tuple(q.shape) != (5, g.ny, g.nx) or q.dtype != self.dtype or not q.is_contiguous():
                raise ValueError(f"state {i} must be a contiguous {self.dtype} tensor of shape {(5, g.ny, g.nx)}")
        ptrs = (ctypes.c_void_p * self.n)(*[q.data_ptr() for q in qs])
        self._chk(self.lib.sgn_batch_set_states(self.h, ptrs))
        self.states = list(qs)

    def init_aux(self):
        self._chk(self.lib.sgn_batch_init_aux(self.h))

    def step(self, dt, nsteps: int = 1):
        self._chk(self.lib.sgn_batch_step(self.h, self._dbl(dt), int(nsteps)))

    def mass_energy(self):
        m = (ctypes.c_double * self.n)()
        e = (ctypes.c_double * self.n)()
        self._chk(self.lib.sgn_batch_mass_energy(self.h, m, e))
        return list(m), list(e)

    def cfl_dt(self, cfl: float = 0.5):
        out = (ctypes.c_double * self.n)()
        self._chk(self.lib.sgn_batch_cfl_dt(self.h, float(cfl), out))
        return list(out)

    def set_step_path(self, path: str):
        """'fused' (one step kernel launch per RK4 step, default) or 'pairs'."""
        self._chk(self.lib.sgn_batch_set_step_path(self.h, {"fused": SGN_PATH_FUSED, "pairs": SGN_PATH_PAIRS,
                                                            "stages": SGN_PATH_STAGES}[path]))

    def set_tiling(self, tile_y: int, blocks_per_cu: int):
        self._chk(self.lib.sgn_batch_set_tiling(self.h, int(tile_y), int(blocks_per_cu)))

    def autotune(self, dt):
        ty, bpc = ctypes.c_int32(), ctypes.c_int32()
        ms = ctypes.c_double()
        self._chk(self.lib.sgn_batch_autotune(self.h, self._dbl(dt), ctypes.byref(ty), ctypes.byref(bpc),
                                              ctypes.byref(ms)))
        return ty.value, bpc.value, ms.value

    def check(self):
        bad = ctypes.c_int32(-1)
        self._chk(self.lib.sgn_batch_check(self.h, ctypes.byref(bad)))
        return bad.value

    def total_nodes(self) -> int:
        n = ctypes.c_int64()
        self._chk(self.lib.sgn_batch_total_nodes(self.h, ctypes.byref(n)))
        return n.value
