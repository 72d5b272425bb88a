"""TEST INFRASTRUCTURE ONLY: ctypes wrapper around the plain FP64 CPU oracle.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (``paper_2601_02540_amd``)
never does; it has no fallback to this code.

Parity status of each oracle function (what pins it) is listed in
``tests/test_oracle_*.py``; every function here is pinned.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sgn_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")

# Plain evaluation order: no FMA contraction, no fast-math.
BUILD_CMD = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-o", _LIB, _SRC]
# The same source with its OpenMP pragmas on: the threaded build used to time
# the oracle on all host cores and to speed up large windows in the tests.
# Its loops split only over disjoint outputs, so it forms the same bits as the
# serial build (tests/test_oracle.py::test_threaded_build_bit_identical).
BUILD_CMD_OMP = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                 "-shared", "-o", _LIB_OMP, _SRC]


def build() -> str:
    subprocess.check_call(BUILD_CMD)
    subprocess.check_call(BUILD_CMD_OMP)
    return _LIB


class _OrcGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("xmin", ctypes.c_double), ("xmax", ctypes.c_double),
                ("ymin", ctypes.c_double), ("ymax", ctypes.c_double),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
                ("g", ctypes.c_double), ("lam", ctypes.c_double)]


_libs = {}
_threaded = False


class threaded:
    """Context manager: oracle calls inside it use the OpenMP build (all host
    cores, or OMP_NUM_THREADS), which forms the same bits as the serial one."""

    def __enter__(self):
        global _threaded
        self._prev = _threaded
        _threaded = True
        return self

    def __exit__(self, *exc):
        global _threaded
        _threaded = self._prev
        return False


def threads_available() -> int:
    """Threads the OpenMP build uses (its omp_get_max_threads())."""
    _load(True)
    lib = _libs[True]
    return int(lib.orc_threads())


def _load(omp=None):
    omp = _threaded if omp is None else omp
    path = _LIB_OMP if omp else _LIB
    if omp not in _libs:
        if not os.path.exists(path):
            build()
        if omp:
            # Keep freed planes of up to 32 MiB (glibc's limit for this
            # setting) in the heap, so that the threaded build's buffers are
            # not faulted in page by page, serially, on every call.
            libc = ctypes.CDLL(None)
            libc.mallopt(-3, 1 << 25)   # M_MMAP_THRESHOLD
            libc.mallopt(-1, 1 << 40)   # M_TRIM_THRESHOLD
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        d = ctypes.c_double
        dp = P(ctypes.c_double)
        fp = P(ctypes.c_float)
        gp = P(_OrcGrid)
        lib.orc_spacing.argtypes = [gp, dp, dp]
        lib.orc_op1d_dense.argtypes = [ctypes.c_int, ctypes.c_int, d, d, dp, dp, dp]
        lib.orc_apply_dx.argtypes = [gp, dp, dp]
        lib.orc_apply_dy.argtypes = [gp, dp, dp]
        lib.orc_rhs.argtypes = [gp, dp, dp, d, ctypes.c_int, dp]
        lib.orc_rhs_f32.argtypes = [gp, fp, fp, d, ctypes.c_int, fp]
        lib.orc_rhs_jvp.argtypes = [gp, dp, dp, dp, dp, dp]
        lib.orc_rk4.argtypes = [gp, dp, dp, d, d, ctypes.c_int64, ctypes.c_int]
        lib.orc_rk4_f32.argtypes = [gp, fp, fp, d, d, ctypes.c_int64, ctypes.c_int]
        lib.orc_init_aux.argtypes = [gp, dp, dp]
        lib.orc_rk4_relax.argtypes = [gp, dp, dp, d, d, ctypes.c_int64, dp, dp]
        lib.orc_mass_energy.argtypes = [gp, dp, dp, dp, dp]
        lib.orc_mass_energy_f32.argtypes = [gp, fp, fp, dp, dp]
        lib.orc_rates.argtypes = [gp, dp, dp, dp, dp, dp]
        lib.orc_cfl_dt.argtypes = [gp, dp, d]
        lib.orc_cfl_dt.restype = d
        lib.orc_mms_fields.argtypes = [gp, d, dp, dp]
        lib.orc_mms_source.argtypes = [gp, d, dp]
        lib.orc_rhs_vjp.argtypes = [gp, dp, dp, dp, dp, dp]
        lib.orc_rk4_vjp.argtypes = [gp, dp, dp, d, dp, dp]
        lib.orc_rk4_jvp.argtypes = [gp, dp, dp, d, dp, dp, dp]
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.orc_gauge_loss.argtypes = [gp, dp, dp, d, ctypes.c_int64, i64p, ctypes.c_int, dp, dp, dp, dp, dp]
        lib.orc_gauge_loss_grad.argtypes = [gp, dp, dp, d, ctypes.c_int64, i64p, ctypes.c_int, dp, dp, dp, dp]
        lib.orc_threads.restype = ctypes.c_int
        lib.orc_fsal35.argtypes = [gp, dp, dp, d, d, d, d, d, ctypes.c_int, ctypes.c_int64, dp, dp, i64p, i64p]
        lib.orc_fsal35.restype = ctypes.c_int64
        lib.orc_fsal35_tableau.argtypes = [dp, dp, dp, dp]
        _libs[omp] = lib
    return _libs[omp]


def _grid(grid) -> _OrcGrid:
    return _OrcGrid(grid.nx, grid.ny, grid.xmin, grid.xmax, grid.ymin, grid.ymax,
                    grid.bc_x, grid.bc_y, grid.g, grid.lam)


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fp(a: np.ndarray):
    assert a.dtype == np.float32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _state(q, grid) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert q.shape == (5, grid.ny, grid.nx), q.shape
    return q


def _plane(b, grid) -> np.ndarray:
    b = np.ascontiguousarray(b, dtype=np.float64)
    assert b.shape == (grid.ny, grid.nx), b.shape
    return b


def spacing(grid) -> Tuple[float, float]:
    dx, dy = ctypes.c_double(), ctypes.c_double()
    _load().orc_spacing(ctypes.byref(_grid(grid)), ctypes.byref(dx), ctypes.byref(dy))
    return dx.value, dy.value


def op1d_dense(n: int, bc: int, lo: float, hi: float):
    D = np.zeros((n, n))
    w = np.zeros(n)
    bn = np.zeros(n)
    _load().orc_op1d_dense(n, bc, lo, hi, _dp(D), _dp(w), _dp(bn))
    return D, w, bn


def apply_dx(grid, f) -> np.ndarray:
    f = _plane(f, grid)
    out = np.empty_like(f)
    _load().orc_apply_dx(ctypes.byref(_grid(grid)), _dp(f), _dp(out))
    return out


def apply_dy(grid, f) -> np.ndarray:
    f = _plane(f, grid)
    out = np.empty_like(f)
    _load().orc_apply_dy(ctypes.byref(_grid(grid)), _dp(f), _dp(out))
    return out


def rhs(grid, q, b, t: float = 0.0, src: int = 0) -> np.ndarray:
    q = _state(q, grid)
    b = _plane(b, grid)
    out = np.empty_like(q)
    _load().orc_rhs(ctypes.byref(_grid(grid)), _dp(q), _dp(b), t, src, _dp(out))
    return out


def rhs_f32(grid, q, b, t: float = 0.0, src: int = 0) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    out = np.empty_like(q)
    _load().orc_rhs_f32(ctypes.byref(_grid(grid)), _fp(q), _fp(b), t, src, _fp(out))
    return out


def rhs_jvp(grid, q, b, dq, db: Optional[np.ndarray] = None) -> np.ndarray:
    """Directional derivative of rhs along (dq, db) by the complex step."""
    q = _state(q, grid)
    b = _plane(b, grid)
    dq = _state(dq, grid)
    out = np.empty_like(q)
    dbp = _dp(_plane(db, grid)) if db is not None else None
    _load().orc_rhs_jvp(ctypes.byref(_grid(grid)), _dp(q), _dp(b), _dp(dq), dbp, _dp(out))
    return out


def rk4(grid, q, b, dt: float, nsteps: int, t0: float = 0.0, src: int = 0) -> np.ndarray:
    q = _state(q, grid).copy()
    b = _plane(b, grid)
    _load().orc_rk4(ctypes.byref(_grid(grid)), _dp(q), _dp(b), dt, t0, nsteps, src)
    return q


def rk4_f32(grid, q, b, dt: float, nsteps: int, t0: float = 0.0, src: int = 0) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float32).copy()
    b = np.ascontiguousarray(b, dtype=np.float32)
    _load().orc_rk4_f32(ctypes.byref(_grid(grid)), _fp(q), _fp(b), dt, t0, nsteps, src)
    return q


def rk4_relax(grid, q, b, dt: float, nsteps: int, t0: float = 0.0):
    """Relaxation RK4 (incremental direction form): returns (q, t_end, gammas)."""
    q = _state(q, grid).copy()
    b = _plane(b, grid)
    t_end = ctypes.c_double()
    gam = np.zeros(max(int(nsteps), 1))
    _load().orc_rk4_relax(ctypes.byref(_grid(grid)), _dp(q), _dp(b), dt, t0, int(nsteps), ctypes.byref(t_end), _dp(gam))
    return q, t_end.value, gam[:nsteps]


def fsal35(grid, q, b, t0: float, t_end: float, dt0: float, rtol: float = 1e-6, atol: float = 1e-6,
           adaptive: bool = True, max_attempts: int = 1_000_000):
    """The adaptive five-stage third-order FSAL pair from t0 to t_end.  Returns
    (q, t_reached, accepted, rejected, rec) with rec[n] = (h, err, accepted) of
    attempt n."""
    q = _state(q, grid).copy()
    b = _plane(b, grid)
    cap = int(max_attempts) if max_attempts < 10_000_000 else 10_000_000
    rec = np.zeros((max(cap, 1), 3))
    t_out = ctypes.c_double()
    na, nr = ctypes.c_int64(), ctypes.c_int64()
    n = _load().orc_fsal35(ctypes.byref(_grid(grid)), _dp(q), _dp(b), t0, t_end, dt0, rtol, atol, int(adaptive),
                           cap, _dp(rec), ctypes.byref(t_out), ctypes.byref(na), ctypes.byref(nr))
    return q, t_out.value, na.value, nr.value, rec[:n]


def fsal35_tableau():
    """(c, A, b, bh) of the adaptive pair: A is 6 x 6 (row 5 is the FSAL stage)."""
    c, A, b, bh = np.zeros(6), np.zeros((6, 6)), np.zeros(6), np.zeros(6)
    _load().orc_fsal35_tableau(_dp(c), _dp(A), _dp(b), _dp(bh))
    return c, A, b, bh


def init_aux(grid, q, b) -> np.ndarray:
    q = _state(q, grid).copy()
    b = _plane(b, grid)
    _load().orc_init_aux(ctypes.byref(_grid(grid)), _dp(q), _dp(b))
    return q


def mass_energy(grid, q, b) -> Tuple[float, float]:
    m, e = ctypes.c_double(), ctypes.c_double()
    if np.asarray(q).dtype == np.float32:
        qf = np.ascontiguousarray(q, dtype=np.float32)
        bf = np.ascontiguousarray(b, dtype=np.float32)
        _load().orc_mass_energy_f32(ctypes.byref(_grid(grid)), _fp(qf), _fp(bf), ctypes.byref(m), ctypes.byref(e))
    else:
        q = _state(q, grid)
        b = _plane(b, grid)
        _load().orc_mass_energy(ctypes.byref(_grid(grid)), _dp(q), _dp(b), ctypes.byref(m), ctypes.byref(e))
    return m.value, e.value


def rates(grid, q, b):
    """(mass_rate, energy_rate, sum M|h_t|, sum M |d_qE . q_t| termwise)."""
    q = _state(q, grid)
    b = _plane(b, grid)
    mr, er = ctypes.c_double(), ctypes.c_double()
    scale = np.zeros(2)
    _load().orc_rates(ctypes.byref(_grid(grid)), _dp(q), _dp(b), ctypes.byref(mr), ctypes.byref(er), _dp(scale))
    return mr.value, er.value, scale[0], scale[1]


def cfl_dt(grid, q, cfl: float = 0.5) -> float:
    q = _state(q, grid)
    return _load().orc_cfl_dt(ctypes.byref(_grid(grid)), _dp(q), cfl)


def mms_fields(grid, t: float):
    q = np.empty((5, grid.ny, grid.nx))
    b = np.empty((grid.ny, grid.nx))
    _load().orc_mms_fields(ctypes.byref(_grid(grid)), t, _dp(q), _dp(b))
    return q, b


def mms_source(grid, t: float) -> np.ndarray:
    S = np.empty((5, grid.ny, grid.nx))
    _load().orc_mms_source(ctypes.byref(_grid(grid)), t, _dp(S))
    return S


def rhs_vjp(grid, q, b, a):
    """(q_bar, b_bar) = J^T a for the right-hand side's Jacobian J wrt (q, b)."""
    q = _state(q, grid)
    b = _plane(b, grid)
    a = _state(a, grid)
    qb = np.zeros_like(q)
    bb = np.zeros_like(b)
    _load().orc_rhs_vjp(ctypes.byref(_grid(grid)), _dp(q), _dp(b), _dp(a), _dp(qb), _dp(bb))
    return qb, bb


def rk4_vjp(grid, q, b, dt: float, qbar):
    """Reverse of one RK4 step from state q: returns (q_bar_n, b_bar) for cotangent qbar of q_{n+1}."""
    q = _state(q, grid)
    b = _plane(b, grid)
    qb = _state(qbar, grid).copy()
    bb = np.zeros_like(b)
    _load().orc_rk4_vjp(ctypes.byref(_grid(grid)), _dp(q), _dp(b), dt, _dp(qb), _dp(bb))
    return qb, bb


def rk4_jvp(grid, q, b, dt: float, dq, db=None):
    """Directional derivative of one RK4 step along (dq, db) by the complex step."""
    q = _state(q, grid)
    b = _plane(b, grid)
    dq = _state(dq, grid)
    out = np.empty_like(q)
    dbp = _dp(_plane(db, grid)) if db is not None else None
    _load().orc_rk4_jvp(ctypes.byref(_grid(grid)), _dp(q), _dp(b), dt, _dp(dq), dbp, _dp(out))
    return out


def _gauges(gidx):
    g = np.ascontiguousarray(gidx, dtype=np.int64)
    return g, g.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def gauge_loss(grid, zeta0, b, dt, nsteps, gauge_nodes, target, dzeta0=None, db=None):
    """(L, dL along (dzeta0, db)) by the complex step; gauge_nodes are row-major node indices."""
    zeta0 = _plane(zeta0, grid)
    b = _plane(b, grid)
    g, gp = _gauges(gauge_nodes)
    target = np.ascontiguousarray(target, dtype=np.float64)
    assert target.shape == (nsteps, g.size)
    L, dL = ctypes.c_double(), ctypes.c_double()
    dz = _dp(_plane(dzeta0, grid)) if dzeta0 is not None else None
    dbp = _dp(_plane(db, grid)) if db is not None else None
    _load().orc_gauge_loss(ctypes.byref(_grid(grid)), _dp(zeta0), _dp(b), dt, nsteps, gp, g.size, _dp(target),
                           dz, dbp, ctypes.byref(L), ctypes.byref(dL))
    return L.value, dL.value


def gauge_loss_grad(grid, zeta0, b, dt, nsteps, gauge_nodes, target):
    """(L, dL/dzeta0, dL/db) by the discrete adjoint."""
    zeta0 = _plane(zeta0, grid)
    b = _plane(b, grid)
    g, gp = _gauges(gauge_nodes)
    target = np.ascontiguousarray(target, dtype=np.float64)
    assert target.shape == (nsteps, g.size)
    L = ctypes.c_double()
    gz = np.zeros_like(zeta0)
    gb = np.zeros_like(b)
    _load().orc_gauge_loss_grad(ctypes.byref(_grid(grid)), _dp(zeta0), _dp(b), dt, nsteps, gp, g.size,
                                _dp(target), ctypes.byref(L), _dp(gz), _dp(gb))
    return L.value, gz, gb
