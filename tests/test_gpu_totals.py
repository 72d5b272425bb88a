"""sgn_step_totals through the C ABI: the step kernel records the total mass and
energy after every step (a6: totals fused into the step's last stage).

* The states are the states of sgn_step, bit for bit (same kernels).
* Each recorded pair equals sgn_mass_energy of the state after that step to
  rounding (the sums are the same nodes' values in another order), and the
  last one the oracle's totals of its RK4 state to 1e-12.
* Graph replays (8 steps) and direct remainders, odd and even counts, both
  step-tile shapes, both boundary types, FP32 storage, repeated calls (the
  series index restarts), and argument errors.
"""

import ctypes
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2601_02540_amd import workloads as W
from gpu_util import dev, host, solver

pytestmark = pytest.mark.gpu

PER, REF = W.PERIODIC, W.REFLECTING


def problem(bc, nx, ny, seed):
    g = W.Grid(nx, ny, -1.0, 1.5, -1.0, 1.0, bc, bc, 9.81, 500.0)
    q, b = W.random_state(g, seed, b_scale=0.1)
    q[1:4] *= 0.3
    return g, oracle.init_aux(g, q, b), b


@pytest.mark.parametrize("bc", [PER, REF])
@pytest.mark.parametrize("ty", [8, 16, 24])
@pytest.mark.parametrize("n", [1, 8, 13])
def test_series_matches_per_step_totals(bc, ty, n):
    g, q0, b = problem(bc, 77, 45, seed=n + ty)
    dt = oracle.cfl_dt(g, q0, 0.5)
    s = solver(g)
    s.set_tile_y(ty)
    s.set_bathymetry(dev(b))
    qd = dev(q0)
    series = host(s.step_totals(qd, dt, n))
    assert series.shape == (n, 2)
    # reference: single steps with a separate totals pass after each
    r = solver(g)
    r.set_bathymetry(dev(b))
    qr = dev(q0)
    for k in range(n):
        r.step(qr, dt, 1)
        m, e = r.mass_energy(qr)
        assert math.isclose(series[k, 0], m, rel_tol=1e-14), (k, series[k, 0], m)
        assert math.isclose(series[k, 1], e, rel_tol=1e-14), (k, series[k, 1], e)
    assert np.array_equal(host(qd), host(qr))
    s.check()
    mo, eo = oracle.mass_energy(g, oracle.rk4(g, q0, b, dt, n), b)
    assert math.isclose(series[-1, 0], mo, rel_tol=1e-12) and math.isclose(series[-1, 1], eo, rel_tol=1e-12)


@pytest.mark.parametrize("path", ["pairs", "stages"])
def test_series_whatever_the_step_path(path):
    """The recorded steps run on the step kernel whatever the selected path;
    every path forms the same states, so the result equals sgn_step's."""
    g, q0, b = problem(REF, 70, 41, seed=11)
    dt = oracle.cfl_dt(g, q0, 0.5)
    s = solver(g)
    s.set_step_path(path)
    s.set_bathymetry(dev(b))
    qa, qb = dev(q0), dev(q0)
    series = host(s.step_totals(qa, dt, 10))
    s.step(qb, dt, 10)
    assert np.array_equal(host(qa), host(qb))
    m, e = s.mass_energy(qb)
    assert math.isclose(series[-1, 0], m, rel_tol=1e-14) and math.isclose(series[-1, 1], e, rel_tol=1e-14)


def test_series_repeated_calls_and_fp32():
    g, q0, b = problem(PER, 96, 64, seed=5)
    dt = oracle.cfl_dt(g, q0, 0.5)
    for dtype in (torch.float64, torch.float32):
        s = solver(g, dtype)
        s.set_bathymetry(dev(b, dtype))
        qd = dev(q0, dtype)
        first = host(s.step_totals(qd, dt, 17))
        second = host(s.step_totals(qd, dt, 3))  # index restarts at 0
        m, e = s.mass_energy(qd)
        assert math.isclose(second[-1, 0], m, rel_tol=1e-13) and math.isclose(second[-1, 1], e, rel_tol=1e-13)
        assert np.all(np.isfinite(first)) and first.shape == (17, 2)
        # mass is conserved to rounding along the whole series
        assert np.abs(first[:, 0] / first[0, 0] - 1.0).max() <= (1e-13 if dtype == torch.float64 else 1e-6)


def test_series_argument_errors():
    from paper_2601_02540_amd.binding import SgnError
    g, q0, b = problem(PER, 32, 32, seed=1)
    s = solver(g)
    s.set_bathymetry(dev(b))
    qd = dev(q0)
    assert s.step_totals(qd, 1e-3, 0).shape == (0, 2)
    assert s.lib.sgn_step_totals(s.ctx, ctypes.c_void_p(qd.data_ptr()), 1e-3, 2, None) == -1  # NULL series
    gm = W.mms_grid(32, PER)
    p = W.mms_initial(gm)
    sm = solver(gm, source=1)
    sm.set_bathymetry(dev(p.b))
    with pytest.raises(SgnError) as ei:
        sm.step_totals(dev(p.q0), 1e-3, 2)
    assert ei.value.status == -3
