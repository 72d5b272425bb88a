"""GPU parity of the adaptive five-stage FSAL pair (sgn_step_adaptive) against
the oracle's pair (oracle.fsal35), through the C ABI.

Both sides initialize the workload themselves and take their own CFL step as
the first attempted step; each records (h, err, accepted) per attempt.  The
attempt sequences must agree: the same accept/reject decisions, steps and error
norms within 1e-10 relative (they differ only by rounding, which the
controller's powers pass on), and the final state within 1e-12 field-relative
(FP64).  Fixed-step runs (every step accepted) are compared the same way, on
both boundary types and both tile heights, and FP32 runs against the FP32
bound of the plain step.  Every case runs on the default step path (the middle
four evaluations of an attempt in one launch of the step tile) and on the
four-stage path (one role kernel per evaluation); the two give the same bits."""

import numpy as np
import pytest
import torch

import oracle
from paper_2601_02540_amd import workloads as W
from gpu_util import STATE_FLOORS, dev, field_rel_err, fp32_bound, host, solver

pytestmark = pytest.mark.gpu

PER, REF = W.PERIODIC, W.REFLECTING
F64_TOL = 1e-12


def compare_records(got, ref):
    """Same decisions; steps within 1e-10 relative; error norms within 1e-10
    relative plus 1e-12 absolute: a small norm is a difference of nearly equal
    rates, whose rounding (~1e-16 |h k| / tol, about 1e-13 on the final, cut
    step of these runs) stays far below the threshold 1 it is compared with."""
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.array_equal(got[:, 2], ref[:, 2])
    np.testing.assert_allclose(got[:, 0], ref[:, 0], rtol=1e-10, atol=0)
    np.testing.assert_allclose(got[:, 1], ref[:, 1], rtol=1e-10, atol=1e-12)


PATHS = ["fused", "stages"]


def run_gpu(g, q0, b, t_end, dt0, dtype=torch.float64, ty=None, path="fused", **kw):
    s = solver(g, dtype)
    if ty is not None:
        s.set_tile_y(ty)
    s.set_step_path(path)
    s.set_bathymetry(dev(b, dtype))
    qd = dev(q0, dtype)
    res, rec = s.step_adaptive(qd, 0.0, t_end, dt0, record=4096, **kw)
    n = res["attempts"]
    rec = host(rec)[:n]
    return res, rec, host(qd)


def adaptive_case(bc):
    """A 64^2 Gaussian bump (periodic, lambda = 500) or a wavy reflecting state."""
    if bc == PER:
        p = W.gaussian_bump_periodic(64, seed=1)
        g, b = p.grid, p.b
        return g, oracle.init_aux(g, p.q0, b), b, 1.0
    g = W.Grid(96, 40, 0.0, 30.0, 0.0, 10.0, REF, REF, 9.81, 500.0)
    q, b = W.random_state(g, 11, b_scale=0.05)
    q[1:4] *= 0.05
    return g, oracle.init_aux(g, q, b), b, 0.2


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("bc", [PER, REF])
def test_adaptive_run_matches_oracle(bc, path):
    """rtol = atol = 1e-6 (the paper's tolerances)."""
    g, q0, b, t_end = adaptive_case(bc)
    dt0 = oracle.cfl_dt(g, q0, 0.5)
    ref, t_ref, na, nr, rec_ref = oracle.fsal35(g, q0, b, 0.0, t_end, dt0)
    res, rec, got = run_gpu(g, q0, b, t_end, dt0, path=path)
    assert res["reached_end"] == 1 and res["t"] == t_ref == t_end
    assert (res["accepted"], res["rejected"]) == (na, nr)
    compare_records(rec, rec_ref)
    err = field_rel_err(got, ref, STATE_FLOORS)
    assert np.all(err <= F64_TOL), err


@pytest.mark.parametrize("ty", [8, 16, 24])
@pytest.mark.parametrize("bc", [PER, REF])
def test_fused_attempt_matches_role_kernels_bitwise(bc, ty):
    """The one-launch middle evaluations and the four role kernels do the same
    arithmetic node by node: same records, same final state, bit for bit (both
    tile shapes of the step tile: 64 x 8 and 32 x 16)."""
    g, q0, b, t_end = adaptive_case(bc)
    dt0 = oracle.cfl_dt(g, q0, 0.5)
    out = [run_gpu(g, q0, b, t_end, dt0, ty=ty, path=path) for path in PATHS]
    (r0, rec0, q0f), (r1, rec1, q1f) = out
    assert r0 == r1
    assert np.array_equal(rec0, rec1)
    assert np.array_equal(q0f, q1f)


def test_switching_paths_on_one_context():
    """One context alternating between the step paths and tile shapes: each
    change drops the captured attempts, and every run gives the first run's
    bits."""
    g, q0, b, t_end = adaptive_case(PER)
    dt0 = oracle.cfl_dt(g, q0, 0.5)
    s = solver(g)
    s.set_bathymetry(dev(b))
    qd = dev(q0)
    q0d = qd.clone()
    outs = []
    # the same state buffer and no record every time: only the path and the tiles tell the runs apart
    for path, ty in (("fused", 16), ("stages", 16), ("fused", 8), ("pairs", 8), ("fused", 16)):
        s.set_tile_y(ty)
        s.set_step_path(path)
        qd.copy_(q0d)
        res = s.step_adaptive(qd, 0.0, t_end, dt0)
        outs.append((res, host(qd)))
    for res, q in outs[1:]:
        assert res == outs[0][0]
        assert np.array_equal(q, outs[0][1])


@pytest.mark.parametrize("path", PATHS)
def test_too_large_first_step_is_rejected_like_the_oracle(path):
    p = W.gaussian_bump_periodic(64, seed=2)
    g, b = p.grid, p.b
    q0 = oracle.init_aux(g, p.q0, b)
    dt_cfl = oracle.cfl_dt(g, q0, 0.5)
    t_end = 30 * dt_cfl
    ref, t_ref, na, nr, rec_ref = oracle.fsal35(g, q0, b, 0.0, t_end, 15 * dt_cfl)
    assert nr >= 1
    res, rec, got = run_gpu(g, q0, b, t_end, 15 * dt_cfl, path=path)
    compare_records(rec, rec_ref)
    assert np.all(field_rel_err(got, ref, STATE_FLOORS) <= F64_TOL)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("ty", [8, 16, 24])
@pytest.mark.parametrize("bcs", [(PER, PER), (REF, REF), (PER, REF), (REF, PER)])
def test_fixed_steps_match_oracle(bcs, ty, path):
    """Fixed steps (adaptive = 0) on a ragged grid: the state after 7 steps and
    the recorded error norms."""
    g = W.Grid(70, 37, -1.0, 2.0, 0.5, 2.0, bcs[0], bcs[1], 9.81, 500.0)
    q, b = W.random_state(g, 5, b_scale=0.05)
    q[1:4] *= 0.1
    q0 = oracle.init_aux(g, q, b)
    dt = 0.3 * oracle.cfl_dt(g, q0, 0.5)
    ref, _, na, _, rec_ref = oracle.fsal35(g, q0, b, 0.0, 7 * dt, dt, adaptive=False)
    res, rec, got = run_gpu(g, q0, b, 7 * dt, dt, ty=ty, path=path, adaptive=False)
    assert res["accepted"] == na == 7 and res["rejected"] == 0
    compare_records(rec, rec_ref)
    assert np.all(field_rel_err(got, ref, STATE_FLOORS) <= F64_TOL)


@pytest.mark.parametrize("shape", [(4, 4), (5, 7), (33, 17)])
@pytest.mark.parametrize("ty", [8, 16, 24])
@pytest.mark.parametrize("bcs", [(PER, PER), (REF, REF), (PER, REF), (REF, PER)])
def test_fused_attempt_on_grids_smaller_than_a_tile(shape, bcs, ty):
    """The attempt kernel where one tile covers the grid (rings and nodes past
    the edge are periodic images or wall copies) or spills over it by one node:
    3 fixed steps against the oracle."""
    nx, ny = shape
    g = W.Grid(nx, ny, -1.0, 2.0, 0.5, 2.0, bcs[0], bcs[1], 9.81, 500.0)
    q, b = W.random_state(g, 3 * nx + ny, b_scale=0.05)
    q[1:4] *= 0.1
    q0 = oracle.init_aux(g, q, b)
    dt = 0.3 * oracle.cfl_dt(g, q0, 0.5)
    ref, _, na, _, rec_ref = oracle.fsal35(g, q0, b, 0.0, 3 * dt, dt, adaptive=False)
    res, rec, got = run_gpu(g, q0, b, 3 * dt, dt, ty=ty, path="fused", adaptive=False)
    assert res["accepted"] == na == 3 and res["rejected"] == 0
    compare_records(rec, rec_ref)
    assert np.all(field_rel_err(got, ref, STATE_FLOORS) <= F64_TOL), (shape, bcs, ty)


@pytest.mark.parametrize("path", PATHS)
def test_fp32_bounded_by_oracle_fp32_error(path):
    """FP32 storage and arithmetic, fixed steps: within the FP32 bound of the
    plain RK4 step over the same interval (the pair's rounding is of the same
    kind), against the FP64 oracle pair."""
    p = W.gaussian_bump_periodic(64, seed=1)
    g = p.grid
    b32 = p.b.astype(np.float32).astype(np.float64)
    q0 = oracle.init_aux(g, p.q0, b32).astype(np.float32).astype(np.float64)
    dt = oracle.cfl_dt(g, q0, 0.5)
    ref, *_ = oracle.fsal35(g, q0, b32, 0.0, 20 * dt, dt, adaptive=False)
    bound = field_rel_err(oracle.rk4_f32(g, q0, b32, dt, 20).astype(np.float64), oracle.rk4(g, q0, b32, dt, 20),
                          STATE_FLOORS)
    res, rec, got = run_gpu(g, q0, b32, 20 * dt, dt, dtype=torch.float32, path=path, adaptive=False)
    assert res["accepted"] == 20
    err = field_rel_err(got, ref, STATE_FLOORS)
    assert np.all(err <= fp32_bound(bound)), (err, bound)


def test_fp32_adaptive_run_reaches_the_fp64_solution():
    """Adaptive stepping with FP32 state and arithmetic (error norm and
    controller in FP64) at the paper's tolerances, 64^2 Gaussian bump to t = 1
    (the paper left FP32 after step-size trouble with adaptive stepping): the
    run reaches t_end, rejects few attempts (here as many as the FP64 run: 2 of
    31), takes within 30% of the FP64 oracle run's accepted steps, and ends
    within 1e-4 field-relative of the oracle's state: about 30 steps each
    allowed a local error of 1e-6 relative, plus the FP32 rounding of the
    state (measured: at most 8e-6)."""
    p = W.gaussian_bump_periodic(64, seed=1)
    g = p.grid
    b32 = p.b.astype(np.float32).astype(np.float64)
    q0 = oracle.init_aux(g, p.q0, b32)
    dt0 = oracle.cfl_dt(g, q0, 0.5)
    ref, t_ref, na, nr, _ = oracle.fsal35(g, q0, b32, 0.0, 1.0, dt0)
    res, rec, got = run_gpu(g, q0.astype(np.float32).astype(np.float64), b32, 1.0, dt0, dtype=torch.float32)
    err = field_rel_err(got, ref, STATE_FLOORS)
    print("fp32 adaptive:", res, "fp64 accepted/rejected", na, nr, "field errors", err)
    assert res["reached_end"] == 1 and res["rejected"] <= 0.1 * res["attempts"], res
    assert abs(res["accepted"] - na) <= 0.3 * na, (res["accepted"], na)
    assert np.all(err <= 1e-4), err


def test_attempt_limit_and_arguments():
    from paper_2601_02540_amd.binding import SgnError
    p = W.gaussian_bump_periodic(32, seed=3)
    g = p.grid
    s = solver(g)
    s.set_bathymetry(dev(p.b))
    qd = dev(oracle.init_aux(g, p.q0, p.b))
    dt = s.cfl_dt(qd, 0.5)
    res = s.step_adaptive(qd, 0.0, 100 * dt, dt, max_attempts=5)
    assert res["reached_end"] == 0 and res["attempts"] == 5 and res["t"] < 100 * dt
    for bad in (dict(t0=1.0, t_end=0.0, dt0=dt), dict(t0=0.0, t_end=1.0, dt0=0.0),
                dict(t0=0.0, t_end=1.0, dt0=dt, rtol=0.0, atol=0.0), dict(t0=0.0, t_end=1.0, dt0=dt, max_attempts=0)):
        with pytest.raises(SgnError) as ei:
            s.step_adaptive(qd, **bad)
        assert ei.value.status == -1
    src = solver(W.mms_grid(32, PER), source=1)
    src.set_bathymetry(dev(np.zeros((32, 32))))
    with pytest.raises(SgnError) as ei:
        src.step_adaptive(dev(np.ones((5, 32, 32))), 0.0, 1.0, 1e-3)
    assert ei.value.status == -3


@pytest.fixture(scope="module")
def obstacle_full_size():
    """The paper's solitary wave over a Gaussian obstacle at its spacing 0.025
    (1600 x 800, periodic) from t = 0 to 0.03 at rtol = atol = 1e-6 (the
    first attempts of the adaptive benchmark run, step growing from the CFL
    step), on the oracle's threaded build (bit-identical to the serial one)."""
    p = W.gaussian_obstacle(1600)
    g, b = p.grid, p.b
    with oracle.threaded():
        q0 = oracle.init_aux(g, p.q0, b)
        dt0 = oracle.cfl_dt(g, q0, 0.5)
        ref, t_ref, na, nr, rec_ref = oracle.fsal35(g, q0, b, 0.0, 0.03, dt0)
    return g, q0, b, dt0, ref, t_ref, na, nr, rec_ref


@pytest.mark.parametrize("path", PATHS)
def test_full_size_obstacle_run_matches_oracle(obstacle_full_size, path):
    g, q0, b, dt0, ref, t_ref, na, nr, rec_ref = obstacle_full_size
    assert na >= 6
    res, rec, got = run_gpu(g, q0, b, 0.03, dt0, path=path)
    assert res["reached_end"] == 1 and res["t"] == t_ref
    assert (res["accepted"], res["rejected"]) == (na, nr)
    compare_records(rec, rec_ref)
    assert np.all(field_rel_err(got, ref, STATE_FLOORS) <= F64_TOL)
