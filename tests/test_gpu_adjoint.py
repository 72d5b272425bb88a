"""GPU tests of the discrete adjoint: RHS and step VJPs against the oracle's
adjoint, the checkpointed loss gradient against the oracle and against
finite differences of the GPU loss, checkpoint-interval invariance and the
autograd wrapper."""

import numpy as np
import pytest
import torch

import oracle
from paper_2601_02540_amd import workloads as W
from paper_2601_02540_amd.adjoint import gauge_misfit_loss
from gpu_util import dev, field_rel_err, host, solver

pytestmark = pytest.mark.gpu

PER, REF = W.PERIODIC, W.REFLECTING
F64_TOL = 1e-12


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("shape", [(4, 4), (13, 11), (61, 17), (130, 37)])
@pytest.mark.parametrize("bcs", [(PER, PER), (REF, REF), (PER, REF), (REF, PER)])
def test_rhs_vjp_matches_oracle(shape, bcs):
    nx, ny = shape
    for lam in (0.0, 500.0):
        g = W.Grid(nx, ny, -1.0, 2.0, 0.5, 2.0, bcs[0], bcs[1], 9.81, lam)
        q, b = W.random_state(g, 3 * nx + ny)
        a = np.random.default_rng(nx + 7 * ny).standard_normal(q.shape)
        qb_ref, bb_ref = oracle.rhs_vjp(g, q, b, a)
        s = solver(g)
        s.set_bathymetry(dev(b))
        qb, bb = s.rhs_vjp(dev(q), dev(a))
        err = field_rel_err(host(qb), qb_ref)
        assert np.all(err <= F64_TOL), (shape, bcs, lam, err)
        assert rel(host(bb), bb_ref) <= F64_TOL


@pytest.mark.parametrize("path", ["fused", "stages"])
@pytest.mark.parametrize("ty", [8, 16, 24])
@pytest.mark.parametrize("bcs", [(PER, PER), (REF, REF), (REF, PER), (PER, REF)])
def test_step_vjp_matches_oracle(bcs, ty, path):
    """One RK4 step's VJP on a ragged 70 x 45 grid: on the fused path two
    two-stage reverse kernels (tiles 64 x 8 or 32 x 16), on the four-stage path
    the four role kernels."""
    g = W.Grid(70, 45, -1.0, 2.0, 0.5, 2.0, bcs[0], bcs[1], 9.81, 500.0)
    q, b = W.random_state(g, 11, b_scale=0.05)
    q[1:4] *= 0.1
    rng = np.random.default_rng(12)
    a = rng.standard_normal(q.shape)
    bb0 = rng.standard_normal(b.shape)
    dt = 0.2 * oracle.cfl_dt(g, q, 0.5)
    qb_ref, bb_ref = oracle.rk4_vjp(g, q, b, dt, a)
    s = solver(g)
    s.set_tile_y(ty)
    s.set_step_path(path)
    s.set_bathymetry(dev(b))
    qb = dev(a)
    bb = dev(bb0)
    s.step_vjp(dev(q), dt, qb, bb)
    assert np.all(field_rel_err(host(qb), qb_ref) <= F64_TOL)
    assert rel(host(bb) - bb0, bb_ref) <= 1e-11


@pytest.mark.parametrize("shape", [(4, 4), (5, 7), (33, 17)])
@pytest.mark.parametrize("ty", [8, 16, 24])
@pytest.mark.parametrize("bcs", [(PER, PER), (REF, REF), (REF, PER), (PER, REF)])
def test_two_stage_reverse_on_grids_smaller_than_a_tile(shape, bcs, ty):
    """The two-stage reverse kernels where one tile covers the grid (its ring
    and its nodes past the edge are periodic images or wall copies) or spills
    over it by one node, against the oracle's RK4 VJP."""
    nx, ny = shape
    g = W.Grid(nx, ny, -1.0, 2.0, 0.5, 2.0, bcs[0], bcs[1], 9.81, 500.0)
    q, b = W.random_state(g, 5 * nx + ny, b_scale=0.05)
    q[1:4] *= 0.1
    rng = np.random.default_rng(nx * ny)
    a = rng.standard_normal(q.shape)
    bb0 = rng.standard_normal(b.shape)
    dt = 0.2 * oracle.cfl_dt(g, q, 0.5)
    qb_ref, bb_ref = oracle.rk4_vjp(g, q, b, dt, a)
    s = solver(g)
    s.set_tile_y(ty)
    s.set_step_path("fused")
    s.set_bathymetry(dev(b))
    qb = dev(a)
    bb = dev(bb0)
    s.step_vjp(dev(q), dt, qb, bb)
    assert np.all(field_rel_err(host(qb), qb_ref) <= F64_TOL), (shape, bcs, ty)
    assert rel(host(bb) - bb0, bb_ref) <= 1e-11


def small_gauge_case(bc=REF, nx=48, ny=20, nsteps=24):
    gp = W.gauge_problem(nx=nx, ny=ny, gauges=6, radius=3.0)
    g = W.Grid(nx, ny, 0.0, 30.0, 0.0, 10.0, bc, bc, 9.81, 500.0)
    h0 = gp.zeta0 - gp.b
    q0 = np.zeros((5, ny, nx))
    q0[0] = h0
    q0[4] = h0
    dt = oracle.cfl_dt(g, q0, 0.5)
    nodes = gp.gauges[:, 0] * nx + gp.gauges[:, 1]
    rng = np.random.default_rng(5)
    target = 1.0 + 0.02 * rng.standard_normal((nsteps, len(nodes)))
    return g, gp, dt, nodes, target


@pytest.mark.parametrize("bc", [PER, REF])
def test_gauge_loss_grad_matches_oracle(bc):
    g, gp, dt, nodes, target = small_gauge_case(bc)
    nsteps = target.shape[0]
    L_ref, gz_ref, gb_ref = oracle.gauge_loss_grad(g, gp.zeta0, gp.b, dt, nsteps, nodes, target)
    s = solver(g)
    s.set_bathymetry(dev(gp.b))
    L, gz, gb = s.gauge_loss_grad(dev(gp.zeta0), nsteps, dt, dev(nodes), dev(target), 5)
    assert abs(L - L_ref) <= 1e-12 * L_ref
    assert rel(host(gz), gz_ref) <= 1e-10
    assert rel(host(gb), gb_ref) <= 1e-10
    series = host(s.gauge_series(dev(gp.zeta0), nsteps, dt, dev(nodes)))
    assert abs(0.5 * np.sum((series - target) ** 2) - L) <= 1e-12 * L


def test_gauge_loss_grad_many_and_repeated_gauges():
    """More gauges than one pass of the gauge kernels' threads, with nodes that
    carry several gauges: the seeds of a shared node add up in gauge order."""
    g, gp, dt, _, _ = small_gauge_case(REF, 48, 20, 9)
    rng = np.random.default_rng(11)
    nodes = rng.integers(0, g.nx * g.ny, size=300)
    nodes[150:170] = nodes[0]  # one node with 21 gauges
    target = 1.0 + 0.02 * rng.standard_normal((9, len(nodes)))
    L_ref, gz_ref, gb_ref = oracle.gauge_loss_grad(g, gp.zeta0, gp.b, dt, 9, nodes, target)
    s = solver(g)
    s.set_bathymetry(dev(gp.b))
    L, gz, gb = s.gauge_loss_grad(dev(gp.zeta0), 9, dt, dev(nodes), dev(target), 3)
    assert abs(L - L_ref) <= 1e-12 * L_ref
    assert rel(host(gz), gz_ref) <= 1e-10
    assert rel(host(gb), gb_ref) <= 1e-10
    series = host(s.gauge_series(dev(gp.zeta0), 9, dt, dev(nodes)))
    assert series.shape == (9, 300) and np.array_equal(series[:, 150:170], np.repeat(series[:, :1], 20, axis=1))


@pytest.mark.parametrize("ty", [8, 16, 24])
@pytest.mark.parametrize("bc", [PER, REF])
def test_gradient_same_on_pair_and_fused_paths(bc, ty):
    """The rollout and the segment recomputation run on the context's step path,
    the reverse on the two-stage reverse kernels (fused path) or the four role
    kernels (pair path).  The pair kernels and the step kernel form the same
    states bit for bit, so the loss and the gauge series agree exactly.  The two
    reverse forms do the same arithmetic node by node, but the compiler fuses
    their multiply-adds differently (the kernels are built separately), so the
    gradients agree to rounding: one step's VJP differs by at most 2e-12
    relative per element; over these 13 steps the fields agree within 1e-11 of
    their maxima (ragged 70 x 36 grid, both tiles)."""
    g, gp, dt, nodes, target = small_gauge_case(bc, 70, 36, 13)
    outs = []
    for path in ("pairs", "fused"):
        s = solver(g)
        s.set_tile_y(ty)
        s.set_step_path(path)
        s.set_bathymetry(dev(gp.b))
        L, gz, gb = s.gauge_loss_grad(dev(gp.zeta0), 13, dt, dev(nodes), dev(target), 4)
        series = host(s.gauge_series(dev(gp.zeta0), 13, dt, dev(nodes)))
        outs.append((L, host(gz), host(gb), series))
    assert outs[0][0] == outs[1][0]
    assert np.array_equal(outs[0][3], outs[1][3])
    for a, b in zip(outs[0][1:3], outs[1][1:3]):
        assert rel(b, a) <= 1e-11


@pytest.mark.parametrize("bcs", [(PER, PER), (REF, REF), (PER, REF)])
def test_two_stage_reverse_independent_of_tile_shape(bcs):
    """The two-stage reverse kernels on 64 x 8 and on 32 x 16 tiles (different
    rings, periodic images and wall copies on a ragged grid) give the same
    cotangents bit for bit."""
    g = W.Grid(70, 45, -1.0, 2.0, 0.5, 2.0, bcs[0], bcs[1], 9.81, 500.0)
    q, b = W.random_state(g, 17, b_scale=0.05)
    q[1:4] *= 0.1
    rng = np.random.default_rng(18)
    a = rng.standard_normal(q.shape)
    bb0 = rng.standard_normal(b.shape)
    dt = 0.2 * oracle.cfl_dt(g, q, 0.5)
    outs = []
    for ty in (8, 16, 24):
        s = solver(g)
        s.set_tile_y(ty)
        s.set_bathymetry(dev(b))
        qb, bb = dev(a), dev(bb0)
        s.step_vjp(dev(q), dt, qb, bb)
        outs.append((host(qb), host(bb)))
    for o in outs[1:]:
        assert np.array_equal(outs[0][0], o[0]) and np.array_equal(outs[0][1], o[1])


@pytest.mark.parametrize("path", ["fused", "pairs"])
def test_kept_rollout_tail_does_not_change_the_gradient(path):
    """Keeping the states and stage states of the last F steps from the forward
    rollout (F = 0, 1, 5, 23, 24 of 24 steps, and a budget beyond the run)
    gives the loss and gradients of the fully recomputed sweep, bit for bit,
    with the default and with explicit checkpoint intervals."""
    g, gp, dt, nodes, target = small_gauge_case()
    state_bytes = 5 * g.nx * g.ny * 8
    results = []
    for f, every in [(0, 0), (1, 0), (5, 0), (5, 4), (23, 0), (24, 0), (40, 0), (0, 7)]:
        s = solver(g)
        s.set_step_path(path)
        s.set_bathymetry(dev(gp.b))
        s.set_adjoint_store((4 * f + 1) * state_bytes + (state_bytes - 1 if f else 0))
        loss, gz, gb = s.gauge_loss_grad(dev(gp.zeta0), len(target), dt, dev(nodes), dev(target), every)
        results.append((f, every, loss, host(gz), host(gb)))
    f0, e0, loss0, gz0, gb0 = results[0]
    for f, every, loss, gz, gb in results[1:]:
        assert loss == loss0, (f, every)
        assert np.array_equal(gz, gz0) and np.array_equal(gb, gb0), (f, every)


def test_adjoint_store_option_rejects_negative_bytes():
    g, gp, dt, nodes, target = small_gauge_case()
    s = solver(g)
    with pytest.raises(RuntimeError):
        s.set_adjoint_store(-1)


def test_checkpoint_interval_does_not_change_the_gradient():
    g, gp, dt, nodes, target = small_gauge_case(REF, 40, 16, 17)
    s = solver(g)
    s.set_bathymetry(dev(gp.b))
    outs = [s.gauge_loss_grad(dev(gp.zeta0), 17, dt, dev(nodes), dev(target), k) for k in (1, 3, 0, 17)]
    for L, gz, gb in outs[1:]:
        assert L == outs[0][0]
        assert np.array_equal(host(gz), host(outs[0][1])) and np.array_equal(host(gb), host(outs[0][2]))


def test_gradient_finite_differences_config_scale():
    """Reflecting [0,30]x[0,10], 1024^2, 2000 steps, 16 gauges: directional derivatives of the
    GPU loss by central differences agree with the adjoint gradient within 1e-6."""
    gp = W.gauge_problem(1024, seed=5)
    g = gp.grid
    h0 = gp.zeta0 - gp.b
    q0 = np.zeros((5, g.ny, g.nx))
    q0[0] = h0
    q0[4] = h0
    dt = oracle.cfl_dt(g, q0, 0.5)
    nsteps = 2000
    nodes = dev(gp.gauges[:, 0] * g.nx + gp.gauges[:, 1])
    s = solver(g)
    s.set_bathymetry(dev(gp.target_b))
    target = s.gauge_series(dev(gp.target_zeta0), nsteps, dt, nodes)
    s.set_bathymetry(dev(gp.b))
    L, gz, gb = s.gauge_loss_grad(dev(gp.zeta0), nsteps, dt, nodes, target)
    gz, gb = host(gz), host(gb)
    X, Y = np.meshgrid(g.x_nodes(), g.y_nodes())
    rng = np.random.default_rng(77)

    def loss(z, b):
        s.set_bathymetry(dev(b))
        ser = host(s.gauge_series(dev(z), nsteps, dt, nodes))
        return 0.5 * np.sum((ser - host(target)) ** 2)

    for k in range(4):
        cx, cy, sig = rng.uniform(8, 22), rng.uniform(2, 8), rng.uniform(1.0, 3.0)
        bump = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * sig * sig))
        dz, db = (bump, 0 * bump) if k % 2 == 0 else (0 * bump, bump)
        e = 1e-4
        fd = (loss(gp.zeta0 + e * dz, gp.b + e * db) - loss(gp.zeta0 - e * dz, gp.b - e * db)) / (2 * e)
        ad = np.sum(gz * dz) + np.sum(gb * db)
        assert abs(ad - fd) <= 1e-6 * max(abs(fd), 1e-3 * L), (k, ad, fd)


def test_autograd_function():
    g, gp, dt, nodes, target = small_gauge_case(REF, 40, 16, 12)
    s = solver(g)
    z = dev(gp.zeta0).requires_grad_(True)
    b = dev(gp.b).requires_grad_(True)
    L = gauge_misfit_loss(z, b, s, 12, dt, dev(nodes), dev(target))
    (3.0 * L).backward()
    L2, gz, gb = s.gauge_loss_grad(dev(gp.zeta0), 12, dt, dev(nodes), dev(target))
    assert abs(float(L.detach()) - L2) <= 1e-14 * L2
    assert torch.allclose(z.grad, 3.0 * gz, rtol=1e-14, atol=0) and torch.allclose(b.grad, 3.0 * gb, rtol=1e-14, atol=0)
