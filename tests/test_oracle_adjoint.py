"""Pins for the oracle's discrete adjoint.

rhs_vjp, rk4_vjp -> dot-product tests <J^T a, v> = <a, J v> with J v from the
                    complex step (exact to rounding), for state and bathymetry
                    directions, both boundary types, lambda in {0, 500}
gauge_loss_grad  -> directional derivatives of the loss by the complex step
                    through the whole rollout (initialization included)
"""

import numpy as np
import pytest

import oracle
from paper_2601_02540_amd import workloads as W

PER, REF = W.PERIODIC, W.REFLECTING


@pytest.mark.parametrize("bcs", [(PER, PER), (REF, REF), (PER, REF)])
@pytest.mark.parametrize("lam", [0.0, 500.0])
def test_rhs_vjp_dot_product(bcs, lam):
    g = W.Grid(9, 7, -1.0, 2.0, 0.5, 2.0, bcs[0], bcs[1], 9.81, lam)
    q, b = W.random_state(g, 41)
    rng = np.random.default_rng(42)
    a = rng.standard_normal(q.shape)
    v = rng.standard_normal(q.shape)
    vb = rng.standard_normal(b.shape)
    Jv = oracle.rhs_jvp(g, q, b, v, vb)
    qb, bb = oracle.rhs_vjp(g, q, b, a)
    lhs = np.sum(a * Jv)
    rhs = np.sum(qb * v) + np.sum(bb * vb)
    assert abs(lhs - rhs) <= 1e-12 * (np.sum(np.abs(a * Jv)) + 1.0), (lhs, rhs)


def test_rhs_vjp_columns_match_dense_jacobian():
    """Every column of J^T (VJP of unit cotangents) equals a row of the dense complex-step Jacobian."""
    g = W.Grid(5, 4, 0.0, 1.0, 0.0, 1.0, REF, PER, 9.81, 500.0)
    q, b = W.random_state(g, 43)
    n = q.size
    J = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        J[:, k] = oracle.rhs_jvp(g, q, b, e.reshape(q.shape)).ravel()
    for k in range(0, n, 7):
        e = np.zeros(n)
        e[k] = 1.0
        qb, _ = oracle.rhs_vjp(g, q, b, e.reshape(q.shape))
        np.testing.assert_allclose(qb.ravel(), J[k, :], rtol=1e-12, atol=1e-12 * np.abs(J).max())


@pytest.mark.parametrize("bc", [PER, REF])
def test_rk4_vjp_dot_product(bc):
    g = W.Grid(8, 6, -1.0, 2.0, 0.5, 2.0, bc, bc, 9.81, 500.0)
    q, b = W.random_state(g, 44)
    q[1:4] *= 0.1
    rng = np.random.default_rng(45)
    a = rng.standard_normal(q.shape)
    v = rng.standard_normal(q.shape)
    vb = rng.standard_normal(b.shape)
    dt = 1e-3
    Jv = oracle.rk4_jvp(g, q, b, dt, v, vb)
    qb, bb = oracle.rk4_vjp(g, q, b, dt, a)
    lhs = np.sum(a * Jv)
    rhs = np.sum(qb * v) + np.sum(bb * vb)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(a * Jv)), (lhs, rhs)


@pytest.mark.parametrize("bc", [PER, REF])
def test_gauge_loss_gradient_matches_complex_step(bc):
    gp = W.gauge_problem(nx=14, ny=10, gauges=4, radius=3.0)
    g = W.Grid(14, 10, 0.0, 30.0, 0.0, 10.0, bc, bc, 9.81, 500.0)
    nsteps = 6
    dt = 0.02
    rng = np.random.default_rng(46)
    target = 1.0 + 0.01 * rng.standard_normal((nsteps, len(gp.gauges)))
    nodes = gp.gauges[:, 0] * g.nx + gp.gauges[:, 1]
    L, gz, gb = oracle.gauge_loss_grad(g, gp.zeta0, gp.b, dt, nsteps, nodes, target)
    for k in range(3):
        dz = rng.standard_normal(g.shape)
        db = rng.standard_normal(g.shape)
        L2, dL = oracle.gauge_loss(g, gp.zeta0, gp.b, dt, nsteps, nodes, target, dz, db)
        assert abs(L2 - L) <= 1e-13 * L
        got = np.sum(gz * dz) + np.sum(gb * db)
        assert abs(got - dL) <= 1e-11 * (abs(dL) + 1e-300), (got, dL)
