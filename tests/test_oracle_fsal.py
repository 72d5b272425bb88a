"""Pins for the oracle's adaptive five-stage, third-order FSAL pair (the kind of
integrator of Section "Numerical Experiments": explicit, third order, five
stages, first same as last, embedded error estimator, adaptive steps with
relative and absolute tolerances 1e-6).  The paper names the method only by
citation; the coefficients are a reading of this project (see the oracle's
comments).  What pins them:

  * the order conditions of the main method (order 3) and of the embedded one
    (order 2, and not 3), evaluated from the oracle's own coefficient table,
    and the first-same-as-last row;
  * the stability polynomial the coefficients were chosen for,
    1 + z + z^2/2 + z^3/6 + z^4/31 + z^5/163, from b^T A^(k-1) 1, and the same
    polynomial seen through the whole oracle: one step scales the energy of a
    small eigenmode of the linearized operator by |R(iy)|^2;
  * observed third order in time with fixed steps, and an error estimate that
    falls as h^3 (the local error of a second-order method);
  * the controller: the run ends exactly at t_end, accepted attempts have
    err <= 1 and rejected ones err > 1, a too-large first step is rejected and
    cut by max(0.2, 0.9 err^(-1/3)), the global error follows the tolerance,
    and mass (a linear invariant) is conserved to rounding."""

import math

import numpy as np
import pytest

import oracle
from paper_2601_02540_amd import workloads as W

PER, REF = W.PERIODIC, W.REFLECTING


def test_tableau_order_conditions():
    c, A, b, bh = oracle.fsal35_tableau()
    Am, bm, cm = A[:5, :5], b[:5], c[:5]
    one = np.ones(5)
    # row sums: c_i = sum_j a_ij, the FSAL stage sits at t_{n+1}
    assert np.allclose(A.sum(axis=1), c, atol=1e-15, rtol=0)
    assert np.array_equal(A[5, :5], bm) and c[5] == 1.0 and b[5] == 0.0
    assert np.all(np.triu(A) == 0)  # explicit
    # main method, order 3
    assert abs(bm @ one - 1) < 1e-15
    assert abs(bm @ cm - 1 / 2) < 1e-15
    assert abs(bm @ cm**2 - 1 / 3) < 1e-15
    assert abs(bm @ Am @ cm - 1 / 6) < 1e-15
    # it is not fourth order (its fourth-order defect is the one chosen for stability)
    assert abs(bm @ Am @ Am @ cm - 1 / 24) > 1e-3
    # embedded method on six stages, order 2 and not 3
    assert abs(bh.sum() - 1) < 1e-15
    assert abs(bh @ c - 1 / 2) < 1e-15
    assert abs(bh @ c**2 - 1 / 3) > 1e-3


def test_stability_polynomial():
    c, A, b, bh = oracle.fsal35_tableau()
    Am, bm = A[:5, :5], b[:5]
    coef = [bm @ np.linalg.matrix_power(Am, k - 1) @ np.ones(5) for k in range(1, 6)]
    np.testing.assert_allclose(coef, [1, 1 / 2, 1 / 6, 1 / 31, 1 / 163], rtol=1e-14, atol=0)
    # stable on the imaginary axis up to |y| ~ 3.9 (classical RK4: 2.83)
    poly = np.array(coef[::-1] + [1.0])  # highest degree first
    ys = np.linspace(0, 3.9, 3901)
    assert np.all(np.abs(np.polyval(poly, 1j * ys)) <= 1 + 1e-12)
    assert abs(np.polyval(poly, 4.0j)) > 1


def smooth_problem(bc=PER, n=24):
    g = W.Grid(n, n, -10.0, 10.0, -10.0, 10.0, bc, bc, 9.81, 50.0)
    p = W.gaussian_bump_periodic(n)
    x = np.linspace(0, 2 * np.pi, n, endpoint=False)
    q = p.q0.copy()
    q[0] = 1.0 + 0.05 * np.sin(x)[None, :] * np.cos(x)[:, None]
    return g, oracle.init_aux(g, q, p.b), p.b


def test_fixed_steps_third_order_in_time():
    g, q0, b = smooth_problem()
    T = 0.2
    ref = oracle.rk4(g, q0, b, T / 512, 512)
    errs = []
    for ns in (10, 20, 40):
        q, t, na, nr, rec = oracle.fsal35(g, q0, b, 0.0, T, T / ns, adaptive=False)
        assert na == ns and nr == 0 and t == T
        errs.append(np.abs(q - ref).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all((orders > 2.8) & (orders < 3.3)), orders


def test_error_estimate_falls_as_h_cubed():
    g, q0, b = smooth_problem()
    errs = []
    for h in (0.02, 0.01, 0.005):
        _, _, _, _, rec = oracle.fsal35(g, q0, b, 0.0, h, h, adaptive=False)
        errs.append(rec[0, 1])
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all((ratios > 7.0) & (ratios < 9.0)), ratios


@pytest.mark.parametrize("y", [3.0, 3.5])
def test_energy_factor_of_a_linear_mode(y):
    """One step scales a small eigenmode of the linearized operator at rest
    (frequency w, y = w h) by R(iy), so the mode's energy changes by |R(iy)|^2
    with R the stability polynomial.  The mode is the fast (relaxation) branch
    of the linearization used by the RK4 pin: the slow branch then sits at
    y w_slow / w_fast, well inside the stability region, so no component that
    the nonlinear terms leave on it can grow; y = 3.5 is near the edge of the
    region (classical RK4 would be unstable there), where the energy change is
    large enough to stand clear of the rounding of the totals (the mode's
    energy is ~1e-9 of the total)."""
    n, h0, lam, k, eps = 32, 1.0, 500.0, 3, 3e-5
    g = W.Grid(n, 4, 0.0, 2 * math.pi, 0.0, 1.0, PER, PER, 9.81, lam)
    dx = g.spacing()[0]
    kt = math.sin(k * dx) / dx
    A = np.array([[0, -h0 * 1j * kt, 0, 0],
                  [-(g.g + lam / (3 * h0)) * 1j * kt, 0, 0, lam / (3 * h0) * 1j * kt],
                  [lam / h0**2, 0, 0, -lam / h0**2],
                  [0, 0, 1, 0]], dtype=complex)
    ev, V = np.linalg.eig(A)
    pos = [i for i in range(4) if ev[i].imag > 0]
    m = max(pos, key=lambda i: ev[i].imag)
    om, v = ev[m].imag, V[:, m] / np.abs(V[:, m]).max()
    x = g.x_nodes()[None, :] * np.ones(g.shape)
    mode = [np.real(c * np.exp(1j * k * x)) for c in v]
    rest = np.zeros((5,) + g.shape)
    rest[0] = h0
    rest[4] = h0
    q = rest.copy()
    q[0] += eps * mode[0]
    q[1] = eps * mode[1]
    q[3] = eps * mode[2]
    q[4] += eps * mode[3]
    b = np.zeros(g.shape)
    _, e_rest = oracle.mass_energy(g, rest, b)
    _, e0 = oracle.mass_energy(g, q, b)
    q1, _, na, _, _ = oracle.fsal35(g, q, b, 0.0, y / om, y / om, adaptive=False)
    assert na == 1
    _, e1 = oracle.mass_energy(g, q1, b)
    R = np.polyval(np.array([1 / 163, 1 / 31, 1 / 6, 1 / 2, 1, 1]), 1j * y)
    factor = abs(R) ** 2
    got = (e1 - e_rest) / (e0 - e_rest)
    assert abs(got - factor) <= 1e-3 * abs(1 - factor), (got, factor)


@pytest.mark.parametrize("bc", [PER, REF])
def test_adaptive_run_controls_error_and_conserves_mass(bc):
    g, q0, b = smooth_problem(bc)
    T = 0.5
    ref = oracle.rk4(g, q0, b, T / 2000, 2000)
    m0, _ = oracle.mass_energy(g, q0, b)
    errs = []
    for tol in (1e-5, 1e-7):
        q, t, na, nr, rec = oracle.fsal35(g, q0, b, 0.0, T, 1e-3, rtol=tol, atol=tol)
        assert t == T and na + nr == len(rec) and na == int(rec[:, 2].sum())
        acc = rec[:, 2] == 1
        assert np.all(rec[acc, 1] <= 1.0) and np.all(rec[~acc, 1] > 1.0)
        assert abs(rec[acc, 0].sum() - T) <= 1e-14 * T
        errs.append(np.abs(q - ref).max())
        m1, _ = oracle.mass_energy(g, q, b)
        assert abs(m1 - m0) <= 1e-13 * abs(m0)
    # a hundred times smaller tolerance: a much smaller error (local error ~ tol)
    assert errs[1] < errs[0] / 10, errs
    assert errs[0] < 1e-3


def test_too_large_first_step_is_rejected_and_cut():
    g, q0, b = smooth_problem()
    dt_cfl = oracle.cfl_dt(g, q0, 0.5)
    q, t, na, nr, rec = oracle.fsal35(g, q0, b, 0.0, 40 * dt_cfl, 20 * dt_cfl)
    assert t == 40 * dt_cfl and nr >= 1
    assert rec[0, 2] == 0 and rec[0, 1] > 1
    assert math.isclose(rec[1, 0], rec[0, 0] * max(0.2, 0.9 * rec[0, 1] ** (-1 / 3)), rel_tol=1e-14)
    # once accepted, the step settles near the stability limit instead of shrinking further
    acc = rec[rec[:, 2] == 1]
    assert acc[:, 0].max() > 0.5 * dt_cfl
