"""Two of the paper's own setups on the default step path, checked against the
oracle by exact windows (see gpu_util.check_windows) and by conservation:

* solitary wave over a Gaussian obstacle (periodic, anisotropic grid) at the
  smallest and the paper's own resolution of its scaling study;
* the long-term cylindrical dam break at its full size, 10000 x 10000 nodes
  (10^8; 4 GB per FP64 state), reflecting walls;
* the Riemann problem at the paper's size ([-600, 600], dx = 0.3, to
  t = 47.434): the mean state and the leading soliton's height against the
  values the paper prints (tests/golden/riemann_problem.txt);
* the paper's check of semi-discrete energy conservation (Section
  "Semi-Discrete Energy Conservation"): along a run of the Gaussian-obstacle
  setup, periodic and reflecting, the energy rate <d_q E, q_t>_M of the GPU's
  right-hand side stays at rounding level.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2601_02540_amd import workloads as W
from gpu_util import check_windows, dev, host, solver

pytestmark = pytest.mark.gpu

STEPS = 8


def run(p, steps=STEPS):
    g = p.grid
    q0 = oracle.init_aux(g, p.q0, p.b)
    dt = oracle.cfl_dt(g, q0, 0.5)
    s = solver(g)
    s.set_bathymetry(dev(p.b))
    qd = dev(q0)
    m0, e0 = s.mass_energy(qd)
    s.step(qd, dt, steps)
    s.check()
    m1, e1 = s.mass_energy(qd)
    got = host(qd)
    del qd, s
    torch.cuda.empty_cache()
    return q0, dt, got, (m0, e0), (m1, e1)


@pytest.mark.parametrize("nx", [1024, 1600])
def test_gaussian_obstacle(nx):
    p = W.gaussian_obstacle(nx)
    g = p.grid
    q0, dt, got, (m0, e0), (m1, e1) = run(p)
    i_obst = int(round(5.0 / g.spacing()[0]))  # x = 0
    i_wave = int(round(2.0 / g.spacing()[0]))  # x = -3, the crest
    j_mid = g.ny // 2
    windows = [(("in", j_mid - 16), ("in", i_wave - 16)), (("in", j_mid - 16), ("in", i_obst - 16)),
               (("in", g.ny - 10), ("in", g.nx - 10)), (("in", 5), ("in", i_wave))]
    check_windows(g, q0, p.b, got, dt, STEPS, windows)
    assert abs(m1 - m0) <= 1e-13 * abs(m0)
    assert abs(e1 - e0) <= 1e-9 * abs(e0)


def test_cylindrical_dam_break_full_size():
    p = W.cylindrical_dam_break(10000, 1100.0)
    g = p.grid
    q0, dt, got, (m0, e0), (m1, e1) = run(p)
    c = g.nx // 2
    front = c + int(round(20.0 / g.spacing()[0]))  # r = 20, the smoothed dam
    windows = [(("in", c - 16), ("in", c - 16)), (("in", c - 16), ("in", front - 16)),
               (("in", front - 16), ("in", front - 16)), (("wall_lo", 0), ("wall_lo", 0)),
               (("wall_hi", 0), ("in", c))]
    check_windows(g, q0, p.b, got, dt, STEPS, windows)
    assert abs(m1 - m0) <= 1e-13 * abs(m0)
    assert abs(e1 - e0) <= 1e-9 * abs(e0)


def test_riemann_problem_matches_the_paper():
    from golden_values import load
    from riemann_check import check_riemann

    G = load("riemann_problem")
    n = int(round((G["x_max"] - G["x_min"]) / G["dx"])) + 1
    g = W.Grid(n, 4, G["x_min"], G["x_max"], 0.0, 1.0, W.REFLECTING, W.PERIODIC, 9.81, G["lambda"])
    x = g.x_nodes()
    q = np.zeros((5,) + g.shape)
    q[0] = (G["h_R"] + 0.5 * (G["h_L"] - G["h_R"]) * (1.0 - np.tanh(0.5 * x)))[None, :]
    s = solver(g)
    s.set_bathymetry(dev(np.zeros(g.shape)))
    qd = dev(q)
    s.init_aux(qd)
    T = G["t_end"]
    ns = int(np.ceil(T / oracle.cfl_dt(g, host(qd), 0.5)))
    m0, _ = s.mass_energy(qd)
    s.step(qd, T / ns, ns)
    s.check()
    m1, _ = s.mass_energy(qd)
    got = host(qd)
    assert abs(m1 - m0) <= 1e-13 * abs(m0)
    plateau, hm = check_riemann(x, got[0][0], G)
    print(f"\nRiemann problem, {n} x 4 nodes, {ns} steps: h* = {plateau:.4f}, h_max = {hm:.4f}")


@pytest.mark.parametrize("bc", [W.PERIODIC, W.REFLECTING])
def test_energy_rate_stays_at_rounding_along_gaussian_obstacle_run(bc):
    p = W.gaussian_obstacle(400, bc=bc)  # spacing 0.1
    g = p.grid
    s = solver(g)
    s.set_bathymetry(dev(p.b))
    qd = dev(p.q0)
    s.init_aux(qd)
    dt = s.cfl_dt(qd, 0.5)
    rows = []
    for chunk in range(6):
        if chunk:
            s.step(qd, dt, 400)
        mr, er = s.rates(qd)
        _, _, sm, se = oracle.rates(g, host(qd), p.b)  # scales: sums of |terms| of each rate
        rows.append((chunk * 400 * dt, mr / sm, er / se))
        assert abs(mr) <= 1e-13 * sm and abs(er) <= 1e-13 * se, rows[-1]
    s.check()
    print("\n(t, mass rate / scale, energy rate / scale):", [tuple(round(v, 3) if i == 0 else float(f"{v:.2e}")
                                                               for i, v in enumerate(r)) for r in rows])
