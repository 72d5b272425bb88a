"""Seeded synthetic inputs for the 2D hyperbolized SGN solver.

This module only *generates inputs*: grids, bathymetries, initial surfaces and
velocities, ensembles and gauge layouts.  It holds none of the method's
arithmetic (no derivative operator, no right-hand side, no time stepping, no
auxiliary-variable initialization), so the HIP path and the test oracle can both
start from the same arrays without sharing any of the computation.

All arrays are float64 numpy arrays in the layout of the C ABI: a state is
``(5, ny, nx)`` holding ``[h, u, v, w, eta]``; the bathymetry is ``(ny, nx)``.
The auxiliary planes ``w`` and ``eta`` are returned as zeros; the caller fills
them with its own initialization (paper eq. (initialization), Section 6).

Node placement (a reading of Section 2.2, where the general grid definition and
the periodic mass matrix disagree): a periodic axis of length ``L`` with ``N``
nodes has spacing ``L/N`` and excludes the right end point; a reflecting axis
has spacing ``L/(N-1)`` and includes both end points.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

PERIODIC = 0
REFLECTING = 1


@dataclasses.dataclass(frozen=True)
class Grid:
    """Grid, boundary types and physical parameters of one problem."""

    nx: int
    ny: int
    xmin: float
    xmax: float
    ymin: float
    ymax: float
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    g: float = 9.81
    lam: float = 500.0

    @property
    def shape(self) -> Tuple[int, int]:
        return (self.ny, self.nx)

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def x_nodes(self) -> np.ndarray:
        return _nodes(self.nx, self.xmin, self.xmax, self.bc_x)

    def y_nodes(self) -> np.ndarray:
        return _nodes(self.ny, self.ymin, self.ymax, self.bc_y)

    def spacing(self) -> Tuple[float, float]:
        return (_spacing(self.nx, self.xmin, self.xmax, self.bc_x),
                _spacing(self.ny, self.ymin, self.ymax, self.bc_y))


def _spacing(n: int, lo: float, hi: float, bc: int) -> float:
    return (hi - lo) / n if bc == PERIODIC else (hi - lo) / (n - 1)


def _nodes(n: int, lo: float, hi: float, bc: int) -> np.ndarray:
    return lo + np.arange(n, dtype=np.float64) * _spacing(n, lo, hi, bc)


@dataclasses.dataclass
class Problem:
    """A grid plus initial data: ``q0`` (5, ny, nx) with w = eta = 0, and ``b``."""

    grid: Grid
    q0: np.ndarray
    b: np.ndarray
    name: str = ""
    seed: Optional[int] = None


def _empty_state(grid: Grid) -> np.ndarray:
    return np.zeros((5, grid.ny, grid.nx), dtype=np.float64)


def _mesh(grid: Grid) -> Tuple[np.ndarray, np.ndarray]:
    X, Y = np.meshgrid(grid.x_nodes(), grid.y_nodes(), indexing="xy")
    return X, Y


def gaussian_sum_bathymetry(grid: Grid, rng: np.random.Generator, count: int = 8,
                            centre_box: Optional[Tuple[float, float, float, float]] = None,
                            sigma_range: Tuple[float, float] = (0.5, 2.0),
                            peak: float = 0.3) -> np.ndarray:
    """Sum of ``count`` Gaussians exp(-r^2/(2 sigma^2)) rescaled so that max b = peak."""
    X, Y = _mesh(grid)
    if centre_box is None:
        centre_box = (grid.xmin, grid.xmax, grid.ymin, grid.ymax)
    x0, x1, y0, y1 = centre_box
    S = np.zeros(grid.shape)
    for _ in range(count):
        cx = rng.uniform(x0, x1)
        cy = rng.uniform(y0, y1)
        sig = rng.uniform(*sigma_range)
        amp = rng.uniform(0.0, 1.0)
        S += amp * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * sig * sig))
    return peak * S / S.max()


def random_phase_bathymetry(grid: Grid, rng: np.random.Generator, amp: float = 0.2,
                            kmax: int = 8) -> np.ndarray:
    """b = amp * S / max|S|, S = sum_{(m,n) != 0, |m|,|n| <= kmax} (m^2+n^2)^-1 cos(2 pi (m x / Lx + n y / Ly) + phi_mn).

    Integer wave numbers make b periodic on the square domain.
    """
    Lx = grid.xmax - grid.xmin
    Ly = grid.ymax - grid.ymin
    ks = np.arange(-kmax, kmax + 1)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=(ks.size, ks.size))
    m2 = ks[None, :] ** 2 + ks[:, None] ** 2
    coef = np.where(m2 > 0, 1.0 / np.maximum(m2, 1), 0.0) * np.exp(1j * phi)  # [n, m]
    Ex = np.exp(2j * math.pi * np.outer(ks, grid.x_nodes() - grid.xmin) / Lx)  # [m, i]
    Ey = np.exp(2j * math.pi * np.outer(ks, grid.y_nodes() - grid.ymin) / Ly)  # [n, j]
    S = np.real(Ey.T @ coef @ Ex)
    return amp * S / np.abs(S).max()


def gaussian_bump(grid: Grid, cx: float, cy: float, amp: float = 0.1, width: float = 5.0) -> np.ndarray:
    X, Y = _mesh(grid)
    return amp * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * width * width))


def classical_soliton(x: np.ndarray, t: float, amp: float, h_inf: float = 1.0, g: float = 9.81,
                      x0: float = 0.0) -> Tuple[np.ndarray, np.ndarray]:
    """Closed-form solitary wave of the classical SGN equations (Section 5):
    h = h_inf (1 + eps sech^2(kappa (x - x0 - C t))), u = C (1 - h_inf/h),
    kappa^2 = 3 eps / (4 h_inf^2 (1 + eps)), C^2 = g h_inf (1 + eps), eps = amp/h_inf.
    """
    eps = amp / h_inf
    kappa = math.sqrt(3.0 * eps / (4.0 * h_inf * h_inf * (1.0 + eps)))
    C = math.sqrt(g * h_inf * (1.0 + eps))
    s = 1.0 / np.cosh(kappa * (x - x0 - C * t))
    h = h_inf * (1.0 + eps * s * s)
    u = C * (1.0 - h_inf / h)
    return h, u


def soliton_speed(amp: float, h_inf: float = 1.0, g: float = 9.81) -> float:
    return math.sqrt(g * h_inf * (1.0 + amp / h_inf))


# ---------------------------------------------------------------------------
# The five workloads.

def gaussian_bump_periodic(n: int = 64, seed: int = 1, lam: float = 500.0) -> Problem:
    """Periodic square [-50,50]^2, flat bottom at depth 1, Gaussian surface bump
    (amplitude 0.1, width 5) at a seeded centre in [-10,10]^2, zero velocity."""
    grid = Grid(n, n, -50.0, 50.0, -50.0, 50.0, PERIODIC, PERIODIC, 9.81, lam)
    rng = np.random.default_rng(seed)
    cx, cy = rng.uniform(-10.0, 10.0, size=2)
    q = _empty_state(grid)
    b = np.zeros(grid.shape)
    q[0] = 1.0 + gaussian_bump(grid, cx, cy)
    return Problem(grid, q, b, f"gaussian_bump_periodic_{n}", seed)


def soliton_over_bathymetry(n: int = 512, seed: int = 2, amp: float = 0.2, x0: float = 10.0,
                            lam: float = 500.0) -> Problem:
    """Reflecting walls on [0,30]x[0,10]; bathymetry = 8 seeded Gaussians scaled to max 0.3
    under a still-water level of 1; classical solitary wave of amplitude ``amp`` at x0
    moving in +x: surface zeta = 1 + A sech^2, h = zeta - b, u from the closed form."""
    grid = Grid(n, n, 0.0, 30.0, 0.0, 10.0, REFLECTING, REFLECTING, 9.81, lam)
    rng = np.random.default_rng(seed)
    b = gaussian_sum_bathymetry(grid, rng)
    X, _ = _mesh(grid)
    zeta, u = classical_soliton(X, 0.0, amp, 1.0, grid.g, x0)
    q = _empty_state(grid)
    q[0] = zeta - b
    q[1] = u
    return Problem(grid, q, b, f"soliton_over_bathymetry_{n}", seed)


def random_phase_large(n: int = 4096, bc: int = PERIODIC, seed: int = 3, lam: float = 500.0) -> Problem:
    """[-50,50]^2 with random-phase bathymetry (amplitude 0.2) under a still-water level of 1,
    a Gaussian surface bump (0.1, width 5) at a seeded centre, zero velocity."""
    grid = Grid(n, n, -50.0, 50.0, -50.0, 50.0, bc, bc, 9.81, lam)
    rng = np.random.default_rng(seed)
    b = random_phase_bathymetry(grid, rng)
    cx, cy = rng.uniform(-10.0, 10.0, size=2)
    q = _empty_state(grid)
    q[0] = 1.0 + gaussian_bump(grid, cx, cy) - b
    return Problem(grid, q, b, f"random_phase_{'periodic' if bc == PERIODIC else 'reflecting'}_{n}", seed)


def ensemble(count: int = 256, seed: int = 4, sizes=(128, 256, 512, 1024), lam: float = 500.0) -> List[Problem]:
    """Ensemble of square problems on [-50,50]^2 with seeded sizes drawn from ``sizes``,
    seeded boundary type (both axes alike), 8-Gaussian bathymetry (max 0.3) and a
    Gaussian surface bump."""
    master = np.random.default_rng(seed)
    out = []
    for k in range(count):
        sub = int(master.integers(0, 2**62))
        rng = np.random.default_rng(sub)
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        bc = int(rng.integers(0, 2))
        grid = Grid(n, n, -50.0, 50.0, -50.0, 50.0, bc, bc, 9.81, lam)
        b = gaussian_sum_bathymetry(grid, rng, 8, (-40.0, 40.0, -40.0, 40.0), (2.0, 6.0), 0.3)
        cx, cy = rng.uniform(-10.0, 10.0, size=2)
        q = _empty_state(grid)
        q[0] = 1.0 + gaussian_bump(grid, cx, cy) - b
        out.append(Problem(grid, q, b, f"ensemble_{k}_{n}_{'p' if bc == 0 else 'r'}", sub))
    return out



# ---------------------------------------------------------------------------
# Two of the paper's own setups (their initial conditions are given in full).

def gaussian_obstacle(nx: int = 1600, ny: Optional[int] = None, lam: float = 500.0, bc: int = PERIODIC) -> Problem:
    """Solitary wave over a Gaussian obstacle (Section "Solitary Wave over a Gaussian
    Obstacle"): periodic [-5,35] x [-10,10], bathymetry b = 0.1 exp(-(x^2+y^2)/2), still
    depth 0.2, a solitary wave of amplitude 0.0365 with its crest at x = -3 moving in +x
    (surface from the classical closed form, h = zeta - b, u from the closed form, v = 0).
    The paper's spacing 0.025 is nx = 1600, ny = 800; its scaling study uses nx = 2^n,
    ny = nx/2 (square cells).  bc: both axes periodic (the setup) or reflecting (the
    paper's semi-discrete energy check runs both)."""
    ny = nx // 2 if ny is None else ny
    grid = Grid(nx, ny, -5.0, 35.0, -10.0, 10.0, bc, bc, 9.81, lam)
    X, Y = _mesh(grid)
    b = 0.1 * np.exp(-(X * X + Y * Y) / 2.0)
    zeta, u = classical_soliton(X, 0.0, 0.0365, 0.2, grid.g, -3.0)
    q = _empty_state(grid)
    q[0] = zeta - b
    q[1] = u
    return Problem(grid, q, b, f"gaussian_obstacle_{nx}x{ny}", 0)


def cylindrical_dam_break(n: int = 10000, half_width: float = 1100.0, lam: float = 500.0) -> Problem:
    """Smoothed cylindrical dam break (Section "Dam Break Problems"; the long-term run
    uses [-1100,1100]^2 at spacing 0.22, i.e. 10000^2 nodes): reflecting walls, flat
    bottom, h = 1 + 0.4 (1 - tanh((r - 20)/6.5)), zero velocity."""
    grid = Grid(n, n, -half_width, half_width, -half_width, half_width, REFLECTING, REFLECTING, 9.81, lam)
    x, y = grid.x_nodes(), grid.y_nodes()
    q = np.zeros((5, n, n))
    for j0 in range(0, n, 1024):  # row blocks keep the temporaries small at 10^8 nodes
        yy = y[j0:j0 + 1024, None]
        r = np.sqrt(x[None, :] ** 2 + yy ** 2)
        q[0, j0:j0 + 1024] = 1.0 + 0.4 * (1.0 - np.tanh((r - 20.0) / 6.5))
    return Problem(grid, q, np.zeros((n, n)), f"cylindrical_dam_break_{n}", 0)

@dataclasses.dataclass
class GaugeProblem:
    """Initial surface zeta0 and bathymetry b (the two parameters), gauge node indices,
    and the seeds of the run and of the target run."""

    grid: Grid
    zeta0: np.ndarray
    b: np.ndarray
    gauges: np.ndarray  # (G, 2) int: (j, i)
    target_zeta0: np.ndarray
    target_b: np.ndarray


def gauge_problem(n: int = 1024, seed: int = 5, gauges: int = 16, radius: float = 4.0,
                  lam: float = 500.0, nx: Optional[int] = None, ny: Optional[int] = None) -> GaugeProblem:
    """Reflecting [0,30]x[0,10]; surface zeta0 = 1 + 0.1 exp(-r^2/(2*2^2)) around a seeded
    centre in [10,20]x[3,7]; bathymetry as the solitary-wave workload; gauges snapped to
    nodes, uniform in a disc of the given radius around the centre.  The target run uses
    another bathymetry seed and a shifted centre."""
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    grid = Grid(nx, ny, 0.0, 30.0, 0.0, 10.0, REFLECTING, REFLECTING, 9.81, lam)
    rng = np.random.default_rng(seed)
    b = gaussian_sum_bathymetry(grid, rng)
    cx = rng.uniform(10.0, 20.0)
    cy = rng.uniform(3.0, 7.0)
    X, Y = _mesh(grid)
    zeta0 = 1.0 + 0.1 * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * 2.0 * 2.0))
    xs, ys = grid.x_nodes(), grid.y_nodes()
    g_idx = []
    while len(g_idx) < gauges:
        rr = radius * math.sqrt(rng.uniform())
        th = rng.uniform(0.0, 2.0 * math.pi)
        gx, gy = cx + rr * math.cos(th), cy + rr * math.sin(th)
        i = int(np.argmin(np.abs(xs - gx)))
        j = int(np.argmin(np.abs(ys - gy)))
        if (j, i) not in g_idx:
            g_idx.append((j, i))
    trng = np.random.default_rng(seed + 1000)
    tb = gaussian_sum_bathymetry(grid, trng)
    tcx, tcy = cx + trng.uniform(-1.0, 1.0), cy + trng.uniform(-1.0, 1.0)
    tzeta0 = 1.0 + 0.1 * np.exp(-((X - tcx) ** 2 + (Y - tcy) ** 2) / (2.0 * 2.0 * 2.0))
    return GaugeProblem(grid, zeta0, b, np.array(g_idx, dtype=np.int64), tzeta0, tb)


def random_state(grid: Grid, seed: int, b_scale: float = 0.3) -> Tuple[np.ndarray, np.ndarray]:
    """A random positive state for property tests: h, eta ~ U[0.5,1.5]; u, v, w ~ N(0,1);
    b ~ b_scale N(0,1).  Used to check identities that hold for any state with h > 0."""
    rng = np.random.default_rng(seed)
    q = np.empty((5, grid.ny, grid.nx))
    q[0] = rng.uniform(0.5, 1.5, grid.shape)
    q[1] = rng.standard_normal(grid.shape)
    q[2] = rng.standard_normal(grid.shape)
    q[3] = rng.standard_normal(grid.shape)
    q[4] = rng.uniform(0.5, 1.5, grid.shape)
    b = b_scale * rng.standard_normal(grid.shape)
    return q, b


def mms_grid(n: int, bc: int, lam: float = 500.0) -> Grid:
    """Grid of the manufactured-solution study (Section 6.1.2): [-1,1]^2."""
    return Grid(n, n, -1.0, 1.0, -1.0, 1.0, bc, bc, 9.81, lam)


def mms_initial(grid: Grid) -> Problem:
    """Initial data of the manufactured solution at t = 0: u = v = 0,
    h = 2 + 1/2 sin(2 pi x) sin(2 pi y) - b,
    b = 0.08 (cos 2 pi x cos 2 pi y + 1/2 cos 4 pi x cos 4 pi y).  (w = 0 and eta = h at
    t = 0 follow from the printed formulas; the caller's initialization reproduces them.)"""
    X, Y = _mesh(grid)
    b = 0.08 * (np.cos(2 * math.pi * X) * np.cos(2 * math.pi * Y)
                + 0.5 * np.cos(4 * math.pi * X) * np.cos(4 * math.pi * Y))
    q = _empty_state(grid)
    q[0] = 2.0 + 0.5 * np.sin(2 * math.pi * X) * np.sin(2 * math.pi * Y) - b
    return Problem(grid, q, b, f"mms_{grid.nx}_{grid.bc_x}")


def solitary_periodic(n: int, ny: int = 4, amp: float = 0.2, lam: float = 30000.0) -> Problem:
    """1D solitary wave repeated in y (Section 6.1.1): periodic [-30,30] x [0, ny*dx]."""
    L = 60.0
    dx = L / n
    grid = Grid(n, ny, -30.0, 30.0, 0.0, ny * dx, PERIODIC, PERIODIC, 9.81, lam)
    X, _ = _mesh(grid)
    h, u = classical_soliton(X, 0.0, amp, 1.0, grid.g, 0.0)
    q = _empty_state(grid)
    q[0] = h
    q[1] = u
    return Problem(grid, q, np.zeros(grid.shape), f"solitary_{n}")
