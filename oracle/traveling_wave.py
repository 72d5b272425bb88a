"""TEST INFRASTRUCTURE ONLY: solitary waves of the SGN equations and of their
hyperbolization, as reference solutions.

Only ``tests/`` may import this module; the product never does.

* ``classical_soliton``: the closed-form solitary wave of the original SGN
  equations (Section "Computing Solitary Waves Numerically",
  eq. (solitary_wave_analytical) with the parameters of
  eq. (solitary_wave_parameters)).
* ``hyperbolic_soliton``: a traveling wave of the hyperbolized system, which has
  no closed form.  Following the same section: with the ansatz q(x - c t) on a
  flat bottom, the one-dimensional equations integrate (integration constants
  of the undisturbed state h = eta = h_inf, u = w = 0) to
    h u = c (h - h_inf),          w = -c h_inf eta' / h,
  and to two equations for (h, eta), taken in the better-conditioned form of
  eq. (solitary_wave_system), with beta = lambda / (c^2 h_inf^2):
    -h + eta'' / beta + eta = h' eta' / (beta h),
    eta / 3 = c^2 h_inf / lambda (1 - h_inf / h) - g h^2 / (2 lambda)
              + eta^2 / (3 h) + g h_inf^2 / (2 lambda).
  They are discretized by Fourier collocation on a periodic interval and solved
  from the classical soliton (h = eta) as the initial guess.

Reading: the paper solves the collocation system with a trust-region method.
Here Newton's method with a backtracking line search is used on the subspace of
profiles even about the wave crest: the system is symmetric under x -> -x, so
the even solution is a solution of the full system, and fixing the crest removes
the translation invariance that makes the full Jacobian singular.  Any
convergent solver reaches the same discrete solution (residual below 1e-12).

Pins (tests/test_oracle_traveling_wave.py): the residual; the distance to the
classical soliton falling as 1/lambda (the paper's observation, against the
closed form); consistency with the oracle's semi-discretization (its
right-hand side at the wave equals -c q_x to second order in the grid spacing);
second-order convergence of the oracle's RK4 solution over one traversal of the
domain, for propagation in x and in y.
"""

from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache

import numpy as np


def soliton_parameters(h_inf: float, A: float, g: float):
    """(epsilon, kappa, C) of eq. (solitary_wave_parameters)."""
    eps = A / h_inf
    kappa = np.sqrt(3.0 * eps / (4.0 * h_inf**2 * (1.0 + eps)))
    C = np.sqrt(g * h_inf * (1.0 + eps))
    return eps, kappa, C


def classical_soliton(x, t: float = 0.0, h_inf: float = 1.0, A: float = 0.5, g: float = 9.81, x0: float = 0.0):
    """(h, u) of the original SGN solitary wave, eq. (solitary_wave_analytical)."""
    eps, kappa, C = soliton_parameters(h_inf, A, g)
    h = h_inf * (1.0 + eps / np.cosh(kappa * (np.asarray(x, dtype=np.float64) - x0 - C * t)) ** 2)
    u = C * (1.0 - h_inf / h)
    return h, u


def fourier_matrices(N: int, L: float):
    """Dense first and second derivative matrices of Fourier collocation on N
    equispaced points of a period L (the unmatched Nyquist mode is dropped from
    the first derivative)."""
    k = 2.0 * np.pi * np.fft.fftfreq(N, d=L / N)
    k1 = k.copy()
    if N % 2 == 0:
        k1[N // 2] = 0.0
    I = np.eye(N)
    FI = np.fft.fft(I, axis=0)
    D1 = np.real(np.fft.ifft(1j * k1[:, None] * FI, axis=0))
    D2 = np.real(np.fft.ifft(-(k**2)[:, None] * FI, axis=0))
    return D1, D2


@dataclass(frozen=True)
class TravelingWave:
    """Profile on x_k = x0 + k L / N (crest at the centre of the interval)."""

    x: np.ndarray
    h: np.ndarray
    eta: np.ndarray
    u: np.ndarray
    w: np.ndarray
    c: float
    lam: float
    h_inf: float
    g: float
    L: float
    residual: float
    iterations: int

    def fields(self):
        return {"h": self.h, "u": self.u, "w": self.w, "eta": self.eta}


def _residual(h, e, D1, D2, c, h_inf, g, lam):
    beta = lam / (c**2 * h_inf**2)
    hx, ex = D1 @ h, D1 @ e
    r1 = -h + (D2 @ e) / beta + e - hx * ex / (beta * h)
    r2 = (e / 3.0 - c**2 * h_inf / lam * (1.0 - h_inf / h) + g / (2.0 * lam) * h**2 - e**2 / (3.0 * h)
          - g * h_inf**2 / (2.0 * lam))
    return np.concatenate([r1, r2])


def _jacobian(h, e, D1, D2, c, h_inf, g, lam):
    N = h.size
    beta = lam / (c**2 * h_inf**2)
    hx, ex = D1 @ h, D1 @ e
    I = np.eye(N)
    J11 = -I - (ex / (beta * h))[:, None] * D1 + np.diag(hx * ex / (beta * h**2))
    J12 = D2 / beta + I - (hx / (beta * h))[:, None] * D1
    J21 = np.diag(-c**2 * h_inf**2 / (lam * h**2) + g * h / lam + e**2 / (3.0 * h**2))
    J22 = np.diag(1.0 / 3.0 - 2.0 * e / (3.0 * h))
    return np.block([[J11, J12], [J21, J22]])


@lru_cache(maxsize=16)
def hyperbolic_soliton(lam: float, L: float = 80.0, N: int = 1024, h_inf: float = 1.0, A: float = 0.5,
                       g: float = 9.81, tol: float = 1e-12, maxit: int = 50) -> TravelingWave:
    """Traveling wave of the hyperbolized system with speed c = C of
    eq. (solitary_wave_parameters), on [-L/2, L/2) with N collocation points."""
    if N % 2:
        raise ValueError("N must be even")
    _, _, c = soliton_parameters(h_inf, A, g)
    x = -0.5 * L + L * np.arange(N) / N
    D1, D2 = fourier_matrices(N, L)
    # even profiles: node k mirrors node (N - k) mod N; unknowns at k = 0..N/2
    half = N // 2 + 1
    mirror = (-np.arange(N)) % N
    E = np.zeros((N, half))
    for k in range(N):
        E[k, min(k, mirror[k])] = 1.0
    Ez = np.block([[E, np.zeros_like(E)], [np.zeros_like(E), E]])
    rows = np.concatenate([np.arange(half), N + np.arange(half)])

    h, _ = classical_soliton(x, 0.0, h_inf, A, g)
    e = h.copy()
    r = _residual(h, e, D1, D2, c, h_inf, g, lam)
    nr = np.abs(r).max()
    it = 0
    while nr > tol and it < maxit:
        J = _jacobian(h, e, D1, D2, c, h_inf, g, lam)
        dz = np.linalg.solve((J @ Ez)[rows], -r[rows])
        dh, de = E @ dz[:half], E @ dz[half:]
        a = 1.0
        while True:
            hn, en = h + a * dh, e + a * de
            if np.all(hn > 0.0):
                rn = _residual(hn, en, D1, D2, c, h_inf, g, lam)
                nrn = np.abs(rn).max()
                if nrn < nr or a < 1e-6:
                    break
            a *= 0.5
        h, e, r, nr = hn, en, rn, nrn
        it += 1
    if not nr <= tol:
        raise RuntimeError(f"traveling wave: residual {nr:.3e} after {it} iterations")
    u = c * (1.0 - h_inf / h)
    w = -c * h_inf * (D1 @ e) / h
    return TravelingWave(x, h, e, u, w, float(c), float(lam), h_inf, g, L, float(nr), it)


def sample(wave: TravelingWave, n: int) -> dict:
    """The profile at n equispaced nodes of the same interval (n divides the
    number of collocation points: the nodes are collocation points)."""
    N = wave.x.size
    if N % n:
        raise ValueError("n must divide the number of collocation points")
    s = N // n
    return {k: v[::s].copy() for k, v in wave.fields().items()}


def state_2d(wave: TravelingWave, n: int, m: int, axis: str = "x") -> np.ndarray:
    """(5, ny, nx) state of the wave propagating along `axis` (n nodes along it,
    repeated over m nodes across it); the transverse velocity is zero."""
    f = sample(wave, n)
    if axis == "x":
        q = np.zeros((5, m, n))
        for k, name in enumerate(("h", "u", None, "w", "eta")):
            if name:
                q[k] = f[name][None, :]
    elif axis == "y":
        q = np.zeros((5, n, m))
        for k, name in enumerate(("h", None, "u", "w", "eta")):
            if name:
                q[k] = f[name][:, None]
    else:
        raise ValueError("axis must be 'x' or 'y'")
    return q
