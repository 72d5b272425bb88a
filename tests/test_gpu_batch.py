"""GPU tests of the ensemble path (sgn_batch_*): uneven grids, mixed boundaries,
one persistent launch per RK4 step (step tiles) or per stage pair (pair tiles).

Each instance must equal, bit for bit, the same problem advanced alone on the
same step path with the same tile shape (same per-tile code), and match the
FP64 oracle within 1e-12 field-relative."""

import math

import numpy as np
import pytest
import torch

import oracle
from paper_2601_02540_amd import workloads as W
from paper_2601_02540_amd.binding import Batch, SgnError, Solver
from gpu_util import STATE_FLOORS, dev, field_rel_err, host

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12


def small_ensemble(seed=7, count=10):
    rng = np.random.default_rng(seed)
    probs = []
    for k in range(count):
        n = int(rng.choice([16, 40, 64, 100, 130]))
        m = int(rng.choice([16, 40, 64, 100, 130]))
        bcx, bcy = int(rng.integers(0, 2)), int(rng.integers(0, 2))
        g = W.Grid(n, m, -5.0, 5.0, -3.0, 4.0, bcx, bcy, 9.81, 500.0)
        q, b = W.random_state(g, 100 + k, b_scale=0.05)
        q[1:4] *= 0.1
        probs.append((g, q, b))
    return probs


def run_batch(probs, dtype, dts, nsteps, tiling=None, path=None):
    batch = Batch([p[0] for p in probs], dtype)
    if path:
        batch.set_step_path(path)
    if tiling:
        batch.set_tiling(*tiling)
    qs = [dev(p[1], dtype) for p in probs]
    for i, p in enumerate(probs):
        batch.set_bathymetry(i, dev(p[2], dtype))
    batch.set_states(qs)
    batch.step(dts, nsteps)
    assert batch.check() == -1
    return batch, [host(q) for q in qs]


# (path, dtype, tile height, blocks per CU): 32 x 24 step tiles exist on the
# fused path only and run one workgroup per tile
BATCH_CASES = [(path, dtype, ty, bpc) for path in ("fused", "pairs")
               for dtype, ty in ((torch.float64, 8), (torch.float64, 16), (torch.float32, 16), (torch.float64, 24),
                                 (torch.float32, 24))
               for bpc in (0, 2) if ty != 24 or (path == "fused" and bpc == 0)]


@pytest.mark.parametrize("path,dtype,ty,bpc", BATCH_CASES)
@pytest.mark.parametrize("nsteps", [1, 2, 11])
def test_batch_equals_single_solver(path, dtype, ty, bpc, nsteps):
    """bpc 0: one workgroup per tile; 2: a persistent grid."""
    probs = small_ensemble()
    dts = [0.2 * oracle.cfl_dt(g, q, 0.5) for g, q, b in probs]
    _, outs = run_batch(probs, dtype, dts, nsteps, (ty, bpc), path)
    for (g, q, b), dt, got in zip(probs, dts, outs):
        s = Solver(g, dtype)
        s.set_step_path(path)
        s.set_tile_y(ty)
        s.set_bathymetry(dev(b, dtype))
        qd = dev(q, dtype)
        s.step(qd, dt, nsteps)
        assert np.array_equal(got, host(qd)), (g, nsteps)


@pytest.mark.parametrize("path", ["fused", "pairs"])
def test_batch_matches_oracle(path):
    probs = small_ensemble(seed=8, count=6)
    dts = [0.2 * oracle.cfl_dt(g, q, 0.5) for g, q, b in probs]
    _, outs = run_batch(probs, torch.float64, dts, 3, path=path)
    for (g, q, b), dt, got in zip(probs, dts, outs):
        ref = oracle.rk4(g, q, b, dt, 3)
        err = field_rel_err(got, ref, STATE_FLOORS)
        assert np.all(err <= F64_TOL), (g, err)


def test_batch_paths_agree_bitwise():
    """The step tiles and the pair tiles form the same values."""
    probs = small_ensemble(seed=12, count=7)
    dts = [0.2 * oracle.cfl_dt(g, q, 0.5) for g, q, b in probs]
    _, a = run_batch(probs, torch.float64, dts, 5, path="fused")
    _, b = run_batch(probs, torch.float64, dts, 5, path="pairs")
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_batch_autotune_reads_states_only():
    probs = small_ensemble(seed=9, count=8)
    batch = Batch([p[0] for p in probs], torch.float64)
    qs = [dev(p[1]) for p in probs]
    for i, p in enumerate(probs):
        batch.set_bathymetry(i, dev(p[2]))
    batch.set_states(qs)
    dts = [0.2 * oracle.cfl_dt(g, q, 0.5) for g, q, b in probs]
    ty, bpc, ms = batch.autotune(dts)
    assert ty in (8, 16, 24) and 0 <= bpc <= 6 and ms > 0 and (ty != 24 or bpc == 0)
    for q, p in zip(qs, probs):
        assert np.array_equal(host(q), p[1])
    batch.step(dts, 2)
    for (g, q, b), dt, qd in zip(probs, dts, qs):
        ref = oracle.rk4(g, q, b, dt, 2)
        assert np.all(field_rel_err(host(qd), ref, STATE_FLOORS) <= F64_TOL)


def test_batch_totals_cfl_init():
    probs = []
    for k, (n, bc) in enumerate([(32, 0), (48, 1), (64, 0), (20, 1)]):
        p = W.soliton_over_bathymetry(n, seed=k) if bc == 1 else W.gaussian_bump_periodic(n, seed=k)
        probs.append((p.grid, p.q0, p.b))
    batch = Batch([p[0] for p in probs], torch.float64)
    qs = [dev(p[1]) for p in probs]
    for i, p in enumerate(probs):
        batch.set_bathymetry(i, dev(p[2]))
    batch.set_states(qs)
    batch.init_aux()
    inits = [oracle.init_aux(g, q, b) for g, q, b in probs]
    for qd, ref in zip(qs, inits):
        assert np.all(field_rel_err(host(qd), ref, STATE_FLOORS) <= F64_TOL)
    dts = batch.cfl_dt(0.5)
    for dt, (g, q, b), q0 in zip(dts, probs, inits):
        assert math.isclose(dt, oracle.cfl_dt(g, q0, 0.5), rel_tol=1e-14)
    m, e = batch.mass_energy()
    for mi, ei, (g, q, b), q0 in zip(m, e, probs, inits):
        mo, eo = oracle.mass_energy(g, q0, b)
        assert math.isclose(mi, mo, rel_tol=1e-13) and math.isclose(ei, eo, rel_tol=1e-13)


def test_batch_flags_name_the_instance():
    probs = small_ensemble(seed=10, count=5)
    probs[3][1][0, 2, 2] = -1.0
    batch = Batch([p[0] for p in probs], torch.float64)
    qs = [dev(p[1]) for p in probs]
    for i, p in enumerate(probs):
        batch.set_bathymetry(i, dev(p[2]))
    batch.set_states(qs)
    batch.step([1e-6] * 5, 2)
    with pytest.raises(SgnError) as ei:
        batch.check()
    assert ei.value.status == -5 and "instance 3" in str(ei.value)
    assert batch.check() == -1


def test_batch_rejects_bad_input():
    g = W.Grid(16, 16, 0.0, 1.0, 0.0, 1.0)
    with pytest.raises(SgnError):
        Batch([g, W.Grid(3, 16, 0.0, 1.0, 0.0, 1.0)])
    batch = Batch([g, g])
    with pytest.raises(SgnError):  # bathymetry not set
        batch.step([1e-3, 1e-3], 1)
    with pytest.raises(SgnError):  # no batch kernel for the four-stage path
        batch.set_step_path("stages")
